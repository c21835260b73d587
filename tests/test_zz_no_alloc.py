"""Allocation-free model training through the C interface:
attn_mlp_train_noalloc keeps its working memory in a fixed device array of
the library instead of allocating.  Two calls in a row, the second with a
smaller input (fewer points, a smaller batch, fewer steps, so the array still
holds the larger first call's data), give the same parameters and per-step
losses as the allocating attn_mlp_train on the same inputs; sizes beyond the
array are refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _data(n, seed):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((n, 3)).astype(np.float32)
    y = (np.tanh(f[:, 0]) - 0.5 * f[:, 1] * f[:, 2]).astype(np.float32)
    return f, y


def test_noalloc_training_matches_allocating_entry_point():
    import torch
    from paper_2507_21236_amd import _lib, ATTN_MLP_PARAMS, AttnError
    w0 = (np.random.default_rng(5).standard_normal(ATTN_MLP_PARAMS) * 0.1).astype(np.float32)
    for n, steps, batch, seed in [(65536, 40, 16384, 1), (8192, 7, 1024, 2)]:
        f, y = _data(n, seed)
        ft, yt = torch.from_numpy(f).cuda(), torch.from_numpy(y).cuda()
        torch.cuda.synchronize()
        w_na, l_na = _lib.attn_mlp_train_noalloc(ft.data_ptr(), yt.data_ptr(), n, steps, batch, 1e-3, w0)
        w_ref, l_ref = _lib.attn_mlp_train(ft.data_ptr(), yt.data_ptr(), n, steps, batch, 1e-3, w0)
        print(f"n={n} steps={steps} batch={batch}: loss {l_na[0]:.4e} -> {l_na[-1]:.4e}, "
              f"max |dw| {np.abs(w_na - w_ref).max():.1e}")
        assert np.all(np.isfinite(w_na)) and l_na[-1] < l_na[0]
        assert np.array_equal(w_na, w_ref)
        assert np.array_equal(l_na, l_ref)
    f, y = _data(40000, 3)
    ft, yt = torch.from_numpy(f).cuda(), torch.from_numpy(y).cuda()
    with pytest.raises(AttnError) as e:
        _lib.attn_mlp_train_noalloc(ft.data_ptr(), yt.data_ptr(), 40000, 2, 32768, 1e-3, w0)
    assert e.value.code == -11
    with pytest.raises(AttnError) as e:
        _lib.attn_mlp_train_noalloc(ft.data_ptr(), yt.data_ptr(), 40000, 70000, 64, 1e-3, w0)
    assert e.value.code == -11
