"""The triangular-lattice Heisenberg model J sum S_i.S_j (Sec. 6.2.2's
model family: XX, YY and ZZ parts on horizontal, vertical and diagonal bonds)
through the C interface.

Small lattices: parity with the FP64 oracle, matvec at every node and sweep
energies.  The 16 x 16 lattice at m = 96 (64 gates; 1.1 TFLOP per H_eff
application at its heaviest node) is beyond the oracle in a test's time
(minutes of set-up and 45 s per matvec on the host), so at that size the test
checks what holds at any size: H_eff symmetric and linear, the FP32 and split
BF16 forms within their rounding bounds of the FP64 path on the same input,
the low-precision eigenvalue within the perturbation bound, and sweep
energies that only go down and stay above the bond bound -3/4 J per bond."""
import numpy as np
import pytest

from problems import config_problem, make_problem
from tests.gpu_util import make_pair, move_both, gpu_matvec, rel

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16x2": 1e-4}   # relative matvec error bounds of the forms


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _lowp_matvec(a, n, x, dtype):
    import torch
    xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda", torch.float32)
    yt = torch.empty_like(xt)
    a.heff_apply(n, xt, yt, dtype=dtype)
    torch.cuda.synchronize()
    return yt.cpu().numpy().astype(np.float64), xt.cpu().numpy().astype(np.float64)


def _n_bonds_triangular(L):
    return 2 * L * (L - 1) + (L - 1) * (L - 1)


@pytest.mark.parametrize("L,m,sweeps", [(4, 8, 3), (8, 16, 2)])
def test_heisenberg_triangular_matches_oracle(L, m, sweeps):
    p = make_problem(f"heis{L}", L, "heisenberg_tri", m, 4, L * L // 4, h=0.0)
    a, o = make_pair(p)
    rng = np.random.default_rng(1)
    for n in range(o.tree.n_nodes):
        move_both(a, o, n)
        x = rng.standard_normal(o.T[n].shape)
        r = rel(gpu_matvec(a, n, x), o.matvec(n, x))
        assert r < 1e-12, (n, o.tree.dims[n], r)
    e_a, _ = a.sweep(sweeps)
    for s in range(sweeps):
        e_o = o.sweep()
        assert abs(e_a[s] - e_o) / p.n_sites < 1e-10, (s, e_a[s], e_o)


def test_heisenberg_16x16_m96_full_size():
    from paper_2507_21236_amd import AttnHandle, ATTN_F32, ATTN_BF16X2, ATTN_F64, solver_opts
    p = config_problem("heis16_m96")
    a = AttnHandle(p)
    a.init_state()
    full = [n for n in range(a.n_nodes) if tuple(a.node_info(n)[0]) == (96, 96, 96)]
    n = max(full, key=lambda q: a.node_info(q)[2])
    a.move_center(n)
    rng = np.random.default_rng(3)
    shape = a.get_tensor(n).shape
    x, y = rng.standard_normal(shape), rng.standard_normal(shape)
    hx, hy = gpu_matvec(a, n, x), gpu_matvec(a, n, y)
    # symmetric and linear
    assert abs(np.vdot(x, hy) - np.vdot(hx, y)) / (np.linalg.norm(hx) * np.linalg.norm(y)) < 1e-14
    assert rel(gpu_matvec(a, n, 2.0 * x - 0.5 * y), 2.0 * hx - 0.5 * hy) < 1e-13
    # the low-precision forms against the FP64 path on the same rounded input
    for name, dt in (("f32", ATTN_F32), ("bf16x2", ATTN_BF16X2)):
        yl, x32 = _lowp_matvec(a, n, x, dt)
        r = rel(yl, gpu_matvec(a, n, x32))
        print(f"{name}: rel err {r:.2e}")
        assert r < TOL[name], (name, r)
    # eigenvalue of the low-precision solve from the same tensor: within the
    # matvec error times the scale of H_eff (||H x|| / ||x|| of a random x)
    scale = np.linalg.norm(hx) / np.linalg.norm(x)
    t0 = a.get_tensor(n)
    th64, _ = a.eigsolve(n, solver_opts(krylov_k=20, precision=ATTN_F64))
    e_pre = th64   # energy of the state the sweep starts from
    t64 = a.get_tensor(n)
    a.set_tensor(n, t0)
    th16, _ = a.eigsolve(n, solver_opts(krylov_k=20, precision=ATTN_BF16X2))
    print(f"theta fp64 {th64:.12f} bf16x2 {th16:.12f} scale {scale:.3f}")
    assert abs(th16 - th64) < 10 * TOL["bf16x2"] * scale
    a.set_tensor(n, t64)
    # one sweep in each precision from the same state: energies go down and
    # stay above -3/4 J per bond; the forms agree to their stated bound per site
    b = AttnHandle(p)
    b.init_state()
    b.move_center(n)
    b.set_tensor(n, t64)
    e64, _ = a.sweep(1, solver_opts(krylov_k=20, precision=ATTN_F64))
    e16, _ = b.sweep(1, solver_opts(krylov_k=20, precision=ATTN_BF16X2))
    bound = -0.75 * _n_bonds_triangular(16)
    for e in (e64[0], e16[0]):
        assert np.isfinite(e) and bound <= e <= e_pre + 1e-9, (e, e_pre, bound)
    d = abs(e16[0] - e64[0]) / p.n_sites
    print(f"sweep energy per site fp64 {e64[0] / p.n_sites:.10f} bf16x2 {e16[0] / p.n_sites:.10f} |dE|/N {d:.2e}")
    assert d < 10 * TOL["bf16x2"]
