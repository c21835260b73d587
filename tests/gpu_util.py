"""Shared helpers of the GPU parity tests (move both implementations through
the same centre path, compare results)."""
import numpy as np

from oracle.ttn import OracleTTN


def make_pair(p, **kw):
    import torch  # noqa: F401
    from paper_2507_21236_amd import AttnHandle
    a = AttnHandle(p, **kw)
    a.init_state()
    o = OracleTTN(p.n_sites, p.d, p.m, p.leaf_order, p.terms, p.de_sites, p.de_u, p.raw_tensors)
    return a, o


def leg_toward(tree, a, b):
    if tree.parent[a] == b:
        return 2
    for side in (0, 1):
        if tree.children[a][side] == ('n', b):
            return side
    raise ValueError((a, b))


def move_both(a, o, target):
    tr = o.tree
    path = tr.path(o.center, target)
    for x, y in zip(path[:-1], path[1:]):
        a.isometrize(x, y)
        a.update_env(x, leg_toward(tr, x, y))
    o.move_center(target)
    assert a.center == target == o.center


def gpu_matvec(a, n, x):
    import torch
    xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    yt = torch.empty_like(xt)
    a.heff_apply(n, xt, yt)
    torch.cuda.synchronize()
    return yt.cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
