"""Degenerate cases of the HIP path through the C interface, against closed
forms and the FP64 oracle.

At the classical Ising point h = 0 the Hamiltonian -sum ZZ is diagonal in the
product basis with a two-fold ground state of energy -(number of bonds); with
identity disentanglers the rotated Hamiltonian (Sec. 3.2) is the same, a
product state is exact at any bond dimension, and once the sweeps have found
it every centre tensor is an eigenvector of its H_eff (the projected
Hamiltonian of Sec. 3.3.2) to rounding, so the local Krylov recursion of the
eigensolver (Sec. 4.4.2) has nothing to add after its first vector."""
import numpy as np
import pytest

from problems import make_problem
from tests.gpu_util import make_pair, gpu_matvec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _bonds(L):
    return 2 * L * (L - 1)   # open square lattice


@pytest.mark.parametrize("L,m,identity", [(4, 4, False), (8, 16, True)])
def test_classical_point_reaches_bond_count(L, m, identity):
    p = make_problem(f"h0_{L}", L, "ising", m, 3 if L == 4 else 5, L * L // 4, h=0.0,
                     identity_de=identity)
    a, o = make_pair(p)
    e_a, _ = a.sweep(3)
    for s in range(3):
        e_o = o.sweep()
        assert abs(e_a[s] - e_o) / p.n_sites < 1e-10, (s, e_a[s], e_o)
        assert e_a[s] >= -_bonds(L) - 1e-9
    assert abs(e_a[-1] + _bonds(L)) < 1e-9


def test_eigsolve_at_exact_eigenvector():
    # 8 x 8, m = 16: the root is a 16 x 16 x 1 node (single-workgroup solver),
    # the nodes below it 16 x 16 x 16 (4096 entries: multi-workgroup solver)
    L = 8
    E0 = -float(_bonds(L))
    p = make_problem("h0_eig", L, "ising", 16, 5, 16, h=0.0, identity_de=True)
    from paper_2507_21236_amd import AttnHandle
    a = AttnHandle(p)
    a.init_state()
    e, _ = a.sweep(3)
    assert abs(e[-1] - E0) < 1e-9
    full = [n for n in range(a.n_nodes) if tuple(a.node_info(n)[0]) == (16, 16, 16)]
    assert full
    for n in [a.center, full[0], full[-1]]:
        a.move_center(n)
        t0 = a.get_tensor(n)
        th, _ = a.eigsolve(n)
        t1 = a.get_tensor(n)
        assert np.all(np.isfinite(t1))
        assert abs(th - E0) < 1e-9, (n, th)
        # the eigenvector is kept, up to its sign
        assert min(np.abs(t1 - t0).max(), np.abs(t1 + t0).max()) < 1e-9, n
        assert abs(np.linalg.norm(t1) - 1.0) < 1e-12
        assert np.abs(gpu_matvec(a, n, t1) - th * t1).max() < 1e-9 * abs(E0), n
