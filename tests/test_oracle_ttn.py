"""Pins for the oracle TTN: brute-force dense effective Hamiltonians, exact
diagonalisation, closed forms and invariants."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from problems import make_problem, make_chain_problem, config_problem
from oracle.ttn import OracleTTN, full_state, embedding_columns, iso_qr
from oracle.ed import ground_energy, hamiltonian_sparse, apply_layer, ising_chain_exact


def _oracle(p, **kw):
    return OracleTTN(p.n_sites, p.d, p.m, p.leaf_order, p.terms, p.de_sites, p.de_u,
                     p.raw_tensors, **kw)


def _dense_heff(o, p, n, H):
    P = embedding_columns(o, n)
    DP = np.array([apply_layer(P[:, k], p.de_sites, p.de_u, p.n_sites)
                   for k in range(P.shape[1])]).T
    return DP.T @ (H @ DP)


def _factorised_heff(o, n):
    sh = o.T[n].shape
    M = int(np.prod(sh))
    prep = o.prepare(n)
    out = np.zeros((M, M))
    for k in range(M):
        e = np.zeros(M)
        e[k] = 1.0
        out[:, k] = o.matvec(n, e.reshape(sh), prep).ravel()
    return out


def _check_all_nodes(p):
    o = _oracle(p)
    H = hamiltonian_sparse(p.terms, p.n_sites)
    for n in range(o.tree.n_nodes):
        o.move_center(n)
        Hd = _dense_heff(o, p, n, H)
        Hf = _factorised_heff(o, n)
        assert np.abs(Hf - Hd).max() < 1e-12 * max(1.0, np.abs(Hd).max()), n


def test_heff_equals_projected_hamiltonian_every_node_4x4():
    # H_eff(n) = P_n^T D^T H D P_n for every node of the 4x4, m = 8 instance
    _check_all_nodes(config_problem("ising4_m8"))


def test_heff_brute_force_relaxed_gates_uneven_tree():
    # 12-site chain (uneven split), gates on non-adjacent sites and terms
    # touching two gates (4-body rotated terms with bond up to 16)
    p = make_chain_problem("c", 12, 1.7, 8, 9, de_pairs=[(1, 3), (4, 6), (8, 10)])
    _check_all_nodes(p)


def test_heff_symmetric():
    p = config_problem("ising4_m8")
    o = _oracle(p)
    rng = np.random.default_rng(2)
    for n in (0, 6, 13, 14):
        o.move_center(n)
        sh = o.T[n].shape
        x, y = rng.standard_normal(sh), rng.standard_normal(sh)
        prep = o.prepare(n)
        a = np.vdot(x, o.matvec(n, y, prep))
        b = np.vdot(o.matvec(n, x, prep), y)
        assert abs(a - b) < 1e-12 * abs(a)


def test_untruncated_root_spectrum_is_exact():
    # m = 256 on 4x4: the tree is exact, lambda_min(H_eff(root)) = E0 of ED
    p = make_problem("u", 4, "ising", 256, 7, 4, h=3.0)
    o = _oracle(p)
    n = o.tree.root
    prep = o.prepare(n)
    sh = o.T[n].shape
    op = spla.LinearOperator((int(np.prod(sh)),) * 2,
                             matvec=lambda v: o.matvec(n, v.reshape(sh), prep).ravel())
    w = spla.eigsh(op, k=1, which='SA', tol=1e-12, return_eigenvectors=False)[0]
    assert abs(w - ground_energy(p.terms, 16)) < 1e-9


def test_initial_tensors_are_isometries():
    p = config_problem("ising8_m32")
    o = _oracle(p)
    for n in range(o.tree.n_nodes):
        ml, mr, mp = o.T[n].shape
        A = o.T[n].reshape(ml * mr, mp)
        if n == o.tree.root:
            assert abs(np.linalg.norm(A) - 1) < 1e-14
        else:
            assert np.allclose(A.T @ A, np.eye(mp), atol=1e-13)


def test_qr_moves_keep_state_and_norm():
    p = config_problem("ising4_m8")
    o = _oracle(p)
    psi0 = full_state(o.tree, o.T)
    for target in (0, 9, 5, 14, 3):
        o.move_center(target)
        psi = full_state(o.tree, o.T)
        assert np.abs(psi - psi0).max() < 1e-13
        assert abs(np.linalg.norm(psi) - np.linalg.norm(o.T[target])) < 1e-13
    Q, R = iso_qr(np.random.default_rng(0).standard_normal((12, 5)))
    assert np.allclose(Q.T @ Q, np.eye(5), atol=1e-14) and np.all(np.diag(R) >= 0)


def test_lanczos_bounds():
    p = config_problem("ising4_m8")
    o = _oracle(p)
    H = hamiltonian_sparse(p.terms, p.n_sites)
    for n in (0, 12, 14):
        o.move_center(n)
        Hd = _dense_heff(o, p, n, H)
        lam = np.linalg.eigvalsh(Hd)[0]
        v = o.T[n].ravel() / np.linalg.norm(o.T[n])
        rq = v @ Hd @ v
        theta = o.eigsolve(n)
        M = Hd.shape[0]
        assert theta >= lam - 1e-10 and theta <= rq + 1e-10
        if M <= 20:        # Krylov space is the whole space
            assert abs(theta - lam) < 1e-10
        x = o.T[n].ravel()
        assert abs(np.linalg.norm(x) - 1) < 1e-13
        assert abs(x @ Hd @ x - theta) < 1e-10


def test_sweeps_variational_and_monotone_4x4():
    p = config_problem("ising4_m8")
    o = _oracle(p)
    E0 = ground_energy(p.terms, p.n_sites)
    prev = np.inf
    H = hamiltonian_sparse(p.terms, p.n_sites)
    for s in range(5):
        e = o.sweep()
        assert e >= E0 - 1e-10 and e <= prev + 1e-10
        prev = e
    # energy of the aTTN state from the full 2^N vector
    psi = apply_layer(full_state(o.tree, o.T), p.de_sites, p.de_u, p.n_sites)
    assert abs(psi @ (H @ psi) - e) < 1e-10


def test_identity_gates_reproduce_plain_ttn():
    pa = make_problem("a", 4, "ising", 4, 21, 4, h=3.0, identity_de=True)
    pb = make_problem("b", 4, "ising", 4, 21, 0, h=3.0)
    # same raw tensor draws: the gate draws come first, so re-draw b with a's tensors
    pb.raw_tensors = pa.raw_tensors
    oa, ob = _oracle(pa), _oracle(pb)
    for s in range(3):
        assert abs(oa.sweep() - ob.sweep()) < 1e-10


def test_ising_h0_reaches_classical_energy():
    p = make_problem("h0", 4, "ising", 4, 3, 4, h=0.0)
    o = _oracle(p)
    for _ in range(3):
        e = o.sweep()
    assert abs(e + 24.0) < 1e-9


def test_chain_against_free_fermions():
    N, h = 32, 3.0
    E0 = ising_chain_exact(N, h)
    prev = np.inf
    for m in (4, 8, 16):
        o = _oracle(make_chain_problem("c", N, h, m, 5))
        for _ in range(3):
            e = o.sweep()
        assert e - E0 >= -1e-10
        assert e - E0 < prev
        prev = e - E0
    assert prev < 1e-9


def test_flop_model_matches_independent_count():
    # per-matvec flops of the full (8, 8, 8) nodes of the 4x4, m = 8 instance:
    # 1.45e-3 GFLOP, and of the heaviest full node of the 16x16, m = 64
    # instance with 64 gates: 76.6 GFLOP over 157 crossing terms (values from
    # an independent structural count of the same readings)
    o = _oracle(config_problem("ising4_m8"), structure_only=True)
    full = [n for n in range(o.tree.n_nodes) if o.tree.dims[n] == (8, 8, 8)]
    assert len(full) == 2
    assert all(abs(o.flops(n) / 1e9 - 0.00145) < 0.000005 for n in full)


@pytest.mark.slow
def test_flop_model_16x16():
    o = _oracle(config_problem("ising16_m64"), structure_only=True)
    full = [n for n in range(o.tree.n_nodes) if o.tree.dims[n] == (64, 64, 64)]
    F = sorted(o.flops(n) / 1e9 for n in full)
    assert len(full) == 30
    assert abs(F[0] - 11.5) < 0.05 and abs(F[-1] - 76.6) < 0.05
    assert max(len(o.crossing_terms(n)) for n in full) == 157
