"""Pins of the oracle's observables and disentangler optimisation
(oracle/measure.py) against definitions on the full 2^N state and against
the closed-form optimum of Sec. 4.1.1.

* expectation values of products and of rotated observables (Sec. 5.2) equal
  <phi| o |phi> with phi = D |psi_TTN> formed explicitly (N = 16);
* the correlation matrix of eq. 7 equals the dense one (N = 9);
* Gamma_k equals the derivative of the energy in the ket copy of u_k taken on
  the full state (definition of eq. 4), and the energy of the terms on the
  disentangler's sites equals the dense one for any gate;
* u = -V U^T attains Tr(u Gamma) = -sum(sigma) (eq. 5) and no orthogonal gate
  does better;
* with the energy shift, the self-consistent iteration never raises the energy;
* optimising the layer lowers the energy of the augmented state, and the
  S_TTN = 1 schedule ends below plain TTN sweeps."""
import numpy as np
import pytest

from problems import config_problem, make_problem
from problems.draws import haar_orthogonal
from problems.models import PX, PZ
from oracle.ttn import OracleTTN, full_state
from oracle.ed import hamiltonian_sparse, apply_layer, term_sparse, apply_two_site
from oracle.measure import (product_expectation, measure, correlation_matrix, de_environment_parts,
                            de_gamma, de_energy, svd_update, optimize_disentangler, optimize_layer,
                            de_terms, term_norm_bound, attn_sweeps)


def _oracle(p, sweeps=1):
    o = OracleTTN(p.n_sites, p.d, p.m, p.leaf_order, p.terms, p.de_sites, p.de_u, p.raw_tensors)
    for _ in range(sweeps):
        o.sweep()
    o.move_center(o.tree.root)
    return o


def test_product_expectation_matches_full_state():
    p = config_problem("ising4_m8")
    o = _oracle(p)
    psi = full_state(o.tree, o.T)
    rng = np.random.default_rng(1)
    for k in (1, 2, 3, 4):
        for _ in range(4):
            sites = [int(s) for s in rng.choice(16, k, replace=False)]
            ops = [rng.standard_normal((2, 2)) for _ in sites]
            ref = psi @ (term_sparse(sites, ops, 1.0, 16) @ psi)
            got = product_expectation(o.tree, o.T, dict(zip(sites, ops)))
            assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (sites, got, ref)


def test_rotated_observables_match_augmented_state():
    p = config_problem("ising4_m8")
    o = _oracle(p)
    phi = apply_layer(full_state(o.tree, o.T), p.de_sites, p.de_u, 16)
    a, b = p.de_sites[0]
    cases = [([a], [PX]), ([a, b], [PZ, PZ]), ([a, 11 if a != 11 else 3], [PX, PZ]),
             ([p.de_sites[1][0], p.de_sites[2][1]], [PZ, PX]), ([5], [PZ])]
    for sites, ops in cases:
        ref = phi @ (term_sparse(sites, ops, 1.0, 16) @ phi)
        got = measure(o.tree, o.T, sites, ops, p.de_sites, p.de_u)
        assert abs(got - ref) <= 1e-12, (sites, got, ref)


def test_correlation_matrix_matches_dense():
    p = make_problem("t", 3, "ising", 4, 11, 2, h=1.3)
    o = _oracle(p, 2)
    phi = apply_layer(full_state(o.tree, o.T), p.de_sites, p.de_u, 9)
    C = correlation_matrix(o.tree, o.T, PZ, PX, p.de_sites, p.de_u)
    for i in range(9):
        for j in range(9):
            op = term_sparse([i], [PZ @ PX], 1.0, 9) if i == j else term_sparse([i, j], [PZ, PX], 1.0, 9)
            assert abs(C[i, j] - phi @ (op @ phi)) <= 1e-12, (i, j)


def _dense_terms_energy(psi, terms, de_sites, k, u, N):
    """sum over the terms on disentangler k's sites of <psi| U^T h U |psi>, U = u on its sites."""
    a, b = de_sites[k]
    v = apply_two_site(psi, u, a, b, N)
    H = sum((term_sparse(s, ops, c, N) for s, ops, c in de_terms(terms, de_sites, k)),
            start=0 * term_sparse([0], [np.eye(2)], 1.0, N))
    return float(v @ (H @ v))


def test_gamma_is_the_derivative_of_the_energy_in_the_ket_gate():
    p = config_problem("ising4_m8")
    o = _oracle(p)
    psi = full_state(o.tree, o.T)
    rng = np.random.default_rng(3)
    for k in range(len(p.de_sites)):
        a, b = p.de_sites[k]
        parts, rho = de_environment_parts(o.tree, o.T, p.terms, p.de_sites, k)
        ut = haar_orthogonal(rng, 4)
        G = de_gamma(parts, rho, ut)
        H = sum((term_sparse(s, ops, c, 16) for s, ops, c in de_terms(p.terms, p.de_sites, k)),
                start=0 * term_sparse([0], [np.eye(2)], 1.0, 16))
        bra = apply_two_site(psi, ut, a, b, 16)      # (u~ x 1) psi
        # E_lin(u) = <psi| (u~ x 1)^T H (u x 1) |psi> = sum_ij u_ij G_ji
        for i in range(4):
            for j in range(4):
                E = np.zeros((4, 4))
                E[i, j] = 1.0
                ket = apply_two_site(psi, E, a, b, 16)
                assert abs(bra @ (H @ ket) - G[j, i]) <= 1e-12, (k, i, j)
        # the energy of the gate's terms for arbitrary orthogonal gates
        for _ in range(3):
            u = haar_orthogonal(rng, 4)
            assert abs(de_energy(parts, u) - _dense_terms_energy(psi, p.terms, p.de_sites, k, u, 16)) <= 1e-12
        assert abs(np.trace(rho) - 1.0) <= 1e-12


def test_svd_update_attains_minus_sum_of_singular_values():
    rng = np.random.default_rng(5)
    for _ in range(20):
        G = rng.standard_normal((4, 4))
        u, ssum = svd_update(G)
        assert np.allclose(u.T @ u, np.eye(4), atol=1e-13)
        assert abs(np.trace(u @ G) + ssum) <= 1e-12
        for _ in range(50):
            w = haar_orthogonal(rng, 4)
            assert np.trace(w @ G) >= -ssum - 1e-12


def test_shifted_iteration_never_raises_the_energy():
    p = config_problem("ising4_m8")
    o = _oracle(p)
    for k in range(len(p.de_sites)):
        parts, rho = de_environment_parts(o.tree, o.T, p.terms, p.de_sites, k)
        c = term_norm_bound(de_terms(p.terms, p.de_sites, k))
        u, es = optimize_disentangler(parts, rho, p.de_u[k], c, max_iter=30)
        assert np.all(np.diff(es) <= 1e-12 * max(1.0, abs(es[0]))), (k, es)
        assert np.allclose(u.T @ u, np.eye(4), atol=1e-12)


def test_layer_optimisation_lowers_the_augmented_energy():
    p = config_problem("ising4_m8")
    o = _oracle(p, 2)
    psi = full_state(o.tree, o.T)
    H = hamiltonian_sparse(p.terms, 16)
    phi0 = apply_layer(psi, p.de_sites, p.de_u, 16)
    new_u, _ = optimize_layer(o.tree, o.T, p.terms, p.de_sites, p.de_u)
    phi1 = apply_layer(psi, p.de_sites, new_u, 16)
    e0, e1 = phi0 @ (H @ phi0), phi1 @ (H @ phi1)
    assert e1 <= e0 + 1e-12
    assert e1 < e0 - 1e-6       # the random gates are far from optimal
    # the oracle's own energy after contracting the new layer agrees
    o.set_disentanglers(p.terms, p.de_sites, new_u)
    r = o.tree.root
    x = o.T[r]
    assert abs(float(np.sum(x * o.matvec(r, x))) - e1) <= 1e-10


def test_attn_schedule_beats_plain_ttn():
    # 4 x 4 Ising at h = 3, m = 4 (truncated bonds), 4 gates starting at the
    # identity: one plain sweep, then the layer optimised before every sweep
    p = make_problem("t", 4, "ising", 4, 1, 4, h=3.0, identity_de=True)
    assert len(p.de_sites) == 4
    o = OracleTTN(p.n_sites, p.d, p.m, p.leaf_order, p.terms, p.de_sites, p.de_u, p.raw_tensors)
    e_attn, u = attn_sweeps(o, p.terms, p.de_sites, p.de_u, 6, s_ttn=1)
    q = OracleTTN(p.n_sites, p.d, p.m, p.leaf_order, p.terms, p.de_sites, p.de_u, p.raw_tensors)
    e_ttn = [q.sweep() for _ in range(6)]
    print("aTTN", e_attn, "TTN", e_ttn)
    assert e_attn[0] == e_ttn[0]
    assert e_attn[-1] < e_ttn[-1] - 1e-6
    from oracle.ed import ground_energy
    assert e_attn[-1] >= ground_energy(p.terms, 16) - 1e-10


def test_riemannian_gradient_matches_finite_differences():
    from oracle.measure import de_riem_grad, cayley
    p = config_problem("ising4_m8")
    o = _oracle(p)
    parts, _ = de_environment_parts(o.tree, o.T, p.terms, p.de_sites, 0)
    rng = np.random.default_rng(7)
    u = haar_orthogonal(rng, 4)
    g = de_riem_grad(parts, u)
    assert np.abs(g + g.T).max() <= 1e-15
    for _ in range(5):
        X = rng.standard_normal((4, 4))
        X = X - X.T
        h = 1e-6
        fd = (de_energy(parts, u @ cayley(h * X)) - de_energy(parts, u @ cayley(-h * X))) / (2 * h)
        assert abs(fd - float(np.sum(g * X))) <= 1e-7 * max(1.0, abs(fd))
        assert np.abs(cayley(X).T @ cayley(X) - np.eye(4)).max() <= 1e-13


def test_rcg_reaches_a_stationary_point_without_raising_the_energy():
    from oracle.measure import optimize_disentangler_rcg, de_riem_grad
    p = config_problem("ising4_m8")
    o = _oracle(p)
    for k in range(len(p.de_sites)):
        parts, rho = de_environment_parts(o.tree, o.T, p.terms, p.de_sites, k)
        u, es = optimize_disentangler_rcg(parts, p.de_u[k], max_iter=200, rel_tol=1e-15)
        assert np.all(np.diff(es) <= 1e-13 * max(1.0, abs(es[0]))), k
        assert np.abs(u.T @ u - np.eye(4)).max() <= 1e-12
        g = de_riem_grad(parts, u)
        assert np.abs(g).max() <= 1e-5 * max(1.0, abs(es[-1])), (k, np.abs(g).max())
        # a local minimum: no small rotation lowers the energy
        rng = np.random.default_rng(k)
        from oracle.measure import cayley
        for _ in range(20):
            X = rng.standard_normal((4, 4))
            X = 1e-3 * (X - X.T)
            assert de_energy(parts, u @ cayley(X)) >= es[-1] - 1e-10
