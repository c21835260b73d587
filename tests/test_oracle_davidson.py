"""Pins for the oracle's Davidson form: the H_eff diagonal against the dense
definition P^T H' P, Davidson against dense eigensolvers (with and without
restarts), the exact Jacobi-Davidson correction against its defining equation,
the MLP gradient against finite differences, special cases of the MLP forward
and of the Adam update."""
import math

import numpy as np

from problems import config_problem, make_chain_problem
from oracle.ed import hamiltonian_sparse
from oracle.davidson import (heff_diagonal, davidson, jacobi_correction, jd_correction,
                             mlp_forward, mlp_loss_grad, mlp_unpack, adam_step, N_PARAMS,
                             mlp_correction, SHAPES)
from tests.test_oracle_ttn import _oracle, _dense_heff


def test_diagonal_equals_dense_definition():
    for p in (config_problem("ising4_m8"),
              make_chain_problem("c", 12, 1.7, 8, 9, de_pairs=[(1, 3), (4, 6), (8, 10)])):
        o = _oracle(p)
        H = hamiltonian_sparse(p.terms, p.n_sites)
        for n in range(o.tree.n_nodes):
            o.move_center(n)
            Hd = _dense_heff(o, p, n, H)
            D = heff_diagonal(o, n)
            assert D.shape == o.T[n].shape
            assert np.abs(D.ravel() - np.diag(Hd)).max() < 1e-12 * max(1.0, np.abs(Hd).max()), n


def test_davidson_reaches_dense_lowest_eigenpair():
    p = config_problem("ising4_m8")
    o = _oracle(p)
    H = hamiltonian_sparse(p.terms, p.n_sites)
    for n, (maxsub, restart) in ((14, (32, 8)), (12, (6, 3)), (0, (32, 8))):
        o.move_center(n)
        Hd = _dense_heff(o, p, n, H)
        ev, U = np.linalg.eigh(Hd)
        D = heff_diagonal(o, n).ravel()
        theta, u, nmv, hist = davidson(lambda v: Hd @ v, o.T[n].ravel(), D, tol=1e-8,
                                       maxsub=maxsub, restart=restart)
        assert hist[-1] <= 1e-8 or Hd.shape[0] <= nmv
        assert abs(theta - ev[0]) < 1e-10 * max(1.0, abs(ev[0])), (n, theta, ev[0])
        assert abs(abs(u @ U[:, 0]) - 1.0) < 1e-8
        assert np.linalg.norm(Hd @ u - theta * u) < 1e-7


def test_davidson_diagonally_dominant_converges_fast():
    # a diagonally dominant matrix: the Jacobi correction is close to the
    # inverse-shift step and Davidson converges before spanning the whole space
    rng = np.random.default_rng(0)
    d = np.sort(rng.uniform(-3.0, 5.0, 60)) + np.arange(60) * 0.1
    S = rng.standard_normal((60, 60)) * 0.01
    H = np.diag(d) + S + S.T
    ev, U = np.linalg.eigh(H)
    theta, u, nmv, hist = davidson(lambda v: H @ v, rng.standard_normal(60), np.diag(H), tol=1e-10)
    assert abs(theta - ev[0]) < 1e-12
    assert nmv < 60, nmv
    # the exact diagonal of a diagonal matrix makes the correction parallel to u
    r = d * U[:, 0] - 1.0 * U[:, 0]
    assert np.allclose(jacobi_correction(r, d, 1.0), -U[:, 0])


def test_jacobi_correction_definition_and_guard():
    r = np.array([1.0, -2.0, 3.0])
    d = np.array([2.0, 0.5, 1.0 + 1e-12])
    t = jacobi_correction(r, d, 1.0)
    assert abs(t[0] - (-1.0)) < 1e-15 and abs(t[1] - (-4.0)) < 1e-15
    assert abs(t[2]) == 3.0 / 1e-8   # |diag - theta| raised to 1e-8 max(1, |theta|)


def test_jd_correction_solves_its_equation():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((30, 30))
    H = A + A.T
    ev, U = np.linalg.eigh(H)
    u = U[:, 0] + 0.05 * rng.standard_normal(30)
    u /= np.linalg.norm(u)
    theta = float(u @ H @ u)
    r = H @ u - theta * u
    t = jd_correction(H, u, theta, r)
    P = np.eye(30) - np.outer(u, u)
    assert abs(u @ t) < 1e-12
    assert np.linalg.norm(P @ (H - theta * np.eye(30)) @ P @ t + r) < 1e-10 * np.linalg.norm(r)


def _rand_weights(rng, scale=0.3):
    return rng.standard_normal(N_PARAMS) * scale


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    w = _rand_weights(rng)
    f = rng.standard_normal((50, 3))
    y = rng.standard_normal(50)
    loss, g = mlp_loss_grad(w, f, y)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in SHAPES])
    idx = [int(rng.integers(offs[k], offs[k + 1])) for k in range(len(SHAPES))] + [N_PARAMS - 1]
    for i in idx:
        h = 1e-6
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (mlp_loss_grad(wp, f, y)[0] - mlp_loss_grad(wm, f, y)[0]) / (2 * h)
        assert abs(fd - g[i]) < 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_mlp_forward_special_cases():
    rng = np.random.default_rng(3)
    f = rng.standard_normal((7, 3))
    # zero hidden weights: output is W4 . tanh(b3) + b4 for every point
    w = np.zeros(N_PARAMS)
    p = mlp_unpack(w)           # views into w
    p["b3"][:] = rng.standard_normal(64)
    p["W4"][:] = rng.standard_normal(64)
    p["b4"][:] = 0.25
    o, _ = mlp_forward(w, f)
    assert np.allclose(o, p["W4"] @ np.tanh(p["b3"]) + 0.25, atol=1e-14)
    # a single path: o = tanh(tanh(tanh(a f0)))
    w = np.zeros(N_PARAMS)
    p = mlp_unpack(w)
    p["W1"][0, 0] = 0.7
    p["W2"][0, 0] = 1.0
    p["W3"][0, 0] = 1.0
    p["W4"][0] = 1.0
    o, _ = mlp_forward(w, f)
    ref = [math.tanh(math.tanh(math.tanh(0.7 * x))) for x in f[:, 0]]
    assert np.allclose(o, ref, atol=1e-15)


def test_mlp_correction_scaling():
    # o = -f1 / f0 would give back the Jacobi correction: check the scaling with
    # a network whose output is the constant c: t = c ||r||_inf / ||diag||_inf
    w = np.zeros(N_PARAMS)
    mlp_unpack(w)["b4"][:] = -0.5
    r = np.array([0.1, -0.4, 0.2])
    d = np.array([3.0, -6.0, 1.0])
    t = mlp_correction(w, r, d, -7.0)
    assert np.allclose(t, -0.5 * 0.4 / 6.0)


def test_adam_first_step_is_signed_learning_rate():
    rng = np.random.default_rng(4)
    w = rng.standard_normal(10)
    g = rng.standard_normal(10)
    w1, m, v = adam_step(w, g, np.zeros(10), np.zeros(10), 1, 0.01)
    # bias-corrected moments are g and g^2 at step 1
    assert np.allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8), atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
