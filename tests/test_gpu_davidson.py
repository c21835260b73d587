"""GPU tests of the Davidson eigensolver form against the oracle: the H_eff
diagonal, Davidson with Jacobi corrections, the correction model's inference
and training step, the exact Jacobi-Davidson corrections used as training data,
and the learned correction with its fallback.

Tolerances: the diagonal is a sum of FP64 products (1e-12 relative).  Both
Davidson solvers stop at ||r|| <= 1e-9, so both Ritz values lie within
||r||^2 / gap of the lowest eigenvalue and agree to 1e-10 relative.  The model
runs in FP32 with FP16 parameters: outputs agree with the FP64 forward of the
same FP16-rounded parameters to 1e-5 relative to their scale; the first Adam
step moves every parameter with a non-negligible gradient by lr sign(g)."""
import numpy as np
import pytest

from problems import config_problem, make_chain_problem
from tests.gpu_util import make_pair, move_both

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _gpu_diag(a, n, shape):
    import torch
    out = torch.empty(int(np.prod(shape)), dtype=torch.float64, device="cuda")
    a.heff_diagonal(n, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(shape)


def test_heff_diagonal_matches_oracle():
    from oracle.davidson import heff_diagonal
    for p in (config_problem("ising8_m16"),
              make_chain_problem("c", 12, 1.7, 8, 9, de_pairs=[(1, 3), (4, 6), (8, 10)])):
        a, o = make_pair(p)
        for n in range(0, o.tree.n_nodes, 3):
            move_both(a, o, n)
            D = heff_diagonal(o, n)
            G = _gpu_diag(a, n, D.shape)
            assert np.abs(G - D).max() <= 1e-12 * max(1.0, np.abs(D).max()), n


def test_davidson_jacobi_matches_oracle():
    from oracle.davidson import heff_diagonal, davidson
    from paper_2507_21236_amd import solver_opts, ATTN_SOLVER_DAVIDSON, ATTN_PRECOND_JACOBI
    p = config_problem("ising8_m16")
    a, o = make_pair(p)
    shapes_seen = set()
    for n in range(o.tree.n_nodes):
        sh = o.tree.dims[n]
        if sh in shapes_seen:
            continue
        shapes_seen.add(sh)
        move_both(a, o, n)
        prep = o.prepare(n)
        D = heff_diagonal(o, n, prep).ravel()
        x0 = o.T[n].ravel().copy()
        th_o, u_o, nmv_o, hist = davidson(lambda v: o.matvec(n, v.reshape(sh), prep).ravel(), x0, D,
                                          tol=1e-9, maxsub=32, restart=8, max_iter=300)
        th_a, nmv = a.eigsolve(n, solver_opts(solver=ATTN_SOLVER_DAVIDSON, krylov_k=32, tol=1e-9,
                                              precond=ATTN_PRECOND_JACOBI, max_iter=300, restart=8))
        print(f"node {n} {sh}: theta {th_a:.14f} oracle {th_o:.14f}  matvecs {nmv} / {nmv_o}")
        assert abs(th_a - th_o) <= 1e-10 * abs(th_o), (n, th_a, th_o)
        u = a.get_tensor(n).ravel()
        assert abs(abs(u @ u_o) - 1.0) < 1e-8
        # keep both sides on the same tensor
        a.set_tensor(n, o.T[n])


def _rand_params(rng, scale=0.25):
    from oracle.davidson import N_PARAMS
    return (rng.standard_normal(N_PARAMS) * scale).astype(np.float32)


def test_mlp_eval_matches_oracle():
    import torch
    from oracle.davidson import mlp_forward
    from paper_2507_21236_amd import mlp_eval
    rng = np.random.default_rng(5)
    w = _rand_params(rng)
    f = rng.standard_normal((5000, 3)).astype(np.float32)
    out = mlp_eval(w, torch.from_numpy(f).cuda()).cpu().numpy()
    w16 = w.astype(np.float16).astype(np.float64)
    ref, _ = mlp_forward(w16, f.astype(np.float64))
    err = np.abs(out - ref).max() / max(1.0, np.abs(ref).max())
    print("model eval max rel err", err)
    assert err < 1e-5


def test_mlp_train_step_matches_oracle():
    import torch
    from oracle.davidson import mlp_loss_grad, adam_step
    from paper_2507_21236_amd import mlp_train
    rng = np.random.default_rng(6)
    w0 = _rand_params(rng)
    f = rng.standard_normal((256, 3)).astype(np.float32)
    y = rng.standard_normal(256).astype(np.float32)
    lr = 1e-3
    w1, loss = mlp_train(torch.from_numpy(f).cuda(), torch.from_numpy(y).cuda(), w0, steps=1,
                         batch=256, lr=lr)
    l_ref, g = mlp_loss_grad(w0.astype(np.float64), f.astype(np.float64), y.astype(np.float64))
    w_ref, _, _ = adam_step(w0.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    assert abs(loss[0] - l_ref) < 1e-5 * l_ref
    big = np.abs(g) > 1e-4
    assert big.sum() > 1000
    assert np.abs(w1[big] - w_ref[big]).max() < 1e-3 * lr
    # two more steps keep decreasing the loss on this batch
    w3, loss3 = mlp_train(torch.from_numpy(f).cuda(), torch.from_numpy(y).cuda(), w0, steps=20,
                          batch=256, lr=lr)
    assert loss3[-1] < loss3[0]


def test_harvested_correction_solves_jd_equation():
    # the first pair is taken at the start vector, so u = T / ||T|| is known and
    # the exact correction can be formed from the dense H_eff on the CPU
    from oracle.davidson import heff_diagonal, jd_correction
    from tests.test_oracle_ttn import _dense_heff
    from oracle.ed import hamiltonian_sparse
    p = config_problem("ising4_m8")
    a, o = make_pair(p)
    H = hamiltonian_sparse(p.terms, p.n_sites)
    n = max(range(o.tree.n_nodes), key=lambda k: np.prod(o.tree.dims[k]))
    move_both(a, o, n)
    Hd = _dense_heff(o, p, n, H)
    # at the random start vector theta lies inside the spectrum: the projected
    # system is indefinite and can be ill-conditioned, so MINRES may need more
    # than M steps
    T_before = a.get_tensor(n)
    f, t, res = a.harvest(n, 2, cg_tol=1e-12, cg_max=4000)
    print("MINRES relative residuals", res)
    assert res[0] < 1e-9
    u = o.T[n].ravel() / np.linalg.norm(o.T[n])
    theta = float(u @ Hd @ u)
    r = Hd @ u - theta * u
    t_ref = jd_correction(Hd, u, theta, r)
    D = heff_diagonal(o, n).ravel()
    s, rinf = np.abs(D).max(), np.abs(r).max()
    M = u.size
    feats = f.cpu().numpy()[:M]
    targ = t.cpu().numpy()[:M].astype(np.float64) * rinf / s
    assert np.allclose(feats[:, 0], (D - theta) / s, atol=1e-6)
    assert np.allclose(feats[:, 1], r / rinf, atol=1e-6)
    assert np.linalg.norm(targ - t_ref) <= 1e-5 * np.linalg.norm(t_ref)
    # the tensor is unchanged
    assert np.array_equal(a.get_tensor(n), T_before)


def test_learned_davidson_trained_and_fallback():
    import torch
    from paper_2507_21236_amd import (solver_opts, ATTN_SOLVER_DAVIDSON, ATTN_PRECOND_JACOBI,
                                      ATTN_PRECOND_LEARNED, mlp_train)
    p = config_problem("ising8_m32")
    a, o = make_pair(p)
    full = [n for n in range(o.tree.n_nodes) if o.tree.dims[n] == (32, 32, 32)]
    move_both(a, o, full[0])
    f, t, res = a.harvest(full[0], 4, cg_tol=1e-8, cg_max=400)
    print("harvest CG residuals", res)
    w0 = _rand_params(np.random.default_rng(7), 0.1)
    w, loss = mlp_train(f, t, w0, steps=300, batch=4096, lr=2e-3)
    print("training loss", loss[0], "->", loss[-1])
    assert np.isfinite(loss).all() and loss[-1] < loss[0]
    n = full[1]
    move_both(a, o, n)
    T0 = a.get_tensor(n)
    opts = dict(solver=ATTN_SOLVER_DAVIDSON, krylov_k=32, tol=1e-8, max_iter=300, restart=8)
    th_j, nmv_j = a.eigsolve(n, solver_opts(precond=ATTN_PRECOND_JACOBI, **opts))
    a.set_tensor(n, T0)
    a.set_precond_weights(w)
    th_l, nmv_l = a.eigsolve(n, solver_opts(precond=ATTN_PRECOND_LEARNED, **opts))
    it, fb, rn, rate = a.solver_stats()
    print(f"jacobi {th_j:.12f} ({nmv_j} matvecs), learned {th_l:.12f} ({nmv_l} matvecs), "
          f"fallbacks {fb}, last residual {rn:.2e}")
    assert abs(th_l - th_j) <= 1e-9 * abs(th_j)
    # non-finite model output: the solve falls back to Jacobi and still converges
    a.set_tensor(n, T0)
    a.set_precond_weights(np.full(w.size, np.nan, dtype=np.float32))
    th_n, _ = a.eigsolve(n, solver_opts(precond=ATTN_PRECOND_LEARNED, **opts))
    assert a.solver_stats()[1] >= fb + 1
    assert abs(th_n - th_j) <= 1e-9 * abs(th_j)
