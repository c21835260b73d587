"""Davidson eigensolver form of the local eigenproblem (oracle side).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper solves the local eigenproblem with the Lanczos method (Sec. 4.4.2,
the cost analysis of the ground-state search); this module defines an alternative eigensolver
form that is not from the paper, written from the published methods it uses:

* ``heff_diagonal`` -- the diagonal of H_eff(n).  H_eff(n) is a sum of
  Kronecker products of leg operators (the summed local operators and the
  items of every crossing term, as assembled by ``OracleTTN.prepare``), and the
  diagonal of a Kronecker product is the Kronecker product of the diagonals.
* ``davidson`` -- Davidson's method (E. R. Davidson, J. Comput. Phys. 17, 87
  (1975)) in float64: Rayleigh-Ritz on an orthonormal basis V, residual
  r = H u - theta u of the lowest Ritz pair, correction t = K(r) from a
  preconditioner, two passes of classical Gram-Schmidt against V, restart
  to the lowest Ritz vectors when the basis is full; stops at ||r|| <= tol.
* ``jacobi_correction`` -- the diagonal preconditioner
  t_i = -r_i / (diag_i - theta), with |diag_i - theta| kept >= 1e-8 max(1, |theta|).
* ``jd_correction`` -- the exact solution of the Jacobi-Davidson correction
  equation (1 - u u^T)(H - theta)(1 - u u^T) t = -r, t orthogonal to u
  (G. L. G. Sleijpen, H. A. van der Vorst, SIAM J. Matrix Anal. Appl. 17, 401
  (1996)), from a dense H: t = -(H - theta)^-1 r + e (H - theta)^-1 u with e
  fixing u^T t = 0.
* ``mlp_*`` -- the pointwise correction model: features per entry
  f_i = ((diag_i - theta)/s, r_i/||r||_inf, theta/s) with s = ||diag||_inf,
  three hidden tanh layers of width 64, one linear output o_i, correction
  t_i = o_i ||r||_inf / s (so the Jacobi correction is o_i = -f_i1 / f_i0).
  Parameters in one flat vector (see ``mlp_unpack``); mean-squared-error loss
  and its gradient by the chain rule; Adam updates (D. P. Kingma, J. Ba,
  arXiv:1412.6980).
"""
from __future__ import annotations

import numpy as np

HIDDEN = 64
N_FEAT = 3
SHAPES = [("W1", (N_FEAT, HIDDEN)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
          ("W3", (HIDDEN, HIDDEN)), ("b3", (HIDDEN,)), ("W4", (HIDDEN,)), ("b4", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


# ---------------------------------------------------------------- H_eff diagonal
def heff_diagonal(ttn, n, prep=None):
    """diag(H_eff(n)) as an (ml, mr, mp) array, from the same items the oracle
    matvec applies (identity factors contribute ones)."""
    El, Er, Ep, groups = prep if prep is not None else ttn.prepare(n)
    ml, mr, mp = ttn.T[n].shape
    dl, dr, dp = np.diag(El), np.diag(Er), np.diag(Ep)
    D = dl[:, None, None] + dr[None, :, None] + dp[None, None, :]
    one = {0: np.ones(ml), 1: np.ones(mr), 2: np.ones(mp)}
    for wc, Op, inner in groups:
        gp = np.diag(Op) if Op is not None else one[2]
        for c, Al, Ar in inner:
            gl = np.diag(Al) if Al is not None else one[0]
            gr = np.diag(Ar) if Ar is not None else one[1]
            D = D + (wc * c) * gl[:, None, None] * gr[None, :, None] * gp[None, None, :]
    return D


# ---------------------------------------------------------------- preconditioners
def jacobi_correction(r, diag, theta):
    eps = 1e-8 * max(1.0, abs(theta))
    den = diag - theta
    den = np.where(np.abs(den) < eps, np.where(den < 0, -eps, eps), den)
    return -r / den


def jd_correction(H, u, theta, r):
    """Exact Jacobi-Davidson correction for a dense symmetric H."""
    A = H - theta * np.eye(H.shape[0])
    a = np.linalg.solve(A, r)
    b = np.linalg.solve(A, u)
    e = float(u @ a) / float(u @ b)
    return -a + e * b


# ---------------------------------------------------------------- Davidson
def davidson(apply_h, x0, diag, tol=1e-8, maxsub=32, restart=8, max_iter=400,
             precond=None):
    """Lowest eigenpair of the symmetric operator apply_h (flat vectors) from
    the start vector x0.  precond(r, theta) -> t (default: Jacobi with diag).
    Returns (theta, u, n_matvec, residual norms per iteration)."""
    if precond is None:
        def precond(r, theta):
            return jacobi_correction(r, diag, theta)
    v = x0 / np.linalg.norm(x0)
    V = [v]
    W = [apply_h(v)]
    nmv = 1
    hist = []
    theta, u = None, None
    for _ in range(max_iter):
        Vm, Wm = np.array(V).T, np.array(W).T
        G = Vm.T @ Wm
        G = 0.5 * (G + G.T)
        ev, Y = np.linalg.eigh(G)
        theta = float(ev[0])
        y = Y[:, 0]
        u = Vm @ y
        r = Wm @ y - theta * u
        rn = float(np.linalg.norm(r))
        hist.append(rn)
        if rn <= tol:
            break
        t = precond(r, theta)
        for _ in range(2):
            t = t - Vm @ (Vm.T @ t)
        nt = float(np.linalg.norm(t))
        if not np.isfinite(nt) or nt <= 1e-14 * max(1.0, float(np.linalg.norm(r))):
            break
        t = t / nt
        if len(V) == maxsub:
            keep = Y[:, :restart]
            V = list((Vm @ keep).T)
            W = list((Wm @ keep).T)
        V.append(t)
        W.append(apply_h(t))
        nmv += 1
    return theta, u / np.linalg.norm(u), nmv, hist


# ---------------------------------------------------------------- pointwise MLP
def mlp_unpack(w):
    w = np.asarray(w, dtype=np.float64)
    assert w.size == N_PARAMS
    out, k = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = w[k:k + n].reshape(shape)
        k += n
    return out


def mlp_features(r, diag, theta):
    s = float(np.max(np.abs(diag)))
    rinf = float(np.max(np.abs(r)))
    f = np.stack([(diag - theta) / s, r / rinf, np.full(r.shape, theta / s)], axis=-1)
    return f.reshape(-1, N_FEAT), s, rinf


def mlp_forward(w, f):
    """Outputs o (n,) and the hidden activations for features f (n, 3)."""
    p = mlp_unpack(w)
    h1 = np.tanh(f @ p["W1"] + p["b1"])
    h2 = np.tanh(h1 @ p["W2"] + p["b2"])
    h3 = np.tanh(h2 @ p["W3"] + p["b3"])
    o = h3 @ p["W4"] + p["b4"][0]
    return o, (h1, h2, h3)


def mlp_correction(w, r, diag, theta):
    f, s, rinf = mlp_features(r.reshape(-1), diag.reshape(-1), theta)
    o, _ = mlp_forward(w, f)
    return (o * rinf / s).reshape(r.shape)


def mlp_loss_grad(w, f, target):
    """Mean squared error over the n points and its gradient (flat)."""
    p = mlp_unpack(w)
    o, (h1, h2, h3) = mlp_forward(w, f)
    n = f.shape[0]
    e = o - target
    loss = float(np.mean(e * e))
    go = 2.0 * e / n                        # dL/do
    g = {"W4": h3.T @ go, "b4": np.array([go.sum()])}
    d3 = np.outer(go, p["W4"]) * (1.0 - h3 * h3)
    g["W3"] = h2.T @ d3
    g["b3"] = d3.sum(axis=0)
    d2 = (d3 @ p["W3"].T) * (1.0 - h2 * h2)
    g["W2"] = h1.T @ d2
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ p["W2"].T) * (1.0 - h1 * h1)
    g["W1"] = f.T @ d1
    g["b1"] = d1.sum(axis=0)
    flat = np.concatenate([g[name].reshape(-1) for name, _ in SHAPES])
    return loss, flat


def adam_step(w, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
