"""Observables and the disentangler-layer optimisation (oracle side).

TEST INFRASTRUCTURE ONLY (see the package header).

* ``product_expectation`` -- <psi_TTN| prod_s A_s |psi_TTN> for a product of
  one-site operators, by contracting the tree from the leaves to the root
  (Sec. 5.1: only the subtree holding the operators needs explicit
  contraction; with the isometry centre at the root every operator-free
  subtree contracts to the identity).
* ``expectation`` -- a dense operator on a few sites, expanded in products of
  one-site matrix units.
* ``measure`` / ``correlation_matrix`` -- observables of the augmented state:
  <psi_aTTN| o |psi_aTTN> = <psi_TTN| o' |psi_TTN> with o' the observable with
  the disentanglers that touch it contracted in (Sec. 5.2, eq. 6; with the
  state read as D|psi_TTN>, o' = U^T o U, the same reading as the rotated
  Hamiltonian); the two-body correlation matrix of eq. 7, C[i][j] =
  <o^a_i o^b_j>, diagonal entries the one-site product o^a o^b (Sec. 5.3).
* ``de_environment`` / ``optimize_disentangler`` / ``optimize_layer`` -- the
  MERA-like optimisation of Sec. 4.1.1.  The energy terms that act on the
  sites of disentangler k depend on u_k (eq. 3, the others form c_k); with the
  copy of u_k in the bra fixed at u~, the energy is linear in the ket copy,
  E = Tr(u_k Gamma_k) (eq. 4), and the minimiser over orthogonal u is
  u = -V U^T for Gamma_k = U sigma V^T, with E = -sum sigma (eq. 5); the step
  is repeated with the new u as u~ until the energy settles, the environment
  (here: the expectation values of the state) staying fixed.
"""
from __future__ import annotations

import itertools

import numpy as np

from .terms import rotate_term, embed
from .ttn import mode


# ---------------------------------------------------------------- expectations on the TTN
def product_expectation(tree, T, ops):
    """<psi| prod_{s in ops} ops[s] |psi> for the TTN with tensors T whose
    isometry centre is the root (every other node an isometry toward its
    parent).  ops: {site: d x d matrix}, element [i][k] = <i|A|k>."""
    children = tree.children

    def rec(child):
        if child[0] == 's':
            return ops.get(child[1])
        n = child[1]
        Rl, Rr = rec(children[n][0]), rec(children[n][1])
        if Rl is None and Rr is None:
            return None
        X = T[n]
        if Rl is not None:
            X = mode(Rl, X, 0)
        if Rr is not None:
            X = mode(Rr, X, 1)
        # <c| P |c'> = sum_{a b} T[a, b, c] (P T)[a, b, c']
        return np.tensordot(T[n], X, axes=([0, 1], [0, 1]))

    R = rec(('n', tree.root))
    if R is None:
        return float(np.sum(T[tree.root] ** 2))
    return float(R[0, 0])


def unit(d, o, i):
    e = np.zeros((d, d))
    e[o, i] = 1.0
    return e


def expectation(tree, T, S, h, d=2):
    """<psi| h |psi> for a dense operator h on the ordered sites S (first site
    most significant), as the sum over its entries of h[o, i] times the
    expectation of the product of one-site units |o_t><i_t|."""
    k = len(S)
    total = 0.0
    for o in range(d ** k):
        for i in range(d ** k):
            v = h[o, i]
            if v == 0.0:
                continue
            od = [(o // d ** (k - 1 - t)) % d for t in range(k)]
            idg = [(i // d ** (k - 1 - t)) % d for t in range(k)]
            ops = {S[t]: unit(d, od[t], idg[t]) for t in range(k)}
            total += v * product_expectation(tree, T, ops)
    return total


def measure(tree, T, sites, ops, de_sites, de_u, coef=1.0, d=2):
    """<psi_aTTN| coef prod ops |psi_aTTN> with the disentanglers contracted into the
    observable (Sec. 5.2)."""
    S, h = rotate_term(tuple(sites), [np.asarray(o, dtype=float) for o in ops], coef,
                       de_sites, de_u, d)
    return expectation(tree, T, list(S), h, d)


def correlation_matrix(tree, T, oa, ob, de_sites, de_u, d=2):
    """C[i][j] = <o^a_i o^b_j> of the augmented state (eq. 7); the diagonal is
    the one-site product o^a o^b."""
    N = tree.N
    C = np.zeros((N, N))
    for i in range(N):
        for j in range(N):
            if i == j:
                C[i, j] = measure(tree, T, [i], [oa @ ob], de_sites, de_u, 1.0, d)
            else:
                C[i, j] = measure(tree, T, [i, j], [oa, ob], de_sites, de_u, 1.0, d)
    return C


# ---------------------------------------------------------------- MERA-like disentangler optimisation
def de_terms(terms, de_sites, k):
    """Terms acting on a site of disentangler k.  The optimisation needs the
    placement restriction of Sec. 4.1 (no term acts on two disentanglers)."""
    a, b = de_sites[k]
    others = {s for j, (x, y) in enumerate(de_sites) if j != k for s in (x, y)}
    out = []
    for sites, ops, coef in terms:
        if a in sites or b in sites:
            if any(s in others for s in sites):
                raise ValueError(f"term on {sites} acts on two disentanglers")
            out.append((sites, ops, coef))
    return out


def de_environment_parts(tree, T, terms, de_sites, k, d=2):
    """The expectation values Gamma_k is built from: for every term h = coef
    P (x) Q acting on a site of disentangler k (P on its other sites R, Q on the
    disentangler's sites (a, b), identity on the untouched one), the d^2 x d^2
    matrix sigma[x, y] = coef <P (x) |y><x|_(a b)>; and rho_ab[x, y] =
    <|y><x|_(a b)> (for the energy shift).  Returns ([(sigma, Q)], rho_ab)."""
    a, b = de_sites[k]
    dd = d * d

    def pair_units(x, y):
        ya, yb, xa, xb = y // d, y % d, x // d, x % d
        return {a: unit(d, ya, xa), b: unit(d, yb, xb)}

    parts = []
    for sites, ops, coef in de_terms(terms, de_sites, k):
        on_pair = [(s, o) for s, o in zip(sites, ops) if s in (a, b)]
        Q = embed(_kron([o for _, o in on_pair]), [s for s, _ in on_pair], [a, b], d)
        rest = {s: np.asarray(o, dtype=float) for s, o in zip(sites, ops) if s not in (a, b)}
        sigma = np.zeros((dd, dd))
        for x in range(dd):
            for y in range(dd):
                o = dict(rest)
                o.update(pair_units(x, y))
                sigma[x, y] = coef * product_expectation(tree, T, o)
        parts.append((sigma, Q))
    rho = np.zeros((dd, dd))
    for x in range(dd):
        for y in range(dd):
            rho[x, y] = product_expectation(tree, T, pair_units(x, y))
    return parts, rho


def _kron(mats):
    out = np.array([[1.0]])
    for m in mats:
        out = np.kron(out, np.asarray(m, dtype=float))
    return out


def de_energy(parts, u):
    """Energy of the terms acting on the disentangler's sites with gate u:
    sum over terms of Tr(u sigma u^T Q)."""
    return float(sum(np.trace(u @ s @ u.T @ Q) for s, Q in parts))


def de_gamma(parts, rho, u_fixed, shift=0.0):
    """Gamma_k of eq. 4 with the bra copy fixed at u_fixed: E_lin(u) = Tr(u Gamma)
    = sum over terms of Tr(u sigma u_fixed^T Q); a shift c of the energy
    (the terms minus c times the identity) adds -c rho_ab u_fixed^T."""
    G = sum(s @ u_fixed.T @ Q for s, Q in parts)
    return G - shift * rho @ u_fixed.T


def svd_update(G):
    """Minimiser of Tr(u G) over orthogonal u: u = -V U^T for G = U sigma V^T
    (eq. 5); returns (u, sum of singular values)."""
    U, s, Vt = np.linalg.svd(G)
    return -Vt.T @ U.T, float(s.sum())


def optimize_disentangler(parts, rho, u0, shift, max_iter=20, rel_tol=1e-12):
    """Self-consistent iteration of Sec. 4.1.1 from u0 with the environment
    fixed: Gamma from the current u, u <- -V U^T, until the relative energy
    change is below rel_tol or max_iter steps.  With shift >= the largest
    eigenvalue of the terms, the energy of every step is at most that of the
    step before (the shifted energy is a concave function of u, so the linear
    model is an upper bound).  Returns (u, [energies, starting with u0's])."""
    u = np.asarray(u0, dtype=float)
    es = [de_energy(parts, u)]
    for _ in range(max_iter):
        G = de_gamma(parts, rho, u, shift)
        u, _ = svd_update(G)
        es.append(de_energy(parts, u))
        if abs(es[-1] - es[-2]) <= rel_tol * max(1.0, abs(es[-1])):
            break
    return u, es


def term_norm_bound(terms):
    """Sum over terms of |coef| prod ||op||_2: an upper bound of the largest
    eigenvalue of their sum (used as the shift)."""
    return float(sum(abs(c) * np.prod([np.linalg.norm(o, 2) for o in ops]) for _, ops, c in terms))


def optimize_layer(tree, T, terms, de_sites, de_u, max_iter=20, rel_tol=1e-12, use_shift=True, d=2,
                   method="mera"):
    """Every disentangler of the layer optimised with the others fixed (they
    act on other terms only, Sec. 4.1), from the TTN state T (centre at the
    root), by the MERA-like update ("mera", Sec. 4.1.1) or Riemannian CG
    ("rcg", Sec. 4.1.2).  Returns (new de_u, per-gate energy histories)."""
    new_u = np.array(de_u, dtype=float, copy=True)
    hist = []
    for k in range(len(de_sites)):
        parts, rho = de_environment_parts(tree, T, terms, de_sites, k, d)
        if method == "rcg":
            u, es = optimize_disentangler_rcg(parts, de_u[k], max_iter, rel_tol)
        else:
            c = term_norm_bound(de_terms(terms, de_sites, k)) if use_shift else 0.0
            u, es = optimize_disentangler(parts, rho, de_u[k], c, max_iter, rel_tol)
        new_u[k] = u
        hist.append(es)
    return new_u, hist


def attn_sweeps(o, terms, de_sites, de_u0, n_sweeps, s_ttn=1, max_iter=20, rel_tol=1e-12,
                use_shift=True, compress=False):
    """The aTTN ground-state recipe of Sec. 4 on the oracle TTN ``o``: every
    sweep from sweep s_ttn on first optimises the disentangler layer on the
    current state (step 1), contracts it into the Hamiltonian (step 2) and then
    runs the TTN sweep (step 3); the first s_ttn sweeps run on the TTN with
    the layer it was given (Sec. 6.3: the best schedule starts from one sweep
    without the layer, S_TTN = 1).  Returns (energies, final de_u)."""
    de_u = np.array(de_u0, dtype=float, copy=True)
    es = []
    for s in range(n_sweeps):
        if s >= s_ttn:
            o.move_center(o.tree.root)
            de_u, _ = optimize_layer(o.tree, o.T, terms, de_sites, de_u, max_iter, rel_tol, use_shift)
            o.set_disentanglers(terms, de_sites, de_u, compress)
        es.append(o.sweep())
    return es, de_u


# ---------------------------------------------------------------- gradient-based optimisation (Sec. 4.1.2)
def de_euclid_grad(parts, u):
    """Gradient of E(u) = sum Tr(u sigma u^T Q) in both copies of u at once:
    dE = Tr(G^T du) with G = sum (Q^T u sigma^T + Q u sigma)."""
    return sum(Q.T @ u @ s.T + Q @ u @ s for s, Q in parts)


def de_riem_grad(parts, u):
    """Riemannian gradient on the orthogonal group, written in the frame of u:
    the tangent vector is u Omega with Omega = skew(u^T G)."""
    A = u.T @ de_euclid_grad(parts, u)
    return 0.5 * (A - A.T)


def cayley(X):
    """(I - X/2)^-1 (I + X/2): orthogonal for skew-symmetric X (the Cayley
    retraction of the orthogonal group)."""
    n = X.shape[0]
    return np.linalg.solve(np.eye(n) - 0.5 * X, np.eye(n) + 0.5 * X)


def optimize_disentangler_rcg(parts, u0, max_iter=50, rel_tol=1e-12):
    """Riemannian conjugate gradient on O(d^2) (Sec. 4.1.2: both copies of
    u_k are varied together and the constraint u^T u = 1 is kept by the
    geometry; the paper points to Riemannian nonlinear CG).  Directions are
    skew matrices Omega (tangent vectors u Omega, carried between points by
    the group translation); Polak-Ribiere+ coefficient; steps u <- u
    cay(t D) with t halved from 1 until the Armijo condition
    E(new) <= E + 1e-4 t <g, D> holds; restart along -g when D is not a
    descent direction.  Stops when the energy changes by at most
    rel_tol max(1, |E|).  Returns (u, energies)."""
    u = np.asarray(u0, dtype=float)
    E = de_energy(parts, u)
    es = [E]
    g = de_riem_grad(parts, u)
    D = -g
    for _ in range(max_iter):
        gg = float(np.sum(g * g))
        if gg == 0.0:
            break
        slope = float(np.sum(g * D))
        if slope >= 0.0:
            D = -g
            slope = -gg
        t = 1.0
        while True:
            un = u @ cayley(t * D)
            En = de_energy(parts, un)
            if En <= E + 1e-4 * t * slope or t < 1e-12:
                break
            t *= 0.5
        if En > E:
            break
        gn = de_riem_grad(parts, un)
        beta = max(0.0, float(np.sum(gn * (gn - g))) / gg)
        D = -gn + beta * D
        done = abs(En - E) <= rel_tol * max(1.0, abs(En))
        u, E, g = un, En, gn
        es.append(E)
        if done:
            break
    return u, es
