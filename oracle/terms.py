"""Hamiltonian terms rotated by the disentangler layer (oracle side).

The aTTN state is D|psi_TTN> with D the product of the two-site gates
(paper Sec. 2, eq. 1), so its energy is <psi_TTN| D^T H D |psi_TTN>.  The
mapped Hamiltonian H' = D^T H D is built term by term (Sec. 4.3, algorithm
"Contract disentangler layer"): a term h is conjugated only by the gates that
touch its support -- gates away from it cancel by unitarity (Sec. 4.1,
figure on the energy split).  A gate lying fully on the term keeps it n-body
(case (a) of the contraction figure); a gate with one site outside extends
the support by that site with an identity (case (b)).  Here the contraction is
written out densely on the extended support (at most 4 sites) instead of
through QR link propagation: h' = U^T (h x 1) U with U the gates on that
support.

Direction of the rotation: the text writes H' = D H D^dagger, the state
definition implies D^dagger H D; the two describe the same variational class
(u <-> u^dagger).  The oracle uses h' = U^T h U (real orthogonal U).

Operators on an ordered site list S are dense d^|S| x d^|S| matrices with the
first listed site as the most significant index.
"""
from __future__ import annotations

import itertools

import numpy as np


def embed(op, op_sites, S, d=2):
    """Matrix of ``op`` (acting on op_sites, first site major) on the ordered
    support S, identity elsewhere.  Written as an explicit loop over basis
    states so that the index bookkeeping is visible."""
    s = len(S)
    pos = [S.index(x) for x in op_sites]
    rest = [i for i in range(s) if i not in pos]
    k = len(op_sites)
    D = d ** s
    out = np.zeros((D, D))
    for o in itertools.product(range(d), repeat=s):
        for i in itertools.product(range(d), repeat=s):
            if any(o[r] != i[r] for r in rest):
                continue
            oi = 0
            ii = 0
            for p in pos:
                oi = oi * d + o[p]
                ii = ii * d + i[p]
            val = op[oi, ii]
            if val == 0.0:
                continue
            ro = 0
            ri = 0
            for t in range(s):
                ro = ro * d + o[t]
                ri = ri * d + i[t]
            out[ro, ri] = val
    return out


def product_op(ops):
    out = np.array([[1.0]])
    for o in ops:
        out = np.kron(out, o)
    return out


def rotate_term(sites, ops, coef, de_sites, de_u, d=2):
    """Return (S', h') for one term: S' = term sites followed by the partner
    sites of every disentangler that meets the term."""
    S = list(sites)
    touching = []
    for k, (a, b) in enumerate(de_sites):
        if a in sites or b in sites:
            touching.append(k)
            for x in (a, b):
                if x not in S:
                    S.append(x)
    h = coef * embed(product_op(ops), list(sites), S, d)
    U = np.eye(d ** len(S))
    for k in touching:
        a, b = de_sites[k]
        U = U @ embed(np.asarray(de_u[k]), [a, b], S, d)
    return tuple(S), U.T @ h @ U


def rotate_all(terms, de_sites, de_u, d=2):
    return [rotate_term(s, o, c, de_sites, de_u, d) for (s, o, c) in terms]


def realign(h, S, groups, d=2):
    """View the operator h on S as a tensor over site groups.

    ``groups`` is a list of site lists partitioning S.  Returns an array with
    one axis per group; the axis of group g has length d^(2|g|) and index
    (out indices of the group's sites, then in indices), so that a vector over
    that axis is an operator on the group in the same layout as ``embed``.
    """
    s = len(S)
    t = h.reshape([d] * (2 * s))
    perm = []
    shape = []
    for g in groups:
        pos = [S.index(x) for x in g]
        perm += pos + [s + p for p in pos]
        shape.append(d ** (2 * len(g)))
    return t.transpose(perm).reshape(shape)


def schmidt(mat, rel_tol=1e-12):
    """SVD of a realigned operator, keeping singular values above
    rel_tol * largest.  Returns (sigma, U, Vt)."""
    u, sv, vt = np.linalg.svd(mat, full_matrices=False)
    if sv.size == 0 or sv[0] == 0.0:
        return sv[:0], u[:, :0], vt[:0]
    keep = sv > rel_tol * sv[0]
    return sv[keep], u[:, keep], vt[keep]


def op_rank(h, S, group_a, group_b, d=2, rel_tol=1e-12):
    """Operator-Schmidt rank of h across the bipartition (group_a | group_b)."""
    mat = realign(h, S, [list(group_a), list(group_b)], d)
    return len(schmidt(mat, rel_tol)[0])


def compress_terms(terms, rterms):
    """Sum the rotated terms whose original supports are the same set of sites
    (Sec. 6.2.2, closing paragraph: the terms acting on the same sites, e.g.
    XX, YY and ZZ on one bond, become one term; after the disentangler layer
    it has one bond of at most d^2 across any cut instead of one such bond per
    term).  Terms with the same support meet the same disentanglers, so their
    rotated supports coincide as sets; each rotated operator is re-expressed
    on the sorted support before the sum.  Order: first occurrence."""
    groups = {}
    order = []
    for (sites, _, _), (S, h) in zip(terms, rterms):
        key = frozenset(sites)
        Sc = tuple(sorted(S))
        hc = embed(h, list(S), list(Sc), int(round(h.shape[0] ** (1.0 / len(S)))))
        if key in groups:
            S0, h0 = groups[key]
            assert S0 == Sc
            groups[key] = (S0, h0 + hc)
        else:
            groups[key] = (Sc, hc)
            order.append(key)
    return [groups[k] for k in order]
