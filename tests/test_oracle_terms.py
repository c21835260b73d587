"""Pins for the rotated terms h' = U^T h U and operator-Schmidt ranks."""
import numpy as np
import pytest

from problems import make_problem
from problems.draws import haar_orthogonal
from problems.models import PX, PZ
from oracle.terms import embed, rotate_all, rotate_term, op_rank, realign
from oracle.ed import hamiltonian_sparse, apply_layer


def test_embed_matches_kron():
    rng = np.random.default_rng(1)
    A, B, C = (rng.standard_normal((2, 2)) for _ in range(3))
    assert np.allclose(embed(np.kron(A, B), [5, 7], [5, 7, 9]), np.kron(np.kron(A, B), np.eye(2)))
    assert np.allclose(embed(np.kron(A, B), [7, 5], [5, 7, 9]), np.kron(np.kron(B, A), np.eye(2)))
    assert np.allclose(embed(C, [9], [5, 7, 9]), np.kron(np.eye(4), C))
    assert np.allclose(embed(C, [7], [5, 7, 9]), np.kron(np.kron(np.eye(2), C), np.eye(2)))


def _dense_from_terms(rterms, N):
    H = np.zeros((2 ** N, 2 ** N))
    for S, h in rterms:
        # embed h (on S) into N sites through the sparse builder: expand h in
        # elementary products and add each one
        k = len(S)
        for o in range(2 ** k):
            for i in range(2 ** k):
                v = h[o, i]
                if v == 0.0:
                    continue
                ops = []
                for t in range(k):
                    E = np.zeros((2, 2))
                    E[(o >> (k - 1 - t)) & 1, (i >> (k - 1 - t)) & 1] = 1.0
                    ops.append(E)
                H += hamiltonian_sparse([(S, ops, v)], N).toarray()
    return H


def test_rotated_terms_sum_to_conjugated_hamiltonian_3x3():
    p = make_problem("t", 3, "ising", 4, 11, 2, h=1.3)
    assert len(p.de_sites) == 2
    N = p.n_sites
    Hp = _dense_from_terms(rotate_all(p.terms, p.de_sites, p.de_u), N)
    H = hamiltonian_sparse(p.terms, N).toarray()
    D = np.array([apply_layer(e, p.de_sites, p.de_u, N) for e in np.eye(2 ** N)]).T
    assert np.allclose(D.T @ D, np.eye(2 ** N), atol=1e-13)
    assert np.abs(Hp - D.T @ H @ D).max() < 1e-12


def test_rotated_terms_4x4_on_random_vectors():
    p = make_problem("t", 4, "ising", 8, 1, 4, h=3.0)
    N = p.n_sites
    H = hamiltonian_sparse(p.terms, N)
    rt = rotate_all(p.terms, p.de_sites, p.de_u)
    rng = np.random.default_rng(0)
    v = rng.standard_normal(2 ** N)
    ref = apply_layer(H @ apply_layer(v, p.de_sites, p.de_u, N), p.de_sites, p.de_u, N,
                      transpose=True)
    out = np.zeros_like(v)
    for S, h in rt:
        t = v.reshape([2] * N)
        t = np.moveaxis(t, list(S), list(range(len(S))))
        sh = t.shape
        t = (h @ t.reshape(2 ** len(S), -1)).reshape(sh)
        out += np.moveaxis(t, list(range(len(S))), list(S)).reshape(-1)
    assert np.abs(out - ref).max() < 1e-11


def test_identity_disentanglers_leave_terms_unchanged():
    p = make_problem("t", 4, "ising", 8, 1, 4, h=3.0, identity_de=True)
    for (sites, ops, coef), (S, h) in zip(p.terms, rotate_all(p.terms, p.de_sites, p.de_u)):
        ref = embed(coef * np.kron(*ops) if len(ops) == 2 else coef * ops[0], list(sites), list(S))
        assert np.allclose(h, ref, atol=1e-15)


def test_schmidt_rank_bounds():
    rng = np.random.default_rng(3)
    u1, u2 = haar_orthogonal(rng, 4), haar_orthogonal(rng, 4)
    # two-site ZZ term with a gate lying fully on it: stays 2-body, rank <= d^2
    S, h = rotate_term((0, 1), [PZ, PZ], -1.0, [(0, 1)], [u1])
    assert S == (0, 1) and op_rank(h, S, [0], [1]) <= 4
    # gate with one site outside: 3-body, each cut rank <= d^2
    S, h = rotate_term((0, 1), [PZ, PZ], -1.0, [(1, 2)], [u1])
    assert set(S) == {0, 1, 2}
    assert op_rank(h, S, [0], [1, 2]) == 1 and op_rank(h, S, [0, 1], [2]) <= 4
    # a local term under a gate becomes (at most) two-body with rank <= d^2
    S, h = rotate_term((0,), [PX], -3.0, [(0, 1)], [u1])
    assert op_rank(h, S, [0], [1]) <= 4
    # a term touching two gates: 4-body, middle cut rank <= d^4
    S, h = rotate_term((1, 2), [PZ, PZ], -1.0, [(0, 1), (2, 3)], [u1, u2])
    assert len(S) == 4
    r = op_rank(h, S, sorted([0, 1]), sorted([2, 3]))
    assert r <= 16 and op_rank(h, S, [0], [1, 2, 3]) <= 4
    # no gate: plain product, rank 1
    S, h = rotate_term((0, 1), [PZ, PZ], -1.0, [], [])
    assert op_rank(h, S, [0], [1]) == 1


def test_realign_roundtrip():
    rng = np.random.default_rng(5)
    h = rng.standard_normal((8, 8))
    t = realign(h, [3, 1, 2], [[1], [2, 3]])
    assert t.shape == (4, 16)
    # element (o1 i1 | o2 o3 i2 i3) for sites sorted as given in the groups
    for o in range(8):
        for i in range(8):
            o3, o1, o2 = (o >> 2) & 1, (o >> 1) & 1, o & 1
            i3, i1, i2 = (i >> 2) & 1, (i >> 1) & 1, i & 1
            assert t[o1 * 2 + i1, ((o2 * 2 + o3) * 2 + i2) * 2 + i3] == h[o, i]
