"""Compression of terms that act on the same sites (paper Sec. 6.2.2, closing
paragraph), oracle side and host build of the library (no GPU).

Pins: the compressed rotated terms still sum to D^T H D as 2^N x 2^N
matrices (dense, N = 9, against the conjugated lattice Hamiltonian); one term
per distinct support; a two-site sum under one disentangler has bond <= d^2
across every cut of its extended support, as the paper states; terms with
distinct supports (the Ising model) are left as they are; and the library's
host build, with ATTN_COMPRESS_TERMS, reproduces the oracle's dims, crossing-term
counts and flop model at every node."""
import numpy as np
import pytest

from problems import make_problem, config_problem
from oracle.terms import rotate_all, compress_terms, op_rank
from oracle.ed import hamiltonian_sparse, apply_layer
from oracle.ttn import OracleTTN
from paper_2507_21236_amd import AttnHandle, ATTN_HOST_ONLY, _lib
from tests.test_oracle_terms import _dense_from_terms

ATTN_COMPRESS_TERMS = 8


def test_flag_value_matches_header():
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "attn.h")).read()
    assert int(re.search(r"#define ATTN_COMPRESS_TERMS\s+(\d+)u", hdr).group(1)) == ATTN_COMPRESS_TERMS


def test_compressed_terms_sum_to_conjugated_hamiltonian():
    p = make_problem("t", 3, "heisenberg_tri", 4, 11, 2)
    assert len(p.de_sites) == 2
    N = p.n_sites
    rt = rotate_all(p.terms, p.de_sites, p.de_u)
    ct = compress_terms(p.terms, rt)
    assert len(ct) == len({frozenset(s) for s, _, _ in p.terms}) == len(p.terms) // 3
    H = hamiltonian_sparse(p.terms, N).toarray()
    D = np.array([apply_layer(e, p.de_sites, p.de_u, N) for e in np.eye(2 ** N)]).T
    assert np.abs(_dense_from_terms(ct, N) - D.T @ H @ D).max() < 1e-12


def test_compressed_bonds_are_at_most_d_squared():
    p = make_problem("t", 4, "heisenberg_tri", 8, 4, 4)
    de_site = {s for ab in p.de_sites for s in ab}
    rt = rotate_all(p.terms, p.de_sites, p.de_u)
    ct = compress_terms(p.terms, rt)
    seen = 0
    for S, h in ct:
        n_de = sum(1 for a, b in p.de_sites if a in S or b in S)
        if n_de != 1:
            continue
        seen += 1
        S = list(S)
        for k in range(1, len(S)):
            for cut in ([S[:k], S[k:]], [[S[k]], S[:k] + S[k + 1:]]):
                assert op_rank(h, S, *cut) <= 4
    assert seen > 0
    # uncompressed: three terms per bond, each already of bond <= d^2, so the
    # crossing blocks add up to three times as many
    assert len(rt) == 3 * len(ct) and de_site


def test_distinct_supports_are_unchanged():
    p = config_problem("ising4_m8")
    rt = rotate_all(p.terms, p.de_sites, p.de_u)
    ct = compress_terms(p.terms, rt)
    assert len(ct) == len(rt)
    for (S, h), (Sc, hc) in zip(rt, ct):
        assert set(S) == set(Sc)
        assert np.abs(np.linalg.eigvalsh(h) - np.linalg.eigvalsh(hc)).max() < 1e-13


def test_compressed_oracle_matvec_equals_uncompressed():
    # the same Hamiltonian in fewer terms: H_eff agrees at every node
    p = make_problem("t", 4, "heisenberg_tri", 8, 4, 4)
    a = OracleTTN(p.n_sites, p.d, p.m, p.leaf_order, p.terms, p.de_sites, p.de_u, p.raw_tensors)
    b = OracleTTN(p.n_sites, p.d, p.m, p.leaf_order, p.terms, p.de_sites, p.de_u, p.raw_tensors,
                  compress=True)
    rng = np.random.default_rng(2)
    for n in range(a.tree.n_nodes):
        a.move_center(n)
        b.move_center(n)
        x = rng.standard_normal(a.T[n].shape)
        ya, yb = a.matvec(n, x), b.matvec(n, x)
        assert np.linalg.norm(ya - yb) <= 1e-12 * np.linalg.norm(ya), n
        assert b.flops(n) <= a.flops(n)
        assert len(b.crossing_terms(n)) <= len(a.crossing_terms(n))


@pytest.mark.parametrize("make", [
    lambda: make_problem("t", 4, "heisenberg_tri", 8, 4, 4),
    lambda: make_problem("t", 8, "heisenberg_tri", 16, 4, 16),
    lambda: config_problem("ising8_m32"),
])
def test_host_build_compressed_matches_oracle_structure(make):
    p = make()
    a = AttnHandle(p, flags=ATTN_HOST_ONLY | ATTN_COMPRESS_TERMS)
    o = OracleTTN(p.n_sites, p.d, p.m, p.leaf_order, p.terms, p.de_sites, p.de_u, p.raw_tensors,
                  structure_only=True, compress=True)
    u = AttnHandle(p, flags=ATTN_HOST_ONLY)
    tot_c = tot_u = 0
    for n in range(a.n_nodes):
        dims, nc, fl = a.node_info(n)
        assert tuple(dims) == tuple(o.tree.dims[n])
        assert nc == len(o.crossing_terms(n)), n
        assert fl == o.flops(n), n
        tot_c += fl
        tot_u += u.node_info(n)[2]
    if p.meta["model"] == "heisenberg_tri":
        assert tot_c < tot_u
    else:
        assert tot_c == tot_u
