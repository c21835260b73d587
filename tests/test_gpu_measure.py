"""Observables through the C interface (attn_expect_products, attn_measure,
attn_correlation) against the oracle (oracle/measure.py) on the same
seeded state: products of one-site operators on the TTN, observables of the
augmented state with the disentanglers contracted in (Sec. 5.2), and the
two-body correlation matrix of eq. 7 (Sec. 5.3)."""
import numpy as np
import pytest

from problems import config_problem, make_problem
from problems.models import PX, PZ, IPY
from oracle.ttn import OracleTTN
from oracle.measure import product_expectation, measure, correlation_matrix

pytestmark = pytest.mark.gpu


def _pair(p, sweeps):
    from paper_2507_21236_amd import AttnHandle
    a = AttnHandle(p)
    a.init_state()
    o = OracleTTN(p.n_sites, p.d, p.m, p.leaf_order, p.terms, p.de_sites, p.de_u, p.raw_tensors)
    if sweeps:
        a.sweep(sweeps)
        for _ in range(sweeps):
            o.sweep()
    o.move_center(o.tree.root)
    # the same tensors on both sides (a sweep leaves rounding-level differences)
    assert a.center == o.tree.root
    for n in range(o.tree.n_nodes):
        a.set_tensor(n, o.T[n])
    return a, o


@pytest.mark.parametrize("key,sweeps", [("ising4_m8", 1), ("ising8_m16", 1)])
def test_products_and_observables_match_oracle(key, sweeps):
    p = config_problem(key)
    a, o = _pair(p, sweeps)
    rng = np.random.default_rng(4)
    N = p.n_sites
    items = []
    for k in (1, 2, 3, 4, 2, 3):
        sites = [int(s) for s in rng.choice(N, k, replace=False)]
        items.append([(s, rng.standard_normal((2, 2))) for s in sites])
    got = a.expect_products(items)
    for it, g in zip(items, got):
        ref = product_expectation(o.tree, o.T, dict(it))
        assert abs(g - ref) <= 1e-12 * max(1.0, abs(ref)), (it, g, ref)
    # observables touching gates: one-site, both sites of a gate, two gates
    (a0, b0), (a1, b1) = p.de_sites[0], p.de_sites[1]
    free = [s for s in range(N) if all(s not in ab for ab in p.de_sites)][0]
    obs = [[(a0, PX)], [(a0, PZ), (b0, PZ)], [(a0, PX), (a1, PZ)], [(free, PZ)], [(b1, IPY), (free, PX)]]
    coef = [1.0, -0.5, 2.0, 1.0, 0.25]
    got = a.measure(obs, coef)
    for it, c, g in zip(obs, coef, got):
        ref = measure(o.tree, o.T, [s for s, _ in it], [x for _, x in it], p.de_sites, p.de_u, c)
        assert abs(g - ref) <= 1e-12 * max(1.0, abs(ref)), (it, g, ref)


def test_correlation_matrix_matches_oracle_4x4():
    p = config_problem("ising4_m8")
    a, o = _pair(p, 2)
    C = a.correlation(PZ, PX)
    rng = np.random.default_rng(2)
    pairs = [(i, i) for i in range(16)] + [tuple(int(x) for x in rng.choice(16, 2, replace=False)) for _ in range(40)]
    pairs += [tuple(ab) for ab in p.de_sites] + [tuple(ab[::-1]) for ab in p.de_sites]
    for i, j in pairs:
        if i == j:
            ref = measure(o.tree, o.T, [i], [PZ @ PX], p.de_sites, p.de_u)
        else:
            ref = measure(o.tree, o.T, [i, j], [PZ, PX], p.de_sites, p.de_u)
        assert abs(C[i, j] - ref) <= 1e-12, (i, j, C[i, j], ref)
    Czz = a.correlation(PZ, PZ)
    assert np.abs(Czz - Czz.T).max() <= 1e-12
    assert np.abs(np.diag(Czz) - 1.0).max() <= 1e-12     # Z Z = 1 on one site


@pytest.mark.timeout(600)
def test_correlation_matrix_16x16_sampled():
    import time
    p = config_problem("ising16_m64")
    from paper_2507_21236_amd import AttnHandle
    a = AttnHandle(p)
    a.init_state()
    t0 = time.time()
    C = a.correlation(PZ, PZ)
    dt = time.time() - t0
    print(f"16 x 16 m = 64 correlation matrix (65536 entries): {dt:.2f} s")
    o = OracleTTN(p.n_sites, p.d, p.m, p.leaf_order, p.terms, p.de_sites, p.de_u, p.raw_tensors)
    de_site = {s for ab in p.de_sites for s in ab}
    free = [s for s in range(256) if s not in de_site]
    rng = np.random.default_rng(8)
    pairs = [tuple(int(x) for x in rng.choice(free, 2, replace=False)) for _ in range(6)]
    pairs += [(p.de_sites[3][0], free[10]), tuple(p.de_sites[5])]
    for i, j in pairs:
        ref = measure(o.tree, o.T, [i, j], [PZ, PZ], p.de_sites, p.de_u)
        assert abs(C[i, j] - ref) <= 1e-11, (i, j, C[i, j], ref)
    assert np.abs(C - C.T).max() <= 1e-11
    assert np.abs(np.diag(C) - 1.0).max() <= 1e-11
