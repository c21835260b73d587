"""Input generator invariants (no method arithmetic is tested here)."""
import numpy as np
import pytest

from problems import config_problem, make_problem, batch_instances
from problems.lattice import hilbert_order, square_bonds, triangular_bonds
from problems.draws import balanced_tree_shapes, haar_orthogonal
from problems.placement import place_disentanglers, _subtree_of_pair, _maxdim


@pytest.mark.parametrize("L", [2, 4, 8, 16, 32])
def test_hilbert_is_permutation_of_neighbours(L):
    order = hilbert_order(L)
    assert sorted(order) == list(range(L * L))
    for a, b in zip(order[:-1], order[1:]):
        xa, ya = divmod(a, L)
        xb, yb = divmod(b, L)
        assert abs(xa - xb) + abs(ya - yb) == 1


@pytest.mark.parametrize("L", [3, 5, 6, 12])
def test_hilbert_non_power_of_two_is_permutation(L):
    assert sorted(hilbert_order(L)) == list(range(L * L))


def test_hilbert_order_4x4():
    # the classic index -> (x, y) construction with site id x * L + y
    assert hilbert_order(4) == [0, 4, 5, 1, 2, 3, 7, 6, 10, 11, 15, 14, 13, 9, 8, 12]


@pytest.mark.parametrize("L", [2, 4, 16])
def test_bond_counts(L):
    assert len(square_bonds(L)) == 2 * L * (L - 1)
    assert len(triangular_bonds(L)) == 3 * L * L - 4 * L + 1


def test_haar_orthogonal():
    rng = np.random.default_rng(0)
    for _ in range(20):
        u = haar_orthogonal(rng, 4)
        assert np.allclose(u.T @ u, np.eye(4), atol=1e-14)
        assert abs(abs(np.linalg.det(u)) - 1) < 1e-13


@pytest.mark.parametrize("key,strict,total", [
    ("ising4_m8", 4, 4), ("ising8_m32", 12, 16), ("ising16_m64", 48, 64),
])
def test_placement_counts_and_constraints(key, strict, total):
    p = config_problem(key)
    assert p.n_de_strict == strict and len(p.de_sites) == total
    used = [s for pr in p.de_sites for s in pr]
    assert len(used) == len(set(used))               # one layer: no shared site
    pos = {s: i for i, s in enumerate(p.leaf_order)}
    de_of = {s: k for k, pr in enumerate(p.de_sites) for s in pr}
    for k, (a, b) in enumerate(p.de_sites):
        assert pos[a] < pos[b]
        _, kl, kr = _subtree_of_pair(p.n_sites, pos[a], pos[b])
        assert _maxdim(2, kl, p.n_sites) > p.m and _maxdim(2, kr, p.n_sites) > p.m
        assert (a, b) in set(square_bonds(p.meta["L"])) or (b, a) in set(square_bonds(p.meta["L"]))
    # pass-1 disentanglers: no term touches two of them
    strict_set = set(range(strict))
    for sites, _, _ in p.terms:
        ks = {de_of[s] for s in sites if s in de_of and de_of[s] in strict_set}
        assert len(ks) <= 1


def test_placement_deterministic():
    a = config_problem("ising8_m32")
    b = config_problem("ising8_m32")
    assert a.de_sites == b.de_sites
    assert np.array_equal(a.de_u, b.de_u)
    assert all(np.array_equal(x, y) for x, y in zip(a.raw_tensors, b.raw_tensors))


def test_tree_shapes_small():
    assert balanced_tree_shapes(16, 8) == (
        [(2, 2, 4)] * 2 + [(4, 4, 8)] + [(2, 2, 4)] * 2 + [(4, 4, 8)] + [(8, 8, 8)]) * 2 + [(8, 8, 1)]


def test_batch_instances_shapes():
    inst = batch_instances(4)
    for p in inst:
        assert p.meta["L"] in (8, 12, 16) and p.m in (16, 32, 48, 64)
        assert 2.5 <= p.meta["h"] <= 3.5
        assert len(p.raw_tensors) == p.n_sites - 1
