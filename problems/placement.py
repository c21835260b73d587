"""Deterministic disentangler placement (input generation).

Follows the automatic positioning strategy of paper Sec. 6.1.2: walk the
candidate positions starting from those that support the highest-layer link,
accept a position that lies fully on an interaction term and breaks none of
the restrictions of Sec. 6.1.1.  The reading used here:

* candidates are the site pairs of the two-site interaction terms;
* priority key: (-size of the subtree of the pair's lowest common ancestor,
  smaller leaf position, larger leaf position) -- the pair whose common
  ancestor is highest in the tree comes first;
* disentanglers never share a site (they form one layer);
* restriction 2 (no disentangler on untruncated links): both child links of
  the pair's lowest common ancestor must have maximal dimension
  min(d^k, d^(N-k)) larger than m;
* pass 1 also enforces restriction 1 (no term touches two disentanglers);
  if pass 1 places fewer than the requested count, pass 2 walks the same
  order again with restriction 1 relaxed.

The tree shape used for the priorities is the balanced binary split of the
leaf order (left part gets ceil(k/2) leaves); it is computed here only to rank
candidate positions.
"""
from __future__ import annotations


def _subtree_of_pair(n_leaves: int, pa: int, pb: int):
    """Walk the balanced split down to the lowest subtree holding both leaf
    positions.  Returns (size, left child size, right child size)."""
    lo, hi = 0, n_leaves
    while True:
        k = hi - lo
        kl = (k + 1) // 2
        mid = lo + kl
        if pb < mid:
            hi = mid
        elif pa >= mid:
            lo = mid
        else:
            return k, kl, k - kl


def _maxdim(d: int, k: int, N: int) -> int:
    return min(d ** min(k, 64), d ** min(N - k, 64))


def place_disentanglers(n_sites: int, leaf_order, terms, target: int, m: int,
                        d: int = 2, strict_only: bool = False):
    """Return ``(pairs, n_strict)``: the placed site pairs (first site listed is
    the one earlier in the leaf order) and how many came from pass 1."""
    pos = {s: i for i, s in enumerate(leaf_order)}
    cand = []
    seen = set()
    for sites, _, _ in terms:
        if len(sites) != 2:
            continue
        a, b = sites
        if pos[a] > pos[b]:
            a, b = b, a
        if (a, b) in seen:
            continue
        seen.add((a, b))
        size, kl, kr = _subtree_of_pair(n_sites, pos[a], pos[b])
        cand.append(((-size, pos[a], pos[b]), (a, b), (kl, kr)))
    cand.sort(key=lambda c: c[0])

    terms_of_site = {s: [] for s in range(n_sites)}
    for ti, (sites, _, _) in enumerate(terms):
        for s in sites:
            terms_of_site[s].append(ti)

    placed = []
    used = set()
    de_of_site = {}

    def ok_r2(kl, kr):
        return _maxdim(d, kl, n_sites) > m and _maxdim(d, kr, n_sites) > m

    def breaks_r1(a, b):
        for s in (a, b):
            for ti in terms_of_site[s]:
                for t in terms[ti][0]:
                    if t in de_of_site and t not in (a, b):
                        return True
        return False

    def run(enforce_r1):
        for _, (a, b), (kl, kr) in cand:
            if len(placed) >= target:
                return
            if a in used or b in used:
                continue
            if not ok_r2(kl, kr):
                continue
            if enforce_r1 and breaks_r1(a, b):
                continue
            placed.append((a, b))
            used.update((a, b))
            de_of_site[a] = len(placed) - 1
            de_of_site[b] = len(placed) - 1

    run(True)
    n_strict = len(placed)
    if not strict_only:
        run(False)
    return placed, n_strict
