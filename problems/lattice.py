"""Lattice geometry for the benchmark models: bonds and the 2D -> 1D site order.

Input generation only: nothing here computes any part of the aTTN method.
Site ids are ``x * L + y`` with ``x`` the row index.

* Square lattice, open boundaries (quantum Ising model, paper Sec. 6, eq. 8).
* Triangular lattice, open boundaries, built as the square lattice plus one
  diagonal per plaquette (Heisenberg model, paper Sec. 6, eq. 9 and the
  triangular-lattice benchmark section); the diagonal is (x, y)-(x+1, y+1).
* Hilbert-curve ordering of the lattice sites (paper Sec. 6, the 2D -> 1D
  mapping used before building the tree).
"""
from __future__ import annotations


def square_bonds(L: int) -> list[tuple[int, int]]:
    """Nearest-neighbour bonds of an L x L open-boundary square lattice."""
    bonds = []
    for x in range(L):
        for y in range(L):
            s = x * L + y
            if x + 1 < L:
                bonds.append((s, (x + 1) * L + y))
            if y + 1 < L:
                bonds.append((s, x * L + y + 1))
    return bonds


def triangular_bonds(L: int) -> list[tuple[int, int]]:
    """Square-lattice bonds plus the (x, y)-(x+1, y+1) diagonal, open boundaries.

    Count: 3 L^2 - 4 L + 1.
    """
    bonds = square_bonds(L)
    for x in range(L - 1):
        for y in range(L - 1):
            bonds.append((x * L + y, (x + 1) * L + y + 1))
    return bonds


def _hilbert_d2xy(n: int, d: int) -> tuple[int, int]:
    """Classic Hilbert-curve index -> (x, y) on an n x n grid, n a power of two."""
    x = y = 0
    s = 1
    t = d
    while s < n:
        rx = 1 & (t // 2)
        ry = 1 & (t ^ rx)
        if ry == 0:
            if rx == 1:
                x = s - 1 - x
                y = s - 1 - y
            x, y = y, x
        x += s * rx
        y += s * ry
        t //= 4
        s *= 2
    return x, y


def hilbert_order(L: int) -> list[int]:
    """Site ids of an L x L lattice in Hilbert-curve order.

    For L not a power of two the curve of the enclosing 2^p x 2^p grid is
    walked and only points inside the lattice are kept, in curve order.
    """
    n = 1
    while n < L:
        n *= 2
    order = []
    for d in range(n * n):
        x, y = _hilbert_d2xy(n, d)
        if x < L and y < L:
            order.append(x * L + y)
    return order
