"""Hamiltonians of the benchmark models as lists of tensor-product terms.

A Hamiltonian is a sum of terms h_a (paper Sec. 3.3, the TPO representation);
each term here is ``(sites, ops, coef)`` with ``ops[i]`` the real d x d matrix
acting on ``sites[i]`` and the term equal to ``coef * (ops[0] x ops[1] ...)``.
Local (one-site) terms are kept one per site and per operator.

Conventions (all real arithmetic):

* Quantum Ising: H = -J sum_<ij> Z_i Z_j - h sum_i X_i  (the paper's eq. 8 up to
  a Hadamard rotation of every site, which leaves the spectrum unchanged).
* Heisenberg: H = J sum_<ij> S_i . S_j with S = sigma / 2 (eq. 9 uses the Pauli
  matrices; the two differ by a factor 4).  Y_i Y_j is written as
  -(iY)_i (iY)_j with iY = [[0, 1], [-1, 0]] so that every operator is real.
"""
from __future__ import annotations

import numpy as np

from .lattice import square_bonds, triangular_bonds

PX = np.array([[0.0, 1.0], [1.0, 0.0]])
PZ = np.array([[1.0, 0.0], [0.0, -1.0]])
IPY = np.array([[0.0, 1.0], [-1.0, 0.0]])  # i * sigma_y, real


def ising_terms(L: int, h: float, J: float = 1.0, bonds=None):
    """Terms of -J sum Z Z - h sum X on an L x L open square lattice."""
    if bonds is None:
        bonds = square_bonds(L)
    terms = []
    for (i, j) in bonds:
        terms.append(((i, j), [PZ, PZ], -J))
    for s in range(L * L):
        terms.append(((s,), [PX], -h))
    return terms


def ising_chain_terms(N: int, h: float, J: float = 1.0):
    """Terms of -J sum Z_i Z_{i+1} - h sum X_i on an open chain of N sites."""
    terms = [((i, i + 1), [PZ, PZ], -J) for i in range(N - 1)]
    terms += [((s,), [PX], -h) for s in range(N)]
    return terms


def ising_terms_xx_form(L: int, h: float):
    """The paper's sign/axis form -sum X X - h sum Z (figure 1 text)."""
    terms = [((i, j), [PX, PX], -1.0) for (i, j) in square_bonds(L)]
    terms += [((s,), [PZ], -h) for s in range(L * L)]
    return terms


def heisenberg_triangular_terms(L: int, J: float = 1.0):
    """Terms of J sum S.S on the L x L open triangular lattice.

    Three terms per bond (XX, YY, ZZ), kept separate.
    """
    terms = []
    for (i, j) in triangular_bonds(L):
        terms.append(((i, j), [PX, PX], 0.25 * J))
        terms.append(((i, j), [IPY, IPY], -0.25 * J))
        terms.append(((i, j), [PZ, PZ], 0.25 * J))
    return terms


def interaction_bonds(terms) -> list[tuple[int, int]]:
    """Distinct site pairs of the two-site terms, in first-appearance order."""
    seen = set()
    out = []
    for sites, _, _ in terms:
        if len(sites) == 2:
            key = tuple(sites)
            if key not in seen:
                seen.add(key)
                out.append(key)
    return out
