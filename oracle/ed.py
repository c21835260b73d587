"""Exact diagonalisation and full-state helpers (oracle side).

H = sum of tensor-product terms (paper Sec. 3.3) as a sparse 2^N x 2^N matrix,
site 0 the most significant bit.  Used to pin the oracle's energies and its
effective Hamiltonians for N <= 16.

Closed form for the open transverse-field Ising chain -J sum Z Z - h sum X:
by the Jordan-Wigner mapping the ground energy is minus the sum of the
singular values of the N x N upper-bidiagonal matrix with h on the diagonal
and J on the superdiagonal (free-fermion modes).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def term_sparse(sites, ops, coef, N, d=2):
    """coef * (ops on sites) as a sparse matrix on N sites."""
    mats = []
    by_site = dict(zip(sites, ops))
    out = sp.identity(1, format='csr')
    for s in range(N):
        if s in by_site:
            out = sp.kron(out, sp.csr_matrix(by_site[s]), format='csr')
        else:
            out = sp.kron(out, sp.identity(d, format='csr'), format='csr')
    del mats
    return coef * out


def hamiltonian_sparse(terms, N, d=2):
    H = sp.csr_matrix((d ** N, d ** N))
    for sites, ops, coef in terms:
        H = H + term_sparse(sites, ops, coef, N, d)
    return H


def ground_energy(terms, N, d=2):
    """Lowest eigenvalue by sparse Lanczos (ARPACK), tolerance 1e-13."""
    H = hamiltonian_sparse(terms, N, d)
    if d ** N <= 256:
        return float(np.linalg.eigvalsh(H.toarray())[0])
    w = spla.eigsh(H, k=1, which='SA', tol=1e-13, return_eigenvectors=False)
    return float(w[0])


def ising_chain_exact(N, h, J=1.0):
    """Ground energy of the open chain -J sum Z_i Z_{i+1} - h sum X_i."""
    B = np.diag(np.full(N, float(h))) + np.diag(np.full(N - 1, float(J)), 1)
    return -float(np.linalg.svd(B, compute_uv=False).sum())


def apply_two_site(psi, u, a, b, N, d=2):
    """Apply the d^2 x d^2 gate u on sites (a, b) (a major) to a 2^N vector."""
    t = psi.reshape([d] * N)
    t = np.moveaxis(t, [a, b], [0, 1])
    sh = t.shape
    t = (u @ t.reshape(d * d, -1)).reshape(sh)
    t = np.moveaxis(t, [0, 1], [a, b])
    return t.reshape(-1)


def apply_layer(psi, de_sites, de_u, N, d=2, transpose=False):
    """D psi (or D^T psi) for the disentangler layer D = prod_k u_k."""
    for (a, b), u in zip(de_sites, de_u):
        psi = apply_two_site(psi, u.T if transpose else u, a, b, N, d)
    return psi
