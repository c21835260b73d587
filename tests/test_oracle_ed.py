"""Pins for exact diagonalisation: closed forms and special cases."""
import numpy as np
import pytest

from problems.models import ising_chain_terms, ising_terms, ising_terms_xx_form
from oracle.ed import ground_energy, ising_chain_exact, hamiltonian_sparse


@pytest.mark.parametrize("N,h", [(8, 0.5), (10, 1.0), (12, 3.0)])
def test_chain_ed_matches_free_fermion_closed_form(N, h):
    assert abs(ground_energy(ising_chain_terms(N, h), N) - ising_chain_exact(N, h)) < 1e-10


def test_chain_closed_form_limits():
    # h = 0: classical ferromagnet, -(N - 1); J = 0 equivalent: h large -> -N h
    assert abs(ising_chain_exact(20, 0.0) + 19.0) < 1e-12
    assert abs(ising_chain_exact(5, 1e6) + 5e6) / 5e6 < 1e-9


def test_square_lattice_h0_is_minus_bond_count():
    assert abs(ground_energy(ising_terms(4, 0.0), 16) + 24.0) < 1e-10
    assert abs(ground_energy(ising_terms(3, 0.0), 9) + 12.0) < 1e-10


def test_ising_axis_forms_agree():
    # -sum ZZ - h sum X and -sum XX - h sum Z differ by a Hadamard on every site
    for h in (0.7, 3.0):
        a = ground_energy(ising_terms(3, h), 9)
        b = ground_energy(ising_terms_xx_form(3, h), 9)
        assert abs(a - b) < 1e-10


def test_sparse_matches_dense_eigvalsh():
    terms = ising_terms(3, 2.0)
    H = hamiltonian_sparse(terms, 9).toarray()
    assert np.allclose(H, H.T)
    w = np.linalg.eigvalsh(H)[0]
    from scipy.sparse.linalg import eigsh
    w2 = eigsh(hamiltonian_sparse(terms, 9), k=1, which='SA', tol=1e-13)[0][0]
    assert abs(w - w2) < 1e-10


def test_hamiltonian_single_term_matrix():
    # one ZZ term on sites (0, 2) of 3 sites is diag(+1,-1,+1,-1,-1,+1,-1,+1)... times coef
    H = hamiltonian_sparse([((0, 2), [np.diag([1., -1.]), np.diag([1., -1.])], 2.0)], 3).toarray()
    bits = [((k >> 2) & 1, (k >> 1) & 1, k & 1) for k in range(8)]
    expect = [2.0 * (1 - 2 * b[0]) * (1 - 2 * b[2]) for b in bits]
    assert np.allclose(np.diag(H), expect) and np.allclose(H, np.diag(expect))
