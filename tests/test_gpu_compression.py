"""Compressed terms (ATTN_COMPRESS_TERMS: terms on the same sites summed
into one, paper Sec. 6.2.2 closing paragraph) through the C interface.

Parity with the oracle's compressed form on the triangular Heisenberg model
(matvec at every node, sweep energies); the compressed and the plain handle
hold the same Hamiltonian, so their matvecs agree on the same tensors and
their sweeps follow the same trajectory; the compressed one needs less
effective-operator storage."""
import numpy as np
import pytest

from problems import make_problem
from tests.gpu_util import move_both, gpu_matvec, rel

pytestmark = pytest.mark.gpu

ATTN_COMPRESS_TERMS = 8


def _pair(p):
    from paper_2507_21236_amd import AttnHandle
    from oracle.ttn import OracleTTN
    a = AttnHandle(p, flags=ATTN_COMPRESS_TERMS)
    a.init_state()
    o = OracleTTN(p.n_sites, p.d, p.m, p.leaf_order, p.terms, p.de_sites, p.de_u, p.raw_tensors,
                  compress=True)
    return a, o


def test_compressed_matvec_every_node_and_sweeps_against_oracle():
    p = make_problem("heis4", 4, "heisenberg_tri", 8, 4, 4)
    a, o = _pair(p)
    rng = np.random.default_rng(6)
    for n in range(o.tree.n_nodes):
        move_both(a, o, n)
        x = rng.standard_normal(o.T[n].shape)
        assert rel(gpu_matvec(a, n, x), o.matvec(n, x)) < 1e-12, n
    a2, o2 = _pair(p)
    e, _ = a2.sweep(3)
    for s in range(3):
        e_o = o2.sweep()
        assert abs(e[s] - e_o) / p.n_sites < 1e-10, (s, e[s], e_o)


def test_compressed_equals_plain_handle():
    from paper_2507_21236_amd import AttnHandle
    p = make_problem("heis8", 8, "heisenberg_tri", 16, 4, 16)
    c = AttnHandle(p, flags=ATTN_COMPRESS_TERMS)
    u = AttnHandle(p)
    assert c.env_bytes < u.env_bytes
    c.init_state()
    u.init_state()
    rng = np.random.default_rng(9)
    for n in (10, 40, u.root - 1, u.root):
        c.move_center(n)
        u.move_center(n)
        x = rng.standard_normal(u.node_info(n)[0])
        assert rel(gpu_matvec(c, n, x), gpu_matvec(u, n, x)) < 1e-12, n
    c.init_state()
    u.init_state()
    ec, _ = c.sweep(2)
    eu, _ = u.sweep(2)
    print("compressed", ec, "plain", eu, "env bytes", c.env_bytes, u.env_bytes)
    assert np.abs(ec - eu).max() / p.n_sites < 1e-9
