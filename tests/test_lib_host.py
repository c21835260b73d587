"""Host-side tests of the C library (no GPU): exported symbols, the rotated-TPO
build and its flop model against the oracle, bounds of every device work list
(dry-run build), and the error codes of the C interface."""
import os
import re

import numpy as np
import pytest

from problems import config_problem, make_chain_problem, batch_instances, make_problem
from paper_2507_21236_amd import AttnHandle, ATTN_HOST_ONLY, ATTN_DRYRUN, ATTN_DE_STRICT, AttnError
from paper_2507_21236_amd import _lib
from oracle.ttn import OracleTTN

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "attn.h")).read()
    declared = sorted(set(re.findall(r"^\s*(?:attn_status|const char\*)\s+(attn_\w+)\(", hdr, re.M)))
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(_lib._lib, name), name
    assert set(declared) == set(_lib.EXPORTED)


def _oracle_structure(p):
    return OracleTTN(p.n_sites, p.d, p.m, p.leaf_order, p.terms, p.de_sites, p.de_u,
                     p.raw_tensors, structure_only=True)


@pytest.mark.parametrize("make", [
    lambda: config_problem("ising4_m8"),
    lambda: config_problem("ising8_m32"),
    lambda: make_chain_problem("c", 12, 1.7, 8, 9, de_pairs=[(1, 3), (4, 6), (8, 10)]),
    lambda: [p for p in batch_instances(8) if p.meta["L"] == 12][0],
])
def test_host_build_matches_oracle_structure(make):
    # dims, number of crossing terms and the flop model (integers) at every node
    p = make()
    a = AttnHandle(p, flags=ATTN_HOST_ONLY)
    o = _oracle_structure(p)
    assert a.n_nodes == o.tree.n_nodes and a.root == o.tree.root
    for n in range(a.n_nodes):
        dims, nc, fl = a.node_info(n)
        assert tuple(dims) == tuple(o.tree.dims[n])
        assert nc == len(o.crossing_terms(n))
        assert fl == o.flops(n), n


@pytest.mark.slow
def test_host_build_matches_oracle_structure_16x16():
    p = config_problem("ising16_m64")
    a = AttnHandle(p, flags=ATTN_HOST_ONLY)
    o = _oracle_structure(p)
    for n in range(a.n_nodes):
        dims, nc, fl = a.node_info(n)
        assert nc == len(o.crossing_terms(n)) and fl == o.flops(n), n


@pytest.mark.parametrize("make", [
    lambda: config_problem("ising4_m8"),
    lambda: config_problem("ising8_m32"),
    lambda: config_problem("ising16_m64"),
    lambda: make_chain_problem("c", 12, 1.7, 8, 9, de_pairs=[(1, 3), (4, 6), (8, 10)]),
] + [(lambda i=i: batch_instances(8)[i]) for i in range(8)])
def test_dryrun_work_lists_in_bounds(make):
    a = AttnHandle(make(), flags=ATTN_DRYRUN)
    a.validate()


def _flat(p):
    nsites, sites, ops, coef = p.flat_terms()
    return dict(n_sites=p.n_sites, d=p.d, m=p.m, leaf_order=p.leaf_order, term_nsites=nsites,
                term_sites=sites, term_ops=ops, term_coef=coef,
                de_sites=np.asarray(p.de_sites, dtype=np.int32).reshape(-1, 2), de_u=p.de_u)


def _code(**kw):
    try:
        h = _lib.attn_build_tpo(**kw)
        _lib.attn_destroy(h)
        return 0
    except AttnError as e:
        return e.code


def test_error_codes():
    p = config_problem("ising4_m8")
    base = _flat(p)
    base["flags"] = ATTN_HOST_ONLY
    assert _code(**base) == 0
    bad = dict(base); bad["de_u"] = base["de_u"].copy(); bad["de_u"][0, 0, 0] += 1e-6
    assert _code(**bad) == -2                                     # NOT_UNITARY
    bad = dict(base); bad["de_sites"] = np.array([[4, 8], [8, 11]], dtype=np.int32)
    bad["de_u"] = base["de_u"][:2]
    assert _code(**bad) == -4                                     # DE_OVERLAP
    bad = dict(base); bad["leaf_order"] = [0] * 16
    assert _code(**bad) == -1                                     # ARG
    bad = dict(base); bad["term_ops"] = base["term_ops"].copy(); bad["term_ops"][1] = 0.5
    assert _code(**bad) == -3                                     # NOT_HERMITIAN
    bad = dict(base); bad["m"] = 0
    assert _code(**bad) == -1
    # strict mode: a term touching two disentanglers (relaxed placement of 8x8)
    q = _flat(config_problem("ising8_m32"))
    q["flags"] = ATTN_HOST_ONLY | ATTN_DE_STRICT
    assert _code(**q) == -5                                       # DE_RESTRICTION
    q["flags"] = ATTN_HOST_ONLY
    assert _code(**q) == 0


def test_device_calls_on_host_only_handle_fail_cleanly():
    a = AttnHandle(config_problem("ising4_m8"), flags=ATTN_HOST_ONLY)
    with pytest.raises(AttnError) as e:
        a.init_state()
    assert e.value.code == -8
    with pytest.raises(AttnError):
        _lib.attn_node_info(a.h, 99)


def test_batch_create_rejects_bad_input_on_host():
    from paper_2507_21236_amd import AttnBatch
    a = AttnHandle(config_problem("ising4_m8"), flags=ATTN_HOST_ONLY)
    with pytest.raises(AttnError) as e:
        AttnBatch([a])
    assert e.value.code == -8          # STATE: handle cannot run on the device
    assert "device" in str(e.value)
    with pytest.raises(AttnError) as e:
        _lib.attn_batch_create([], 20)
    assert e.value.code == -1          # ARG: no handles
    with pytest.raises(AttnError) as e:
        _lib.attn_batch_create([a.h, a.h], 20)
    assert e.value.code in (-1, -8)


def test_binding_loads_torch_before_library():
    # torch carries its own HIP runtime; the binding imports it before loading
    # libattn.so so that one runtime serves both in a process
    import sys
    assert "torch" in sys.modules
    assert _lib.LIB_PATH.endswith("libattn.so")


def test_disentangler_optimisation_needs_the_strict_placement():
    # 8 x 8 relaxed placement: four gates share a term with another gate
    a = AttnHandle(config_problem("ising8_m32"), flags=ATTN_HOST_ONLY)
    with pytest.raises(AttnError) as e:
        a.optimize_disentanglers()
    assert e.value.code == -5
    b = AttnHandle(config_problem("ising8_m32", strict_only=True), flags=ATTN_HOST_ONLY)
    with pytest.raises(AttnError) as e:
        b.optimize_disentanglers()
    assert e.value.code == -8          # strict placement accepted, then: no device state
    u = b.get_disentanglers()
    assert u.shape == (len(b.problem.de_sites), 4, 4)
    assert np.allclose(u, np.asarray(b.problem.de_u))
