"""Seeded synthetic problem instances shared by the oracle and the GPU library.

This package only generates inputs (lattices, Hamiltonian terms, the site
order, disentangler positions, random draws).  It contains no part of the
method's arithmetic; both implementations receive its arrays and compute
everything else themselves.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .lattice import hilbert_order, square_bonds, triangular_bonds
from .models import (ising_terms, ising_chain_terms, heisenberg_triangular_terms,
                     ising_terms_xx_form, PX, PZ, IPY)
from .placement import place_disentanglers
from .draws import draw_inputs, balanced_tree_shapes, haar_orthogonal


@dataclass
class Problem:
    name: str
    n_sites: int
    d: int
    m: int
    leaf_order: list
    terms: list                     # [(sites, [ops], coef)]
    de_sites: list                  # [(a, b)]
    de_u: np.ndarray                # [n_de, d^2, d^2], row index |s_a s_b>, a major
    raw_tensors: list               # Gaussian blocks per node, post-order
    n_de_strict: int = 0
    meta: dict = field(default_factory=dict)

    # flat arrays in the layout of the C interface
    def flat_terms(self):
        nsites = np.array([len(t[0]) for t in self.terms], dtype=np.int32)
        sites = np.array([s for t in self.terms for s in t[0]], dtype=np.int32)
        ops = np.concatenate([np.asarray(o, dtype=np.float64).ravel()
                              for t in self.terms for o in t[1]])
        coef = np.array([t[2] for t in self.terms], dtype=np.float64)
        return nsites, sites, ops, coef

    def raw_concat(self):
        return np.concatenate([r.ravel() for r in self.raw_tensors]) if self.raw_tensors \
            else np.zeros(0)


def make_problem(name, L, model, m, seed, n_de_target, h=3.0, J=1.0,
                 strict_only=False, identity_de=False, d=2):
    """Build an L x L instance.

    model: "ising" (-sum ZZ - h sum X) or "heisenberg_tri" (J sum S.S).
    """
    N = L * L
    order = hilbert_order(L)
    if model == "ising":
        terms = ising_terms(L, h, J)
    elif model == "heisenberg_tri":
        terms = heisenberg_triangular_terms(L, J)
    else:
        raise ValueError(model)
    pairs, n_strict = place_disentanglers(N, order, terms, n_de_target, m, d,
                                          strict_only=strict_only)
    shapes = balanced_tree_shapes(N, m, d)
    us, raw = draw_inputs(seed, len(pairs), shapes, d)
    if identity_de:
        us = np.stack([np.eye(d * d)] * len(pairs)) if pairs else us
    return Problem(name=name, n_sites=N, d=d, m=m, leaf_order=order, terms=terms,
                   de_sites=pairs, de_u=us, raw_tensors=raw, n_de_strict=n_strict,
                   meta=dict(L=L, model=model, h=h, J=J, seed=seed))


def make_chain_problem(name, N, h, m, seed, de_pairs=(), d=2):
    """Open Ising chain of N sites in natural order, optional disentanglers."""
    order = list(range(N))
    terms = ising_chain_terms(N, h)
    shapes = balanced_tree_shapes(N, m, d)
    us, raw = draw_inputs(seed, len(de_pairs), shapes, d)
    return Problem(name=name, n_sites=N, d=d, m=m, leaf_order=order, terms=terms,
                   de_sites=list(de_pairs), de_u=us, raw_tensors=raw,
                   meta=dict(model="ising_chain", h=h, seed=seed))


# The benchmark workloads (seeded, synthetic; the paper's models and sizes).
CONFIGS = {
    # 4x4 Ising, h = 3, m = 8, 4 disentanglers, 5 sweeps, seed 1
    "ising4_m8": dict(L=4, model="ising", h=3.0, m=8, seed=1, n_de=4, sweeps=5),
    # 8x8 Ising, h = 3.05, m = 32, 16 disentanglers, 8 sweeps, seed 2
    "ising8_m32": dict(L=8, model="ising", h=3.05, m=32, seed=2, n_de=16, sweeps=8),
    "ising8_m16": dict(L=8, model="ising", h=3.05, m=16, seed=2, n_de=16, sweeps=8),
    # 16x16 Ising, h = 3, m = 64, 64 disentanglers, seed 16 (headline workload)
    "ising16_m64": dict(L=16, model="ising", h=3.0, m=64, seed=16, n_de=64, sweeps=12),
    # 16x16 triangular Heisenberg, m = 96, 64 disentanglers, seed 4
    "heis16_m96": dict(L=16, model="heisenberg_tri", h=0.0, m=96, seed=4, n_de=64, sweeps=6),
    # 32x32 Ising, h = 3.05, m = 128, 256 disentanglers, seed 5
    "ising32_m128": dict(L=32, model="ising", h=3.05, m=128, seed=5, n_de=256, sweeps=3),
    # 16x16 Ising at m = 128: the (128, 128, 128) node shape of the 32x32 workload
    # on a lattice the oracle can hold in memory
    "ising16_m128": dict(L=16, model="ising", h=3.0, m=128, seed=16, n_de=64, sweeps=3),
}


def config_problem(key, **over):
    c = dict(CONFIGS[key])
    c.update(over)
    return make_problem(key, c["L"], c["model"], c["m"], c["seed"], c["n_de"],
                        h=c.get("h", 3.0), strict_only=c.get("strict_only", False),
                        identity_de=c.get("identity_de", False))


def batch_instances(n=32, base_seed=3):
    """Independent Ising instances of uneven size: L in {8,12,16},
    m in {16,32,48,64}, h ~ U[2.5, 3.5], L^2/4 disentanglers, seed 1000+i."""
    rng = np.random.default_rng(base_seed)
    out = []
    for i in range(n):
        L = int(rng.choice([8, 12, 16]))
        m = int(rng.choice([16, 32, 48, 64]))
        h = float(rng.uniform(2.5, 3.5))
        out.append(make_problem(f"batch{i}", L, "ising", m, 1000 + i, L * L // 4, h=h))
    return out
