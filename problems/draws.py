"""Seeded random inputs: disentangler unitaries and raw initial tensors.

All draws come from ``numpy.random.default_rng(seed)`` in a fixed order:
first one 4 x 4 Gaussian per disentangler (placement order), then one
Gaussian block per tree node in post-order.  The raw node blocks are handed to
both implementations unchanged; each side turns them into isometries itself.
"""
from __future__ import annotations

import numpy as np


def haar_orthogonal(rng: np.random.Generator, n: int) -> np.ndarray:
    """Haar-distributed real orthogonal n x n matrix (QR of a Gaussian with the
    signs of R's diagonal moved into Q; Mezzadri's construction)."""
    a = rng.standard_normal((n, n))
    q, r = np.linalg.qr(a)
    return q * np.sign(np.diag(r))[None, :]


def balanced_tree_shapes(n_sites: int, m: int, d: int = 2):
    """Node shapes (m_l, m_r, m_p) in post-order for the balanced binary split
    with a single root whose parent leg has dimension 1.

    Dimension of the link above a k-site subtree: min(m, d^k, d^(N-k)).
    Used only to size the raw Gaussian draws.
    """
    N = n_sites

    def dim(k):
        if k == N:
            return 1
        return min(m, d ** min(k, 62), d ** min(N - k, 62))

    shapes = []

    def rec(k):
        if k == 1:
            return
        kl = (k + 1) // 2
        rec(kl)
        rec(k - kl)
        shapes.append((dim(kl), dim(k - kl), dim(k)))

    rec(N)
    return shapes


def draw_inputs(seed: int, n_de: int, shapes, d: int = 2):
    """Returns (de_unitaries [n_de, d^2, d^2], raw node blocks list)."""
    rng = np.random.default_rng(seed)
    us = np.stack([haar_orthogonal(rng, d * d) for _ in range(n_de)]) if n_de else \
        np.zeros((0, d * d, d * d))
    raw = [rng.standard_normal(s) for s in shapes]
    return us, raw
