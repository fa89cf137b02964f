"""Submap-fusion distillation loss of eq. 14 in NumPy float64 -- TEST INFRASTRUCTURE.

Section III-C fuses two submaps alpha and beta after a loop closure by
rendering both at the poses of the m keyframes of their overlap and
penalising the squared differences of the rendered colour and depth.  Per
keyframe k with images rendered from alpha (C_a [3,H,W], D_a [H,W]) and from
beta (C_b, D_b):

    l_k = mean over channels and pixels of (C_a - C_b)^2
        + mean over pixels of (D_a - D_b)^2

and L = (1/m) sum_k l_k.  Both submaps receive gradients (the loss merges
them): dL/dC_a = 2 (C_a - C_b) / (m 3 H W) = -dL/dC_b, and likewise for the
depth with 1/(m H W).
"""
from __future__ import annotations

import numpy as np

__all__ = ["pair_terms", "distill_loss"]


def pair_terms(ca, da, cb, db):
    """(colour MSE, depth MSE) of one keyframe, float64."""
    ca, da, cb, db = (np.asarray(x, np.float64) for x in (ca, da, cb, db))
    return float(np.mean((ca - cb) ** 2)), float(np.mean((da - db) ** 2))


def distill_loss(pairs):
    """pairs: list of (C_a, D_a, C_b, D_b) per keyframe.  Returns (L, terms
    [m, 2], grads) with grads[k] = (dL/dC_a, dL/dD_a, dL/dC_b, dL/dD_b)."""
    m = len(pairs)
    terms = np.zeros((m, 2))
    grads = []
    for k, (ca, da, cb, db) in enumerate(pairs):
        ca, da, cb, db = (np.asarray(x, np.float64) for x in (ca, da, cb, db))
        terms[k] = pair_terms(ca, da, cb, db)
        gc = 2.0 * (ca - cb) / (m * ca.size)
        gd = 2.0 * (da - db) / (m * da.size)
        grads.append((gc, gd, -gc, -gd))
    return float(terms.sum() / m) if m else 0.0, terms, grads
