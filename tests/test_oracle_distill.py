"""Pins of the distillation-loss oracle (eq. 14) on the CPU: constant-image
closed form, central differences, zero at identical renders, and the
exchange symmetry of the two submaps."""
import math

import numpy as np

from oracle import distill


def _pairs(seed, m=3, H=7, W=9):
    rng = np.random.default_rng(seed)
    return [(rng.uniform(0, 1, (3, H, W)), rng.uniform(1, 5, (H, W)), rng.uniform(0, 1, (3, H, W)),
             rng.uniform(1, 5, (H, W))) for _ in range(m)]


def test_constant_images_closed_form():
    H, W = 4, 5
    vals = [(0.2, 1.5, 0.7, 2.5), (0.9, 3.0, 0.4, 3.25)]
    pairs = [(np.full((3, H, W), a), np.full((H, W), d), np.full((3, H, W), b), np.full((H, W), e))
             for a, d, b, e in vals]
    L, terms, _ = distill.distill_loss(pairs)
    want = [(a - b) ** 2 + (d - e) ** 2 for a, d, b, e in vals]
    assert np.allclose(terms.sum(axis=1), want, rtol=1e-15)
    assert math.isclose(L, sum(want) / 2, rel_tol=1e-15)


def test_gradient_matches_central_differences():
    pairs = _pairs(1)
    L, _, grads = distill.distill_loss(pairs)
    rng = np.random.default_rng(2)
    h = 1e-6
    for _ in range(16):
        k, which = int(rng.integers(0, 3)), int(rng.integers(0, 4))
        arr = pairs[k][which]
        idx = tuple(int(rng.integers(0, s)) for s in arr.shape)
        plus = [list(p) for p in pairs]
        minus = [list(p) for p in pairs]
        plus[k][which] = arr.copy(); plus[k][which][idx] += h
        minus[k][which] = arr.copy(); minus[k][which][idx] -= h
        fd = (distill.distill_loss(plus)[0] - distill.distill_loss(minus)[0]) / (2 * h)
        assert abs(fd - grads[k][which][idx]) < 1e-8, (k, which, idx, fd, grads[k][which][idx])


def test_identical_renders_and_exchange_symmetry():
    pairs = _pairs(3)
    same = [(ca, da, ca.copy(), da.copy()) for ca, da, _, _ in pairs]
    L, terms, grads = distill.distill_loss(same)
    assert L == 0.0 and not terms.any() and all(not g.any() for gs in grads for g in gs)
    L1, t1, g1 = distill.distill_loss(pairs)
    L2, t2, g2 = distill.distill_loss([(cb, db, ca, da) for ca, da, cb, db in pairs])
    assert L1 == L2 and np.array_equal(t1, t2)
    for a, b in zip(g1, g2):
        assert np.array_equal(a[0], b[2]) and np.array_equal(a[1], b[3])
