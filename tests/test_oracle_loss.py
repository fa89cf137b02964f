"""Pins of the mapping-loss oracle (eq. 7-9) against closed forms, a
brute-force SSIM and central differences (CPU)."""
import math

import numpy as np
import pytest

from oracle import loss


def _imgs(seed, H=14, W=17):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, (3, H, W))
    y = np.clip(x + rng.normal(0, 0.1, x.shape), 0, 1)
    d = rng.uniform(1, 5, (H, W))
    t = d + rng.normal(0, 0.2, d.shape)
    t[rng.uniform(size=t.shape) < 0.2] = 0.0  # pixels without a target depth
    return x, d, y, t


def test_window_is_the_normalised_gaussian():
    g = loss.window_1d()
    assert g.shape == (11,) and abs(g.sum() - 1.0) < 1e-15
    assert np.allclose(g, g[::-1])
    # ratio of neighbouring taps exp(((k - 5)^2 - (k - 4)^2) / (2 * 1.5^2))
    for k in range(1, 11):
        assert math.isclose(g[k] / g[k - 1], math.exp(-((k - 5) ** 2 - (k - 6) ** 2) / 4.5), rel_tol=1e-12)


def test_ssim_matches_bruteforce_window_sums():
    x, _, y, _ = _imgs(1, H=9, W=13)
    fast = loss.ssim_map(x, y).numpy()
    brute = loss.ssim_map_bruteforce(x, y)
    assert np.max(np.abs(fast - brute)) < 1e-12


def test_ssim_of_identical_images_is_one_and_has_zero_gradient():
    x, d, _, _ = _imgs(2)
    s = loss.ssim_map(x, x).numpy()
    assert np.allclose(s, 1.0, atol=1e-12)
    # with depth equal too, the only loss term is 0 and so is the gradient
    gx, gd = loss.view_loss_grad(x, d, x, d)
    assert np.abs(gx).max() < 1e-15 and np.abs(gd).max() == 0.0  # SSIM's stationary point, up to rounding
    assert loss.view_loss(x, d, x, d)["total"] == 0.0


def test_ssim_of_constant_images_interior_closed_form():
    # away from the border (5 px) the local variances vanish and SSIM is the
    # luminance term (2ab + C1) / (a^2 + b^2 + C1)
    a, b = 0.3, 0.7
    x = np.full((1, 24, 24), a)
    y = np.full((1, 24, 24), b)
    s = loss.ssim_map(x, y).numpy()[0, 5:-5, 5:-5]
    want = (2 * a * b + loss.C1) / (a * a + b * b + loss.C1)
    assert np.allclose(s, want, rtol=1e-12)


def test_l1_and_depth_terms_closed_form():
    x, d, y, t = _imgs(3)
    terms = loss.view_loss(x, d, y, t, lam_ssim=0.2, lam_d=0.7)
    l1 = np.abs(x - y).mean()
    valid = t > 0
    ld = np.abs(d - t)[valid].mean()
    assert math.isclose(terms["L_c"], l1, rel_tol=1e-13)
    assert math.isclose(terms["L_d"], ld, rel_tol=1e-13)
    ssim = loss.ssim_map(x, y).numpy().mean()
    assert math.isclose(terms["L_ssim"], 0.8 * l1 + 0.2 * (1 - ssim), rel_tol=1e-13)
    assert math.isclose(terms["total"], l1 + 0.8 * l1 + 0.2 * (1 - ssim) + 0.7 * ld, rel_tol=1e-13)


def test_gradient_matches_central_differences():
    x, d, y, t = _imgs(4, H=10, W=12)
    gx, gd = loss.view_loss_grad(x, d, y, t, 0.2, 1.0)
    rng = np.random.default_rng(5)
    h = 1e-6
    f = lambda xx, dd: loss.view_loss(xx, dd, y, t, 0.2, 1.0)["total"]
    for _ in range(12):
        c, i, j = rng.integers(0, 3), rng.integers(0, 10), rng.integers(0, 12)
        if abs(x[c, i, j] - y[c, i, j]) < 1e-3:
            continue  # the L1 kink
        xp, xm = x.copy(), x.copy()
        xp[c, i, j] += h; xm[c, i, j] -= h
        fd = (f(xp, d) - f(xm, d)) / (2 * h)
        assert abs(fd - gx[c, i, j]) < 1e-7 * max(1.0, abs(fd)), (c, i, j, fd, gx[c, i, j])
    for _ in range(8):
        i, j = rng.integers(0, 10), rng.integers(0, 12)
        if t[i, j] > 0 and abs(d[i, j] - t[i, j]) < 1e-3:
            continue
        dp, dm = d.copy(), d.copy()
        dp[i, j] += h; dm[i, j] -= h
        fd = (f(x, dp) - f(x, dm)) / (2 * h)
        assert abs(fd - gd[i, j]) < 1e-7 * max(1.0, abs(fd))
    # pixels without a target depth get no depth gradient
    assert np.all(gd[t <= 0] == 0.0)


def test_volume_term_closed_form():
    rng = np.random.default_rng(6)
    l = rng.normal(-3, 0.5, (50, 3))
    val, g = loss.volume_loss(l, 0.001)
    prod = np.exp(l).prod(axis=1)
    assert math.isclose(val, 0.001 * prod.sum(), rel_tol=1e-13)
    # d/dl_k prod(exp(l)) = prod(exp(l))
    assert np.allclose(g, 0.001 * prod[:, None], rtol=1e-13)
