"""Pins of the submap-expansion statistics oracle (Section III-A) on the CPU.

The screen-space gradient is pinned against a closed form (one isotropic
Gaussian on the optical axis) and against central differences of the
oracle's forward under a shift of the principal point, which moves every
projected centre by the same amount and nothing else; visibility and
frustum counts against hand-built cases; the anchor reduction against a
hand-computed dyadic example and invariants; the expansion sampler against
raster-order enumeration, a half-covered render and a re-projection round
trip.
"""
import math

import numpy as np
import pytest

import oracle
import scenes
from oracle import densify


def _one(mean, log_scale, quat, opacity, color=(0.5, 0.4, 0.3)):
    f = lambda a: np.ascontiguousarray(np.asarray(a, np.float64)[None].astype(np.float32))
    return scenes.GaussianSet(f(mean), f(log_scale), f(quat), np.asarray([opacity], np.float32), f(color))


def _zeros(cam):
    H, W = cam.height, cam.width
    return np.zeros((3, H, W)), np.zeros((H, W)), np.zeros((H, W))


def test_isotropic_on_axis_gradient_closed_form():
    # on the optical axis J = diag(f/z) and the 2-D covariance is
    # ((f s / z)^2 + 0.3) I (the renderer's constants are float32 values);
    # with an alpha-only upstream L = sum_p alpha_p and
    # dL/du = sum_p alpha_p (x_p - u) / sigma^2 over the blended pixels
    W, H, f, cx, cy = 40, 30, 50.0, 19.8, 15.3
    cam = scenes.identity_camera(W, H, f, f, cx, cy)
    z, ls, o = 3.0, math.log(0.08), 0.6
    g = _one((0.0, 0.0, z), (ls, ls, ls), (1.0, 0.0, 0.0, 0.0), o)
    gr, gd, ga = _zeros(cam)
    ga[:] = 1.0
    acc, scale, _ = densify.view_accum(g, cam, gr, gd, ga)
    s = math.exp(float(np.float32(ls)))
    sig2 = (f * s / z) ** 2 + float(np.float32(0.3))
    xs, ys = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    ucx, vcy = float(np.float32(cx)), float(np.float32(cy))
    alpha = float(np.float32(o)) * np.exp(-((xs - ucx) ** 2 + (ys - vcy) ** 2) / (2 * sig2))
    alpha = np.where(alpha >= float(np.float32(1) / np.float32(255)), alpha, 0.0)
    gu = float((alpha * (xs - ucx)).sum() / sig2)
    gv = float((alpha * (ys - vcy)).sum() / sig2)
    assert abs(gu) > 1e-3 and abs(gv) > 1e-3
    assert acc[0, 0] == pytest.approx(math.hypot(gu, gv), rel=1e-9)
    assert acc[0, 1] == 1.0 and acc[0, 3] == 1.0 and acc[0, 2] == pytest.approx(o, rel=1e-7)
    assert scale[0] >= acc[0, 0]
    ndc, _, _ = densify.view_accum(g, cam, gr, gd, ga, grad_space=1)
    assert ndc[0, 0] == pytest.approx(math.hypot(gu * W / 2, gv * H / 2), rel=1e-9)


def _loss(g, cam, w):
    r = oracle.render(g, cam)
    return float((w[0] * r["rgb"]).sum() + (w[1] * r["depth"]).sum() + (w[2] * r["alpha"]).sum())


@pytest.mark.parametrize("seed", [3, 4])
def test_gradient_norm_matches_principal_point_shift(seed):
    # u = fx x / z + cx, so d/dcx of the loss is dL/du of the single Gaussian
    rng = np.random.default_rng(seed)
    q = rng.standard_normal(4)
    g = _one((rng.uniform(-0.2, 0.2), rng.uniform(-0.2, 0.2), rng.uniform(2.5, 3.5)),
             rng.normal(-2.2, 0.3, 3), q / np.linalg.norm(q), 0.7, rng.uniform(0, 1, 3))
    cam = scenes.identity_camera(32, 24, 40.0, 40.0, 16.0, 12.0)
    w = scenes.upstream_weights(seed, [cam])[0]
    assert not oracle.render(g, cam, margins=(2e-3, 2e-3, 2e-3))["flags"].any()
    h = 2.0 ** -8  # exact in float32, the precision the intrinsics are taken in
    fd = []
    for attr in ("cx", "cy"):
        cp, cm = cam.copy(), cam.copy()
        setattr(cp, attr, getattr(cam, attr) + h)
        setattr(cm, attr, getattr(cam, attr) - h)
        fd.append((_loss(g, cp, w) - _loss(g, cm, w)) / (2 * h))
    acc, _, _ = densify.view_accum(g, cam, *[x.astype(np.float64) for x in w])
    assert math.hypot(*fd) > 1e-2
    assert acc[0, 0] == pytest.approx(math.hypot(*fd), rel=1e-4)


def test_visibility_and_frustum_counts():
    cam = scenes.identity_camera(40, 30, 50.0, 50.0, 20.0, 15.0)
    cases = [  # mean, log-scale, opacity -> (rendered, in frustum, opacity term)
        ((0.1, 0.0, 3.0), -2.5, 0.5, (1, 1, 0.5)),       # plain visible Gaussian
        ((0.1, 0.0, -2.0), -2.5, 0.5, (0, 0, 0.0)),      # behind the camera
        ((0.1, 0.1, 3.0), -2.5, 0.002, (0, 1, 0.002)),   # in view, below the 1/255 cutoff
        ((-1.38, 0.0, 3.0), -1.0, 0.9, (1, 0, 0.0)),     # centre 3 px left of the image, footprint inside
        ((0.0, 0.95, 3.0), -1.0, 0.9, (1, 0, 0.0)),      # centre 0.8 px below the image, footprint inside
        ((0.0, -0.1, 3.0), -2.5, -0.3, (0, 1, 0.0)),     # negative (invalid) decoded opacity
        ((0.0, 0.0, 0.1), -2.5, 0.5, (0, 0, 0.0)),       # in front of the near plane
    ]
    for mean, ls, o, (ren, inv, op) in cases:
        g = _one(mean, (ls, ls, ls), (1.0, 0.0, 0.0, 0.0), o)
        gr, gd, ga = _zeros(cam)
        gd[:] = 1.0
        acc, _, _ = densify.view_accum(g, cam, gr, gd, ga)
        assert (acc[0, 1], acc[0, 3]) == (ren, inv), (mean, o, acc[0])
        assert acc[0, 2] == pytest.approx(op, rel=1e-7), (mean, o)
        if not ren:
            assert acc[0, 0] == 0.0
        else:
            assert acc[0, 0] > 0.0


def test_anchor_stats_dyadic_example():
    acc = np.array([[0.5, 1, 0.25, 1], [1.5, 2, 0.75, 2], [0, 0, 0, 1],   # anchor 0
                    [0, 0, 0, 0], [0, 0, 0, 0], [0, 0, 0, 0]], np.float32)  # anchor 1: never seen
    st, grow, prune = densify.anchor_stats(acc, 3, tau_g=0.5, tau_o=0.3)
    assert st[0].tolist() == [np.float32(2) / np.float32(3), 3.0, 1.0, 4.0]
    assert st[1].tolist() == [0.0, 0.0, 0.0, 0.0]
    assert grow.tolist() == [True, False] and prune.tolist() == [True, False]  # 1 < 0.3 * 4
    _, grow, prune = densify.anchor_stats(acc, 3, tau_g=0.7, tau_o=0.2)
    assert grow.tolist() == [False, False] and prune.tolist() == [False, False]  # 1 >= 0.2 * 4


def test_anchor_stats_invariants():
    rng = np.random.default_rng(9)
    m, k = 200, 10
    acc = np.zeros((m * k, 4), np.float32)
    acc[:, 1] = rng.integers(0, 5, m * k)
    acc[:, 3] = acc[:, 1] + rng.integers(0, 3, m * k)
    acc[:, 0] = (rng.uniform(0, 2e-3, m * k) * acc[:, 1]).astype(np.float32)
    acc[:, 2] = (rng.uniform(0, 1, m * k) * acc[:, 3]).astype(np.float32)
    st, grow, prune = densify.anchor_stats(acc, k, 1e-3, 0.4)
    # permuting the Gaussians of an anchor changes only rounding
    perm = np.concatenate([a * k + rng.permutation(k) for a in range(m)])
    st2, _, _ = densify.anchor_stats(acc[perm], k, 1e-3, 0.4)
    assert np.array_equal(st[:, 1], st2[:, 1]) and np.array_equal(st[:, 3], st2[:, 3])
    assert np.allclose(st, st2, rtol=1e-6, atol=0)
    # the totals are the column sums, and k = 1 leaves every Gaussian its own anchor
    assert st[:, 1].sum() == acc[:, 1].sum() and st[:, 3].sum() == acc[:, 3].sum()
    one, _, _ = densify.anchor_stats(acc, 1, 1e-3, 0.4)
    seen = acc[:, 1] > 0
    assert np.array_equal(one[seen, 0], acc[seen, 0] / acc[seen, 1]) and np.all(one[~seen, 0] == 0)
    # thresholds act monotonically
    assert np.all(grow <= densify.anchor_stats(acc, k, 5e-4, 0.4)[1])
    assert np.all(prune <= densify.anchor_stats(acc, k, 1e-3, 0.6)[2])
    assert grow.any() and (~grow).any() and prune.any() and (~prune).any()


def test_expansion_candidates_of_a_half_covered_view():
    # an opaque wall of Gaussians over the left half only: the uncovered right
    # half (alpha ~ 0) is where new anchors are sampled; the target depth is
    # the rendered depth itself, so the depth test adds nothing on the left
    cam = scenes.identity_camera(48, 32, 40.0, 40.0, 24.0, 16.0)
    xs, ys = np.meshgrid(np.linspace(-1.9, -0.05, 40), np.linspace(-1.4, 1.4, 30))
    n = xs.size
    means = np.stack([xs.ravel(), ys.ravel(), np.full(n, 3.0)], axis=1)
    g = scenes.GaussianSet(means.astype(np.float32), np.full((n, 3), -2.7, np.float32),
                           np.tile(np.float32([1, 0, 0, 0]), (n, 1)), np.full(n, 0.95, np.float32),
                           np.full((n, 3), 0.5, np.float32))
    r = oracle.render(g, cam)
    alpha, depth = r["alpha"].astype(np.float32), r["depth"].astype(np.float32)
    t = depth.copy()
    t[:, 24:] = 3.0
    cand = densify.expansion_candidates(alpha, depth, t, 0.5, 0.1)
    assert cand[:, 30:].all() and not cand[:, :20].any()
    # the depth test alone flags the right half, where D ~ 0 and T = 3
    assert np.array_equal(densify.expansion_candidates(alpha, depth, t, 0.0, 0.1)[:, 30:], cand[:, 30:])
    # pixels without a target depth never qualify
    t0 = t.copy()
    t0[:, 40:] = 0.0
    assert not densify.expansion_candidates(alpha, depth, t0, 0.5, 0.1)[:, 40:].any()


def test_expansion_sample_ranks_and_round_trip():
    rng = np.random.default_rng(2)
    H, W = 12, 17
    cam = scenes.camera_look((0.3, -0.2, 1.1), 0.4, -0.1, 0.05, W, H, 20.0, 21.0, 8.1, 6.3)
    cand = rng.uniform(size=(H, W)) < 0.3
    t = rng.uniform(0.5, 4.0, (H, W)).astype(np.float32)
    rgb = rng.uniform(0, 1, (3, H, W)).astype(np.float32)
    c = int(cand.sum())
    # u = (r + 1/2) / c enumerates the candidates in raster order
    u = ((np.arange(c) + 0.5) / c).astype(np.float32)
    pix, pts, col = densify.expansion_sample(cand, u, t, rgb, cam)
    order = [y * W + x for y in range(H) for x in range(W) if cand[y, x]]
    assert pix.tolist() == order
    # the ends of [0, 1)
    assert densify.expansion_sample(cand, np.float32([0.0, np.nextafter(np.float32(1), np.float32(0))]),
                                    t, rgb, cam)[0].tolist() == [order[0], order[-1]]
    # re-projecting a sample lands on its pixel centre at the target depth (to
    # the orthogonality of a float32 rotation, R^T standing for its inverse)
    w2c = cam.world_to_cam.astype(np.float64)
    for p, X, cl in zip(pix, pts, col):
        x, y = p % W, p // W
        pc = w2c[:, :3] @ X + w2c[:, 3]
        assert pc[2] == pytest.approx(t[y, x], rel=1e-6)
        assert cam.fx * pc[0] / pc[2] + cam.cx == pytest.approx(x + 0.5, abs=1e-5)
        assert cam.fy * pc[1] / pc[2] + cam.cy == pytest.approx(y + 0.5, abs=1e-5)
        assert np.array_equal(cl, rgb[:, y, x].astype(np.float64))
    # a view without candidates yields -1
    pix, pts, _ = densify.expansion_sample(np.zeros((H, W), bool), u[:3], t, rgb, cam)
    assert pix.tolist() == [-1, -1, -1] and not pts.any()
