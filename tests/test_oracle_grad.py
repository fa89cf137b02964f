"""Pins of the FP64 oracle's gradients (CPU only).

The dual-number gradients are checked against central finite differences of
the oracle's own forward, a linear closed form for the colours, and the
translation identity of the left se(3) pose increment (the gradient that
photometric tracking descends, Section III-B).
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import scenes


class G64:
    """A float64 copy of a Gaussian set, so finite differences can perturb it."""

    def __init__(self, g):
        self.means = g.means.astype(np.float64)
        self.log_scales = g.log_scales.astype(np.float64)
        self.quats = g.quats.astype(np.float64)
        self.opacities = g.opacities.astype(np.float64)
        self.colors = g.colors.astype(np.float64)

    @property
    def n(self):
        return self.means.shape[0]


def _loss(h, cam, w):
    r = oracle.render(h, cam)
    return float((w[0] * r["rgb"]).sum() + (w[1] * r["depth"]).sum() + (w[2] * r["alpha"]).sum())


def _clear_scene(seed):
    """A tiny scene with no pixel near a threshold, so the loss is smooth."""
    for s in range(seed, seed + 50):
        sc = scenes.tiny_scene(s, n=8, width=20, height=16, f=24.0)
        r = oracle.render(sc.sets[0], sc.cameras[0], margins=(2e-3, 2e-3, 2e-3))
        if not r["flags"].any() and r["n_blend"].sum() > 200:
            return sc
    raise RuntimeError("no clear scene")


@pytest.mark.parametrize("seed", [0, 100])
def test_dual_gradients_match_central_differences(seed):
    sc = _clear_scene(seed)
    cam = sc.cameras[0]
    h = G64(sc.sets[0])
    w = [a.astype(np.float64) for a in sc.weights[0]]
    G, S = oracle.grad(h, cam, *w)
    for name in ("means", "log_scales", "quats", "opacities", "colors"):
        arr = getattr(h, name)
        for idx in np.ndindex(arr.shape):
            old = arr[idx]
            step = 1e-6 * max(1.0, abs(old))
            arr[idx] = old + step
            lp = _loss(h, cam, w)
            arr[idx] = old - step
            lm = _loss(h, cam, w)
            arr[idx] = old
            fd = (lp - lm) / (2 * step)
            assert abs(fd - G[name][idx]) <= 1e-6 * S[name][idx] + 1e-8, (name, idx, fd, G[name][idx])


def _perturbed_camera(cam, xi):
    """Left increment: [R|t] <- Exp(xi) [R|t] with xi = (rho, phi)."""
    R = cam.world_to_cam[:, :3].astype(np.float64)
    t = cam.world_to_cam[:, 3].astype(np.float64)
    Rp = Rotation.from_rotvec(xi[3:]).as_matrix()
    c = cam.copy()
    c.world_to_cam = np.concatenate([Rp @ R, (Rp @ t + xi[:3])[:, None]], axis=1)
    return c


class _Cam64:
    """Camera whose pose stays in float64 (the oracle reads it as given)."""

    def __init__(self, cam, w2c):
        self.width, self.height = cam.width, cam.height
        self.fx, self.fy, self.cx, self.cy, self.near = cam.fx, cam.fy, cam.cx, cam.cy, cam.near
        self.world_to_cam = w2c


def test_pose_gradient_matches_central_differences(monkeypatch):
    sc = _clear_scene(7)
    cam = scenes.camera_look((0.05, -0.03, 0.02), 0.02, -0.01, 0.01, 20, 16, 24.0, 24.0, 10.0, 8.0)
    cam.world_to_cam = cam.world_to_cam.astype(np.float64)
    # build the scene in front of this camera: reuse the tiny scene's means
    h = G64(sc.sets[0])
    h.means = h.means[:, [2, 0, 1]] * np.array([1.0, -1.0, -1.0])  # the camera looks along +x
    w = [a.astype(np.float64) for a in sc.weights[0]]
    # keep the pose in float64 so that finite differences see the perturbation
    monkeypatch.setattr(oracle, "_cam_arrays", lambda c: (
        np.array([c.fx, c.fy, c.cx, c.cy, c.near], np.float64), np.ascontiguousarray(c.world_to_cam, np.float64)))
    r = oracle.render(h, cam, margins=(2e-3, 2e-3, 2e-3))
    assert r["n_blend"].sum() > 100
    G, S = oracle.grad(h, cam, *w)
    for k in range(6):
        step = 1e-6
        e = np.zeros(6); e[k] = step
        lp = _loss(h, _Cam64(cam, _perturbed_camera(cam, e).world_to_cam), w)
        lm = _loss(h, _Cam64(cam, _perturbed_camera(cam, -e).world_to_cam), w)
        fd = (lp - lm) / (2 * step)
        assert abs(fd - G["pose"][k]) <= 1e-6 * S["pose"][k] + 1e-8, (k, fd, G["pose"][k])


def test_color_gradient_linear_closed_form():
    """dL/dc_i = sum_p w_i(p) g_rgb(p): the blend weight of Gaussian i is the
    rendered colour when i alone has colour one."""
    sc = scenes.tiny_scene(31, n=10, width=24, height=20)
    g, cam = sc.sets[0], sc.cameras[0]
    gr, gd, ga = (a.astype(np.float64) for a in sc.weights[0])
    G, _ = oracle.grad(g, cam, gr, gd, ga)
    for i in range(g.n):
        h = G64(g)
        h.colors[:] = 0.0
        h.colors[i] = 1.0
        wi = oracle.render(h, cam)["rgb"][0]
        np.testing.assert_allclose(G["colors"][i], [(wi * gr[ch]).sum() for ch in range(3)], rtol=1e-10, atol=1e-12)


def test_opacity_gradient_vanishes_where_clamped():
    """A Gaussian whose alpha is clamped at 0.99 everywhere it is blended has
    zero opacity gradient (the derivative of the clamp)."""
    cam = scenes.identity_camera(8, 8, 10.0, 10.0, 4.0, 4.0)
    g = scenes.GaussianSet(np.array([[0, 0, 2.0]], np.float32), np.full((1, 3), np.log(30.0), np.float32),
                           np.array([[1, 0, 0, 0]], np.float32), np.array([0.999], np.float32),
                           np.array([[0.3, 0.6, 0.9]], np.float32))
    ones = np.ones((3, 8, 8)); o1 = np.ones((8, 8))
    G, _ = oracle.grad(g, cam, ones, o1, o1)
    assert G["opacities"][0] == 0.0
    assert abs(G["colors"][0, 0] - float(np.float32(0.99)) * 64) < 1e-12


def test_translation_identity():
    """dL/drho = R sum_i dL/dmu_i: a camera translation moves every camera-space mean."""
    sc = scenes.make_c1(n=300)
    g, cam = sc.sets[0], sc.cameras[0]
    w = [a.astype(np.float64) for a in sc.weights[0]]
    G, S = oracle.grad(g, cam, *w)
    R = cam.world_to_cam[:, :3].astype(np.float64)
    lhs = G["pose"][:3]
    rhs = R @ G["means"].sum(axis=0)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-10 * S["pose"][:3].max())


def test_translation_identity_rotated_camera():
    sc = scenes.make_c2(n=4000)
    g, cam = sc.sets[0], sc.cameras[0]
    cam = cam.copy(); cam.width, cam.height, cam.cx, cam.cy = 160, 120, 80.0, 60.0
    cam.fx = cam.fy = 131.25
    w = scenes.upstream_weights(5, [cam])[0]
    G, S = oracle.grad(g, cam, *[a.astype(np.float64) for a in w])
    R = cam.world_to_cam[:, :3].astype(np.float64)
    # dL/dmu_i = R^T dL/dp_i; the float32 R is orthonormal only to rounding, so invert R^T
    np.testing.assert_allclose(G["pose"][:3], np.linalg.solve(R.T, G["means"].sum(axis=0)), rtol=0,
                               atol=1e-10 * S["pose"][:3].max())
    assert np.abs(G["pose"]).max() > 0


def test_skip_mask_removes_pixels():
    sc = scenes.tiny_scene(41, n=10, width=24, height=20)
    g, cam = sc.sets[0], sc.cameras[0]
    gr, gd, ga = (a.astype(np.float64) for a in sc.weights[0])
    skip = np.zeros((20, 24), np.uint8); skip[:, 12:] = 1
    G1, _ = oracle.grad(g, cam, gr, gd, ga, skip=skip)
    keep = 1 - skip
    G2, _ = oracle.grad(g, cam, gr * keep, gd * keep, ga * keep)
    for k in G1:
        np.testing.assert_allclose(G1[k], G2[k], rtol=1e-12, atol=1e-14)
