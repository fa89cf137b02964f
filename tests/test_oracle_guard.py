"""Pins of the oracle's field-of-view guard on the EWA Jacobian (CPU only).

The projection linearises the pinhole map at each Gaussian's camera-space
mean.  Far outside the image that linearisation blows up, so the direction
x/z (and y/z) at which it is taken is clamped to 1.3 times the half field of
view; with the principal point at the image centre that is the pixel-margin
form [-0.15 W, 1.15 W] x [-0.15 H, 1.15 H].  The projected centre itself is
not clamped.  These tests pin that reading with quantities the oracle does
not compute the same way:

* the guard limits come from the field of view, 1.3 tan(fov / 2) (the method's
  FP32 literals 0.15 and 1.15 move them by under 4e-8 relative, which sets
  the tolerances below);
* the covariance of a Gaussian past the guard equals J' Sigma J'^T + 0.3 I
  where J' is the central-difference Jacobian of the pinhole map at the
  clamped point (scipy builds the rotation of the covariance);
* the clamped axis carries no derivative: moving the mean along it leaves
  the covariance unchanged, while inside the guard it changes it;
* a Gaussian centred past the guard whose footprint reaches the image is
  rendered with that covariance around its unclamped centre;
* the oracle's gradient of such a Gaussian matches central differences of
  its forward.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import scenes

DILATE = float(np.float32(0.3))
A_MIN = float(np.float32(1.0) / np.float32(255.0))
A_MAX = float(np.float32(0.99))

W, H, F = 128, 96, 100.0


class G64:
    def __init__(self, means, ls, quats, opac, cols):
        self.means = np.asarray(means, np.float64).reshape(-1, 3)
        self.log_scales = np.asarray(ls, np.float64).reshape(-1, 3)
        self.quats = np.asarray(quats, np.float64).reshape(-1, 4)
        self.opacities = np.asarray(opac, np.float64).reshape(-1)
        self.colors = np.asarray(cols, np.float64).reshape(-1, 3)

    @property
    def n(self):
        return self.means.shape[0]


def _cam():
    return scenes.identity_camera(W, H, F, F, W / 2.0, H / 2.0)


def _fov_limits(cam):
    """1.3 x tan(half field of view) per axis, from the image size alone."""
    return 1.3 * (cam.width / 2.0) / cam.fx, 1.3 * (cam.height / 2.0) / cam.fy


def _pinhole_jacobian_fd(cam, p):
    """Central differences of (fx x/z + cx, fy y/z + cy) at camera point p."""
    def pi(q):
        return np.array([cam.fx * q[0] / q[2] + cam.cx, cam.fy * q[1] / q[2] + cam.cy])
    J = np.zeros((2, 3))
    for k in range(3):
        h = 1e-5 * max(1.0, abs(p[k]))
        e = np.zeros(3); e[k] = h
        J[:, k] = (pi(p + e) - pi(p - e)) / (2 * h)
    return J


def _sigma(ls, q):
    """World covariance R_q diag(exp(2 l)) R_q^T, rotation from scipy (w, x, y, z)."""
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    return R @ np.diag(np.exp(2.0 * np.asarray(ls, np.float64))) @ R.T


def _expected_cov2d(cam, mean, ls, q):
    lx, ly = _fov_limits(cam)
    z = mean[2]
    tx = np.clip(mean[0] / z, -lx, lx)
    ty = np.clip(mean[1] / z, -ly, ly)
    J = _pinhole_jacobian_fd(cam, np.array([tx * z, ty * z, z]))
    C = J @ _sigma(ls, q) @ J.T
    return C[0, 0] + DILATE, C[0, 1], C[1, 1] + DILATE


def test_guard_limits_are_the_widened_field_of_view():
    cam = _cam()
    lx, ly = _fov_limits(cam)
    # with the principal point at the image centre, 1.3 tan(fov/2) is the
    # pixel-margin form (1.15 W - cx) / fx = (cx + 0.15 W) / fx
    assert math.isclose(lx, (1.15 * W - cam.cx) / cam.fx, rel_tol=1e-15)
    assert math.isclose(lx, (cam.cx + 0.15 * W) / cam.fx, rel_tol=1e-15)
    assert math.isclose(ly, (1.15 * H - cam.cy) / cam.fy, rel_tol=1e-15)


@pytest.mark.parametrize("axis,sign", [(0, 1), (0, -1), (1, 1), (1, -1)])
@pytest.mark.parametrize("where", [0.97, 1.03, 1.6])
def test_covariance_past_the_guard_uses_the_clamped_jacobian(axis, sign, where):
    """Inside (0.97 of the limit) the Jacobian is taken at the mean; past it
    (1.03, 1.6) at the point on the guard, on that axis only."""
    cam = _cam()
    lim = _fov_limits(cam)[axis]
    z = 2.5
    mean = np.array([0.1 * z, -0.05 * z, z])
    mean[axis] = sign * where * lim * z
    ls = np.log([0.05, 0.11, 0.03])
    q = np.array([0.8, 0.3, -0.4, 0.33])
    q /= np.linalg.norm(q)
    g = G64(mean, ls, q, [0.9], [0.5, 0.5, 0.5])
    p = oracle.project(g, cam)
    a, b, c = _expected_cov2d(cam, mean, ls, q)
    np.testing.assert_allclose([p["a"][0], p["b"][0], p["c"][0]], [a, b, c], rtol=2e-7)
    # the unclamped Jacobian would give another covariance past the guard
    J = _pinhole_jacobian_fd(cam, mean)
    C = J @ _sigma(ls, q) @ J.T
    differs = not np.allclose([p["a"][0], p["b"][0], p["c"][0]], [C[0, 0] + DILATE, C[0, 1], C[1, 1] + DILATE],
                              rtol=1e-4)
    assert differs == (where > 1.0)
    # the centre is not clamped (F7)
    assert math.isclose(p["u"][0], cam.fx * mean[0] / z + cam.cx, rel_tol=1e-13)
    assert math.isclose(p["v"][0], cam.fy * mean[1] / z + cam.cy, rel_tol=1e-13)


@pytest.mark.parametrize("axis", [0, 1])
def test_clamped_axis_has_no_derivative(axis):
    """Central differences of the covariance with respect to the mean along
    the clamped axis vanish past the guard and not inside it."""
    cam = _cam()
    lim = _fov_limits(cam)[axis]
    z = 3.0
    ls = np.log([0.08, 0.05, 0.12])
    q = np.array([0.6, -0.2, 0.5, 0.59])
    q /= np.linalg.norm(q)

    def mean_at(x):
        mean = np.array([0.05 * z, 0.07 * z, z])
        mean[axis] = x
        return mean

    def cov(x):
        p = oracle.project(G64(mean_at(x), ls, q, [0.9], [0.5, 0.5, 0.5]), cam)
        return np.array([p["a"][0], p["b"][0], p["c"][0]])

    h = 1e-4
    outside = 1.25 * lim * z
    d_out = (cov(outside + h) - cov(outside - h)) / (2 * h)
    assert np.all(d_out == 0.0), d_out
    inside = 0.8 * lim * z
    d_in = (cov(inside + h) - cov(inside - h)) / (2 * h)
    d_exp = (np.array(_expected_cov2d(cam, mean_at(inside + h), ls, q)) -
             np.array(_expected_cov2d(cam, mean_at(inside - h), ls, q))) / (2 * h)
    assert np.abs(d_in).max() > 0.1, d_in
    np.testing.assert_allclose(d_in, d_exp, rtol=1e-3, atol=1e-6 * np.abs(d_exp).max())


def _guard_gaussian():
    """An isotropic Gaussian centred past the right guard (x/z = 1.0 against
    a limit of 0.832) whose footprint still covers the right image border."""
    z, s = 2.0, 0.3
    return G64([1.0 * z, 0.1 * z, z], np.log([s, s, s]), [1, 0, 0, 0], [0.9], [0.2, 0.6, 0.9])


def test_gaussian_past_the_guard_renders_with_the_clamped_covariance():
    cam = _cam()
    g = _guard_gaussian()
    a, b, c = _expected_cov2d(cam, g.means[0], g.log_scales[0], g.quats[0])
    det = a * c - b * b
    Qa, Qb, Qc = c / det, -b / det, a / det
    u = cam.fx * g.means[0, 0] / g.means[0, 2] + cam.cx
    v = cam.fy * g.means[0, 1] / g.means[0, 2] + cam.cy
    assert u > 1.15 * W  # centred past the guard
    px = np.arange(W)[None, :] + 0.5 - u
    py = np.arange(H)[:, None] + 0.5 - v
    sigma = 0.5 * (Qa * px * px + Qc * py * py) + Qb * px * py
    alpha = np.minimum(A_MAX, g.opacities[0] * np.exp(-sigma))
    alpha = np.where(alpha >= A_MIN, alpha, 0.0)
    assert (alpha > 0).sum() > 200  # the footprint reaches the image
    r = oracle.render(g, cam)
    np.testing.assert_allclose(r["alpha"], alpha, rtol=1e-6, atol=1e-12)
    for ch in range(3):
        np.testing.assert_allclose(r["rgb"][ch], alpha * g.colors[0, ch], rtol=1e-6, atol=1e-12)


def test_gradient_past_the_guard_matches_central_differences():
    cam = _cam()
    g = _guard_gaussian()
    g.quats[0] = [0.9, 0.1, -0.3, 0.2]           # anisotropic, rotated
    g.log_scales[0] = np.log([0.3, 0.2, 0.4])
    w = scenes.upstream_weights(11, [cam])[0]
    r = oracle.render(g, cam, margins=(1e-3, 1e-3, 1e-3))
    keep = (~r["flags"]).astype(np.float64)
    wr, wd, wa = (x.astype(np.float64) * keep for x in w)
    G, S = oracle.grad(g, cam, wr, wd, wa)

    def loss():
        rr = oracle.render(g, cam)
        return float((wr * rr["rgb"]).sum() + (wd * rr["depth"]).sum() + (wa * rr["alpha"]).sum())

    for name in ("means", "log_scales", "quats", "opacities"):
        arr = getattr(g, name)
        for idx in np.ndindex(arr.shape):
            old = arr[idx]
            h = 1e-6 * max(1.0, abs(old))
            arr[idx] = old + h; lp = loss()
            arr[idx] = old - h; lm = loss()
            arr[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - G[name][idx]) <= 1e-6 * S[name][idx] + 1e-8, (name, idx, fd, G[name][idx])
