"""Pins of the FP64 oracle's forward render against closed forms, invariants,
library routines and brute force (CPU only).

The forward follows the compositing cutoffs of the method (alpha >= 1/255,
clamp at 0.99, stop before blending once the transmittance would fall under
1e-4) over EWA-projected Gaussians (eq. 6 renders colour and opacity of the
submaps; depth feeds the L1 depth loss of eq. 7).
"""
import math

import numpy as np
import pytest

import oracle
import scenes
from scenes import Camera, GaussianSet

# FP32 literals of the method, promoted to double (the oracle's constants).
A_MIN = float(np.float32(1.0) / np.float32(255.0))
A_MAX = float(np.float32(0.99))
T_MIN = float(np.float32(1e-4))
DILATE = float(np.float32(0.3))


def f32(x):
    """The float32 value of x, as the renderer receives it."""
    return np.asarray(x, np.float32).astype(np.float64)


def _gs(means, ls, quats, opac, cols):
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return GaussianSet(f(means), f(ls), f(quats), f(opac), f(cols))


def _cam(W=40, H=30, f=50.0):
    return scenes.identity_camera(W, H, f, f, W / 2.0, H / 2.0)


def _pix_r2(cam, u, v):
    px = np.arange(cam.width) + 0.5
    py = np.arange(cam.height) + 0.5
    return (px[None, :] - u) ** 2 + (py[:, None] - v) ** 2


def test_single_isotropic_gaussian_closed_form():
    cam = _cam(80, 60)
    z, o = 3.0, float(f32(0.9999))
    ls = np.float32(math.log(0.5))
    col = f32([0.2, 0.5, 0.9])
    g = _gs([[0, 0, z]], [[ls, ls, ls]], [[0.3, -0.5, 0.1, 0.8]], [o], [col])
    r = oracle.render(g, cam)
    s = math.exp(float(ls))
    var = (cam.fx * s / z) ** 2 + DILATE
    alpha = np.minimum(A_MAX, o * np.exp(-_pix_r2(cam, cam.cx, cam.cy) / (2 * var)))
    alpha = np.where(alpha >= A_MIN, alpha, 0.0)
    assert (alpha >= A_MAX).any() and (alpha == 0).any()
    np.testing.assert_allclose(r["alpha"], alpha, rtol=1e-12, atol=1e-15)
    for ch in range(3):
        np.testing.assert_allclose(r["rgb"][ch], alpha * col[ch], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(r["depth"], alpha * z, rtol=1e-12, atol=1e-15)
    assert not r["flags"].any()


def test_two_gaussians_front_to_back():
    cam = _cam()
    s1, s2 = 0.08, 0.15
    z1, z2 = 2.5, 4.0
    o1, o2 = float(f32(0.6)), float(f32(0.9))
    c1, c2 = f32([1.0, 0.0, 0.2]), f32([0.0, 1.0, 0.7])
    g = _gs([[0, 0, z2], [0, 0, z1]], np.log([[s2] * 3, [s1] * 3]), [[1, 0, 0, 0]] * 2, [o2, o1], [c2, c1])
    r = oracle.render(g, cam)
    r2 = _pix_r2(cam, cam.cx, cam.cy)
    s1f, s2f = math.exp(float(np.float32(math.log(s1)))), math.exp(float(np.float32(math.log(s2))))
    z1, z2 = float(f32(z1)), float(f32(z2))
    a1 = o1 * np.exp(-r2 / (2 * ((cam.fx * s1f / z1) ** 2 + DILATE)))
    a2 = o2 * np.exp(-r2 / (2 * ((cam.fx * s2f / z2) ** 2 + DILATE)))
    both = (a1 > 2 * A_MIN) & (a2 > 2 * A_MIN)
    assert both.sum() > 20
    exp_c = a1[..., None] * c1 + ((1 - a1) * a2)[..., None] * c2
    np.testing.assert_allclose(np.moveaxis(r["rgb"], 0, -1)[both], exp_c[both], rtol=1e-12)
    np.testing.assert_allclose(r["depth"][both], (a1 * z1 + (1 - a1) * a2 * z2)[both], rtol=1e-12)
    np.testing.assert_allclose(r["alpha"][both], (1 - (1 - a1) * (1 - a2))[both], rtol=1e-12)
    none = (a1 < 0.5 * A_MIN) & (a2 < 0.5 * A_MIN)
    assert none.sum() > 20
    assert np.all(r["rgb"][:, none] == 0) and np.all(r["alpha"][none] == 0)


def test_termination_stack_stops_before_blending():
    """Four co-centred wide Gaussians, o = 0.95: after three blends T is about
    0.05^3 = 1.25e-4, so the fourth would take T under 1e-4 and is not blended."""
    cam = _cam()
    zs = [3.0, 3.2, 3.4, 3.6]
    cols = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]], float)
    s = 0.6
    g = _gs([[0, 0, z] for z in zs], np.log([[s] * 3] * 4), [[1, 0, 0, 0]] * 4, [0.95] * 4, cols)
    r = oracle.render(g, cam)
    sf = math.exp(float(np.float32(math.log(s))))
    r2 = _pix_r2(cam, cam.cx, cam.cy)
    zs = list(f32(zs))
    al = [f32(0.95) * np.exp(-r2 / (2 * ((cam.fx * sf / z) ** 2 + DILATE))) for z in zs]
    T3 = (1 - al[0]) * (1 - al[1]) * (1 - al[2])
    T4 = T3 * (1 - al[3])
    regime = (T3 > 1.05 * T_MIN) & (T4 < 0.95 * T_MIN)
    assert regime.sum() >= 4
    Ts = [np.ones_like(r2), 1 - al[0], (1 - al[0]) * (1 - al[1])]
    exp_c = sum((al[i] * Ts[i])[..., None] * cols[i] for i in range(3))
    exp_d = sum(al[i] * Ts[i] * zs[i] for i in range(3))
    np.testing.assert_allclose(np.moveaxis(r["rgb"], 0, -1)[regime], exp_c[regime], rtol=1e-12)
    np.testing.assert_allclose(r["depth"][regime], exp_d[regime], rtol=1e-12)
    np.testing.assert_allclose(r["alpha"][regime], 1 - T3[regime], rtol=1e-12)
    assert np.all(r["n_blend"][regime] == 3)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_weights_plus_final_transmittance_is_one(seed):
    sc = scenes.tiny_scene(seed, n=30, width=32, height=24)
    g = sc.sets[0]
    g.colors[:] = 1.0
    r = oracle.render(g, sc.cameras[0])
    for ch in range(3):
        np.testing.assert_allclose(r["rgb"][ch] + r["T_final"], 1.0, rtol=0, atol=1e-13)
    assert r["n_blend"].max() > 3


@pytest.mark.parametrize("seed", [3, 4, 5, 6])
def test_brute_force_equals_box_accelerated(seed):
    sc = scenes.tiny_scene(seed, n=20, width=32, height=32)
    g, cam = sc.sets[0], sc.cameras[0]
    a = oracle.render(g, cam)
    b = oracle.render(g, cam, brute_force=True)
    for k in ("rgb", "depth", "alpha", "T_final", "n_blend"):
        assert np.array_equal(a[k], b[k]), k


def test_brute_force_equals_box_accelerated_c1():
    sc = scenes.make_c1()
    a = oracle.render(sc.sets[0], sc.cameras[0])
    b = oracle.render(sc.sets[0], sc.cameras[0], brute_force=True)
    for k in ("rgb", "depth", "alpha", "n_blend"):
        assert np.array_equal(a[k], b[k]), k
    assert a["n_blend"].sum() > 50_000


def test_box_is_conservative():
    """Every pixel where a Gaussian reaches alpha >= 1/255 lies in its box."""
    sc = scenes.tiny_scene(11, n=40, width=48, height=40)
    g, cam = sc.sets[0], sc.cameras[0]
    p = oracle.project(g, cam)
    px = np.arange(cam.width) + 0.5
    py = np.arange(cam.height) + 0.5
    checked = 0
    for i in np.nonzero(p["valid"])[0]:
        dx = p["u"][i] - px[None, :]
        dy = p["v"][i] - py[:, None]
        sig = 0.5 * (p["Qa"][i] * dx * dx + p["Qc"][i] * dy * dy) + p["Qb"][i] * dx * dy
        hit = np.minimum(A_MAX, g.opacities[i] * np.exp(-sig)) >= A_MIN
        x0, x1, y0, y1 = p["box"][i]
        ys, xs = np.nonzero(hit)
        assert np.all((xs >= x0) & (xs <= x1) & (ys >= y0) & (ys <= y1))
        checked += hit.sum()
    assert checked > 100


def _rotation_xyzw(q):
    from scipy.spatial.transform import Rotation
    q = np.asarray(q, np.float64)
    return Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()


def test_projection_matches_library_rotation_and_fd_jacobian():
    """Sigma2D = J R Sigma R^T J^T + 0.3 I with R_q from scipy and J from a
    central difference of the pinhole map."""
    rng = np.random.default_rng(7)
    cam = scenes.camera_look((0.3, -0.2, 0.1), 0.4, 0.2, 0.1, 64, 48, 70.0, 72.0, 31.0, 25.0)
    Rc = cam.world_to_cam[:, :3].astype(np.float64)
    tc = cam.world_to_cam[:, 3].astype(np.float64)
    n = 25
    fwd = Rc.T @ np.array([0, 0, 1.0])
    means = (np.array([0.3, -0.2, 0.1]) + fwd * rng.uniform(2, 4, (n, 1))
             + rng.uniform(-0.4, 0.4, (n, 3))).astype(np.float32)
    g = _gs(means, rng.normal(-2.5, 0.5, (n, 3)), rng.standard_normal((n, 4)),
            rng.uniform(0.3, 0.9, n), rng.uniform(0, 1, (n, 3)))
    p = oracle.project(g, cam)

    def pin(pc):
        return np.array([cam.fx * pc[0] / pc[2] + cam.cx, cam.fy * pc[1] / pc[2] + cam.cy])

    for i in range(n):
        pc = Rc @ g.means[i].astype(np.float64) + tc
        J = np.zeros((2, 3))
        for k in range(3):
            h = 1e-6
            e = np.zeros(3); e[k] = h
            J[:, k] = (pin(pc + e) - pin(pc - e)) / (2 * h)
        Rq = _rotation_xyzw(g.quats[i])
        S = np.diag(np.exp(2 * g.log_scales[i].astype(np.float64)))
        Sig = Rq @ S @ Rq.T
        ev = np.linalg.eigvalsh(Sig)
        np.testing.assert_allclose(np.sort(ev), np.sort(np.exp(2 * g.log_scales[i].astype(np.float64))), rtol=1e-10)
        S2 = J @ Rc @ Sig @ Rc.T @ J.T + DILATE * np.eye(2)
        np.testing.assert_allclose([p["a"][i], p["b"][i], p["c"][i]], [S2[0, 0], S2[0, 1], S2[1, 1]],
                                   rtol=1e-6, atol=1e-9)
        det = S2[0, 0] * S2[1, 1] - S2[0, 1] ** 2
        np.testing.assert_allclose([p["Qa"][i], p["Qb"][i], p["Qc"][i]],
                                   [S2[1, 1] / det, -S2[0, 1] / det, S2[0, 0] / det], rtol=1e-5)
        np.testing.assert_allclose([p["u"][i], p["v"][i], p["z"][i]], [*pin(pc), pc[2]], rtol=1e-12)


def test_projection_on_axis_closed_form():
    cam = _cam(64, 48, 80.0)
    s, z = 0.05, 2.0
    g = _gs([[0, 0, z]], np.log([[s] * 3]), [[0.2, 0.9, -0.3, 0.4]], [0.7], [[0.5] * 3])
    p = oracle.project(g, cam)
    sf = math.exp(float(np.float32(math.log(s))))
    var = (cam.fx * sf / z) ** 2 + DILATE
    np.testing.assert_allclose([p["a"][0], p["c"][0]], [var, var], rtol=1e-12)
    assert abs(p["b"][0]) < 1e-12
    assert p["u"][0] == cam.cx and p["v"][0] == cam.cy


def test_quaternion_sign_and_norm_invariance():
    sc = scenes.tiny_scene(21, n=15)
    g, cam = sc.sets[0], sc.cameras[0]
    a = oracle.render(g, cam)
    g2 = _gs(g.means, g.log_scales, -2.0 * g.quats, g.opacities, g.colors)
    b = oracle.render(g2, cam)
    for k in ("rgb", "depth", "alpha"):
        np.testing.assert_allclose(a[k], b[k], rtol=1e-12, atol=1e-14)


def test_fp32_spec_values_match_ieee_float32():
    """The FP32 values that decide integers (depth bits, projected centres)
    equal an IEEE float32 evaluation in the stated operation order."""
    sc = scenes.make_c2(n=3000)
    g, cam = sc.sets[0], sc.cameras[0]
    p = oracle.project(g, cam)
    R = cam.world_to_cam[:, :3].astype(np.float32)
    t = cam.world_to_cam[:, 3].astype(np.float32)
    m = g.means
    f32 = np.float32
    x = ((R[0, 0] * m[:, 0] + R[0, 1] * m[:, 1]) + R[0, 2] * m[:, 2]) + t[0]
    y = ((R[1, 0] * m[:, 0] + R[1, 1] * m[:, 1]) + R[1, 2] * m[:, 2]) + t[1]
    z = ((R[2, 0] * m[:, 0] + R[2, 1] * m[:, 1]) + R[2, 2] * m[:, 2]) + t[2]
    u = f32(cam.fx) * (x / z) + f32(cam.cx)
    v = f32(cam.fy) * (y / z) + f32(cam.cy)
    assert z.dtype == np.float32 and u.dtype == np.float32
    assert np.array_equal(p["z32"].view(np.uint32), z.view(np.uint32))
    front = z > f32(0.2)
    assert np.array_equal(p["u32"][front].view(np.uint32), u[front].view(np.uint32))
    assert np.array_equal(p["v32"][front].view(np.uint32), v[front].view(np.uint32))


def test_culling_rules():
    cam = _cam()
    g = _gs([[0, 0, 0.1], [0, 0, 3.0], [0, 0, 3.0], [0, 0, 3.0], [0, 0, 3.0]],
            np.log([[0.1] * 3] * 5),
            [[1, 0, 0, 0], [1, 0, 0, 0], [0, 0, 0, 0], [1, 0, 0, 0], [1, 0, 0, 0]],
            [0.5, 0.5, 0.5, float(np.float32(1.0) / np.float32(255.0)), 0.5],
            [[1, 1, 1]] * 5)
    g.means[4] = [50.0, 0.0, 3.0]    # far outside the image
    p = oracle.project(g, cam)
    # behind near plane, normal, zero quaternion, o == 1/255, off-screen
    assert list(p["valid"]) == [False, True, False, False, False]
