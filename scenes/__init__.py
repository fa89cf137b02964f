"""Seeded synthetic inputs for the Gaussian-splatting render path.

This module only draws random numbers and lays them out.  It holds none of
the renderer's or the decoder's arithmetic, so both the HIP path and the CPU
oracle can be fed from it without sharing any computation.

The paper's datasets (Replica, ScanNet, KITTI, VKITTI2, Newer College;
Section IV, "Datasets") are not available, so each workload below is a
synthetic stand-in with the shape, size and value distribution of the
paper's setting:

* ``c1``  1 000 random Gaussians, one 128x96 view (small parity case).
* ``c2``  200 k Gaussians on planar patches of a 6x5x3 m room, one 640x480
          RGB-D view at a random interior pose (the tracking step; room size
          chosen near the Replica/ScanNet rooms of Section IV).
* ``c3``  50 k voxel anchors (0.1 m grid) with 32-d features, k = 10 neural
          Gaussians each through a width-64 MLP decoder (Section III-A,
          eq. 1-5), one 1200x680 view.
* ``c4``  1 M Gaussians in a 24x8x3 m corridor shared by 8 keyframes of
          mixed resolution on a 20 m path (the mapping window).
* ``c5``  4 submaps x 1.5 M Gaussians along a 200 m street (ground and
          facades), 16 keyframes at 1242x375 (KITTI-like street frames).
* ``street scan``  1.5 M map points on an 80 m street with boxes, one
          64-beam LiDAR sweep in the sensor frame, the true and a perturbed
          pose (the voxel-map registration of the fine tracking stage).

Seeds are ``100 * config + purpose`` (1 scene, 2 poses, 3 loss weights)
unless a caller overrides them.  Every array is float32, C-contiguous.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Camera", "GaussianSet", "AnchorSet", "Decoder", "Scene",
    "camera_look", "random_gaussians", "upstream_weights",
    "make_c1", "make_c2", "make_c3", "make_c4", "make_c5", "make_config", "StreetScan", "make_street_scan",
    "tiny_scene",
]


@dataclasses.dataclass
class Camera:
    """Pinhole camera. ``world_to_cam`` is the 3x4 row-major [R|t]."""
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    world_to_cam: np.ndarray  # (3, 4) float32
    near: float = 0.2

    def copy(self) -> "Camera":
        return dataclasses.replace(self, world_to_cam=self.world_to_cam.copy())


@dataclasses.dataclass
class GaussianSet:
    means: np.ndarray       # (n, 3)
    log_scales: np.ndarray  # (n, 3)
    quats: np.ndarray       # (n, 4) (w, x, y, z)
    opacities: np.ndarray   # (n,)   post-activation
    colors: np.ndarray      # (n, 3) post-activation

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def arrays(self):
        return (self.means, self.log_scales, self.quats, self.opacities, self.colors)


@dataclasses.dataclass
class AnchorSet:
    xyz: np.ndarray      # (m, 3) voxel centres
    feat: np.ndarray     # (m, 32)
    scale: np.ndarray    # (m, 3) > 0
    offsets: np.ndarray  # (m, k, 3)

    @property
    def m(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def k(self) -> int:
        return int(self.offsets.shape[1])


@dataclasses.dataclass
class Decoder:
    """Three independent LINEAR-ReLU-LINEAR heads (opacity, colour, covariance).

    Weights use the (out, in) row-major convention; head h maps
    ``in_dim -> width -> out_h`` with out = (k, 3k, 7k).
    """
    in_dim: int
    width: int
    k: int
    W1: List[np.ndarray]
    b1: List[np.ndarray]
    W2: List[np.ndarray]
    b2: List[np.ndarray]


@dataclasses.dataclass
class Scene:
    """A workload: Gaussian sets (or anchors + decoder), views, loss weights."""
    name: str
    sets: List[GaussianSet]
    cameras: List[Camera]
    view_set: List[int]                     # which set each view renders
    weights: Optional[list] = None          # per view: (g_rgb[3,H,W], g_depth[H,W], g_alpha[H,W])
    anchors: Optional[AnchorSet] = None
    decoder: Optional[Decoder] = None


# ----------------------------------------------------------------------------
# camera helpers
# ----------------------------------------------------------------------------

def _rot_axis(axis: np.ndarray, ang: float) -> np.ndarray:
    axis = axis / np.linalg.norm(axis)
    x, y, z = axis
    c, s = math.cos(ang), math.sin(ang)
    C = 1.0 - c
    return np.array([[c + x * x * C, x * y * C - z * s, x * z * C + y * s],
                     [y * x * C + z * s, c + y * y * C, y * z * C - x * s],
                     [z * x * C - y * s, z * y * C + x * s, c + z * z * C]])


def camera_look(center, yaw: float, pitch: float, roll: float, width: int, height: int,
                fx: float, fy: float, cx: float, cy: float, near: float = 0.2) -> Camera:
    """World z is up.  The camera looks along (yaw, pitch); image x is right, y down."""
    center = np.asarray(center, dtype=np.float64)
    fwd = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
    up = np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    if roll != 0.0:
        Rr = _rot_axis(fwd, roll)
        right, down = Rr @ right, Rr @ down
    c2w = np.stack([right, down, fwd], axis=1)
    R = c2w.T
    t = -R @ center
    w2c = np.concatenate([R, t[:, None]], axis=1).astype(np.float32)
    return Camera(width, height, float(fx), float(fy), float(cx), float(cy), w2c, near)


def _look_at(center, target, width, height, fx, fy, cx, cy) -> Camera:
    d = np.asarray(target, np.float64) - np.asarray(center, np.float64)
    yaw = math.atan2(d[1], d[0])
    pitch = math.atan2(d[2], math.hypot(d[0], d[1]))
    return camera_look(center, yaw, pitch, 0.0, width, height, fx, fy, cx, cy)


def identity_camera(width: int, height: int, fx: float, fy: float, cx: float, cy: float) -> Camera:
    w2c = np.zeros((3, 4), np.float32)
    w2c[0, 0] = w2c[1, 1] = w2c[2, 2] = 1.0
    return Camera(width, height, fx, fy, cx, cy, w2c)


# ----------------------------------------------------------------------------
# Gaussian attribute draws
# ----------------------------------------------------------------------------

def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _unit_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def random_gaussians(rng, means, ls_mu, ls_sigma, opa_mu, opa_sigma) -> GaussianSet:
    n = means.shape[0]
    ls = rng.normal(ls_mu, ls_sigma, (n, 3))
    q = _unit_quats(rng, n)
    o = _sigmoid(rng.normal(opa_mu, opa_sigma, n))
    c = rng.uniform(0.0, 1.0, (n, 3))
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return GaussianSet(f(means), f(ls), f(q), f(o), f(c))


def upstream_weights(seed: int, cams: Sequence[Camera]):
    """Loss weights w ~ N(0, 1) per output element, one triple per view."""
    rng = np.random.default_rng(seed)
    out = []
    for cam in cams:
        H, W = cam.height, cam.width
        out.append((rng.standard_normal((3, H, W)).astype(np.float32),
                    rng.standard_normal((H, W)).astype(np.float32),
                    rng.standard_normal((H, W)).astype(np.float32)))
    return out


# ----------------------------------------------------------------------------
# surface models: boxes (room / corridor) plus random rectangles
# ----------------------------------------------------------------------------

def _box_faces(size):
    """The 6 inner faces of an axis-aligned box [0, size] as (origin, e1, e2)."""
    X, Y, Z = size
    o = np.zeros(3)
    ex, ey, ez = np.array([X, 0, 0.]), np.array([0, Y, 0.]), np.array([0, 0, Z])
    return [(o, ex, ey), (o + ez, ex, ey), (o, ex, ez), (o + ey, ex, ez), (o, ey, ez), (o + ex, ey, ez)]


def _random_rects(rng, count, size, side_lo=0.3, side_hi=1.5):
    rects = []
    size = np.asarray(size, np.float64)
    for _ in range(count):
        a, b = rng.uniform(side_lo, side_hi, 2)
        R = _rot_axis(rng.standard_normal(3), rng.uniform(0, 2 * math.pi))
        ctr = rng.uniform(0.15 * size, 0.85 * size)
        e1, e2 = R[:, 0] * a, R[:, 1] * b
        rects.append((ctr - 0.5 * e1 - 0.5 * e2, e1, e2))
    return rects


def _sample_patches(rng, patches, n):
    areas = np.array([np.linalg.norm(np.cross(e1, e2)) for (_, e1, e2) in patches])
    idx = rng.choice(len(patches), size=n, p=areas / areas.sum())
    uv = rng.uniform(0.0, 1.0, (n, 2))
    O = np.stack([p[0] for p in patches])[idx]
    E1 = np.stack([p[1] for p in patches])[idx]
    E2 = np.stack([p[2] for p in patches])[idx]
    return O + uv[:, :1] * E1 + uv[:, 1:] * E2


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def make_c1(seed: Optional[int] = None, n: int = 1000, width: int = 128, height: int = 96) -> Scene:
    """1 000 random Gaussians in front of an identity camera (128x96, f = 100)."""
    rng = np.random.default_rng(101 if seed is None else seed)
    means = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(2, 6, n)], axis=1)
    g = random_gaussians(rng, means, -3.0, 0.5, 0.0, 1.0)
    cam = identity_camera(width, height, 100.0, 100.0, width / 2.0, height / 2.0)
    sc = Scene("c1", [g], [cam], [0])
    sc.weights = upstream_weights(103 if seed is None else seed + 2, sc.cameras)
    return sc


def make_c2(seed: Optional[int] = None, n: int = 200_000) -> Scene:
    """200 k Gaussians on planar patches of a 6x5x3 m room, one 640x480 view."""
    rng = np.random.default_rng(201 if seed is None else seed)
    size = (6.0, 5.0, 3.0)
    patches = _box_faces(size) + _random_rects(rng, 24, size)
    means = _sample_patches(rng, patches, n)
    g = random_gaussians(rng, means, -4.0, 0.4, 1.0, 1.0)
    prng = np.random.default_rng(202 if seed is None else seed + 1)
    ctr = prng.uniform([0.5, 0.5, 0.5], [5.5, 4.5, 2.5])
    cam = camera_look(ctr, prng.uniform(0, 2 * math.pi), math.radians(prng.uniform(-20, 20)),
                      math.radians(prng.uniform(-5, 5)), 640, 480, 525.0, 525.0, 320.0, 240.0)
    sc = Scene("c2", [g], [cam], [0])
    sc.weights = upstream_weights(203 if seed is None else seed + 2, sc.cameras)
    return sc


def make_decoder(rng, width: int, k: int, in_dim: int = 36) -> Decoder:
    outs = (k, 3 * k, 7 * k)
    W1, b1, W2, b2 = [], [], [], []
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    for o in outs:
        lim1 = 1.0 / math.sqrt(in_dim)
        lim2 = 1.0 / math.sqrt(width)
        W1.append(f(rng.uniform(-lim1, lim1, (width, in_dim))))
        b1.append(f(rng.uniform(-lim1, lim1, width)))
        W2.append(f(rng.uniform(-lim2, lim2, (o, width))))
        b2.append(f(rng.uniform(-lim2, lim2, o)))
    return Decoder(in_dim, width, k, W1, b1, W2, b2)


def make_anchors(rng, m: int, k: int, size=(12.0, 8.0, 4.0), voxel: float = 0.1) -> AnchorSet:
    size = np.asarray(size)
    patches = _box_faces(size) + _random_rects(rng, 40, size, 0.5, 3.0)
    keys = np.zeros((0, 3), np.int64)
    batch = 4 * m
    while keys.shape[0] < m:
        pts = _sample_patches(rng, patches, batch)
        keys = np.unique(np.concatenate([keys, np.floor(pts / voxel).astype(np.int64)]), axis=0)
    keys = keys[rng.permutation(keys.shape[0])[:m]]
    xyz = (keys + 0.5) * voxel
    feat = rng.standard_normal((m, 32))
    scale = voxel * np.exp(rng.normal(0.0, 0.1, (m, 3)))
    offs = rng.normal(0.0, 0.5, (m, k, 3))
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return AnchorSet(f(xyz), f(feat), f(scale), f(offs))


def make_c3(seed: Optional[int] = None, m: int = 50_000, k: int = 10, width: int = 64,
            img=(1200, 680)) -> Scene:
    """50 k voxel anchors + a width-64 decoder (k = 10), one 1200x680 view."""
    rng = np.random.default_rng(301 if seed is None else seed)
    anchors = make_anchors(rng, m, k)
    dec = make_decoder(rng, width, k)
    prng = np.random.default_rng(302 if seed is None else seed + 1)
    centroid = anchors.xyz.astype(np.float64).mean(axis=0)
    d = prng.standard_normal(3)
    d[2] = abs(d[2]) * 0.3
    d /= np.linalg.norm(d)
    W, H = img
    cam = _look_at(centroid + 3.0 * d, centroid, W, H, 600.0, 600.0, W / 2.0, H / 2.0)
    sc = Scene("c3", [], [cam], [0], anchors=anchors, decoder=dec)
    sc.weights = upstream_weights(303 if seed is None else seed + 2, sc.cameras)
    return sc


C4_SIZES = ((640, 480), (960, 540), (1200, 680))


def make_c4(seed: Optional[int] = None, n: int = 1_000_000, views: int = 8, sizes=None,
            weights: bool = True) -> Scene:
    """1 M Gaussians in a 24x8x3 m corridor seen by 8 keyframes on a 20 m path.

    ``sizes`` fixes every view to one (W, H); by default each view draws its
    resolution from {640x480, 960x540, 1200x680}.
    """
    rng = np.random.default_rng(401 if seed is None else seed)
    size = (24.0, 8.0, 3.0)
    patches = _box_faces(size) + _random_rects(rng, 200, size)
    means = _sample_patches(rng, patches, n)
    g = random_gaussians(rng, means, -4.0, 0.4, 1.0, 1.0)
    prng = np.random.default_rng(402 if seed is None else seed + 1)
    cams = []
    for i in range(views):
        s = i / max(views - 1, 1)
        x = 2.0 + 20.0 * s
        y = 4.0 + 1.5 * math.sin(2 * math.pi * s)
        dydx = 1.5 * 2 * math.pi * math.cos(2 * math.pi * s) / 20.0
        yaw = math.atan2(dydx, 1.0) + math.radians(prng.uniform(-30, 30))
        pitch = math.radians(prng.uniform(-10, 10))
        W, H = sizes if sizes is not None else C4_SIZES[prng.integers(0, 3)]
        cams.append(camera_look((x, y, 1.5), yaw, pitch, 0.0, W, H, W / 2.0, W / 2.0, W / 2.0, H / 2.0))
    sc = Scene("c4", [g], cams, [0] * views)
    if weights:
        sc.weights = upstream_weights(403 if seed is None else seed + 2, cams)
    return sc


def make_c5(seed: Optional[int] = None, n_per: int = 1_500_000, submaps: int = 4, views_per: int = 4,
            weights: bool = True) -> Scene:
    """4 submaps x 1.5 M Gaussians on ground and facades of a 200 m street."""
    rng = np.random.default_rng(501 if seed is None else seed)
    sets = []
    for j in range(submaps):
        x0, x1 = 50.0 * j, 50.0 * j + 80.0
        n_ground = n_per // 3
        n_fac = n_per - n_ground
        gx = rng.uniform(x0, x1, n_ground)
        gy = rng.uniform(-6.0, 6.0, n_ground)
        gz = rng.normal(0.0, 0.05, n_ground)
        fx_ = rng.uniform(x0, x1, n_fac)
        side = np.where(rng.uniform(size=n_fac) < 0.5, -8.0, 8.0)
        fy_ = side + rng.normal(0.0, 0.05, n_fac)
        fz = rng.uniform(0.0, 15.0, n_fac)
        means = np.concatenate([np.stack([gx, gy, gz], 1), np.stack([fx_, fy_, fz], 1)])
        sets.append(random_gaussians(rng, means, -2.5, 0.6, 1.0, 1.0))
    prng = np.random.default_rng(502 if seed is None else seed + 1)
    cams, vset = [], []
    for j in range(submaps):
        for i in range(views_per):
            x = 50.0 * j + 5.0 + 10.0 * i + prng.uniform(-1, 1)
            y = prng.uniform(-2.0, 2.0)
            yaw = math.radians(prng.uniform(-5, 5))
            pitch = math.radians(prng.uniform(-5, 5))
            cams.append(camera_look((x, y, 1.7), yaw, pitch, 0.0, 1242, 375, 720.0, 720.0, 621.0, 187.5))
            vset.append(j)
    sc = Scene("c5", sets, cams, vset)
    if weights:
        sc.weights = upstream_weights(503 if seed is None else seed + 2, cams)
    return sc


@dataclasses.dataclass
class StreetScan:
    """A voxel-map registration case: map points on a street's surfaces, one
    LiDAR sweep of the same street in the sensor frame, the sensor's true
    pose and a perturbed initial guess (sensor-to-world [R | t], float64)."""
    map_points: np.ndarray  # (n, 3) float32, world frame
    scan: np.ndarray        # (m, 3) float32, sensor frame
    pose_gt: np.ndarray     # (3, 4)
    pose_init: np.ndarray   # (3, 4)
    voxel: float


def _street_boxes(rng, length, half_width, count):
    """Axis-aligned boxes standing on the ground: parked cars, poles, kiosks."""
    kinds = np.array([[4.5, 1.8, 1.5], [0.3, 0.3, 4.0], [2.0, 2.0, 2.5]])
    k = rng.integers(0, 3, count)
    size = kinds[k] * rng.uniform(0.8, 1.2, (count, 3))
    ctr = np.stack([rng.uniform(0.0, length, count), rng.uniform(-half_width + 1.5, half_width - 1.5, count),
                    np.zeros(count)], axis=1)
    lo = ctr - 0.5 * size * np.array([1, 1, 0])
    hi = lo + size
    return lo, hi


def _street_surfaces(length, half_width, height, lo, hi):
    """Rectangles (origin, e1, e2) of the ground, both facades and the
    visible faces (top and four sides) of every box."""
    rects = [(np.array([0.0, -half_width, 0.0]), np.array([length, 0, 0.]), np.array([0, 2 * half_width, 0.])),
             (np.array([0.0, -half_width, 0.0]), np.array([length, 0, 0.]), np.array([0, 0, height])),
             (np.array([0.0, half_width, 0.0]), np.array([length, 0, 0.]), np.array([0, 0, height]))]
    for a, b in zip(lo, hi):
        d = b - a
        ex, ey, ez = np.array([d[0], 0, 0]), np.array([0, d[1], 0]), np.array([0, 0, d[2]])
        rects += [(a + ez, ex, ey), (a, ex, ez), (a + ey, ex, ez), (a, ey, ez), (a + ex, ey, ez)]
    return rects


def _cast_street(origin, dirs, length, half_width, height, lo, hi, max_range):
    """Ray parameter of the first hit of each unit direction with the
    street (ground z = 0, facades y = +-half_width up to height, boxes),
    restricted to 0 <= x <= length; inf for a miss."""
    t_best = np.full(dirs.shape[0], np.inf)

    def keep(t):
        p = origin + t[:, None] * dirs
        ok = (t > 0.1) & (t <= max_range) & (p[:, 0] >= 0) & (p[:, 0] <= length)
        return np.where(ok, t, np.inf), p

    with np.errstate(divide="ignore", invalid="ignore"):
        t, p = keep(-origin[2] / dirs[:, 2])
        t = np.where(np.abs(p[:, 1]) <= half_width, t, np.inf)
        t_best = np.minimum(t_best, t)
        for side in (-half_width, half_width):
            t, p = keep((side - origin[1]) / dirs[:, 1])
            t = np.where((p[:, 2] >= 0) & (p[:, 2] <= height), t, np.inf)
            t_best = np.minimum(t_best, t)
        inv = 1.0 / dirs
        for a, b in zip(lo, hi):  # slab test
            t0 = (a - origin) * inv
            t1 = (b - origin) * inv
            tn = np.max(np.minimum(t0, t1), axis=1)
            tf = np.min(np.maximum(t0, t1), axis=1)
            hit = (tf >= tn) & (tn > 0.1) & (tn <= max_range)
            t_best = np.where(hit & (tn < t_best), tn, t_best)
    return t_best


def make_street_scan(seed: Optional[int] = None, n_map: int = 1_500_000, beams: int = 64, azimuths: int = 2048,
                     length: float = 80.0, voxel: float = 1.0, noise: float = 0.02,
                     init_error=(0.5, 0.3, 0.05, 2.0)) -> StreetScan:
    """Frame-to-map registration on a street (the outdoor fine-tracking case).

    The map is n_map points drawn area-weighted on the ground (16 m wide),
    two facades (15 m high) and 50 boxes (cars, poles, kiosks) of an 80 m
    street, with normal noise 0.02 m: the means of a submap's Gaussians.
    The scan is one sweep of a 64-beam LiDAR (elevations -24.8..+2 deg,
    2048 azimuths, 80 m range, range noise 0.02 m) from a sensor 1.8 m above
    the road at x in [30, 50], in the sensor frame.  The initial guess is the
    true pose moved by init_error = (dx, dy, dz metres, yaw degrees).
    """
    rng = np.random.default_rng(601 if seed is None else seed)
    half_width, height = 8.0, 15.0
    lo, hi = _street_boxes(rng, length, half_width, 50)
    pts = _sample_patches(rng, _street_surfaces(length, half_width, height, lo, hi), n_map)
    pts += rng.normal(0.0, noise, pts.shape)
    prng = np.random.default_rng(602 if seed is None else seed + 1)
    pos = np.array([prng.uniform(30.0, 50.0), prng.uniform(-3.0, 3.0), 1.8])
    yaw = prng.uniform(-0.3, 0.3)
    R = _rot_axis(np.array([0.0, 0.0, 1.0]), yaw)
    el = np.radians(np.linspace(-24.8, 2.0, beams))
    az = np.linspace(-math.pi, math.pi, azimuths, endpoint=False)
    E, A = np.meshgrid(el, az, indexing="ij")
    d_sensor = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], axis=-1).reshape(-1, 3)
    d_world = d_sensor @ R.T
    t = _cast_street(pos, d_world, length, half_width, height, lo, hi, 80.0)
    hit = np.isfinite(t)
    r = t[hit] + prng.normal(0.0, noise, int(hit.sum()))
    scan = d_sensor[hit] * r[:, None]
    gt = np.concatenate([R, pos[:, None]], axis=1)
    dx, dy, dz, dyaw = init_error
    Ri = _rot_axis(np.array([0.0, 0.0, 1.0]), yaw + math.radians(dyaw))
    init = np.concatenate([Ri, (pos + np.array([dx, dy, dz]))[:, None]], axis=1)
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return StreetScan(f(pts), f(scan), gt, init, voxel)


def make_config(i: int, **kw) -> Scene:
    return {1: make_c1, 2: make_c2, 3: make_c3, 4: make_c4, 5: make_c5}[i](**kw)


def tiny_scene(seed: int, n: int = 12, width: int = 24, height: int = 20, f: float = 30.0,
               ls_mu: float = -1.6, ls_sigma: float = 0.4) -> Scene:
    """A few Gaussians in front of a small camera, for brute-force checks."""
    rng = np.random.default_rng(seed)
    means = np.stack([rng.uniform(-1, 1, n), rng.uniform(-0.8, 0.8, n), rng.uniform(2, 5, n)], axis=1)
    g = random_gaussians(rng, means, ls_mu, ls_sigma, 0.0, 1.5)
    cam = identity_camera(width, height, f, f, width / 2.0, height / 2.0)
    sc = Scene("tiny", [g], [cam], [0])
    sc.weights = upstream_weights(seed + 7, [cam])
    return sc
