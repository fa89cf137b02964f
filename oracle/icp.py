"""Voxel-map frame-to-map registration of Section III-B (eq. 10-12) in NumPy -- TEST INFRASTRUCTURE.

The fine tracking stage registers a scan against the voxelised map of 3D
Gaussian means, in the manner of the cited KISS-ICP:

* voxels: a point p falls in voxel floor(p / v) (FP32 division, per axis);
* downsampling keeps one original point per voxel, the first by index (the
  scan is downsampled twice, at two voxel sizes);
* the map keeps, per voxel, the first max_per_voxel points by index;
* eq. 10: source points are the scan under the predicted pose, s = T p;
* correspondences: the nearest map point among the 27 voxels around the
  voxel of s (squared distance in FP32, ties to the lower index), kept if
  its squared distance is below tau^2 (C(tau_t) of eq. 11);
* eq. 11-12: the pose minimises sum rho(||T s - m||) with the Geman-McClure
  kernel rho(e) = (e^2 / 2) / (kappa + e^2), kappa = sigma_t / 3 as printed;
  each Gauss-Newton step solves H dx = -g with the iteratively reweighted
  system H = sum w J^T J, g = sum w J^T r, r = T s - m, w = rho'(e) / e =
  kappa / (kappa + e^2)^2 and J = [I, -[T s]x], the derivative of
  Exp(xi) T s at xi = 0 for a left increment xi = (rho, phi); then
  T <- Exp(dx) T, until |dx| < eps or max_iter steps.

Decisions that turn floats into integers (voxel, nearest neighbour,
threshold) are taken in FP32 with the operation order the kernels use:
s = ((R00 p_x + R01 p_y) + R02 p_z) + t_x with R, t rounded to float32, and
d^2 = ((dx dx + dy dy) + dz dz).  Everything else is float64.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["voxel_coords", "downsample", "VoxelMap", "transform32", "correspond", "gm_rho", "gm_weight",
           "normal_equations", "se3_exp", "register"]

_F = np.float32


def voxel_coords(points, voxel: float) -> np.ndarray:
    """Integer voxel coordinates floor(p / v), the division in float32."""
    p = np.asarray(points, _F)
    return np.floor(p / _F(voxel)).astype(np.int64)


def downsample(points, voxel: float) -> np.ndarray:
    """Indices (ascending) of the first point of every occupied voxel."""
    seen = {}
    for i, key in enumerate(map(tuple, voxel_coords(points, voxel))):
        if key not in seen:
            seen[key] = i
    return np.array(sorted(seen.values()), np.int64)


class VoxelMap:
    """Per voxel, the indices of its first max_per_voxel points by index."""

    def __init__(self, points, voxel: float, max_per_voxel: int):
        self.points = np.asarray(points, _F)
        self.voxel = float(voxel)
        self.cells = {}
        for i, key in enumerate(map(tuple, voxel_coords(self.points, voxel))):
            lst = self.cells.setdefault(key, [])
            if len(lst) < max_per_voxel:
                lst.append(i)


def transform32(src, pose) -> np.ndarray:
    """T p in float32 with the kernels' operation order (no fused products)."""
    P = np.asarray(pose, np.float64).reshape(3, 4).astype(_F)
    s = np.asarray(src, _F)
    out = np.empty_like(s)
    for r in range(3):
        out[:, r] = ((P[r, 0] * s[:, 0] + P[r, 1] * s[:, 1]) + P[r, 2] * s[:, 2]) + P[r, 3]
    return out


_OFFSETS = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]


def correspond(vmap: VoxelMap, q32, tau: float):
    """Nearest map point of each float32 query among the 27 voxels around
    its own: (index int64, -1 if none below tau; squared distance float32,
    +inf if no candidate at all)."""
    q = np.asarray(q32, _F)
    n = q.shape[0]
    vox = voxel_coords(q, vmap.voxel)
    cand = [[] for _ in range(n)]
    for i in range(n):
        x, y, z = vox[i]
        for a, b, c in _OFFSETS:
            lst = vmap.cells.get((x + a, y + b, z + c))
            if lst:
                cand[i].extend(lst)
    best = np.full(n, -1, np.int64)
    d2 = np.full(n, np.inf, _F)
    tau2 = _F(tau) * _F(tau)
    for i in range(n):
        if not cand[i]:
            continue
        idx = np.array(cand[i], np.int64)
        m = vmap.points[idx]
        dx, dy, dz = q[i, 0] - m[:, 0], q[i, 1] - m[:, 1], q[i, 2] - m[:, 2]
        dd = (dx * dx + dy * dy) + dz * dz
        k = np.lexsort((idx, dd))[0]
        d2[i] = dd[k]
        if dd[k] < tau2:
            best[i] = idx[k]
    return best, d2


def gm_rho(e2, sigma: float):
    kappa = sigma / 3.0
    return 0.5 * e2 / (kappa + e2)


def gm_weight(e2, sigma: float):
    kappa = sigma / 3.0
    return kappa / (kappa + e2) ** 2


def _skew(v):
    x, y, z = v
    return np.array([[0.0, -z, y], [z, 0.0, -x], [-y, x, 0.0]])


def normal_equations(p, m, sigma: float):
    """(H [6,6], g [6], count, sum rho) over the pairs (p_i, m_i), float64."""
    p = np.asarray(p, np.float64)
    m = np.asarray(m, np.float64)
    r = p - m
    e2 = np.einsum("ij,ij->i", r, r)
    w = gm_weight(e2, sigma)
    H = np.zeros((6, 6))
    g = np.zeros(6)
    for i in range(p.shape[0]):
        J = np.concatenate([np.eye(3), -_skew(p[i])], axis=1)
        H += w[i] * J.T @ J
        g += w[i] * J.T @ r[i]
    return H, g, int(p.shape[0]), float(gm_rho(e2, sigma).sum())


def se3_exp(xi) -> np.ndarray:
    """Exp of xi = (rho, phi) as a 3x4 [R | t]: R = Rodrigues(phi), t = V rho."""
    rho, phi = np.asarray(xi[:3], np.float64), np.asarray(xi[3:], np.float64)
    th = float(np.linalg.norm(phi))
    K = _skew(phi)
    if th < 1e-8:
        R = np.eye(3) + K + 0.5 * K @ K
        V = np.eye(3) + 0.5 * K + K @ K / 6.0
    else:
        a, b = math.sin(th) / th, (1.0 - math.cos(th)) / th ** 2
        c = (th - math.sin(th)) / th ** 3
        R = np.eye(3) + a * K + b * K @ K
        V = np.eye(3) + b * K + c * K @ K
    return np.concatenate([R, (V @ rho)[:, None]], axis=1)


def _compose(A, B):
    Ra, ta = A[:, :3], A[:, 3]
    Rb, tb = B[:, :3], B[:, 3]
    return np.concatenate([Ra @ Rb, (Ra @ tb + ta)[:, None]], axis=1)


def register(vmap: VoxelMap, src, pose_init, tau: float, sigma: float, max_iter: int = 500, eps: float = 1e-4):
    """Gauss-Newton with Geman-McClure weights from pose_init (3x4).
    Returns dict(pose, iterations, count, rho, converged)."""
    T = np.asarray(pose_init, np.float64).reshape(3, 4).copy()
    count, rho, it, converged = 0, 0.0, 0, False
    for it in range(1, max_iter + 1):
        q = transform32(src, T)
        nn, _ = correspond(vmap, q, tau)
        ok = nn >= 0
        H, g, count, rho = normal_equations(q[ok], vmap.points[nn[ok]], sigma)
        if count < 6:
            it -= 1
            break
        dx = -np.linalg.solve(H, g)
        T = _compose(se3_exp(dx), T)
        if np.linalg.norm(dx) < eps:
            converged = True
            break
    return dict(pose=T, iterations=it, count=count, rho=rho, converged=converged)
