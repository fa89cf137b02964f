"""Submap-expansion statistics of Section III-A in NumPy -- TEST INFRASTRUCTURE.

Section III-A grows and prunes the anchors of a submap from three kinds of
evidence, and this module defines each as plainly as the paper allows:

* Pixels where new anchors are sampled: the posed point cloud of the input
  frame is sampled where the rendered accumulated alpha is below a
  threshold or the rendered depth disagrees markedly with the measured one.
  Here a pixel is a candidate iff its target depth T > 0 (it has a point)
  and (A < alpha_threshold or |D - T| > depth_threshold).  A sample takes
  the candidate of rank floor(u c) (raster order, at most c - 1) for a
  given uniform u in [0, 1) and c candidates, and back-projects its pixel
  centre with the target depth: X = R^T (T K^-1 (x + 1/2, y + 1/2, 1) - t).
* Anchor growth: per voxel, the averaged gradient of its neural Gaussians,
  grown where it exceeds tau_g.  Per Gaussian and view, the gradient is the
  norm of dL/d(u, v), the gradient with respect to the projected centre,
  counted in the views that render the Gaussian; an anchor's value is the
  sum of those norms over its k Gaussians divided by the number of
  (Gaussian, view) observations.
* Anchor pruning: the accumulated opacity of its neural Gaussians, summed
  as max(opacity, 0) over the views whose frustum holds each Gaussian's
  centre, and pruned when its mean per observation is below tau_o.

Per-Gaussian gradients come from the float64 render gradient of
``oracle.grad`` (its d L / d(u, v) quantities).  Decisions that turn floats
into integers (visibility, frustum, candidate, rank, threshold) are taken in
float32 on the float32 values the renderer itself uses, and the anchor
reductions sum in float32 in index order, so both sides decide alike.
"""
from __future__ import annotations

import numpy as np

import oracle

__all__ = ["view_accum", "anchor_stats", "expansion_candidates", "expansion_sample"]


def view_accum(g, cam, g_rgb, g_depth, g_alpha, grad_space: int = 0):
    """Per-Gaussian contributions of one view, float64 [n, 4]:
    (|dL/d(u, v)| if rendered, 1 if rendered, max(o, 0) if the centre is in
    the frustum, 1 if it is), and the error scales of column 0: the
    summation scale and the float32 forward bound of the norm.

    grad_space 1 measures the gradient in normalised device coordinates,
    x_ndc = 2 u / W - 1: (W/2 dL/du, H/2 dL/dv)."""
    W, H = cam.width, cam.height
    p = oracle.project(g, cam)
    G, S = oracle.grad(g, cam, np.asarray(g_rgb, np.float64), np.asarray(g_depth, np.float64),
                       np.asarray(g_alpha, np.float64), quantities=True)
    su, sv = (W / 2.0, H / 2.0) if grad_space == 1 else (1.0, 1.0)
    gu, gv = G["quantity"][:, 0] * su, G["quantity"][:, 1] * sv
    rendered = p["valid"]
    out = np.zeros((g.n, 4))
    out[:, 0] = np.where(rendered, np.hypot(gu, gv), 0.0)
    out[:, 1] = rendered
    z, u, v = p["z32"], p["u32"], p["v32"]
    near = np.float32(cam.near if cam.near > 0 else 0.2)
    with np.errstate(invalid="ignore"):
        in_view = (z > near) & (u >= 0) & (u < np.float32(W)) & (v >= 0) & (v < np.float32(H))
    out[:, 2] = np.where(in_view, np.maximum(np.asarray(g.opacities, np.float64), 0.0), 0.0)
    out[:, 3] = in_view
    scale = np.where(rendered, np.hypot(S["quantity"][:, 0] * su, S["quantity"][:, 1] * sv), 0.0)
    bound = np.where(rendered, np.hypot(S["quantity_fp32"][:, 0] * su, S["quantity_fp32"][:, 1] * sv), 0.0)
    return out, scale, bound


def anchor_stats(accum, k: int, tau_g: float, tau_o: float):
    """Anchor statistics from the [m*k, 4] float32 accumulators of its
    Gaussians (anchor-major).  Returns (stats float32 [m, 4], grow bool [m],
    prune bool [m]) with S_c the float32 sum over j = 0..k-1 in order:
    stats = (S_0 / S_1 or 0, S_1, S_2, S_3); grow = stats_0 > tau_g;
    prune = S_3 > 0 and S_2 < tau_o S_3."""
    a = np.asarray(accum, np.float32).reshape(-1, k, 4)
    m = a.shape[0]
    s = np.zeros((m, 4), np.float32)
    for j in range(k):
        s = s + a[:, j]  # float32 + float32 -> float32, one rounding per add
    with np.errstate(divide="ignore", invalid="ignore"):
        avg = np.where(s[:, 1] > 0, s[:, 0] / np.where(s[:, 1] > 0, s[:, 1], np.float32(1)), np.float32(0))
    stats = np.stack([avg.astype(np.float32), s[:, 1], s[:, 2], s[:, 3]], axis=1)
    grow = stats[:, 0] > np.float32(tau_g)
    prune = (s[:, 3] > 0) & (s[:, 2] < np.float32(tau_o) * s[:, 3])
    return stats, grow, prune


def expansion_candidates(alpha, depth, t_depth, alpha_threshold: float, depth_threshold: float):
    """Candidate mask (bool [H, W]) of one view from its float32 rendered
    alpha and depth and its target depth."""
    a = np.asarray(alpha, np.float32)
    d = np.asarray(depth, np.float32)
    t = np.asarray(t_depth, np.float32)
    err = np.abs(d - t)  # float32 subtraction, exact rounding as on the device
    return (t > 0) & ((a < np.float32(alpha_threshold)) | (err > np.float32(depth_threshold)))


def expansion_sample(cand, uniforms, t_depth, t_rgb, cam):
    """Samples of one view: (pixel int32 [M] (-1 if there is no candidate),
    world points float64 [M, 3], target colours float64 [M, 3])."""
    H, W = cand.shape
    idx = np.flatnonzero(np.asarray(cand).reshape(-1))
    c = idx.size
    u = np.asarray(uniforms, np.float32)
    M = u.size
    pix = np.full(M, -1, np.int32)
    pts = np.zeros((M, 3))
    col = np.zeros((M, 3))
    if c == 0:
        return pix, pts, col
    w2c = np.asarray(cam.world_to_cam, np.float32).astype(np.float64)
    R, t = w2c[:, :3], w2c[:, 3]
    fx, fy, cx, cy = (float(np.float32(x)) for x in (cam.fx, cam.fy, cam.cx, cam.cy))
    td = np.asarray(t_depth, np.float32).reshape(-1)
    rgb = np.asarray(t_rgb, np.float32).reshape(3, -1)
    for i in range(M):
        r = min(int(u[i] * np.float32(c)), c - 1)  # float32 product, truncated
        p = int(idx[r])
        x, y = p % W, p // W
        T = float(td[p])
        cam_pt = np.array([(x + 0.5 - cx) / fx * T, (y + 0.5 - cy) / fy * T, T])
        pix[i] = p
        pts[i] = R.T @ (cam_pt - t)
        col[i] = rgb[:, p]
    return pix, pts, col
