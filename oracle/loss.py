"""Mapping loss of eq. 7-9 in plain PyTorch CPU float64 -- TEST INFRASTRUCTURE.

Per view (rendered colour X [3,H,W] and depth D [H,W] against a target colour
Y and depth T):

* L_c     = mean over channels and pixels of |X - Y|            (eq. 7)
* L_SSIM  = (1 - lambda_ssim) mean|X - Y| + lambda_ssim (1 - SSIM(X, Y))   (eq. 8)
* L_d     = mean over pixels with a target depth (T > 0) of |D - T|  (eq. 7)
* L_view  = L_c + L_SSIM + lambda_d L_d                        (eq. 7)

SSIM is the structural similarity of Wang et al. (2004) as used by 3DGS
renderers: an 11x11 Gaussian window with sigma 1.5 (normalised), local
statistics by zero-padded "same" filtering of X, Y, X^2, Y^2, XY per
channel, C1 = 0.01^2, C2 = 0.03^2 (dynamic range 1), and the map averaged
over channels and pixels.  The volume term of eq. 9 is
lambda_vol * sum_i prod(exp(l_i)) over the Gaussians of a set (l the
log-scales).  A window's loss is the sum over its views.

Gradients are torch autograd of these forwards; d|x|/dx is taken as 0 at 0.
"""
from __future__ import annotations

import math

import numpy as np
import torch

__all__ = ["WINDOW", "SIGMA", "C1", "C2", "window_1d", "ssim_map", "ssim_map_bruteforce", "view_loss",
           "view_loss_grad", "view_grad_bounds", "volume_loss"]

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2


def _t(a):
    if isinstance(a, torch.Tensor):
        return a.to(torch.float64)
    return torch.as_tensor(np.asarray(a)).to(torch.float64)


def window_1d(size: int = WINDOW, sigma: float = SIGMA) -> np.ndarray:
    """Normalised 1-D Gaussian taps g_k ~ exp(-(k - c)^2 / (2 sigma^2))."""
    c = (size - 1) / 2.0
    g = np.array([math.exp(-((k - c) ** 2) / (2.0 * sigma * sigma)) for k in range(size)])
    return g / g.sum()


def _filter(img: torch.Tensor) -> torch.Tensor:
    """Zero-padded 'same' correlation of [C,H,W] planes with the 2-D window
    outer(g, g) (symmetric, so correlation equals convolution)."""
    g = _t(window_1d())
    w2 = torch.outer(g, g)[None, None]
    pad = WINDOW // 2
    return torch.nn.functional.conv2d(img[:, None], w2, padding=pad)[:, 0]


def ssim_map(x, y) -> torch.Tensor:
    x, y = _t(x), _t(y)
    mu1, mu2 = _filter(x), _filter(y)
    s11 = _filter(x * x) - mu1 * mu1
    s22 = _filter(y * y) - mu2 * mu2
    s12 = _filter(x * y) - mu1 * mu2
    return ((2 * mu1 * mu2 + C1) * (2 * s12 + C2)) / ((mu1 * mu1 + mu2 * mu2 + C1) * (s11 + s22 + C2))


def ssim_map_bruteforce(x, y) -> np.ndarray:
    """The same SSIM map from explicit window sums per pixel (small images
    only): the definition written out, independent of the filtering path."""
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    g = window_1d()
    C, H, W = x.shape
    r = WINDOW // 2
    out = np.zeros((C, H, W))
    for c in range(C):
        for i in range(H):
            for j in range(W):
                m1 = m2 = e11 = e22 = e12 = 0.0
                for a in range(-r, r + 1):
                    for b in range(-r, r + 1):
                        ii, jj = i + a, j + b
                        if 0 <= ii < H and 0 <= jj < W:
                            w = g[a + r] * g[b + r]
                            xv, yv = x[c, ii, jj], y[c, ii, jj]
                            m1 += w * xv; m2 += w * yv
                            e11 += w * xv * xv; e22 += w * yv * yv; e12 += w * xv * yv
                s11, s22, s12 = e11 - m1 * m1, e22 - m2 * m2, e12 - m1 * m2
                out[c, i, j] = ((2 * m1 * m2 + C1) * (2 * s12 + C2)) / ((m1 * m1 + m2 * m2 + C1) * (s11 + s22 + C2))
    return out


def _abs(v: torch.Tensor) -> torch.Tensor:
    # |v| with derivative sign(v) (0 at 0)
    return v * torch.sign(v).detach()


def _view_terms(x, dep, y, tdep, lam_ssim, lam_d):
    l1 = _abs(x - y).mean()
    ssim = ssim_map(x, y).mean()
    valid = (tdep > 0).to(torch.float64)
    nvalid = float(valid.sum())
    ld = (_abs(dep - tdep) * valid).sum() / nvalid if nvalid > 0 else dep.sum() * 0.0
    l_c = l1
    l_ssim = (1.0 - lam_ssim) * l1 + lam_ssim * (1.0 - ssim)
    total = l_c + l_ssim + lam_d * ld
    return l_c, l_ssim, ld, total, ssim


def view_loss(rgb, depth, t_rgb, t_depth, lam_ssim=0.2, lam_d=1.0) -> dict:
    """Loss terms of one view (floats): L_c, L_SSIM, L_d, total, and the mean SSIM."""
    with torch.no_grad():
        l_c, l_ssim, ld, total, ssim = _view_terms(_t(rgb), _t(depth), _t(t_rgb), _t(t_depth), lam_ssim, lam_d)
    return dict(L_c=float(l_c), L_ssim=float(l_ssim), L_d=float(ld), total=float(total), ssim=float(ssim))


def view_loss_grad(rgb, depth, t_rgb, t_depth, lam_ssim=0.2, lam_d=1.0):
    """Gradient of the view's total loss w.r.t. the rendered colour and depth
    (float64 numpy [3,H,W], [H,W])."""
    x = _t(rgb).requires_grad_(True)
    dep = _t(depth).requires_grad_(True)
    _, _, _, total, _ = _view_terms(x, dep, _t(t_rgb), _t(t_depth), lam_ssim, lam_d)
    gx, gd = torch.autograd.grad(total, (x, dep), allow_unused=True)
    gd = torch.zeros_like(dep) if gd is None else gd
    return gx.numpy(), gd.numpy()


def volume_loss(log_scales, lam_vol=0.001):
    """(lambda_vol * sum_i prod(exp(l_i)), its gradient w.r.t. the log-scales [n,3])."""
    l = _t(log_scales)
    prod = torch.exp(l.sum(dim=1))
    val = lam_vol * float(prod.sum())
    grad = (lam_vol * prod)[:, None].expand(-1, 3).numpy().copy()
    return val, grad


def view_grad_bounds(rgb, t_rgb, lam_ssim=0.2, lam_d=1.0):
    """Error scales of the colour gradient (float64 [3,H,W] each), for
    comparing a float32 evaluation:

    * scale: the magnitude of its terms, |w| (G*|P1| + 2|X| G*|P2| + |Y| G*|P3|)
      + the L1 weight, with P1..P3 the partials of the SSIM map with respect to
      the local mean of X, E[X^2] and E[XY] and w = -lambda_ssim / N;
    * fp32: the same filtered sum with each pixel's partials weighted by the
      amplification of float32 rounding in its statistics,
      (E[X^2] + mu_x^2 + E[Y^2] + mu_y^2 + 2|E[XY]| + 2|mu_x mu_y|) / min(B2, |A2|),
      times 2^-24 (the variance-like terms are differences of filtered
      squares, and A2, B2 are the denominators of the structure term)."""
    x, y = _t(rgb), _t(t_rgb)
    n = x.numel()
    m1, m2 = _filter(x), _filter(y)
    e11, e22, e12 = _filter(x * x), _filter(y * y), _filter(x * y)
    A1 = 2 * m1 * m2 + C1
    A2 = 2 * (e12 - m1 * m2) + C2
    B1 = m1 * m1 + m2 * m2 + C1
    B2 = (e11 - m1 * m1) + (e22 - m2 * m2) + C2
    S = A1 * A2 / (B1 * B2)
    P1 = 2 * S * (m2 / A1 - m2 / A2 - m1 / B1 + m1 / B2)
    P2 = -S / B2
    P3 = 2 * S / A2
    w = lam_ssim / n
    wl1 = (2.0 - lam_ssim) / n
    scale = w * (_filter(P1.abs()) + 2 * x.abs() * _filter(P2.abs()) + y.abs() * _filter(P3.abs())) + wl1
    kappa = (e11 + m1 * m1 + e22 + m2 * m2 + 2 * e12.abs() + 2 * (m1 * m2).abs()) / torch.minimum(B2, A2.abs())
    fp32 = w * (_filter(P1.abs() * kappa) + 2 * x.abs() * _filter(P2.abs() * kappa) +
                y.abs() * _filter(P3.abs() * kappa)) * 2.0 ** -24
    return scale.numpy(), fp32.numpy()
