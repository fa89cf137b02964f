"""Helpers shared by the GPU parity tests: device transfer, the tolerance
gates and the near-tie masks (test infrastructure)."""
from __future__ import annotations

import numpy as np
import torch

import oracle

# Margins of the near-tie mask: a pixel is excluded from the image gate (and
# its upstream weights are zeroed for the gradient gate) if any Gaussian
# evaluated there has alpha within a relative 2e-4 of 1/255, o*G within 1e-5
# of the 0.99 clamp, or T(1 - alpha) within a relative 1e-4 of 1e-4 -- the
# places where an FP32 evaluation can take the other branch of a cutoff.
# Each margin is widened by the oracle's own first-order estimate of the FP32
# error that reaches that test (projected-centre and exponent rounding, and
# for the transmittance its accumulation over the pixel's blends).  The FP32
# build of the oracle takes the other branch only at flagged pixels.
MARGINS = (2e-4, 1e-5, 1e-4)

# Ceilings of the flagged-pixel fraction per workload.  The fraction grows
# with the blends per pixel, as the accumulated transmittance error widens
# the termination margin: about 8 blends per pixel at C1 (0.11 % flagged),
# 44 at C2 (0.54 %), 60-70 on corridor and anchor keyframes (1.0-2.3 %), and
# about 110 (up to 350) on street frames (2.6 %).
MASK_CEILING = {"c1": 0.005, "c2": 0.01, "c3": 0.03, "c4": 0.015, "c5": 0.035}

IMAGE_RTOL = 1e-5     # norm-wise, per plane, FP32 vs the FP64 oracle
GRAD_TOL = 1e-4       # per element against the error scale, and norm-wise


def to_dev(arrs, dev="cuda"):
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in arrs)


def np_(t):
    return t.detach().cpu().numpy()


def assert_mask_fraction(mask, workload):
    """The near-tie mask must not grow past the workload's ceiling (it would
    silently drop pixels from the image gate); returns the fraction."""
    frac = float(np.mean(mask))
    assert frac <= MASK_CEILING[workload], f"{workload}: {frac:.3%} of pixels flagged, ceiling {MASK_CEILING[workload]:.1%}"
    return frac


def image_errors(got, ref, mask):
    """Norm-wise relative errors of the five planes over unmasked pixels."""
    rgb, depth, alpha = (np_(t).astype(np.float64) for t in got)
    keep = ~mask
    out = {}
    for name, g, e in (("r", rgb[0], ref["rgb"][0]), ("g", rgb[1], ref["rgb"][1]), ("b", rgb[2], ref["rgb"][2]),
                       ("depth", depth, ref["depth"]), ("alpha", alpha, ref["alpha"])):
        num = np.linalg.norm((g - e)[keep])
        den = np.linalg.norm(e[keep])
        out[name] = num / den if den > 0 else num
    return out


def assert_images(got, ref, mask, rtol=IMAGE_RTOL):
    errs = image_errors(got, ref, mask)
    bad = {k: v for k, v in errs.items() if not v <= rtol}
    assert not bad, f"image parity failed: {errs} (masked {int(mask.sum())} px)"
    return errs


# Multiple of the oracle's FP32 propagation bound B in the gradient gate.
B_FACTOR = 2.0


def assert_grads(got: dict, G: dict, S: dict, tol=GRAD_TOL, keys=None):
    """Per element |g - g_ref| <= tol * scale + B_FACTOR * fp32_bound (plus a
    tiny floor), and norm-wise ||g - g_ref|| <= tol ||g_ref|| + B_FACTOR ||fp32_bound||.

    scale is the summation error scale of the element; fp32_bound (B) is the
    oracle's first-order bound on how far float32 rounding of the projected
    centres and of the transmittance of long stacks moves that element (the
    forward's own deviation, not a summation error).  The FP32 build of the
    oracle stays within tol * scale + B; the GPU's float32 evaluation (its
    exponent, its reverse walk by division) is another one of the same order.

    Returns {key: (gate fraction used, error / (tol * scale) alone, error /
    (tol * scale + B), norm-wise error)}."""
    report = {}
    for k in keys or [x for x in G.keys() if x in got]:
        g = np.asarray(got[k], np.float64)
        e, s = G[k], S[k]
        b = S.get(k + "_fp32", np.zeros_like(s))
        floor = 1e-7 * (s.max() if s.size else 0.0)
        err = np.abs(g - e)
        base = tol * s + tol * floor + 1e-30
        worst = float(np.max(err / (base + B_FACTOR * b))) if err.size else 0.0
        s_only = float(np.max(err / base)) if err.size else 0.0
        with_b = float(np.max(err / (base + b))) if err.size else 0.0
        nrm = float(np.linalg.norm(g - e) / max(np.linalg.norm(e), 1e-30))
        nrm_gate = tol + B_FACTOR * float(np.linalg.norm(b)) / max(np.linalg.norm(e), 1e-30)
        report[k] = (round(worst, 4), round(s_only, 4), round(with_b, 4), float(f"{nrm:.3e}"))
        assert worst <= 1.0, f"{k}: per-element error {worst:.3f} of the gate ({report})"
        assert nrm <= nrm_gate or np.linalg.norm(e) < 1e-6 * np.linalg.norm(s), \
            f"{k}: norm-wise {nrm:.3e} exceeds {nrm_gate:.3e} ({report})"
    return report


def masked_weights(weights, mask):
    gr, gd, ga = (np.array(w, np.float32) for w in weights)
    gr[:, mask] = 0.0
    gd[mask] = 0.0
    ga[mask] = 0.0
    return gr, gd, ga


def oracle_reference(g, cam, weights=None):
    """FP64 render (with near-tie flags) and, if weights are given, the masked
    gradients and their error scales."""
    ref = oracle.render(g, cam, margins=MARGINS)
    mask = ref["flags"]
    if weights is None:
        return ref, mask, None
    w = masked_weights(weights, mask)
    G, S = oracle.grad(g, cam, *[x.astype(np.float64) for x in w])
    return ref, mask, (w, G, S)
