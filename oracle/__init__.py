"""CPU oracle for the Gaussian-splatting render path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it
and shares no code with it.

* ``render``, ``grad``, ``project``, ``binning``: ctypes wrappers over the
  FP64 C++ reference in ``oracle.cpp`` (see its header for the definition);
  ``render`` and ``grad`` also run its float32 evaluation (``fp32=True``).
* ``decode``: the anchor -> neural-Gaussian decoder of Section III-A
  (eq. 1-5) in plain PyTorch CPU float64 with autograd (``decode.py``).
* ``loss``: the mapping loss of eq. 7-9 (``loss.py``).
* ``densify``: the submap-expansion statistics of Section III-A -- screen-space
  gradient and opacity accumulators, anchor growth and pruning, expansion
  candidates and samples (``densify.py``).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIBS = {}

_D = ctypes.POINTER(ctypes.c_double)
_F = ctypes.POINTER(ctypes.c_float)
_U8 = ctypes.POINTER(ctypes.c_uint8)
_I32 = ctypes.POINTER(ctypes.c_int32)
_U32 = ctypes.POINTER(ctypes.c_uint32)
_U64 = ctypes.POINTER(ctypes.c_uint64)


def lib(fp32: bool = False):
    """The FP64 reference, or with fp32=True the same definition evaluated in
    float32 (every step rounded to float32)."""
    if fp32 not in _LIBS:
        path = os.path.join(HERE, "liboracle32.so" if fp32 else "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        i64, c_int = ctypes.c_int64, ctypes.c_int
        L.oracle_project.argtypes = [c_int, c_int, _D, _D, i64, _D, _D, _D, _D, _D, _D, _F, _U8, _I32]
        L.oracle_render.argtypes = [c_int, c_int, _D, _D, i64, _D, _D, _D, _D, _D, c_int,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    _D, _D, _D, _D, _I32, _I32, _U8]
        L.oracle_grad.argtypes = [c_int, c_int, _D, _D, i64, _D, _D, _D, _D, _D, _D, _D, _D, _U8,
                                  _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D,
                                  _D, _D]
        L.oracle_binning.argtypes = [i64, _U8, _F, _F, _F, _F, _U32, c_int, c_int, c_int, c_int,
                                     ctypes.c_uint32, ctypes.c_uint32, i64, _U64, _U32, _U32]
        L.oracle_binning.restype = i64
        L.oracle_num_threads.restype = c_int
        _LIBS[fp32] = L
    return _LIBS[fp32]


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def _p(a, t):
    return a.ctypes.data_as(t)


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _cam_arrays(cam):
    intr = np.array([cam.fx, cam.fy, cam.cx, cam.cy, cam.near], np.float32).astype(np.float64)
    w2c = np.asarray(cam.world_to_cam, np.float32).astype(np.float64).reshape(3, 4)
    return intr, np.ascontiguousarray(w2c)


def _gauss_arrays(g):
    return tuple(_d(a) for a in (g.means, g.log_scales, g.quats, g.opacities, g.colors))


def project(g, cam):
    """Per-Gaussian FP64 projection: dict of u, v, z, a, b, c, Qa, Qb, Qc, hx, hy,
    the FP32 spec values u32, v32, z32, the validity mask and the pixel box."""
    n = g.n
    intr, w2c = _cam_arrays(cam)
    m, l, q, o, c = _gauss_arrays(g)
    f64 = np.zeros((n, 11), np.float64)
    f32 = np.zeros((n, 3), np.float32)
    valid = np.zeros(n, np.uint8)
    box = np.zeros((n, 4), np.int32)
    lib().oracle_project(cam.width, cam.height, _p(intr, _D), _p(w2c, _D), n, _p(m, _D), _p(l, _D),
                         _p(q, _D), _p(o, _D), _p(c, _D), _p(f64, _D), _p(f32, _F), _p(valid, _U8),
                         _p(box, _I32))
    names = ["u", "v", "z", "a", "b", "c", "Qa", "Qb", "Qc", "hx", "hy"]
    out = {k: f64[:, i].copy() for i, k in enumerate(names)}
    out.update(u32=f32[:, 0].copy(), v32=f32[:, 1].copy(), z32=f32[:, 2].copy(),
               valid=valid.astype(bool), box=box)
    return out


def render(g, cam, brute_force: bool = False, margins=(1e-4, 1e-4, 1e-4), fp32: bool = False):
    """FP64 forward render of one view (fp32=True: evaluated in float32).
    Returns rgb[3,H,W], depth, alpha, T_final, n_blend, n_eval and the
    near-tie pixel flags."""
    W, H = cam.width, cam.height
    intr, w2c = _cam_arrays(cam)
    m, l, q, o, c = _gauss_arrays(g)
    rgb = np.zeros((3, H, W)); depth = np.zeros((H, W)); alpha = np.zeros((H, W)); T = np.zeros((H, W))
    nb = np.zeros((H, W), np.int32); ne = np.zeros((H, W), np.int32); fl = np.zeros((H, W), np.uint8)
    lib(fp32).oracle_render(W, H, _p(intr, _D), _p(w2c, _D), g.n, _p(m, _D), _p(l, _D), _p(q, _D), _p(o, _D),
                        _p(c, _D), int(brute_force), float(margins[0]), float(margins[1]), float(margins[2]),
                        _p(rgb, _D), _p(depth, _D), _p(alpha, _D), _p(T, _D), _p(nb, _I32), _p(ne, _I32),
                        _p(fl, _U8))
    return dict(rgb=rgb, depth=depth, alpha=alpha, T_final=T, n_blend=nb, n_eval=ne, flags=fl.astype(bool))


def grad(g, cam, g_rgb, g_depth, g_alpha, skip: Optional[np.ndarray] = None, quantities: bool = False,
         fp32: bool = False):
    """FP64 gradient of sum(g_rgb*RGB + g_depth*D + g_alpha*A) (fp32=True: the
    same definition evaluated in float32, its scales and bounds too).

    Returns (grads, scales): dicts with means, log_scales, quats, opacities,
    colors and pose (rho, phi) -- the gradient and its summation error scale.
    scales also holds "<name>_fp32": a first-order bound on how far a float32
    evaluation of the same forward moves the gradient (rounding of the
    projected centres, propagated through the transmittance).  With
    quantities=True grads also holds "quantity": [n, 10] gradients with
    respect to (u, v, Qa, Qb, Qc, opacity, r, g, b, z) of every Gaussian, and
    scales the matching "quantity" and "quantity_fp32" arrays."""
    W, H = cam.width, cam.height
    n = g.n
    intr, w2c = _cam_arrays(cam)
    m, l, q, o, c = _gauss_arrays(g)
    gr, gd, ga = _d(g_rgb), _d(g_depth), _d(g_alpha)
    sk = None if skip is None else np.ascontiguousarray(skip, dtype=np.uint8)
    outs = [np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 4)), np.zeros(n), np.zeros((n, 3)), np.zeros(6)]
    scl = [np.zeros_like(a) for a in outs]
    bnd = [np.zeros_like(a) for a in outs]
    qg = np.zeros((n, 10)) if quantities else None
    qs = np.zeros((n, 10)) if quantities else None
    qb = np.zeros((n, 10)) if quantities else None
    lib(fp32).oracle_grad(W, H, _p(intr, _D), _p(w2c, _D), n, _p(m, _D), _p(l, _D), _p(q, _D), _p(o, _D),
                      _p(c, _D), _p(gr, _D), _p(gd, _D), _p(ga, _D),
                      None if sk is None else _p(sk, _U8),
                      *[_p(a, _D) for a in outs], *[_p(a, _D) for a in scl],
                      None if qg is None else _p(qg, _D), *[_p(a, _D) for a in bnd],
                      None if qs is None else _p(qs, _D), None if qb is None else _p(qb, _D))
    keys = ["means", "log_scales", "quats", "opacities", "colors", "pose"]
    G = dict(zip(keys, outs))
    S = dict(zip(keys, scl))
    S.update({k + "_fp32": b for k, b in zip(keys, bnd)})
    if quantities:
        G["quantity"] = qg
        S["quantity"] = qs
        S["quantity_fp32"] = qb
    return G, S


def binning(valid, u, v, hx, hy, zbits, W, H, tw, th, tile_base=0, index_base=0, cap=None):
    """Integer binning on given FP32 per-Gaussian values: sorted keys, values
    and the per-tile [start, end) ranges."""
    n = len(u)
    valid = np.ascontiguousarray(valid, np.uint8)
    u, v, hx, hy = (np.ascontiguousarray(a, np.float32) for a in (u, v, hx, hy))
    zbits = np.ascontiguousarray(zbits, np.uint32)
    tiles = ((W + tw - 1) // tw) * ((H + th - 1) // th)
    if cap is None:
        cap = max(1, n) * tiles if n * tiles < 50_000_000 else 50_000_000
    keys = np.zeros(cap, np.uint64)
    vals = np.zeros(cap, np.uint32)
    ranges = np.zeros((tiles, 2), np.uint32)
    P = lib().oracle_binning(n, _p(valid, _U8), _p(u, _F), _p(v, _F), _p(hx, _F), _p(hy, _F),
                             _p(zbits, _U32), W, H, tw, th, tile_base, index_base, cap,
                             _p(keys, _U64), _p(vals, _U32), _p(ranges, _U32))
    if P < 0:
        raise ValueError("pair capacity exceeded")
    return keys[:P].copy(), vals[:P].copy(), ranges
