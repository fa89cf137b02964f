"""Voxel map and frame-to-map registration (Section III-B, eq. 10-12):
argument marshalling over the C ABI of ``include/vpgs.h``."""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import check, load
from .render import Context, _ptr, _stream, get_context

__all__ = ["VoxelMap", "voxel_downsample", "icp_correspond", "icp_linearize", "icp_linearize_noalloc", "icp_register"]


def _points(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.dim() != 2 or t.shape[1] != 3 or t.dtype != torch.float32 \
            or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 GPU tensor [n, 3]")
    return t


def _pose(p) -> ctypes.Array:
    a = np.ascontiguousarray(np.asarray(p, np.float64).reshape(3, 4))
    return (ctypes.c_double * 12)(*a.reshape(-1).tolist())


class VoxelMap:
    """The first max_per_voxel points (by index) of every occupied voxel of
    size `voxel`, with a hash table over the voxels."""

    def __init__(self, points: torch.Tensor, voxel: float, max_per_voxel: int = 20, ctx: Optional[Context] = None):
        self.ctx = ctx or get_context()
        _points(points, "points")
        h = ctypes.c_void_p()
        check(load().vpgs_voxel_map_create(self.ctx.handle, _ptr(points), int(points.shape[0]), float(voxel),
                                           int(max_per_voxel), ctypes.byref(h), _stream()),
              self.ctx.handle, "vpgs_voxel_map_create")
        self.handle = h
        self.voxel = float(voxel)
        self.max_per_voxel = int(max_per_voxel)

    def info(self):
        """(points given, occupied voxels); synchronises the stream."""
        n, v = ctypes.c_int64(), ctypes.c_int64()
        check(load().vpgs_voxel_map_info(self.handle, ctypes.byref(n), ctypes.byref(v), _stream()),
              self.ctx.handle, "vpgs_voxel_map_info")
        return n.value, v.value

    def close(self):
        if getattr(self, "handle", None):
            load().vpgs_voxel_map_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def voxel_downsample(points: torch.Tensor, voxel: float, ctx: Optional[Context] = None) -> torch.Tensor:
    """Ascending indices (int64) of the first point of every occupied voxel;
    synchronises the stream to read their number."""
    ctx = ctx or get_context()
    _points(points, "points")
    n = int(points.shape[0])
    idx = torch.empty((max(n, 1),), dtype=torch.int32, device=points.device)
    cnt = torch.empty((1,), dtype=torch.int32, device=points.device)
    check(load().vpgs_voxel_downsample(ctx.handle, _ptr(points), n, float(voxel), _ptr(idx), _ptr(cnt), _stream()),
          ctx.handle, "vpgs_voxel_downsample")
    return idx[: int(cnt.item())].long()


def icp_correspond(vmap: VoxelMap, src: torch.Tensor, pose, tau: float):
    """(nn int32 [n] (-1 = none within tau), d2 float32 [n]) under pose (3x4)."""
    _points(src, "src")
    n = int(src.shape[0])
    nn = torch.empty((n,), dtype=torch.int32, device=src.device)
    d2 = torch.empty((n,), dtype=torch.float32, device=src.device)
    check(load().vpgs_icp_correspond(vmap.ctx.handle, vmap.handle, _ptr(src), n, _pose(pose), float(tau), _ptr(nn),
                                     _ptr(d2), _stream()), vmap.ctx.handle, "vpgs_icp_correspond")
    return nn, d2


def icp_linearize(vmap: VoxelMap, src: torch.Tensor, pose, tau: float, sigma: float) -> torch.Tensor:
    """The 29 Gauss-Newton terms (float64 device tensor): H upper triangle
    (21), g (6), correspondence count, sum rho."""
    _points(src, "src")
    out = torch.empty((29,), dtype=torch.float64, device=src.device)
    check(load().vpgs_icp_linearize(vmap.ctx.handle, vmap.handle, _ptr(src), int(src.shape[0]), _pose(pose),
                                    float(tau), float(sigma), _ptr(out), _stream()),
          vmap.ctx.handle, "vpgs_icp_linearize")
    return out


def icp_linearize_noalloc(vmap: VoxelMap, src: torch.Tensor, pose, tau: float, sigma: float,
                          out: torch.Tensor) -> torch.Tensor:
    """icp_linearize into a caller-given float64 [29] device tensor, with no
    allocation in the library (its partial sums use a static per-device
    scratch array, so overlapping calls on one device race)."""
    _points(src, "src")
    if out.dtype != torch.float64 or tuple(out.shape) != (29,) or not out.is_cuda or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 [29] GPU tensor")
    check(load().vpgs_icp_linearize_noalloc(vmap.ctx.handle, vmap.handle, _ptr(src), int(src.shape[0]), _pose(pose),
                                            float(tau), float(sigma), _ptr(out), _stream()),
          vmap.ctx.handle, "vpgs_icp_linearize_noalloc")
    return out


def icp_register(vmap: VoxelMap, src: torch.Tensor, prev_pose, pred_pose=None, tau: float = 1.0,
                 sigma: float = 1.0, max_iterations: int = 500, eps: float = 1e-4):
    """Registration of src (sensor frame) from prev_pose * pred_pose.
    Returns (pose float64 [3, 4], result dict)."""
    _points(src, "src")
    opts = _lib.IcpOpts(float(tau), float(sigma), int(max_iterations), 0, float(eps))
    out = (ctypes.c_double * 12)()
    res = _lib.IcpResult()
    check(load().vpgs_icp_register(vmap.ctx.handle, vmap.handle, _ptr(src), int(src.shape[0]), _pose(prev_pose),
                                   None if pred_pose is None else _pose(pred_pose), ctypes.byref(opts), out,
                                   ctypes.byref(res), _stream()), vmap.ctx.handle, "vpgs_icp_register")
    return np.array(out[:], np.float64).reshape(3, 4), {f: getattr(res, f) for f, _ in _lib.IcpResult._fields_
                                                         if f != "reserved"}
