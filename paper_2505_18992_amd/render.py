"""PyTorch-facing API of the renderer and decoder.

PyTorch supplies device memory, the current HIP stream and autograd; every
step of the computation runs in ``libvpgs.so``.

* ``render(...)``          forward render of one or more views (no autograd).
* ``render_backward(...)`` its backward.
* ``RenderFn``             ``torch.autograd.Function`` over one Gaussian set
                           and its views, with an optional se(3) pose leaf.
* ``render_views(...)``    autograd render of several sets and views.
"""
from __future__ import annotations

import ctypes
import sys
import threading
from typing import List, Optional, Sequence

import torch

from . import _lib
from ._lib import check, load

__all__ = ["Context", "get_context", "render", "render_backward", "Saved", "RenderFn", "render_views",
           "camera_struct", "decode_forward", "decode_backward", "DecodeFn", "decode", "RenderWindow",
           "mapping_loss", "volume_loss"]


class _TorchWorkspace:
    """The library's device workspace through torch's caching allocator: a
    block is a uint8 tensor held until the library hands it back (the
    library synchronises the device first)."""

    def __init__(self, device: int):
        self.device = torch.device("cuda", device)
        self.blocks = {}
        # late-bound, so a test can swap the allocation policy of a live context
        self.alloc_cb = _lib.ALLOC_FN(lambda n, u: self._alloc(n, u))
        self.free_cb = _lib.FREE_FN(lambda p, u: self._free(p, u))

    def _alloc(self, nbytes, _user):
        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        except Exception:  # out of memory: the library reports VPGS_ENOMEM
            return None
        self.blocks[t.data_ptr()] = t
        return t.data_ptr()

    def _free(self, ptr, _user):
        self.blocks.pop(ptr, None)

    def bytes_held(self) -> int:
        return sum(t.numel() for t in self.blocks.values())


class Context:
    """One library context per device (the library requires one per stream
    user).  Its workspace comes from torch's caching allocator unless
    ``torch_workspace`` is False (then the library calls hipMalloc)."""

    def __init__(self, device: int = 0, torch_workspace: bool = True):
        L = load()
        h = ctypes.c_void_p()
        self.workspace = _TorchWorkspace(device) if torch_workspace else None
        if self.workspace is not None:
            st = L.vpgs_create(ctypes.byref(h), int(device), ctypes.cast(self.workspace.alloc_cb, ctypes.c_void_p),
                               ctypes.cast(self.workspace.free_cb, ctypes.c_void_p), None)
        else:
            st = L.vpgs_create(ctypes.byref(h), int(device), None, None, None)
        if st != 0:
            raise _lib.VpgsError(st, f"vpgs_create(device={device}) failed: {L.vpgs_status_string(st).decode()}")
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            load().vpgs_destroy(self.handle)
            self.handle = None

    def profile(self, on: bool = True):
        """Enable (and reset) or disable per-stage HIP-event timing."""
        check(load().vpgs_profile_enable(self.handle, int(on)), self.handle, "vpgs_profile_enable")

    def profile_read(self) -> dict:
        """{stage name: (launch sequences recorded, total milliseconds)}."""
        L = load()
        out = {}
        for i in range(_lib.NUM_STAGES):
            name, calls, ms = ctypes.c_char_p(), ctypes.c_int64(), ctypes.c_double()
            check(L.vpgs_profile_read(self.handle, i, ctypes.byref(name), ctypes.byref(calls), ctypes.byref(ms)),
                  self.handle, "vpgs_profile_read")
            out[name.value.decode()] = (calls.value, ms.value)
        return out

    def measure_peaks(self) -> dict:
        """Measured device rates (vpgs_measure_peaks): LDS read GB/s with
        distinct and with broadcast addresses, FP32 FMA TFLOP/s, exp2 T/s and
        HBM copy GB/s."""
        out = (ctypes.c_double * 5)()
        check(load().vpgs_measure_peaks(self.handle, out, _stream()), self.handle, "vpgs_measure_peaks")
        return {"lds_GBs": out[0], "lds_broadcast_GBs": out[1], "fp32_fma_TFLOPs": out[2], "exp2_Tps": out[3],
                "hbm_copy_GBs": out[4]}

    def __del__(self):
        try:
            if not sys.is_finalizing():  # the allocator callbacks need a live interpreter
                self.close()
        except Exception:
            pass


_CTX = {}
_CTX_LOCK = threading.Lock()


def get_context(device: Optional[int] = None) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    key = (threading.get_ident(), device)
    with _CTX_LOCK:
        if key not in _CTX:
            _CTX[key] = Context(device)
        return _CTX[key]


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _check_tensor(t, name, shape_tail, n=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 GPU tensor")
    if tuple(t.shape[1:]) != tuple(shape_tail) or (n is not None and t.shape[0] != n):
        raise ValueError(f"{name}: bad shape {tuple(t.shape)}")


def camera_struct(cam) -> _lib.Camera:
    """Any object with width, height, fx, fy, cx, cy, world_to_cam (3x4) and
    optional near."""
    c = _lib.Camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.near_plane = float(getattr(cam, "near", 0.2))
    w2c = torch.as_tensor(cam.world_to_cam, dtype=torch.float32).reshape(-1).tolist()
    for k in range(12):
        c.world_to_cam[k] = w2c[k]
    return c


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Saved:
    """Handle of a forward's saved state; released on close or garbage collection."""

    def __init__(self, ctx: Context, handle, n_views, n_sets, set_sizes, view_sizes, keep_alive=()):
        self.ctx = ctx
        # the library reads the Gaussian buffers again in the backward: hold them
        self._keep_alive = tuple(keep_alive)
        self.handle = handle
        self.n_views = n_views
        self.n_sets = n_sets
        self.set_sizes = set_sizes
        self.view_sizes = view_sizes

    def stats(self) -> dict:
        s = _lib.Stats()
        st = load().vpgs_saved_stats(self.ctx.handle, self.handle, ctypes.byref(s), _stream())
        d = {f: getattr(s, f) for f, _ in _lib.Stats._fields_}
        if st not in (0, _lib.VPGS_ECAPACITY):
            check(st, self.ctx.handle, "vpgs_saved_stats")
        return d

    def export(self, what: int, dtype=torch.float32) -> torch.Tensor:
        L = load()
        size = ctypes.c_size_t(0)
        check(L.vpgs_saved_export(self.ctx.handle, self.handle, what, None, 0, ctypes.byref(size), _stream()),
              self.ctx.handle, "export size")
        itemsize = torch.tensor([], dtype=dtype).element_size()
        out = torch.empty(max(size.value // itemsize, 1), dtype=dtype, device="cuda")
        check(L.vpgs_saved_export(self.ctx.handle, self.handle, what, _ptr(out), out.numel() * itemsize, None,
                                  _stream()), self.ctx.handle, "export")
        return out[: size.value // itemsize]

    def close(self):
        if self.handle:
            load().vpgs_saved_release(self.ctx.handle, self.handle)
            self.handle = None
        self._keep_alive = ()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _set_struct(s) -> _lib.Gaussians:
    means, log_scales, quats, opacities, colors = s
    n = means.shape[0]
    _check_tensor(means, "means", (3,), n)
    _check_tensor(log_scales, "log_scales", (3,), n)
    _check_tensor(quats, "quats", (4,), n)
    _check_tensor(opacities, "opacities", (), n)
    _check_tensor(colors, "colors", (3,), n)
    g = _lib.Gaussians()
    g.n = n
    g.means, g.log_scales, g.quats, g.opacities, g.colors = (t.data_ptr() for t in s)
    return g


def render(sets: Sequence[Sequence[torch.Tensor]], cameras: Sequence, view_set: Optional[Sequence[int]] = None,
           tile=(16, 16), pair_capacity: int = 0, keep: bool = True, ctx: Optional[Context] = None,
           lds_batch: int = 0, grid_ctas: int = 0, count: bool = True):
    """Forward render.  ``sets`` is a list of (means, log_scales, quats,
    opacities, colors) tuples; view v renders sets[view_set[v]] with
    cameras[v].  lds_batch: entries staged per compositing batch (0 = the
    tile's pixel count); grid_ctas: persistent compositing workgroups (0 =
    one per tile); count: count evaluations and blends (Saved.stats).  Returns (list of (rgb[3,H,W], depth[H,W], alpha[H,W]),
    Saved or None)."""
    ctx = ctx or get_context()
    L = load()
    nv = len(cameras)
    if view_set is None:
        view_set = [0] * nv
    gs = (_lib.Gaussians * len(sets))(*[_set_struct(s) for s in sets])
    cams = (_lib.Camera * nv)(*[camera_struct(c) for c in cameras])
    vs = (ctypes.c_int32 * nv)(*view_set)
    outs, ims = [], (_lib.Images * nv)()
    dev = sets[0][0].device
    for v, c in enumerate(cameras):
        H, W = int(c.height), int(c.width)
        rgb = torch.empty((3, H, W), dtype=torch.float32, device=dev)
        depth = torch.empty((H, W), dtype=torch.float32, device=dev)
        alpha = torch.empty((H, W), dtype=torch.float32, device=dev)
        ims[v].rgb, ims[v].depth, ims[v].alpha = rgb.data_ptr(), depth.data_ptr(), alpha.data_ptr()
        outs.append((rgb, depth, alpha))
    opts = _lib.RenderOpts()
    opts.tile_w, opts.tile_h = tile
    opts.lds_batch = int(lds_batch)
    opts.grid_ctas = int(grid_ctas)
    opts.pair_capacity = int(pair_capacity)
    opts.skip_counts = 0 if count else 1
    h = ctypes.c_void_p()
    st = L.vpgs_render_forward(ctx.handle, len(sets), gs, nv, vs, cams, ims, ctypes.byref(opts),
                               ctypes.byref(h) if keep else None, _stream())
    check(st, ctx.handle, "vpgs_render_forward")
    saved = Saved(ctx, h, nv, len(sets), [s[0].shape[0] for s in sets],
                  [(int(c.height), int(c.width)) for c in cameras],
                  keep_alive=[t for s in sets for t in s]) if keep else None
    return outs, saved


def _accum_struct(accum, set_sizes, grad_space: int):
    """DensifyAccum over per-set [n,4] float32 tensors (None entries allowed);
    returns (struct, keep-alive array)."""
    if len(accum) != len(set_sizes):
        raise ValueError("one accumulator (or None) per set")
    arr = (ctypes.c_void_p * max(len(accum), 1))()
    for s, (a, n) in enumerate(zip(accum, set_sizes)):
        if a is None:
            continue
        if tuple(a.shape) != (n, 4) or a.dtype != torch.float32 or not a.is_contiguous():
            raise ValueError(f"set {s}: accumulators must be contiguous float32 [{n}, 4]")
        arr[s] = a.data_ptr()
    return _lib.DensifyAccum(ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p)), int(grad_space), 0), arr


def render_backward(saved: Saved, grad_images: Sequence, want_pose: bool = True, accum: Optional[Sequence] = None,
                    grad_space: int = 0):
    """Backward of ``render``.  grad_images[v] = (g_rgb, g_depth, g_alpha),
    any of them None.  Returns (list of per-set gradient tuples, d_pose[V,6] or None).

    accum: optional per-set [n,4] float32 expansion accumulators (or None per
    set) that the same pass adds to: (sum of |dL/d(u,v)| and count over the
    views that render each Gaussian, sum of max(opacity,0) and count over the
    views whose frustum holds its centre); grad_space 1 measures the gradient
    in normalised device coordinates."""
    L = load()
    nv, ns = saved.n_views, saved.n_sets
    gi = (_lib.ImageGrads * nv)()
    keep_alive = []
    for v, (gr, gd, ga) in enumerate(grad_images):
        H, W = saved.view_sizes[v]
        for t, shp in ((gr, (3, H, W)), (gd, (H, W)), (ga, (H, W))):
            if t is not None and (tuple(t.shape) != shp or t.dtype != torch.float32 or not t.is_contiguous()):
                raise ValueError(f"upstream gradient of view {v} must be contiguous float32 of shape {shp}")
        gi[v].rgb, gi[v].depth, gi[v].alpha = (t.data_ptr() if t is not None else None for t in (gr, gd, ga))
        keep_alive += [gr, gd, ga]
    grads, gb = [], (_lib.GaussBuffers * ns)()
    for s, n in enumerate(saved.set_sizes):
        g = (torch.empty((n, 3), dtype=torch.float32, device="cuda"),
             torch.empty((n, 3), dtype=torch.float32, device="cuda"),
             torch.empty((n, 4), dtype=torch.float32, device="cuda"),
             torch.empty((n,), dtype=torch.float32, device="cuda"),
             torch.empty((n, 3), dtype=torch.float32, device="cuda"))
        gb[s].means, gb[s].log_scales, gb[s].quats, gb[s].opacities, gb[s].colors = (t.data_ptr() for t in g)
        grads.append(g)
    d_pose = torch.empty((nv, 6), dtype=torch.float32, device="cuda") if want_pose else None
    if accum is None:
        st = L.vpgs_render_backward(saved.ctx.handle, saved.handle, gi, gb, _ptr(d_pose) if want_pose else None,
                                    _stream())
        check(st, saved.ctx.handle, "vpgs_render_backward")
    else:
        acc, _keep = _accum_struct(accum, saved.set_sizes, grad_space)
        st = L.vpgs_render_backward_accum(saved.ctx.handle, saved.handle, gi, gb,
                                          _ptr(d_pose) if want_pose else None, ctypes.byref(acc), _stream())
        check(st, saved.ctx.handle, "vpgs_render_backward_accum")
    return grads, d_pose


class _RenderViews(torch.autograd.Function):
    @staticmethod
    def forward(ctx, cfg, pose_delta, *flat):
        cameras, view_set, tile, cap = cfg
        sets = [tuple(flat[5 * s: 5 * s + 5]) for s in range(len(flat) // 5)]
        sets = [tuple(t.detach().contiguous() for t in s) for s in sets]
        outs, saved = render(sets, cameras, view_set, tile=tile, pair_capacity=cap, keep=True)
        ctx.saved_handle = saved
        ctx.n_sets = len(sets)
        ctx.want_pose = pose_delta is not None
        flat_out = []
        for o in outs:
            flat_out += list(o)
        return tuple(flat_out)

    @staticmethod
    def backward(ctx, *g):
        saved = ctx.saved_handle
        grads_img = []
        for v in range(saved.n_views):
            trip = g[3 * v: 3 * v + 3]
            grads_img.append(tuple(t.contiguous() if t is not None else None for t in trip))
        grads, d_pose = render_backward(saved, grads_img, want_pose=ctx.want_pose)
        saved.close()
        ctx.saved_handle = None
        flat = []
        for gset in grads:
            flat += list(gset)
        return (None, d_pose, *flat)


def render_views(sets, cameras, view_set=None, pose_delta: Optional[torch.Tensor] = None, tile=(16, 16),
                 pair_capacity: int = 0):
    """Differentiable render of several Gaussian sets and views.

    ``pose_delta`` ([V, 6], zeros) is a leaf whose gradient is the gradient of
    the loss with respect to a left se(3) increment (rho, phi) of each view's
    pose; the render itself is at the given poses.  Returns a list of
    (rgb, depth, alpha) per view."""
    nv = len(cameras)
    if view_set is None:
        view_set = [0] * nv
    flat = []
    for s in sets:
        flat += list(s)
    out = _RenderViews.apply((list(cameras), list(view_set), tuple(tile), int(pair_capacity)), pose_delta, *flat)
    return [tuple(out[3 * v: 3 * v + 3]) for v in range(nv)]


# The autograd function: RenderFn.apply((cameras, view_set, tile, capacity), pose_delta, *set_tensors)
RenderFn = _RenderViews


# ---------------------------------------------------------------------------
# mapping window: all views bound once, tuned once, replayed as graph launches
# ---------------------------------------------------------------------------

class RenderWindow:
    """Batched forward+backward of a fixed set of views (a mapping window).

    ``outputs[v]`` = (rgb, depth, alpha) written by each forward;
    ``grad_out[v]`` = (g_rgb, g_depth, g_alpha) read by each backward (fill
    them in place, e.g. with a loss gradient, between the two parts);
    ``grads[s]`` = the 5 gradient tensors of set s; ``d_pose`` [V, 6].
    The Gaussian tensors are read in place, so an optimiser may update them
    between runs."""

    def __init__(self, sets, cameras, view_set=None, tile=None, persistent: int = -1, use_graph: bool = True,
                 pair_capacity: int = 0, tune_reps: int = 3, ctx: Optional[Context] = None, lds_batch: int = 0,
                 tune_cache: Optional[str] = None, count: bool = True):
        self.ctx = ctx or get_context()
        L = load()
        nv = len(cameras)
        view_set = [0] * nv if view_set is None else list(view_set)
        self.sets = [tuple(s) for s in sets]
        dev = self.sets[0][0].device
        f = lambda *shape: torch.zeros(shape, dtype=torch.float32, device=dev)
        self.outputs = [(f(3, c.height, c.width), f(c.height, c.width), f(c.height, c.width)) for c in cameras]
        self.grad_out = [(f(3, c.height, c.width), f(c.height, c.width), f(c.height, c.width)) for c in cameras]
        self.grads = [(f(s[0].shape[0], 3), f(s[0].shape[0], 3), f(s[0].shape[0], 4), f(s[0].shape[0]),
                       f(s[0].shape[0], 3)) for s in self.sets]
        self.d_pose = f(nv, 6)
        gs = (_lib.Gaussians * len(self.sets))(*[_set_struct(s) for s in self.sets])
        cams = (_lib.Camera * nv)(*[camera_struct(c) for c in cameras])
        vs = (ctypes.c_int32 * nv)(*view_set)
        ims = (_lib.Images * nv)()
        gis = (_lib.ImageGrads * nv)()
        for v in range(nv):
            ims[v].rgb, ims[v].depth, ims[v].alpha = (t.data_ptr() for t in self.outputs[v])
            gis[v].rgb, gis[v].depth, gis[v].alpha = (t.data_ptr() for t in self.grad_out[v])
        gb = (_lib.GaussBuffers * len(self.sets))()
        for s, g in enumerate(self.grads):
            gb[s].means, gb[s].log_scales, gb[s].quats, gb[s].opacities, gb[s].colors = (t.data_ptr() for t in g)
        o = _lib.WindowOpts()
        o.tile_w, o.tile_h = tile if tile is not None else (0, 0)
        o.persistent = int(persistent)
        o.use_graph = int(use_graph)
        o.pair_capacity = int(pair_capacity)
        o.tune_reps = int(tune_reps)
        o.lds_batch = int(lds_batch)
        o.tune_cache = None if tune_cache is None else str(tune_cache).encode()
        o.skip_counts = 0 if count else 1
        h = ctypes.c_void_p()
        check(L.vpgs_window_create(self.ctx.handle, len(self.sets), gs, nv, vs, cams, ims, gis, gb,
                                   _ptr(self.d_pose), ctypes.byref(o), ctypes.byref(h), _stream()),
              self.ctx.handle, "vpgs_window_create")
        self.handle = h
        self.n_views = nv

    def set_cameras(self, cameras):
        cams = (_lib.Camera * self.n_views)(*[camera_struct(c) for c in cameras])
        check(load().vpgs_window_set_cameras(self.handle, cams), self.ctx.handle, "vpgs_window_set_cameras")

    def set_accum(self, accum: Optional[Sequence], grad_space: int = 0):
        """Binds per-set [n,4] expansion accumulators (see ``render_backward``)
        that every later backward run adds to; None unbinds."""
        L = load()
        if accum is None:
            check(L.vpgs_window_set_accum(self.handle, None), self.ctx.handle, "vpgs_window_set_accum")
            self._accum = None
            return
        acc, keep = _accum_struct(accum, [s[0].shape[0] for s in self.sets], grad_space)
        check(L.vpgs_window_set_accum(self.handle, ctypes.byref(acc)), self.ctx.handle, "vpgs_window_set_accum")
        self._accum = list(accum)  # the window keeps the device pointers

    def run(self, forward: bool = True, backward: bool = True):
        parts = (_lib.WINDOW_FORWARD if forward else 0) | (_lib.WINDOW_BACKWARD if backward else 0)
        check(load().vpgs_window_run(self.handle, parts, _stream()), self.ctx.handle, "vpgs_window_run")

    def stats(self) -> dict:
        s = _lib.Stats()
        st = load().vpgs_window_stats(self.handle, ctypes.byref(s), _stream())
        if st not in (0, _lib.VPGS_ECAPACITY):
            check(st, self.ctx.handle, "vpgs_window_stats")
        return {f: getattr(s, f) for f, _ in _lib.Stats._fields_}

    def config(self) -> dict:
        o = _lib.WindowOpts()
        check(load().vpgs_window_config(self.handle, ctypes.byref(o)), self.ctx.handle, "vpgs_window_config")
        return {f: getattr(o, f) for f, _ in _lib.WindowOpts._fields_ if f not in ("tune_cache", "reserved")}

    def close(self):
        if getattr(self, "handle", None):
            load().vpgs_window_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# anchor decoder
# ---------------------------------------------------------------------------

def _anchors_struct(xyz, feat, scale, offsets) -> _lib.Anchors:
    m, k = offsets.shape[0], offsets.shape[1]
    _check_tensor(xyz, "xyz", (3,), m)
    _check_tensor(feat, "feat", (32,), m)
    _check_tensor(scale, "scale", (3,), m)
    _check_tensor(offsets, "offsets", (k, 3), m)
    a = _lib.Anchors()
    a.m, a.k = m, k
    a.xyz, a.feat, a.scale, a.offsets = xyz.data_ptr(), feat.data_ptr(), scale.data_ptr(), offsets.data_ptr()
    return a


def _mlp_struct(W1, b1, W2, b2) -> _lib.Mlp:
    mlp = _lib.Mlp()
    mlp.in_dim = int(W1[0].shape[1])
    mlp.width = int(W1[0].shape[0])
    for h in range(3):
        for t, nm in ((W1[h], "W1"), (b1[h], "b1"), (W2[h], "W2"), (b2[h], "b2")):
            if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{nm}[{h}] must be a contiguous float32 GPU tensor")
        mlp.W1[h], mlp.b1[h], mlp.W2[h], mlp.b2[h] = (W1[h].data_ptr(), b1[h].data_ptr(), W2[h].data_ptr(),
                                                      b2[h].data_ptr())
    return mlp


def _cam3(cam_center):
    c = [float(x) for x in torch.as_tensor(cam_center).reshape(-1).tolist()]
    return (ctypes.c_float * 3)(*c)


def decode_forward(anchors, mlp, cam_center, ctx: Optional[Context] = None):
    """Decode m*k neural Gaussians from anchors (xyz, feat, scale, offsets)
    and decoder weights (W1, b1, W2, b2: lists of 3 tensors).  Returns
    (means, log_scales, quats, opacities, colors)."""
    ctx = ctx or get_context()
    xyz, feat, scale, offsets = anchors
    m, k = offsets.shape[0], offsets.shape[1]
    n = m * k
    dev = xyz.device
    out = (torch.empty((n, 3), dtype=torch.float32, device=dev), torch.empty((n, 3), dtype=torch.float32, device=dev),
           torch.empty((n, 4), dtype=torch.float32, device=dev), torch.empty((n,), dtype=torch.float32, device=dev),
           torch.empty((n, 3), dtype=torch.float32, device=dev))
    gb = _lib.GaussBuffers()
    gb.means, gb.log_scales, gb.quats, gb.opacities, gb.colors = (t.data_ptr() for t in out)
    a = _anchors_struct(xyz, feat, scale, offsets)
    w = _mlp_struct(*mlp)
    check(load().vpgs_decode_forward(ctx.handle, ctypes.byref(a), ctypes.byref(w), _cam3(cam_center),
                                     ctypes.byref(gb), _stream()), ctx.handle, "vpgs_decode_forward")
    return out


def decode_backward(anchors, mlp, cam_center, upstream, ctx: Optional[Context] = None):
    """Gradients of sum(upstream . decoded) w.r.t. feat, scale, offsets and the
    weights.  Returns (d_feat, d_scale, d_offsets, (dW1, db1, dW2, db2))."""
    ctx = ctx or get_context()
    xyz, feat, scale, offsets = anchors
    W1, b1, W2, b2 = mlp
    up = tuple(t.contiguous() for t in upstream)
    for t, shp in zip(up, ((3,), (3,), (4,), (), (3,))):
        if t.dtype != torch.float32 or tuple(t.shape[1:]) != shp:
            raise ValueError("upstream gradients must be float32 with the decoded shapes")
    gb = _lib.GaussBuffers()
    gb.means, gb.log_scales, gb.quats, gb.opacities, gb.colors = (t.data_ptr() for t in up)
    d_feat, d_scale, d_off = torch.empty_like(feat), torch.empty_like(scale), torch.empty_like(offsets)
    dW1 = [torch.empty_like(t) for t in W1]
    db1 = [torch.empty_like(t) for t in b1]
    dW2 = [torch.empty_like(t) for t in W2]
    db2 = [torch.empty_like(t) for t in b2]
    g = _lib.MlpGrads()
    for h in range(3):
        g.W1[h], g.b1[h], g.W2[h], g.b2[h] = dW1[h].data_ptr(), db1[h].data_ptr(), dW2[h].data_ptr(), db2[h].data_ptr()
    a = _anchors_struct(xyz, feat, scale, offsets)
    w = _mlp_struct(W1, b1, W2, b2)
    check(load().vpgs_decode_backward(ctx.handle, ctypes.byref(a), ctypes.byref(w), _cam3(cam_center),
                                      ctypes.byref(gb), _ptr(d_feat), _ptr(d_scale), _ptr(d_off), ctypes.byref(g),
                                      _stream()), ctx.handle, "vpgs_decode_backward")
    return d_feat, d_scale, d_off, (dW1, db1, dW2, db2)


class DecodeFn(torch.autograd.Function):
    """DecodeFn.apply(cam_center, xyz, feat, scale, offsets, W1_0, W1_1, W1_2,
    b1_0.., W2_0.., b2_0..) -> (means, log_scales, quats, opacities, colors).
    Gradients flow to feat, scale, offsets and the 12 weight tensors (the
    anchor positions and the camera are constants of the decode)."""

    @staticmethod
    def forward(ctx, cam_center, xyz, feat, scale, offsets, *w):
        W1, b1, W2, b2 = list(w[0:3]), list(w[3:6]), list(w[6:9]), list(w[9:12])
        anchors = tuple(t.detach().contiguous() for t in (xyz, feat, scale, offsets))
        mlp = tuple([t.detach().contiguous() for t in lst] for lst in (W1, b1, W2, b2))
        ctx.save_for_backward(*anchors, *[t for lst in mlp for t in lst])
        ctx.cam_center = cam_center
        return decode_forward(anchors, mlp, cam_center)

    @staticmethod
    def backward(ctx, *g):
        saved = ctx.saved_tensors
        anchors = saved[:4]
        mlp = (list(saved[4:7]), list(saved[7:10]), list(saved[10:13]), list(saved[13:16]))
        up = []
        for t, ref in zip(g, decode_forward_shapes(anchors)):
            up.append(t if t is not None else torch.zeros(ref, dtype=torch.float32, device=anchors[0].device))
        d_feat, d_scale, d_off, (dW1, db1, dW2, db2) = decode_backward(anchors, mlp, ctx.cam_center, up)
        return (None, None, d_feat, d_scale, d_off, *dW1, *db1, *dW2, *db2)


def decode_forward_shapes(anchors):
    m, k = anchors[3].shape[0], anchors[3].shape[1]
    n = m * k
    return ((n, 3), (n, 3), (n, 4), (n,), (n, 3))


def decode(anchors, mlp, cam_center):
    """Differentiable decode: anchors = (xyz, feat, scale, offsets); mlp =
    (W1, b1, W2, b2) lists of 3 tensors each."""
    W1, b1, W2, b2 = mlp
    return DecodeFn.apply(cam_center, *anchors, *W1, *b1, *W2, *b2)


# ---------------------------------------------------------------------------
# mapping loss (eq. 7-9)
# ---------------------------------------------------------------------------
def mapping_loss(images: Sequence, targets: Sequence, cameras: Sequence, lambda_ssim: float = 0.2,
                 lambda_depth: float = 1.0, ctx: Optional[Context] = None):
    """Mapping loss of eq. 7-8 of every view and its gradient planes.

    images: per view (rgb [3,H,W], depth [H,W], ...) as rendered; targets:
    per view (rgb [3,H,W], depth [H,W]) with depth <= 0 = no target.  Returns
    (terms [n_views, 4] = (L_c, L_SSIM, L_d, L) on the device, grads) with
    grads[v] = (g_rgb, g_depth, g_alpha) -- the upstream planes of the render
    backward for the summed loss (g_alpha is zero)."""
    ctx = ctx or get_context()
    nv = len(images)
    if not (len(targets) == nv and len(cameras) == nv):
        raise ValueError("images, targets and cameras must have one entry per view")
    dev = images[0][0].device if nv else torch.device("cuda")
    cams = (_lib.Camera * max(nv, 1))()
    ims = (_lib.Images * max(nv, 1))()
    tgs = (_lib.Targets * max(nv, 1))()
    gbs = (_lib.Images * max(nv, 1))()
    grads = []
    for v in range(nv):
        rgb, depth = images[v][0], images[v][1]
        trgb, tdepth = targets[v][0], targets[v][1]
        H, W = int(depth.shape[0]), int(depth.shape[1])
        for t, shape, name in ((rgb, (3, H, W), "rgb"), (depth, (H, W), "depth"), (trgb, (3, H, W), "target rgb"),
                               (tdepth, (H, W), "target depth")):
            if tuple(t.shape) != shape or t.dtype != torch.float32 or not t.is_contiguous():
                raise ValueError(f"view {v}: {name} must be contiguous float32 {shape}")
        cams[v] = camera_struct(cameras[v]) if not isinstance(cameras[v], _lib.Camera) else cameras[v]
        if cams[v].width != W or cams[v].height != H:
            raise ValueError(f"view {v}: camera size {cams[v].width}x{cams[v].height} differs from the image {W}x{H}")
        ims[v].rgb, ims[v].depth, ims[v].alpha = rgb.data_ptr(), depth.data_ptr(), None
        tgs[v].rgb, tgs[v].depth = trgb.data_ptr(), tdepth.data_ptr()
        g = (torch.empty_like(rgb), torch.empty_like(depth), torch.empty_like(depth))
        gbs[v].rgb, gbs[v].depth, gbs[v].alpha = (t.data_ptr() for t in g)
        grads.append(g)
    terms = torch.empty((max(nv, 1), 4), dtype=torch.float32, device=dev)
    opts = _lib.LossOpts(float(lambda_ssim), float(lambda_depth), 0, 0)
    check(load().vpgs_mapping_loss(ctx.handle, nv, cams, ims, tgs, ctypes.byref(opts), terms.data_ptr(), gbs,
                                   _stream()), ctx.handle, "vpgs_mapping_loss")
    return terms[:nv], grads


def volume_loss(sets: Sequence, grads: Sequence, lambda_vol: float = 0.001, ctx: Optional[Context] = None):
    """Volume term of eq. 9 per Gaussian set; adds its gradient into
    grads[s][1] (the log-scale gradients).  Returns the per-set losses
    (device tensor [n_sets])."""
    ctx = ctx or get_context()
    ns = len(sets)
    if len(grads) != ns:
        raise ValueError("one gradient tuple per set")
    gs = (_lib.Gaussians * max(ns, 1))()
    gb = (_lib.GaussBuffers * max(ns, 1))()
    for s in range(ns):
        gs[s] = _set_struct(sets[s])
        dls = grads[s][1]
        if tuple(dls.shape) != tuple(sets[s][1].shape) or dls.dtype != torch.float32 or not dls.is_contiguous():
            raise ValueError(f"set {s}: log-scale gradient must match the log-scales")
        gb[s].log_scales = dls.data_ptr()
    dev = sets[0][0].device if ns else torch.device("cuda")
    out = torch.empty((max(ns, 1),), dtype=torch.float32, device=dev)
    check(load().vpgs_volume_loss(ctx.handle, ns, gs, float(lambda_vol), out.data_ptr(), gb, _stream()), ctx.handle,
          "vpgs_volume_loss")
    return out[:ns]


# ---------------------------------------------------------------------------
# submap expansion statistics
# ---------------------------------------------------------------------------

def anchor_stats(accum: torch.Tensor, k: int, tau_g: float, tau_o: float, ctx: Optional[Context] = None):
    """Per-anchor statistics from the [m*k, 4] accumulators of decoded
    Gaussians (anchor-major): (stats [m,4] = (averaged gradient, rendered
    views, accumulated opacity, frustum views), grow uint8 [m], prune uint8 [m])."""
    ctx = ctx or get_context()
    if accum.dim() != 2 or accum.shape[1] != 4 or accum.dtype != torch.float32 or not accum.is_contiguous():
        raise ValueError("accumulators must be contiguous float32 [m*k, 4]")
    if k < 1 or accum.shape[0] % k:
        raise ValueError("the accumulator rows must be a multiple of k")
    m = accum.shape[0] // k
    stats = torch.empty((m, 4), dtype=torch.float32, device=accum.device)
    grow = torch.empty((m,), dtype=torch.uint8, device=accum.device)
    prune = torch.empty((m,), dtype=torch.uint8, device=accum.device)
    check(load().vpgs_anchor_stats(ctx.handle, m, int(k), _ptr(accum), float(tau_g), float(tau_o), _ptr(stats),
                                   _ptr(grow), _ptr(prune), _stream()), ctx.handle, "vpgs_anchor_stats")
    return stats, grow, prune


def expansion_sample(images: Sequence, targets: Sequence, cameras: Sequence, alpha_threshold: float,
                     depth_threshold: float, uniforms: Optional[torch.Tensor] = None, want_mask: bool = True,
                     ctx: Optional[Context] = None) -> dict:
    """Expansion candidates and samples of every view (Section III-A).

    images[v] = (rgb, depth, alpha) as rendered (depth and alpha are read);
    targets[v] = (rgb [3,H,W], depth [H,W]); uniforms [n_views, M] float32
    in [0, 1) or None (no samples).  Returns a dict with counts [V] int32,
    masks (list of uint8 [H,W], or None), and for M > 0 pixels [V,M] int32,
    points [V,M,3] and colors [V,M,3]."""
    ctx = ctx or get_context()
    nv = len(images)
    if not (len(targets) == nv and len(cameras) == nv):
        raise ValueError("images, targets and cameras must have one entry per view")
    dev = images[0][1].device if nv else torch.device("cuda")
    M = 0
    if uniforms is not None:
        if uniforms.dim() != 2 or uniforms.shape[0] != nv or uniforms.dtype != torch.float32 \
                or not uniforms.is_contiguous():
            raise ValueError("uniforms must be contiguous float32 [n_views, M]")
        M = int(uniforms.shape[1])
    cams = (_lib.Camera * max(nv, 1))()
    ims = (_lib.Images * max(nv, 1))()
    tgs = (_lib.Targets * max(nv, 1))()
    outs = (_lib.ExpandOut * max(nv, 1))()
    masks = []
    pixels = torch.empty((nv, M), dtype=torch.int32, device=dev)
    points = torch.empty((nv, M, 3), dtype=torch.float32, device=dev)
    colors = torch.empty((nv, M, 3), dtype=torch.float32, device=dev)
    for v in range(nv):
        depth, alpha = images[v][1], images[v][2]
        trgb, tdepth = targets[v][0], targets[v][1]
        H, W = int(depth.shape[0]), int(depth.shape[1])
        for t, shape, name in ((depth, (H, W), "depth"), (alpha, (H, W), "alpha"), (trgb, (3, H, W), "target rgb"),
                               (tdepth, (H, W), "target depth")):
            if tuple(t.shape) != shape or t.dtype != torch.float32 or not t.is_contiguous():
                raise ValueError(f"view {v}: {name} must be contiguous float32 {shape}")
        cams[v] = camera_struct(cameras[v]) if not isinstance(cameras[v], _lib.Camera) else cameras[v]
        if cams[v].width != W or cams[v].height != H:
            raise ValueError(f"view {v}: camera size {cams[v].width}x{cams[v].height} differs from the image {W}x{H}")
        ims[v].rgb, ims[v].depth, ims[v].alpha = None, depth.data_ptr(), alpha.data_ptr()
        tgs[v].rgb, tgs[v].depth = trgb.data_ptr(), tdepth.data_ptr()
        mk = torch.empty((H, W), dtype=torch.uint8, device=dev) if want_mask else None
        masks.append(mk)
        outs[v].mask = _ptr(mk)
        if M > 0:
            outs[v].pixel, outs[v].points, outs[v].colors = (pixels[v].data_ptr(), points[v].data_ptr(),
                                                              colors[v].data_ptr())
    counts = torch.empty((max(nv, 1),), dtype=torch.int32, device=dev)
    opts = _lib.ExpandOpts(float(alpha_threshold), float(depth_threshold), M, 0)
    check(load().vpgs_expansion_sample(ctx.handle, nv, cams, ims, tgs, ctypes.byref(opts), _ptr(uniforms),
                                       counts.data_ptr(), outs, _stream()), ctx.handle, "vpgs_expansion_sample")
    out = {"counts": counts[:nv], "masks": masks if want_mask else None}
    if M > 0:
        out.update(pixels=pixels, points=points, colors=colors)
    return out


# ---------------------------------------------------------------------------
# submap fusion
# ---------------------------------------------------------------------------

def distill_loss(images_a: Sequence, images_b: Sequence, cameras: Sequence, grad_a: Optional[Sequence] = None,
                 grad_b: Optional[Sequence] = None, want_grads: bool = True, ctx: Optional[Context] = None):
    """Distillation loss of eq. 14 between two submaps rendered at the m
    keyframes of their overlap: images_a[k] / images_b[k] = (rgb, depth, ...)
    from submap alpha / beta.  Returns (loss [1], terms [m, 2], grads_a,
    grads_b); grads are per keyframe (g_rgb, g_depth, g_alpha) written into
    grad_a / grad_b when given (e.g. a window's upstream planes), else
    allocated when want_grads (None otherwise)."""
    ctx = ctx or get_context()
    m = len(images_a)
    if not (len(images_b) == m and len(cameras) == m):
        raise ValueError("images_a, images_b and cameras must have one entry per keyframe")
    dev = images_a[0][0].device if m else torch.device("cuda")
    cams = (_lib.Camera * max(m, 1))()
    ia = (_lib.Images * max(m, 1))()
    ib = (_lib.Images * max(m, 1))()
    ga = (_lib.Images * max(m, 1))()
    gb = (_lib.Images * max(m, 1))()
    outs = {"a": grad_a, "b": grad_b}
    for side in ("a", "b"):
        if outs[side] is None and want_grads:
            outs[side] = [tuple(torch.empty_like(x) for x in (img[0], img[1], img[1]))
                          for img in (images_a if side == "a" else images_b)]
    for k in range(m):
        for side, src in (("a", images_a[k]), ("b", images_b[k])):
            rgb, depth = src[0], src[1]
            H, W = int(depth.shape[0]), int(depth.shape[1])
            for t, shape, name in ((rgb, (3, H, W), "rgb"), (depth, (H, W), "depth")):
                if tuple(t.shape) != shape or t.dtype != torch.float32 or not t.is_contiguous():
                    raise ValueError(f"keyframe {k} ({side}): {name} must be contiguous float32 {shape}")
            dst = ia if side == "a" else ib
            dst[k].rgb, dst[k].depth, dst[k].alpha = rgb.data_ptr(), depth.data_ptr(), None
            g = outs[side]
            if g is not None:
                gg = ga if side == "a" else gb
                gg[k].rgb, gg[k].depth, gg[k].alpha = (t.data_ptr() if t is not None else None for t in g[k])
        cams[k] = camera_struct(cameras[k]) if not isinstance(cameras[k], _lib.Camera) else cameras[k]
        if cams[k].width != int(images_a[k][1].shape[1]) or cams[k].height != int(images_a[k][1].shape[0]):
            raise ValueError(f"keyframe {k}: camera size differs from the images")
        if tuple(images_b[k][1].shape) != tuple(images_a[k][1].shape):
            raise ValueError(f"keyframe {k}: the two renders differ in size")
    terms = torch.empty((max(m, 1), 2), dtype=torch.float32, device=dev)
    loss = torch.empty((1,), dtype=torch.float32, device=dev)
    check(load().vpgs_distill_loss(ctx.handle, m, cams, ia, ib, terms.data_ptr(), loss.data_ptr(),
                                   ga if outs["a"] is not None else None, gb if outs["b"] is not None else None,
                                   _stream()), ctx.handle, "vpgs_distill_loss")
    return loss, terms[:m], outs["a"], outs["b"]
