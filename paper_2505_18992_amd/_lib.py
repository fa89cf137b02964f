"""ctypes binding of ``libvpgs.so`` -- argument marshalling only.

The structures mirror ``include/vpgs.h`` field for field.  Loading fails
loudly when the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvpgs.so")

c_float_p = ctypes.POINTER(ctypes.c_float)
c_void_p = ctypes.c_void_p

VPGS_OK = 0
VPGS_EINVAL = -1
VPGS_ENOMEM = -2
VPGS_EHIP = -3
VPGS_ECAPACITY = -4
VPGS_EUNSUPPORTED = -5
MAX_VIEWS = 64
MAX_SETS = 64
NUM_STAGES = 20
WINDOW_FORWARD, WINDOW_BACKWARD = 1, 2

BUF_PROJ, BUF_EXTENT, BUF_COUNT, BUF_KEYS, BUF_VALUES, BUF_RANGES, BUF_TFINAL, BUF_NCONTRIB = range(1, 9)


class Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("near_plane", ctypes.c_float), ("world_to_cam", ctypes.c_float * 12)]


class Gaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("means", c_void_p), ("log_scales", c_void_p), ("quats", c_void_p),
                ("opacities", c_void_p), ("colors", c_void_p)]


class Images(ctypes.Structure):
    _fields_ = [("rgb", c_void_p), ("depth", c_void_p), ("alpha", c_void_p)]


class ImageGrads(ctypes.Structure):
    _fields_ = [("rgb", c_void_p), ("depth", c_void_p), ("alpha", c_void_p)]


class GaussBuffers(ctypes.Structure):
    _fields_ = [("means", c_void_p), ("log_scales", c_void_p), ("quats", c_void_p), ("opacities", c_void_p),
                ("colors", c_void_p)]


class RenderOpts(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("lds_batch", ctypes.c_int32),
                ("grid_ctas", ctypes.c_int32), ("pair_capacity", ctypes.c_int64), ("skip_counts", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("n_records", ctypes.c_int64), ("n_visible", ctypes.c_int64), ("n_pairs", ctypes.c_int64),
                ("n_evaluated", ctypes.c_int64), ("n_blended", ctypes.c_int64), ("pair_capacity", ctypes.c_int64),
                ("n_tiles", ctypes.c_int64), ("n_pixels", ctypes.c_int64), ("overflow", ctypes.c_int32),
                ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("lds_batch", ctypes.c_int32),
                ("n_fwd_steps", ctypes.c_int64), ("n_bwd_steps", ctypes.c_int64), ("n_bwd_active", ctypes.c_int64)]


class WindowOpts(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("pair_capacity", ctypes.c_int64), ("tune_reps", ctypes.c_int32),
                ("lds_batch", ctypes.c_int32), ("tune_cache", ctypes.c_char_p), ("skip_counts", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Anchors(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("k", ctypes.c_int32), ("reserved", ctypes.c_int32), ("xyz", c_void_p),
                ("feat", c_void_p), ("scale", c_void_p), ("offsets", c_void_p)]


class Mlp(ctypes.Structure):
    _fields_ = [("in_dim", ctypes.c_int32), ("width", ctypes.c_int32), ("W1", c_void_p * 3), ("b1", c_void_p * 3),
                ("W2", c_void_p * 3), ("b2", c_void_p * 3)]


class MlpGrads(ctypes.Structure):
    _fields_ = [("W1", c_void_p * 3), ("b1", c_void_p * 3), ("W2", c_void_p * 3), ("b2", c_void_p * 3)]


class Targets(ctypes.Structure):
    _fields_ = [("rgb", c_void_p), ("depth", c_void_p)]


class LossOpts(ctypes.Structure):
    _fields_ = [("lambda_ssim", ctypes.c_float), ("lambda_depth", ctypes.c_float), ("reserved0", ctypes.c_int32),
                ("reserved1", ctypes.c_int32)]


class DensifyAccum(ctypes.Structure):
    _fields_ = [("accum", ctypes.POINTER(c_void_p)), ("grad_space", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class ExpandOpts(ctypes.Structure):
    _fields_ = [("alpha_threshold", ctypes.c_float), ("depth_threshold", ctypes.c_float),
                ("n_samples", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class ExpandOut(ctypes.Structure):
    _fields_ = [("mask", c_void_p), ("pixel", c_void_p), ("points", c_void_p), ("colors", c_void_p)]


class IcpOpts(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_float), ("sigma", ctypes.c_float), ("max_iterations", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("eps", ctypes.c_double)]


class IcpResult(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32), ("count", ctypes.c_int32),
                ("degenerate", ctypes.c_int32), ("rho", ctypes.c_float), ("reserved", ctypes.c_int32)]


# every entry point of include/vpgs.h, with its ctypes signature
SIGNATURES = {
    "vpgs_create": (ctypes.c_int, [ctypes.POINTER(c_void_p), ctypes.c_int, c_void_p, c_void_p, c_void_p]),
    "vpgs_destroy": (ctypes.c_int, [c_void_p]),
    "vpgs_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "vpgs_last_error": (ctypes.c_char_p, [c_void_p]),
    "vpgs_version": (ctypes.c_int, []),
    "vpgs_render_forward": (ctypes.c_int, [c_void_p, ctypes.c_int, ctypes.POINTER(Gaussians), ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(Camera),
                                           ctypes.POINTER(Images), ctypes.POINTER(RenderOpts),
                                           ctypes.POINTER(c_void_p), c_void_p]),
    "vpgs_render_backward": (ctypes.c_int, [c_void_p, c_void_p, ctypes.POINTER(ImageGrads),
                                            ctypes.POINTER(GaussBuffers), c_void_p, c_void_p]),
    "vpgs_saved_stats": (ctypes.c_int, [c_void_p, c_void_p, ctypes.POINTER(Stats), c_void_p]),
    "vpgs_saved_export": (ctypes.c_int, [c_void_p, c_void_p, ctypes.c_int, c_void_p, ctypes.c_size_t,
                                         ctypes.POINTER(ctypes.c_size_t), c_void_p]),
    "vpgs_saved_release": (ctypes.c_int, [c_void_p, c_void_p]),
    "vpgs_window_create": (ctypes.c_int, [c_void_p, ctypes.c_int, ctypes.POINTER(Gaussians), ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(Camera),
                                          ctypes.POINTER(Images), ctypes.POINTER(ImageGrads),
                                          ctypes.POINTER(GaussBuffers), c_void_p, ctypes.POINTER(WindowOpts),
                                          ctypes.POINTER(c_void_p), c_void_p]),
    "vpgs_window_set_cameras": (ctypes.c_int, [c_void_p, ctypes.POINTER(Camera)]),
    "vpgs_window_run": (ctypes.c_int, [c_void_p, ctypes.c_int, c_void_p]),
    "vpgs_window_stats": (ctypes.c_int, [c_void_p, ctypes.POINTER(Stats), c_void_p]),
    "vpgs_window_config": (ctypes.c_int, [c_void_p, ctypes.POINTER(WindowOpts)]),
    "vpgs_window_destroy": (ctypes.c_int, [c_void_p]),
    "vpgs_profile_enable": (ctypes.c_int, [c_void_p, ctypes.c_int]),
    "vpgs_profile_read": (ctypes.c_int, [c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_char_p),
                                         ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]),
    "vpgs_decode_forward": (ctypes.c_int, [c_void_p, ctypes.POINTER(Anchors), ctypes.POINTER(Mlp),
                                           ctypes.POINTER(ctypes.c_float), ctypes.POINTER(GaussBuffers), c_void_p]),
    "vpgs_decode_backward": (ctypes.c_int, [c_void_p, ctypes.POINTER(Anchors), ctypes.POINTER(Mlp),
                                            ctypes.POINTER(ctypes.c_float), ctypes.POINTER(GaussBuffers), c_void_p,
                                            c_void_p, c_void_p, ctypes.POINTER(MlpGrads), c_void_p]),
    "vpgs_mapping_loss": (ctypes.c_int, [c_void_p, ctypes.c_int, ctypes.POINTER(Camera), ctypes.POINTER(Images),
                                         ctypes.POINTER(Targets), ctypes.POINTER(LossOpts), c_void_p,
                                         ctypes.POINTER(Images), c_void_p]),
    "vpgs_volume_loss": (ctypes.c_int, [c_void_p, ctypes.c_int, ctypes.POINTER(Gaussians), ctypes.c_float,
                                        c_void_p, ctypes.POINTER(GaussBuffers), c_void_p]),
    "vpgs_render_backward_accum": (ctypes.c_int, [c_void_p, c_void_p, ctypes.POINTER(ImageGrads),
                                                  ctypes.POINTER(GaussBuffers), c_void_p,
                                                  ctypes.POINTER(DensifyAccum), c_void_p]),
    "vpgs_window_set_accum": (ctypes.c_int, [c_void_p, ctypes.POINTER(DensifyAccum)]),
    "vpgs_anchor_stats": (ctypes.c_int, [c_void_p, ctypes.c_int64, ctypes.c_int32, c_void_p, ctypes.c_float,
                                         ctypes.c_float, c_void_p, c_void_p, c_void_p, c_void_p]),
    "vpgs_expansion_sample": (ctypes.c_int, [c_void_p, ctypes.c_int, ctypes.POINTER(Camera), ctypes.POINTER(Images),
                                             ctypes.POINTER(Targets), ctypes.POINTER(ExpandOpts), c_void_p, c_void_p,
                                             ctypes.POINTER(ExpandOut), c_void_p]),
    "vpgs_distill_loss": (ctypes.c_int, [c_void_p, ctypes.c_int, ctypes.POINTER(Camera), ctypes.POINTER(Images),
                                         ctypes.POINTER(Images), c_void_p, c_void_p, ctypes.POINTER(Images),
                                         ctypes.POINTER(Images), c_void_p]),
    "vpgs_voxel_map_create": (ctypes.c_int, [c_void_p, c_void_p, ctypes.c_int64, ctypes.c_float, ctypes.c_int32,
                                             ctypes.POINTER(c_void_p), c_void_p]),
    "vpgs_voxel_map_info": (ctypes.c_int, [c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                           c_void_p]),
    "vpgs_voxel_map_destroy": (ctypes.c_int, [c_void_p]),
    "vpgs_voxel_downsample": (ctypes.c_int, [c_void_p, c_void_p, ctypes.c_int64, ctypes.c_float, c_void_p, c_void_p,
                                             c_void_p]),
    "vpgs_icp_correspond": (ctypes.c_int, [c_void_p, c_void_p, c_void_p, ctypes.c_int64,
                                           ctypes.POINTER(ctypes.c_double), ctypes.c_float, c_void_p, c_void_p,
                                           c_void_p]),
    "vpgs_icp_linearize": (ctypes.c_int, [c_void_p, c_void_p, c_void_p, ctypes.c_int64,
                                          ctypes.POINTER(ctypes.c_double), ctypes.c_float, ctypes.c_float, c_void_p,
                                          c_void_p]),
    "vpgs_icp_linearize_noalloc": (ctypes.c_int, [c_void_p, c_void_p, c_void_p, ctypes.c_int64,
                                                  ctypes.POINTER(ctypes.c_double), ctypes.c_float, ctypes.c_float,
                                                  c_void_p, c_void_p]),
    "vpgs_measure_peaks": (ctypes.c_int, [c_void_p, ctypes.POINTER(ctypes.c_double), c_void_p]),
    "vpgs_icp_register": (ctypes.c_int, [c_void_p, c_void_p, c_void_p, ctypes.c_int64,
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(IcpOpts), ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(IcpResult), c_void_p]),
}

_LIB = None


def load():
    """Load the built library (raises if it is missing)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2505_18992_amd.build.build() "
                              "(or __graft_entry__.build()) first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


# vpgs_create's workspace allocator callbacks
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class VpgsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


def check(status: int, ctx=None, what: str = ""):
    if status != VPGS_OK:
        L = load()
        detail = L.vpgs_last_error(ctx).decode() if ctx else ""
        name = L.vpgs_status_string(status).decode()
        raise VpgsError(status, f"{what}: {name} ({status}) {detail}")
