"""The C ABI library: it loads, exports every entry point its header
declares, and its host-side status/validation paths work without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vpgs.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vpgs_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2505_18992_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libvpgs.so not built")
    return _lib.load()


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("vpgs_create", "vpgs_destroy", "vpgs_render_forward", "vpgs_render_backward",
                     "vpgs_decode_forward", "vpgs_decode_backward", "vpgs_saved_release", "vpgs_status_string"):
        assert required in names
    assert len(names) >= 14


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_binding_covers_every_declared_symbol():
    from paper_2505_18992_amd import _lib
    assert set(_declared()) <= set(_lib.SIGNATURES), set(_declared()) - set(_lib.SIGNATURES)


def test_status_strings_and_version(lib):
    assert lib.vpgs_version() >= 1
    assert lib.vpgs_status_string(0) == b"ok"
    assert lib.vpgs_status_string(-1) == b"invalid argument"
    assert lib.vpgs_status_string(-4) == b"pair list capacity exceeded"
    assert lib.vpgs_status_string(12345) == b"unknown status"


def test_null_context_is_rejected_without_touching_the_device(lib):
    from paper_2505_18992_amd import _lib
    assert lib.vpgs_render_forward(None, 1, None, 1, None, None, None, None, None, None) == _lib.VPGS_EINVAL
    assert lib.vpgs_render_backward(None, None, None, None, None, None) == _lib.VPGS_EINVAL
    assert lib.vpgs_decode_forward(None, None, None, None, None, None) == _lib.VPGS_EINVAL
    assert lib.vpgs_decode_backward(None, None, None, None, None, None, None, None, None, None) == _lib.VPGS_EINVAL
    assert lib.vpgs_saved_release(None, None) == _lib.VPGS_EINVAL
    assert lib.vpgs_destroy(None) == _lib.VPGS_EINVAL
    assert lib.vpgs_render_backward_accum(None, None, None, None, None, None, None) == _lib.VPGS_EINVAL
    assert lib.vpgs_window_set_accum(None, None) == _lib.VPGS_EINVAL
    assert lib.vpgs_anchor_stats(None, 1, 1, None, 0.0, 0.0, None, None, None, None) == _lib.VPGS_EINVAL
    assert lib.vpgs_expansion_sample(None, 1, None, None, None, None, None, None, None, None) == _lib.VPGS_EINVAL
    assert lib.vpgs_distill_loss(None, 1, None, None, None, None, None, None, None, None) == _lib.VPGS_EINVAL
    assert lib.vpgs_voxel_map_create(None, None, 0, 1.0, 1, None, None) == _lib.VPGS_EINVAL
    assert lib.vpgs_voxel_map_info(None, None, None, None) == _lib.VPGS_EINVAL
    assert lib.vpgs_voxel_map_destroy(None) == _lib.VPGS_EINVAL
    assert lib.vpgs_voxel_downsample(None, None, 0, 1.0, None, None, None) == _lib.VPGS_EINVAL
    assert lib.vpgs_icp_correspond(None, None, None, 0, None, 1.0, None, None, None) == _lib.VPGS_EINVAL
    assert lib.vpgs_icp_linearize(None, None, None, 0, None, 1.0, 1.0, None, None) == _lib.VPGS_EINVAL
    assert lib.vpgs_icp_linearize_noalloc(None, None, None, 0, None, 1.0, 1.0, None, None) == _lib.VPGS_EINVAL
    assert lib.vpgs_icp_register(None, None, None, 0, None, None, None, None, None, None) == _lib.VPGS_EINVAL
    assert lib.vpgs_create(None, 0, None, None, None) == _lib.VPGS_EINVAL
    assert lib.vpgs_last_error(None) == b"NULL context"


def test_structure_layouts_match_the_header():
    """Field offsets of the ctypes mirrors follow the C layout rules for the
    header's structs (checked against hand-computed offsets)."""
    from paper_2505_18992_amd import _lib
    assert ctypes.sizeof(_lib.Camera) == 4 * 7 + 4 * 12
    assert _lib.Gaussians.means.offset == 8 and ctypes.sizeof(_lib.Gaussians) == 48
    assert ctypes.sizeof(_lib.RenderOpts) == 32 and _lib.RenderOpts.pair_capacity.offset == 16
    assert _lib.RenderOpts.skip_counts.offset == 24
    assert _lib.RenderOpts.lds_batch.offset == 8 and _lib.RenderOpts.grid_ctas.offset == 12
    assert ctypes.sizeof(_lib.WindowOpts) == 48 and _lib.WindowOpts.lds_batch.offset == 28
    assert _lib.WindowOpts.tune_cache.offset == 32 and _lib.WindowOpts.skip_counts.offset == 40
    assert _lib.Anchors.xyz.offset == 16
    assert _lib.Mlp.W1.offset == 8 and ctypes.sizeof(_lib.Mlp) == 8 + 12 * 8
    assert ctypes.sizeof(_lib.Stats) == 8 * 8 + 4 * 4 + 3 * 8
