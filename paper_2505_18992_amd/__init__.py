"""MI355X (gfx950) differentiable Gaussian-splatting renderer and anchor
decoder for the VPGS-SLAM hot path.

The computation runs in hand-written HIP kernels behind the C ABI of
``include/vpgs.h`` (``libvpgs.so``); this package marshals PyTorch tensors
into that ABI.  Importing it does not load the library; the first call does,
and fails loudly if the library is not built.
"""
from .render import (Context, DecodeFn, RenderFn, Saved, anchor_stats, camera_struct, decode,  # noqa: F401
                     decode_backward, decode_forward, distill_loss, expansion_sample, get_context, mapping_loss, render,
                     render_backward, render_views, RenderWindow, volume_loss)

from .registration import (VoxelMap, icp_correspond, icp_linearize, icp_linearize_noalloc, icp_register,  # noqa: F401
                           voxel_downsample)

__version__ = "0.1.0"
