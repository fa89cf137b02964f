// runtime.h -- host-side state shared by the C ABI translation units: the
// context, the saved forward state, grow-only device buffers, error
// reporting and stage timing.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <string>
#include <vector>

#include "internal.h"

namespace vpgs {

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

enum Stage { ST_PROJECT, ST_SCAN, ST_EMIT, ST_SORT, ST_RANGES, ST_FWD, ST_BWD, ST_PROJ_BWD, ST_POSE, ST_FILL,
             ST_DEC_FWD, ST_DEC_BWD, ST_DEPTH, ST_LOSS, ST_VOLUME, ST_ANCHOR, ST_EXPAND, ST_DISTILL, ST_VOXEL,
             ST_ICP };
extern const char* const kStageNames[VPGS_NUM_STAGES];

}  // namespace vpgs

struct vpgs_saved {
  vpgs_ctx* ctx = nullptr;  // whose allocator holds the buffers
  // host and device call tables (the host copy is uploaded through the
  // context's ring of pinned staging buffers)
  vpgs::CallTables* h_tab = nullptr;
  vpgs::DevBuf tab, rec, count, zkey, rect, drect, hitmask, scan_ws, keys, vals, keys_alt, vals_alt, sort_ws, ranges,
      tfinal, ncontrib, counters, acc, pose_partial, dk, dk_alt, dv, dv_alt, dcount, dpoff, key64, order;
  int result_in_alt = 0;
  int depth_in_alt = 0;
  int tile_w = 16, tile_h = 16;
  int lds_batch = 256;  // entries staged per compositing batch
  bool count_work = true;  // the forward counts its evaluations and blends
  int key_bits = 16;  // tile-id bits sorted
  uint32_t persistent_blocks = 0;  // 0: one compositing workgroup per tile
  uint32_t capacity = 0;
  uint32_t n_pixels = 0;
  bool in_use = false;
};

struct vpgs_ctx {
  static constexpr int kTabRing = 8;
  int device = 0;
  // pinned staging buffers of the call-table uploads, each reused only once
  // the copy that last read it has completed (an event per slot), so the
  // host runs ahead of the device by up to kTabRing uploads
  vpgs::CallTables* tab_ring = nullptr;
  hipEvent_t tab_ring_ev[kTabRing] = {};
  int tab_ring_next = 0;
  // device workspace allocator: the caller's callbacks, or hipMalloc/hipFree
  // when none were given
  void* (*alloc)(size_t, void*) = nullptr;
  void (*free_)(void*, void*) = nullptr;
  void* alloc_user = nullptr;
  std::string last_error;
  std::vector<vpgs_saved*> pool;
  void* h_pinned = nullptr;  // small pinned buffer for counter readback
  // decode workspace
  vpgs::DevBuf dec_partial;
  // mapping-loss workspace: SSIM partials of one view, block sums
  vpgs::DevBuf loss_ws, loss_sums;
  // expansion sampling: candidate masks not given by the caller, block counts and offsets
  vpgs::DevBuf expand_mask, expand_blocks;
  // distillation loss: FP64 partial sums per keyframe
  vpgs::DevBuf distill_ws;
  // registration: temporaries of voxel-map builds and downsampling; the
  // per-iteration partial sums and state
  vpgs::DevBuf icp_build, icp_ws;
  // device-rate microbenchmarks: source and destination of the copy
  vpgs::DevBuf peak_ws;
  // stage timing
  bool profiling = false;
  std::vector<hipEvent_t> ev_free;
  struct Pending { int stage; hipEvent_t a, b; };
  std::vector<Pending> pending;
  double stage_ms[VPGS_NUM_STAGES] = {};
  int64_t stage_calls[VPGS_NUM_STAGES] = {};
};

namespace vpgs {

constexpr int kMaxDevices = 64;
constexpr int kMaxGridCtas = 65536;  // persistent compositing workgroups at most

// Looks up, once per device and with it current, the device address of the
// allocation-free entry points' scratch array (icp.hip).
int init_scratch(vpgs_ctx* ctx);

// Records the message as the context's last error and returns code.
int fail(vpgs_ctx* ctx, int code, const char* fmt, ...);
// Grows b to at least `bytes` through the context's allocator (the old
// buffer is released first; contents are not kept).
int ensure(vpgs_ctx* ctx, DevBuf& b, size_t bytes);
// Releases b through the context's allocator.
void free_buf(vpgs_ctx* ctx, DevBuf& b);

// Forward/backward pipeline of one call, shared by the eager entry points
// and the captured window.  The host call tables must be built first.
int build_tables(vpgs_ctx* ctx, CallTables& T, int n_sets, const vpgs_gaussians* sets, int n_views,
                 const int32_t* view_set, const vpgs_camera* cams, const vpgs_images* out, int tw, int th);
int validate_forward(vpgs_ctx* ctx, int n_sets, const vpgs_gaussians* sets, int n_views, const int32_t* view_set,
                     const vpgs_camera* cams, const vpgs_images* out, const vpgs_render_opts* opts);
// Binds the gradient outputs (and unbinds any expansion accumulators).
int bind_backward(vpgs_ctx* ctx, CallTables& T, const vpgs_image_grads* grad_out, const vpgs_gauss_grads* grads);
// Binds expansion accumulators (acc may be NULL: none).
int bind_accum(vpgs_ctx* ctx, CallTables& T, const vpgs_densify_accum* acc);
int upload_tables(vpgs_ctx* ctx, vpgs_saved* sv, hipStream_t st);
int prepare_front(vpgs_ctx* ctx, vpgs_saved* sv);
int ensure_pairs(vpgs_ctx* ctx, vpgs_saved* sv, uint32_t cap);
int ensure_backward(vpgs_ctx* ctx, vpgs_saved* sv, hipStream_t st);
int read_pair_count(vpgs_ctx* ctx, vpgs_saved* sv, hipStream_t st, uint32_t* out);
int enqueue_front(vpgs_ctx* ctx, vpgs_saved* sv, hipStream_t st);
int enqueue_back(vpgs_ctx* ctx, vpgs_saved* sv, hipStream_t st);
int enqueue_backward(vpgs_ctx* ctx, vpgs_saved* sv, float* d_pose, hipStream_t st);
int new_saved(vpgs_ctx* ctx, vpgs_saved** out);
void destroy_saved(vpgs_saved* s);

// Records a HIP event pair around one stage when profiling is on.
struct StageTimer {
  vpgs_ctx* ctx;
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr;
  StageTimer(vpgs_ctx* c, int s, hipStream_t stream);
  ~StageTimer();
};

}  // namespace vpgs

#define HIP_TRY(expr)                                                                              \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) return vpgs::fail(ctx, VPGS_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)
