/*
 * vpgs.h -- C ABI of the MI355X (gfx950) differentiable Gaussian-splatting
 * renderer and anchor decoder.
 *
 * The operations are those of the paper's scene representation and its
 * rasterisation (VPGS-SLAM, Section III-A; eq. 1-6): neural Gaussians are
 * decoded from voxel anchors (eq. 1-5) and the Gaussians of a submap are
 * splatted into colour, depth and opacity images (eq. 6), whose L1 / SSIM /
 * depth losses drive mapping (eq. 7) and photometric pose tracking
 * (Section III-B, coarse stage).  The renderer computes:
 *
 *   projection   p = R mu + t; visible iff FP32 depth z > near; unit quaternion
 *                q/|q|; Sigma = R_q diag(exp(2 l)) R_q^T; J the pinhole
 *                Jacobian with a 1.3x field-of-view guard clamp;
 *                Sigma2D = J R Sigma R^T J^T + 0.3 I; conic = Sigma2D^-1;
 *                (u, v) = (fx x/z + cx, fy y/z + cy); opacity-aware box
 *                { d^T conic d <= 2 ln(255 o) } padded by one pixel.
 *   binning      one (tile id << 32 | FP32 depth bits, index) key per overlapped
 *                tile, sorted, so the per-pixel order is (depth, index).
 *   compositing  per pixel (centre at +0.5) front to back:
 *                alpha = min(0.99, o exp(-d^T conic d / 2)); skip alpha < 1/255;
 *                stop before blending once T (1 - alpha) < 1e-4;
 *                RGB = sum alpha T c, depth = sum alpha T z, alpha = 1 - T.
 *   backward     gradients of sum(gRGB . RGB + gD D + gA A) to means, log-scales,
 *                quaternions, opacities, colours, and to a left se(3) pose
 *                increment xi = (rho, phi) at 0: [R|t] <- Exp(xi) [R|t].
 *
 * Conventions
 *   - Every pointer is a DEVICE pointer unless marked "host".  All floating
 *     point data are FP32, C-contiguous, row-major.  Image planes are [H, W]
 *     (RGB is [3, H, W], channel-major).
 *   - Quaternions are (w, x, y, z) with any non-zero norm.  Opacities and
 *     colours are post-activation values.
 *   - Camera poses are world-to-camera [R | t], row-major 3x4, in host memory.
 *   - Calls are asynchronous on the given HIP stream (hipStream_t passed as
 *     void*; NULL = the default stream) unless stated otherwise.
 *   - Ownership: the caller owns every input and output buffer.  The library
 *     owns its workspace (allocated through the caller's callbacks when
 *     vpgs_create was given them) and the saved-state handles (until
 *     released).
 *   - Errors: every entry point returns a status code; no exception crosses
 *     the ABI.  Arguments are validated on the host before any launch: an
 *     invalid argument returns VPGS_EINVAL and enqueues nothing.
 *   - Thread safety: a context is used by one host thread at a time; use one
 *     context per concurrent stream user.
 */
#ifndef VPGS_H_
#define VPGS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VPGS_OK 0
#define VPGS_EINVAL (-1)        /* invalid argument; nothing was enqueued */
#define VPGS_ENOMEM (-2)        /* device or host allocation failed */
#define VPGS_EHIP (-3)          /* a HIP runtime call failed */
#define VPGS_ECAPACITY (-4)     /* the (tile, Gaussian) pair list overflowed */
#define VPGS_EUNSUPPORTED (-5)  /* option combination not built */

#define VPGS_MAX_VIEWS 64       /* views per call */
#define VPGS_MAX_SETS 64        /* distinct Gaussian sets per call */
#define VPGS_MAX_DIM 8192       /* image width and height limit */
#define VPGS_MAX_RECORDS 107374182  /* (view, Gaussian) records per call: sum over views of their set's size */

typedef struct vpgs_ctx vpgs_ctx;
typedef struct vpgs_saved vpgs_saved;
typedef struct vpgs_window vpgs_window;

/* Pinhole camera.  near_plane <= 0 selects the default 0.2. */
typedef struct {
  int32_t width, height;
  float fx, fy, cx, cy;
  float near_plane;
  float world_to_cam[12]; /* host: row-major 3x4 [R | t] */
} vpgs_camera;

/* A Gaussian set of n Gaussians (SoA arrays of length n). */
typedef struct {
  int64_t n;
  const float* means;      /* [n,3] */
  const float* log_scales; /* [n,3] */
  const float* quats;      /* [n,4] (w,x,y,z) */
  const float* opacities;  /* [n] */
  const float* colors;     /* [n,3] */
} vpgs_gaussians;

/* Rendered planes of one view (outputs, written in full). */
typedef struct {
  float* rgb;   /* [3,H,W] */
  float* depth; /* [H,W] */
  float* alpha; /* [H,W] */
} vpgs_images;

/* Upstream gradients of one view; a NULL plane counts as zero. */
typedef struct {
  const float* rgb;   /* [3,H,W] */
  const float* depth; /* [H,W] */
  const float* alpha; /* [H,W] */
} vpgs_image_grads;

/* Writable per-Gaussian arrays (shapes as in vpgs_gaussians): the gradients
 * of a set, or the Gaussians a decode writes.  Written in full. */
typedef struct {
  float* means;
  float* log_scales;
  float* quats;
  float* opacities;
  float* colors;
} vpgs_gauss_buffers;
typedef vpgs_gauss_buffers vpgs_gauss_grads;

/* Render options.  Zero fields take defaults (16x16 tiles, one LDS batch per
 * tile's pixel count, one compositing workgroup per tile, automatic pair
 * capacity).
 *   tile_w x tile_h  one of the compiled shapes 16x16, 16x8, 8x8, 32x8.
 *   lds_batch        Gaussian entries staged in LDS per compositing batch:
 *                    half, once or twice the tile's pixel count, a multiple
 *                    of 64 (16x16 and 32x8: 128, 256, 512; 16x8: 64, 128,
 *                    256; 8x8: 64, 128).  Any other value: VPGS_EUNSUPPORTED.
 *   grid_ctas        0: one compositing workgroup per tile; > 0 (at most
 *                    65536): that many persistent workgroups taking tiles
 *                    from a queue, longest list first.
 *   pair_capacity    0 sizes the pair list exactly (one host synchronisation
 *                    per forward); > 0 fixes it (no synchronisation; an
 *                    overflow is reported as VPGS_ECAPACITY by
 *                    vpgs_saved_stats and the outputs of that call are
 *                    invalid).
 *   skip_counts      1: the forward compositor does not count its (pixel,
 *                    Gaussian) evaluations and blends (vpgs_stats then
 *                    reports them as 0); 0 counts them (instrumentation
 *                    that costs about a seventh of the compositor's
 *                    per-step instructions).
 * The images do not depend on any of these (the forward is bit-identical
 * across them); the backward's gradients differ only in the order of their
 * floating-point atomic sums. */
typedef struct {
  int32_t tile_w, tile_h;
  int32_t lds_batch;
  int32_t grid_ctas;
  int64_t pair_capacity;
  int32_t skip_counts;
  int32_t reserved;
} vpgs_render_opts;

/* Counters of one forward, filled by vpgs_saved_stats. */
typedef struct {
  int64_t n_records;   /* (view, Gaussian) records projected */
  int64_t n_visible;   /* records with a non-empty tile rectangle */
  int64_t n_pairs;     /* (tile, Gaussian) pairs emitted */
  int64_t n_evaluated; /* (pixel, Gaussian) alpha evaluations */
  int64_t n_blended;   /* (pixel, Gaussian) blends */
  int64_t pair_capacity;
  int64_t n_tiles;
  int64_t n_pixels;
  int32_t overflow;    /* 1 if the pair list overflowed */
  int32_t tile_w, tile_h;
  int32_t lds_batch;   /* entries staged per compositing batch */
  /* compositing work in wavefront steps: one step is one wavefront (64
   * pixels) taking one Gaussian of its hit list.  The backward counts add up
   * over the backward calls of a forward. */
  int64_t n_fwd_steps;   /* forward steps */
  int64_t n_bwd_steps;   /* backward steps */
  int64_t n_bwd_active;  /* backward steps in which some pixel takes a gradient */
} vpgs_stats;

/* ---- context ------------------------------------------------------------- */

/* Create a context on HIP device `device`.  The context keeps a grow-only
 * device workspace (the forward's records, pair lists, sort buffers, hit
 * masks and gradient accumulators, and the scratch of the other calls),
 * released by vpgs_destroy.  With alloc and free_ given (both or neither,
 * else VPGS_EINVAL), every workspace block comes from alloc(bytes, user) --
 * device memory, 256-byte aligned, NULL if it cannot -- and goes back
 * through free_(ptr, user), e.g. a framework's caching allocator; the library
 * synchronises the device before handing a block back, so a caller may
 * recycle it at once.  With neither, it uses hipMalloc / hipFree. */
int vpgs_create(vpgs_ctx** out, int device, void* (*alloc)(size_t bytes, void* user),
                void (*free_)(void* ptr, void* user), void* user);
int vpgs_destroy(vpgs_ctx* ctx);
const char* vpgs_status_string(int status);
/* Text of the last error on this context (valid until the next call). */
const char* vpgs_last_error(const vpgs_ctx* ctx);
int vpgs_version(void);

/* ---- renderer -------------------------------------------------------------- */

/* Forward render of n_views views.  View v renders Gaussian set view_set[v]
 * (host array; several views may share a set) with camera cams[v] (host)
 * into out[v] (host array of device planes).  If `saved` is non-NULL a
 * saved-state handle for vpgs_render_backward is returned; it must be
 * released with vpgs_saved_release.  The Gaussian and camera buffers must not
 * change between the forward and its backward.  VPGS_EINVAL if the views hold
 * more than VPGS_MAX_RECORDS records in all (the backward addresses each
 * record's 40-byte gradient row with a 32-bit byte offset). */
int vpgs_render_forward(vpgs_ctx* ctx, int n_sets, const vpgs_gaussians* sets, int n_views,
                        const int32_t* view_set, const vpgs_camera* cams, const vpgs_images* out,
                        const vpgs_render_opts* opts, vpgs_saved** saved, void* stream);

/* Backward of a forward.  grad_out[v] (host array) holds the upstream planes
 * of view v; grads[s] (host array) receives the gradient of set s summed over
 * the views that render it; d_pose (device, [n_views,6] as (rho, phi), may be
 * NULL) receives the pose-increment gradient of every view.  Per-pixel alpha
 * is recomputed, not stored. */
int vpgs_render_backward(vpgs_ctx* ctx, const vpgs_saved* saved, const vpgs_image_grads* grad_out,
                         const vpgs_gauss_grads* grads, float* d_pose, void* stream);

/* Synchronise the stream and read the counters of a forward.  Returns
 * VPGS_ECAPACITY if its pair list overflowed. */
int vpgs_saved_stats(vpgs_ctx* ctx, const vpgs_saved* saved, vpgs_stats* out, void* stream);

/* Internal buffers of a forward, for inspection and tests.  Copies (device to
 * device, on `stream`) `what` into dst, which must hold `bytes`; returns
 * VPGS_EINVAL if bytes is smaller than the buffer (whose size in bytes is
 * returned through *size when size is non-NULL, and dst may then be NULL):
 *   VPGS_BUF_PROJ    float [R,12]: u, v, z, opacity, Qa, Qb, Qc, 0, r, g, b, 0
 *                    (rows of culled records, count 0, are unspecified)
 *   VPGS_BUF_EXTENT  float [R,2]: half extents hx, hy of the box (0 if culled)
 *   VPGS_BUF_COUNT   uint32 [R]: tiles overlapped (0 = culled)
 *   VPGS_BUF_KEYS    uint64 [P]: sorted keys
 *   VPGS_BUF_VALUES  uint32 [P]: sorted record indices
 *   VPGS_BUF_RANGES  uint32 [T,2]: [start, end) of every tile
 *   VPGS_BUF_TFINAL  float [sum H*W]: final transmittance, views concatenated
 *   VPGS_BUF_NCONTRIB uint32 [sum H*W]: list length up to the last blend
 * R = records (views in order, each the size of its set); T = tiles (views in
 * order, row-major per view). */
#define VPGS_BUF_PROJ 1
#define VPGS_BUF_EXTENT 2
#define VPGS_BUF_COUNT 3
#define VPGS_BUF_KEYS 4
#define VPGS_BUF_VALUES 5
#define VPGS_BUF_RANGES 6
#define VPGS_BUF_TFINAL 7
#define VPGS_BUF_NCONTRIB 8
int vpgs_saved_export(vpgs_ctx* ctx, const vpgs_saved* saved, int what, void* dst, size_t bytes,
                      size_t* size, void* stream);

int vpgs_saved_release(vpgs_ctx* ctx, vpgs_saved* saved);

/* ---- mapping window: batched, graph-captured forward + backward ---------- */

/* A window binds every buffer of a repeated multi-view forward+backward (the
 * keyframes of a mapping window, or the views of several submaps) once, picks
 * the tile shape, LDS batch and compositing grid with a timed search on the
 * actual inputs, and captures the launch sequence of all views in two HIP
 * graphs:
 * the forward (projection, binning, sort, ranges, forward compositing) and
 * the backward (backward compositing, projection backward, pose reduction).
 * A run is one graph launch per part; the pair list has a fixed capacity (no
 * host synchronisation), and an overflow is reported by vpgs_window_stats.
 *
 * The search times every candidate over tune_reps runs of the whole forward
 * and backward on the bound inputs: first each tile shape with each
 * compositing grid (one workgroup per tile, or 2, 4 or 8 persistent
 * workgroups per compute unit) at one batch per tile's pixel count, then the
 * other LDS batch sizes of the best shape and grid.  Fields given in opts
 * are not searched.  With tune_cache set, a result stored under the same
 * key -- the device (architecture name and compute units), the number of
 * views and their sizes, and ceil(log2) of the (view, Gaussian) record count
 * -- is taken without searching, and a new search result is written to the
 * file (a JSON object of entries; other keys are kept).  A cache that cannot
 * be read or parsed is ignored; one that cannot be written is reported. */
typedef struct {
  int32_t tile_w, tile_h;   /* 0 = chosen by the search */
  int32_t persistent;       /* -1 = chosen by the search; 0 = one workgroup per tile;
                               > 0 = that many persistent workgroups on a tile queue */
  int32_t use_graph;        /* 1 = capture in a HIP graph (default); 0 = launch eagerly */
  int64_t pair_capacity;    /* 0 = pairs measured at creation plus 25% headroom */
  int32_t tune_reps;        /* timed runs per candidate in the search (0 = 3) */
  int32_t lds_batch;        /* 0 = chosen by the search; else as in vpgs_render_opts */
  const char* tune_cache;   /* host path of a JSON tuning cache, or NULL for none */
  int32_t skip_counts;      /* as in vpgs_render_opts (the search times the window's own setting) */
  int32_t reserved;
} vpgs_window_opts;

/* Inputs and outputs as in vpgs_render_forward / vpgs_render_backward, all
 * bound for the life of the window (host arrays are copied; the device
 * buffers they point to must stay allocated).  opts may be NULL (full search,
 * graph on).  Runs the search on `stream` (it overwrites the bound outputs). */
int vpgs_window_create(vpgs_ctx* ctx, int n_sets, const vpgs_gaussians* sets, int n_views,
                       const int32_t* view_set, const vpgs_camera* cams, const vpgs_images* out,
                       const vpgs_image_grads* grad_out, const vpgs_gauss_grads* grads, float* d_pose,
                       const vpgs_window_opts* opts, vpgs_window** win, void* stream);
/* New poses and intrinsics for the bound views (image sizes must not change);
 * takes effect at the next run. */
int vpgs_window_set_cameras(vpgs_window* win, const vpgs_camera* cams);
/* parts = 1: forward of every view; 2: backward (uses the upstream planes
 * as they are when it runs, so a loss gradient can be computed between the
 * two); 3: both.  Each part is one graph launch on `stream`.  The forward
 * ends by raising a sticky flag in mapped host memory if its pair list
 * overflowed; every later run (and part) then returns VPGS_ECAPACITY without
 * launching anything, so an overflow is never silent even when nothing
 * synchronises: the outputs of the run that overflowed are invalid, and the
 * window must be recreated with a larger pair_capacity. */
#define VPGS_WINDOW_FORWARD 1
#define VPGS_WINDOW_BACKWARD 2
int vpgs_window_run(vpgs_window* win, int parts, void* stream);
/* Synchronise and read the counters of the last run (VPGS_ECAPACITY on
 * overflow: grow pair_capacity and recreate the window). */
int vpgs_window_stats(vpgs_window* win, vpgs_stats* out, void* stream);
/* The configuration the window runs with. */
int vpgs_window_config(const vpgs_window* win, vpgs_window_opts* out);
int vpgs_window_destroy(vpgs_window* win);

/* ---- stage timing (diagnostics) ------------------------------------------ */

/* When enabled, every launch sequence of the context records a pair of HIP
 * events on its stream around each stage (projection, scan, emission, sort,
 * ranges, forward compositing, backward compositing, projection backward,
 * pose reduction, fills, decode forward, decode backward, depth ordering of
 * the visible records, mapping loss, volume loss, anchor statistics,
 * expansion sampling, distillation loss, voxel map and downsampling,
 * registration).  vpgs_profile_read
 * synchronises on the recorded events and returns, for stage index `stage`
 * (0 <= stage < VPGS_NUM_STAGES), its name, the number of recorded launches
 * and their summed duration in milliseconds since the last enable.  Disabled
 * by default; enabling resets the totals. */
#define VPGS_NUM_STAGES 20
int vpgs_profile_enable(vpgs_ctx* ctx, int on);
int vpgs_profile_read(vpgs_ctx* ctx, int stage, const char** name, int64_t* calls, double* total_ms);

/* Microbenchmarks of the device rates the kernels of this library are held
 * against (diagnostics; synchronous on `stream`).  Writes out (host, 5
 * doubles):
 *   [0] LDS read bandwidth, a distinct 16-byte address per lane (GB/s of
 *       data delivered to lanes)
 *   [1] LDS read bandwidth, one 16-byte address per wavefront (a broadcast,
 *       the compositors' pattern; GB/s delivered to lanes)
 *   [2] FP32 fused-multiply-add rate, 2 FLOP each (TFLOP/s; the library is
 *       built without packed FP32 instructions)
 *   [3] exp2 rate (T/s)
 *   [4] HBM copy bandwidth (GB/s of bytes read plus written)
 * Eight workgroups of 256 lanes per compute unit; the copy uses a 512 MiB
 * workspace buffer of the context. */
int vpgs_measure_peaks(vpgs_ctx* ctx, double* out, void* stream);

/* ---- anchor decoder (Section III-A, eq. 1-5) ------------------------------- */

/* m anchors with k Gaussians each (1 <= k <= 16). */
typedef struct {
  int64_t m;
  int32_t k;
  int32_t reserved;
  const float* xyz;     /* [m,3] anchor positions (voxel centres) */
  const float* feat;    /* [m,32] anchor features */
  const float* scale;   /* [m,3] anchor scaling l, > 0 */
  const float* offsets; /* [m,k,3] learnable offsets */
} vpgs_anchors;

/* Three independent LINEAR-ReLU-LINEAR heads (h = 0 opacity, 1 colour,
 * 2 covariance) on the 36-vector [feat(32), view direction(3), distance(1)];
 * weights are (out, in) row-major: W1[h] [width,36], b1[h] [width],
 * W2[h] [out_h,width], b2[h] [out_h] with out = (k, 3k, 7k).  The covariance
 * head emits [scale(3) | quaternion(4)] per Gaussian.  width <= 128. */
typedef struct {
  int32_t in_dim; /* must be 36 */
  int32_t width;
  const float* W1[3];
  const float* b1[3];
  const float* W2[3];
  const float* b2[3];
} vpgs_mlp;

typedef struct {
  float* W1[3];
  float* b1[3];
  float* W2[3];
  float* b2[3];
} vpgs_mlp_grads;

/* Decode m*k neural Gaussians (anchor-major: Gaussian a*k + j):
 *   mean = xyz + offsets * scale (eq. 1); opacity = tanh (<= 0 is culled by the
 *   renderer); colour = sigmoid (eq. 4); log-scale = log_sigmoid + log scale
 *   (eq. 5); quaternion = normalised (norm floored at 1e-12).
 * cam_center (host, 3 floats) is the camera position of eq. 3. */
int vpgs_decode_forward(vpgs_ctx* ctx, const vpgs_anchors* anchors, const vpgs_mlp* mlp,
                        const float* cam_center, const vpgs_gauss_buffers* out, void* stream);

/* Gradients of sum(upstream . decoded) with respect to feat, scale, offsets
 * and every weight and bias (all written in full; the camera is constant).
 * `upstream` uses the vpgs_gauss_grads layout as input.  The weight gradients
 * are sums over anchors taken in a fixed order, so repeated calls agree bit
 * for bit; their partial sums live in a context-owned device buffer of up to
 * 2112 rows of sum_h out_h (width + 1) + 3 width 37 floats (one row per 64
 * anchors, 57 KB at width 64 and k = 10), grown on demand (VPGS_ENOMEM if it
 * cannot be). */
int vpgs_decode_backward(vpgs_ctx* ctx, const vpgs_anchors* anchors, const vpgs_mlp* mlp,
                         const float* cam_center, const vpgs_gauss_grads* upstream, float* d_feat,
                         float* d_scale, float* d_offsets, const vpgs_mlp_grads* d_mlp, void* stream);

/* ---- mapping loss (Section III-A, eq. 7-9) -------------------------------- */

/* Target frame of one view: colour [3,H,W] and depth [H,W] (device); pixels
 * whose target depth is <= 0 carry no depth. */
typedef struct {
  const float* rgb;
  const float* depth;
} vpgs_targets;

typedef struct {
  float lambda_ssim;  /* weight of the SSIM term inside L_SSIM (eq. 8); the paper uses 0.2 */
  float lambda_depth; /* weight of the depth term in eq. 7 (not given in the paper; 1 is the default) */
  int32_t reserved0, reserved1;
} vpgs_loss_opts;

/* Mapping loss of eq. 7-8 for n_views rendered views against their targets:
 *   L_c    = mean |X - Y| over channels and pixels (X rendered, Y target colour)
 *   L_SSIM = (1 - lambda_ssim) mean |X - Y| + lambda_ssim (1 - mean SSIM(X, Y))
 *   L_d    = mean |D - T| over pixels with target depth T > 0 (0 if none)
 *   L      = L_c + L_SSIM + lambda_depth L_d
 * SSIM: 11x11 Gaussian window of sigma 1.5, zero-padded same-size filtering
 * per channel, C1 = 0.01^2, C2 = 0.03^2, averaged over channels and pixels.
 * Only cams[v].width/height are read.  rendered[v].rgb/.depth are read.
 * Writes terms[4 v + k] (device floats: L_c, L_SSIM, L_d, L) and the gradient
 * of sum_v L_v with respect to the rendered planes into grad[v].rgb and
 * grad[v].depth (written in full; d|x|/dx is 0 at 0); grad[v].alpha, if
 * non-NULL, is zeroed.  These planes are the upstream gradients the render
 * backward takes.  opts NULL = (0.2, 1).  A workspace of 36 bytes per pixel of
 * all views is kept in the context.  Asynchronous on `stream`. */
int vpgs_mapping_loss(vpgs_ctx* ctx, int n_views, const vpgs_camera* cams, const vpgs_images* rendered,
                      const vpgs_targets* targets, const vpgs_loss_opts* opts, float* terms,
                      const vpgs_images* grad, void* stream);

/* Volume regulariser of eq. 9 for n_sets Gaussian sets:
 * loss[s] (device float) = lambda_vol * sum_i prod(exp(log_scales_i)), and its
 * gradient lambda_vol * prod(exp(log_scales_i)) is ADDED to each of the three
 * entries of grads[s].log_scales (run it after the render backward, which
 * writes those gradients).  The paper uses lambda_vol = 0.001. */
int vpgs_volume_loss(vpgs_ctx* ctx, int n_sets, const vpgs_gaussians* sets, float lambda_vol, float* loss,
                     const vpgs_gauss_grads* grads, void* stream);

/* ---- submap expansion statistics (Section III-A) ------------------------- */

/* Anchors grow where the averaged gradient of the neural Gaussians of a voxel
 * is large, and are pruned when the accumulated opacity of their neural
 * Gaussians is small; new anchors are sampled where the map does not yet
 * explain the frame (low accumulated alpha or a large depth discrepancy).
 *
 * Per-Gaussian accumulators of one set: [n,4] floats, 16-byte aligned, ADDED
 * to by every backward that is given them (zero them to start an interval):
 *   [0] sum of |dL/d(u, v)|, the norm of the gradient of the loss with
 *       respect to the Gaussian's projected centre, over the views that render
 *       it (those where it overlaps a tile: the forward's visibility);
 *   [1] the number of those views;
 *   [2] sum of max(opacity, 0) over the views whose frustum holds its centre:
 *       FP32 camera depth z > near, 0 <= u < W and 0 <= v < H, the centre as
 *       the projection computes it, whether or not the Gaussian is rendered;
 *   [3] the number of those views.
 * Counts are exact (integers held in floats, below 2^24).  grad_space 0
 * measures the gradient in pixels; 1 in normalised device coordinates
 * (x_ndc = 2 u / W - 1): the norm of (W/2 dL/du, H/2 dL/dv). */
typedef struct {
  float* const* accum; /* host array [n_sets]: device [n,4] buffer of set s, or NULL for none */
  int32_t grad_space;  /* 0 = pixels, 1 = normalised device coordinates */
  int32_t reserved;
} vpgs_densify_accum;

/* vpgs_render_backward, plus the accumulation above in the same pass (the
 * projection backward reads each Gaussian's accumulators once and writes them
 * once).  acc may be NULL (then it is vpgs_render_backward). */
int vpgs_render_backward_accum(vpgs_ctx* ctx, const vpgs_saved* saved, const vpgs_image_grads* grad_out,
                               const vpgs_gauss_grads* grads, float* d_pose, const vpgs_densify_accum* acc,
                               void* stream);

/* Binds accumulators to a window (host array copied; the buffers must stay
 * allocated); every later backward run of the window adds to them.  NULL
 * unbinds.  Takes effect at the next run (no re-capture). */
int vpgs_window_set_accum(vpgs_window* win, const vpgs_densify_accum* acc);

/* Anchor statistics from the accumulators of m*k decoded Gaussians
 * (anchor-major, Gaussian a*k + j, as vpgs_decode_forward writes them).  With
 * S_c the FP32 sum over j = 0..k-1, in that order, of accum[4 (a k + j) + c]:
 *   stats[4a + 0] = S_0 / S_1, or 0 when S_1 = 0: the averaged gradient
 *   stats[4a + 1] = S_1, stats[4a + 2] = S_2 (accumulated opacity), stats[4a + 3] = S_3
 *   grow[a]  = 1 if stats[4a + 0] > tau_g, else 0
 *   prune[a] = 1 if S_3 > 0 and S_2 < tau_o * S_3 (FP32 product), else 0
 * accum and stats are device [m*k,4] / [m,4] floats, 16-byte aligned; grow and
 * prune (device bytes [m]) may be NULL.  1 <= k <= 64. */
int vpgs_anchor_stats(vpgs_ctx* ctx, int64_t m, int32_t k, const float* accum, float tau_g, float tau_o,
                      float* stats, uint8_t* grow, uint8_t* prune, void* stream);

typedef struct {
  float alpha_threshold; /* candidate where the rendered alpha is below this ... */
  float depth_threshold; /* ... or where |D - T| is above this */
  int32_t n_samples;     /* samples drawn per view (>= 0) */
  int32_t reserved;
} vpgs_expand_opts;

/* Outputs of one view (device).  mask may be NULL; the sample arrays are
 * needed when n_samples > 0. */
typedef struct {
  uint8_t* mask;  /* [H,W]: 1 at candidate pixels, else 0 */
  int32_t* pixel; /* [n_samples]: sampled pixel y*W + x, or -1 if the view has no candidate */
  float* points;  /* [n_samples,3]: world points (0 if none) */
  float* colors;  /* [n_samples,3]: target colour at the pixel (0 if none) */
} vpgs_expand_out;

/* Expansion sampling of n_views frames.  A pixel of view v is a candidate iff
 * its target depth T > 0 and (rendered alpha A < alpha_threshold or
 * |D - T| > depth_threshold), in FP32 (rendered[v].alpha and .depth, and
 * targets[v].depth and .rgb are read).  counts[v] (device int32) receives the
 * number c of candidates.  Sample i of view v takes the candidate of rank
 * r = min((int)(u c), c - 1) in raster order, u = uniforms[v n_samples + i]
 * in [0, 1) (device floats, FP32 product), and back-projects its pixel centre
 * with the target depth: X = R^T (T ((x + 1/2 - cx)/fx, (y + 1/2 - cy)/fy, 1)
 * - t), with [R | t] = cams[v].world_to_cam.  The workspace holds one byte
 * per pixel when a mask is NULL, and 8 bytes per 1024 pixels. */
int vpgs_expansion_sample(vpgs_ctx* ctx, int n_views, const vpgs_camera* cams, const vpgs_images* rendered,
                          const vpgs_targets* targets, const vpgs_expand_opts* opts, const float* uniforms,
                          int32_t* counts, const vpgs_expand_out* out, void* stream);

/* ---- submap fusion (Section III-C, eq. 14) -------------------------------- */

/* Distillation loss between two submaps alpha and beta rendered at the poses
 * of the m keyframes of their overlap (rend_a[k] from alpha, rend_b[k] from
 * beta, both of cams[k]'s size; .rgb and .depth are read):
 *   l_k = mean over channels and pixels of (C_a - C_b)^2
 *       + mean over pixels of (D_a - D_b)^2,      L = (1/m) sum_k l_k.
 * terms (device [m,2] floats: the colour and depth means of each keyframe)
 * and loss (device float) may be NULL.  grad_a / grad_b (host arrays of
 * device planes, or NULL for no gradient on that side) receive
 * dL/dC_a = 2 (C_a - C_b) / (3 m H W) = -dL/dC_b and
 * dL/dD_a = 2 (D_a - D_b) / (m H W) = -dL/dD_b (a NULL plane is skipped;
 * .alpha planes, when given, are zeroed): the upstream planes of the render
 * backward of both submaps.  1 <= m <= VPGS_MAX_VIEWS. */
int vpgs_distill_loss(vpgs_ctx* ctx, int m, const vpgs_camera* cams, const vpgs_images* rend_a,
                      const vpgs_images* rend_b, float* terms, float* loss, const vpgs_images* grad_a,
                      const vpgs_images* grad_b, void* stream);

/* ---- voxel map and frame-to-map registration (Section III-B, eq. 10-12) --- */

/* Voxels: point p lies in voxel floor(p / voxel), per axis, the division in
 * FP32; coordinates must satisfy |p / voxel| < 2^20.  A voxel map holds, for
 * every occupied voxel, its first max_per_voxel points by index (a copy, so
 * the input may be freed once the stream has passed the build).  Lookups go
 * through a hash table over the occupied voxels. */
typedef struct vpgs_voxel_map vpgs_voxel_map;

/* Builds the map of n points (device [n,3] floats, n < 2^31) asynchronously
 * on `stream`.  Release with vpgs_voxel_map_destroy. */
int vpgs_voxel_map_create(vpgs_ctx* ctx, const float* points, int64_t n, float voxel, int32_t max_per_voxel,
                          vpgs_voxel_map** map, void* stream);
/* Synchronises `stream` and reports the points given and the occupied voxels. */
int vpgs_voxel_map_info(vpgs_voxel_map* map, int64_t* n_points, int64_t* n_voxels, void* stream);
int vpgs_voxel_map_destroy(vpgs_voxel_map* map);

/* Downsampling that keeps one original point per voxel: the first one by
 * index.  out_idx (device int32 [n]) receives the kept indices in ascending
 * order, *out_count (device int32) their number.  The fine tracking stage
 * downsamples a scan twice (two voxel sizes). */
int vpgs_voxel_downsample(vpgs_ctx* ctx, const float* points, int64_t n, float voxel, int32_t* out_idx,
                          int32_t* out_count, void* stream);

/* Correspondences of n source points (device [n,3]) under pose (host 3x4
 * row-major [R | t], float64, rounded to FP32 for the transform): s = R p + t
 * in FP32 as ((R00 p_x + R01 p_y) + R02 p_z) + t_x, with no fused products;
 * the nearest stored point among the 27 voxels around the voxel of s, by
 * FP32 squared distance ((dx dx + dy dy) + dz dz), ties to the lower index.
 * nn[i] (device int32, may be NULL) = its original index if d^2 < tau^2
 * (FP32), else -1; d2[i] (device float, may be NULL) = its d^2 (+inf when
 * no neighbouring voxel has points). */
int vpgs_icp_correspond(vpgs_ctx* ctx, const vpgs_voxel_map* map, const float* src, int64_t n, const double* pose,
                        float tau, int32_t* nn, float* d2, void* stream);

/* Gauss-Newton terms of the robust registration cost of eq. 11 at pose, over
 * the correspondences above: with r = s - m, e^2 = |r|^2 and the
 * Geman-McClure kernel of eq. 12, rho(e) = (e^2 / 2) / (kappa + e^2), kappa =
 * sigma / 3, the weight w = rho'(e) / e = kappa / (kappa + e^2)^2 and
 * J = [I, -[s]x] (left increment xi = (rho, phi)):
 *   terms[0..20]  H = sum w J^T J, upper triangle row by row
 *   terms[21..26] g = sum w J^T r
 *   terms[27]     number of correspondences, terms[28] sum rho(e)
 * terms: device, 29 doubles. */
int vpgs_icp_linearize(vpgs_ctx* ctx, const vpgs_voxel_map* map, const float* src, int64_t n, const double* pose,
                       float tau, float sigma, double* terms, void* stream);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight tracking loops, harnesses that forbid allocation:
 * vpgs_icp_linearize with no allocation of any kind.  Its workgroup partial
 * sums live in a static device array of the library (58 KiB: 512 rows of 29
 * floats, enough for any n, as a pass has at most 512 workgroups), whose
 * address on each device is looked up once by vpgs_create.  Arguments,
 * results and errors are those of vpgs_icp_linearize (VPGS_EINVAL if a pass
 * would need more rows than the array holds).  Every call on one device
 * shares that device's array: calls that overlap on one device (on different
 * streams, or from several threads) race and must be serialised by the
 * caller.  Nothing needs clearing between calls. */
int vpgs_icp_linearize_noalloc(vpgs_ctx* ctx, const vpgs_voxel_map* map, const float* src, int64_t n,
                               const double* pose, float tau, float sigma, double* terms, void* stream);

typedef struct {
  float tau;              /* correspondence threshold (map units) */
  float sigma;            /* kernel scale sigma_t of eq. 12 (kappa = sigma / 3) */
  int32_t max_iterations; /* Gauss-Newton steps at most (>= 0) */
  int32_t reserved;
  double eps;             /* stop once |dx| < eps */
} vpgs_icp_opts;

typedef struct {
  int32_t iterations;     /* steps taken */
  int32_t converged;      /* 1 if the last step was below eps */
  int32_t count;          /* correspondences of the last linearisation */
  int32_t degenerate;     /* 1 if it stopped on fewer than 6 correspondences or a singular system */
  float rho;              /* sum rho(e) of the last linearisation */
  int32_t reserved;
} vpgs_icp_result;

/* Frame-to-map registration of a scan (device [n,3], sensor frame): the
 * initial pose is prev_pose * pred_pose (eq. 10: the previous pose and the
 * predicted relative motion, host 3x4 float64; pred_pose may be NULL), then
 * Gauss-Newton steps H dx = -g (FP64 Cholesky on the device) with
 * T <- Exp(dx) T (SE(3) exponential), until |dx| < eps or max_iterations, or a
 * degenerate system.  The pose stays on the device between steps; the host
 * checks the stop flag every eight steps.  Synchronous: returns the final
 * pose (pose_out, host 3x4 float64) and, if result is non-NULL, the
 * counters. */
int vpgs_icp_register(vpgs_ctx* ctx, const vpgs_voxel_map* map, const float* src, int64_t n,
                      const double* prev_pose, const double* pred_pose, const vpgs_icp_opts* opts, double* pose_out,
                      vpgs_icp_result* result, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* VPGS_H_ */
