// runtime.cpp -- host side of the C ABI: argument validation, the context and
// its grow-only buffers, the saved forward state, and the launch sequence of
// the render forward and backward.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "runtime.h"

using namespace vpgs;

namespace vpgs {

const char* const kStageNames[VPGS_NUM_STAGES] = {
    "project", "scan", "emit", "sort", "ranges", "composite_forward", "composite_backward",
    "project_backward", "pose_reduce", "fill", "decode_forward", "decode_backward", "depth_order",
    "mapping_loss", "volume_loss", "anchor_stats", "expansion", "distillation", "voxel_map", "icp"};

int fail(vpgs_ctx* ctx, int code, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->last_error = buf;
  }
  return code;
}

hipEvent_t take_event(vpgs_ctx* ctx) {
  if (!ctx->ev_free.empty()) {
    hipEvent_t e = ctx->ev_free.back();
    ctx->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

StageTimer::StageTimer(vpgs_ctx* c, int s, hipStream_t stream) : ctx(c), stage(s), st(stream) {
  if (ctx->profiling) {
    a = take_event(ctx);
    if (a) (void)hipEventRecord(a, st);
  }
}

StageTimer::~StageTimer() {
  if (!a) return;
  hipEvent_t b = take_event(ctx);
  if (!b) return;
  (void)hipEventRecord(b, st);
  ctx->pending.push_back({stage, a, b});
}

namespace {

// Device memory through the caller's callbacks when it gave them (a caching
// allocator that recycles blocks needs the device idle before a block comes
// back: the library synchronises the device first), else hipMalloc/hipFree.
int alloc_device(vpgs_ctx* ctx, size_t bytes, void** p) {
  *p = nullptr;
  if (ctx->alloc) {
    *p = ctx->alloc(bytes, ctx->alloc_user);
    if (!*p) return fail(ctx, VPGS_ENOMEM, "allocator callback returned NULL for %zu bytes", bytes);
    if (reinterpret_cast<uintptr_t>(*p) & 255u) {
      ctx->free_(*p, ctx->alloc_user);
      *p = nullptr;
      return fail(ctx, VPGS_EINVAL, "allocator callback returned a block that is not 256-byte aligned");
    }
    return VPGS_OK;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(ctx, VPGS_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  }
  return VPGS_OK;
}

int release_device(vpgs_ctx* ctx, void* p) {
  if (!p) return VPGS_OK;
  if (ctx->free_) {
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->free_(p, ctx->alloc_user);
    return VPGS_OK;
  }
  hipError_t e = hipFree(p);
  if (e != hipSuccess) return fail(ctx, VPGS_EHIP, "hipFree: %s", hipGetErrorString(e));
  return VPGS_OK;
}

}  // namespace

int ensure(vpgs_ctx* ctx, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.cap >= bytes) return VPGS_OK;
  if (b.p) {
    void* old = b.p;
    b.p = nullptr;
    b.cap = 0;
    const int rc = release_device(ctx, old);
    if (rc) return rc;
  }
  const size_t want = bytes + bytes / 4;
  const int rc = alloc_device(ctx, want, &b.p);
  if (rc) return rc;
  b.cap = want;
  return VPGS_OK;
}

void free_buf(vpgs_ctx* ctx, DevBuf& b) {
  if (b.p) (void)release_device(ctx, b.p);
  b.p = nullptr;
  b.cap = 0;
}

}  // namespace vpgs

namespace vpgs {

void destroy_saved(vpgs_saved* s) {
  DevBuf* bufs[] = {&s->tab, &s->rec, &s->count, &s->zkey, &s->rect, &s->drect, &s->hitmask, &s->scan_ws,
                    &s->keys, &s->vals, &s->keys_alt, &s->vals_alt, &s->sort_ws, &s->ranges, &s->tfinal,
                    &s->ncontrib, &s->counters, &s->acc, &s->pose_partial, &s->dk, &s->dk_alt, &s->dv,
                    &s->dv_alt, &s->dcount, &s->dpoff, &s->key64, &s->order};
  for (DevBuf* b : bufs) free_buf(s->ctx, *b);
  delete s->h_tab;
  delete s;
}

int new_saved(vpgs_ctx* ctx, vpgs_saved** out) {
  vpgs_saved* s = new (std::nothrow) vpgs_saved();
  if (!s) return fail(ctx, VPGS_ENOMEM, "out of host memory");
  s->ctx = ctx;
  s->h_tab = new (std::nothrow) CallTables();
  if (!s->h_tab) {
    delete s;
    return fail(ctx, VPGS_ENOMEM, "out of host memory");
  }
  std::memset(s->h_tab, 0, sizeof(CallTables));
  *out = s;
  return VPGS_OK;
}

int acquire_saved(vpgs_ctx* ctx, vpgs_saved** out) {
  for (vpgs_saved* s : ctx->pool)
    if (!s->in_use) {
      s->in_use = true;
      *out = s;
      return VPGS_OK;
    }
  vpgs_saved* s = nullptr;
  int rc = new_saved(ctx, &s);
  if (rc) return rc;
  s->in_use = true;
  ctx->pool.push_back(s);
  *out = s;
  return VPGS_OK;
}

bool finite(float x) { return std::isfinite(x); }

int check_camera(vpgs_ctx* ctx, const vpgs_camera& c, int v) {
  if (c.width < 1 || c.height < 1 || c.width > VPGS_MAX_DIM || c.height > VPGS_MAX_DIM)
    return fail(ctx, VPGS_EINVAL, "view %d: image size %dx%d outside [1, %d]", v, c.width, c.height, VPGS_MAX_DIM);
  if (!(finite(c.fx) && finite(c.fy) && c.fx > 0 && c.fy > 0))
    return fail(ctx, VPGS_EINVAL, "view %d: focal lengths must be finite and positive", v);
  if (!(finite(c.cx) && finite(c.cy) && finite(c.near_plane)))
    return fail(ctx, VPGS_EINVAL, "view %d: principal point and near plane must be finite", v);
  for (int k = 0; k < 12; ++k)
    if (!finite(c.world_to_cam[k])) return fail(ctx, VPGS_EINVAL, "view %d: non-finite pose", v);
  return VPGS_OK;
}

int ilog2_ceil(uint64_t x) {
  int r = 0;
  while ((1ull << r) < x) ++r;
  return r;
}

// Builds the host call tables (without gradient pointers).
int build_tables(vpgs_ctx* ctx, CallTables& T, int n_sets, const vpgs_gaussians* sets, int n_views,
                 const int32_t* view_set, const vpgs_camera* cams, const vpgs_images* out, int tw, int th) {
  std::memset(&T, 0, sizeof(T));
  T.n_views = n_views;
  T.n_sets = n_sets;
  uint64_t rec = 0, tiles = 0, pix = 0;
  for (int v = 0; v < n_views; ++v) {
    const vpgs_camera& c = cams[v];
    ViewDesc& V = T.views[v];
    const int s = view_set[v];
    V.W = c.width;
    V.H = c.height;
    V.tiles_x = (c.width + tw - 1) / tw;
    V.tiles_y = (c.height + th - 1) / th;
    V.tile_base = (uint32_t)tiles;
    V.rec_base = (uint32_t)rec;
    V.pix_base = (uint32_t)pix;
    V.set = s;
    V.fx = c.fx; V.fy = c.fy; V.cx = c.cx; V.cy = c.cy;
    V.near_z = c.near_plane > 0.f ? c.near_plane : kDefaultNear;
    V.glx = (-kGuardLo * (float)c.width - c.cx) / c.fx;
    V.ghx = (kGuardHi * (float)c.width - c.cx) / c.fx;
    V.gly = (-kGuardLo * (float)c.height - c.cy) / c.fy;
    V.ghy = (kGuardHi * (float)c.height - c.cy) / c.fy;
    for (int r = 0; r < 3; ++r) {
      for (int k = 0; k < 3; ++k) V.R[3 * r + k] = c.world_to_cam[4 * r + k];
      V.t[r] = c.world_to_cam[4 * r + 3];
    }
    V.rgb = out[v].rgb;
    V.depth = out[v].depth;
    V.alpha = out[v].alpha;
    rec += (uint64_t)sets[s].n;
    tiles += (uint64_t)V.tiles_x * V.tiles_y;
    pix += (uint64_t)c.width * c.height;
  }
  if (rec > VPGS_MAX_RECORDS)
    return fail(ctx, VPGS_EINVAL, "too many (view, Gaussian) records: %llu (at most %d)", (unsigned long long)rec,
                VPGS_MAX_RECORDS);
  if (pix >= 0xffffffffull) return fail(ctx, VPGS_EINVAL, "too many pixels");
  T.n_records = (uint32_t)rec;
  T.n_tiles = (uint32_t)tiles;
  // sets: contiguous block ranges and the list of views of each set
  uint32_t block = 0;
  int nv = 0;
  for (int s = 0; s < n_sets; ++s) {
    SetDesc& S = T.sets[s];
    S.means = sets[s].means;
    S.log_scales = sets[s].log_scales;
    S.quats = sets[s].quats;
    S.opacities = sets[s].opacities;
    S.colors = sets[s].colors;
    S.n = sets[s].n;
    S.block_base = block;
    block += (uint32_t)((sets[s].n + 255) / 256);
    S.view_first = nv;
    for (int v = 0; v < n_views; ++v)
      if (view_set[v] == s) T.set_views[nv++] = v;
    S.view_count = nv - S.view_first;
  }
  return VPGS_OK;
}

int upload_tables(vpgs_ctx* ctx, vpgs_saved* sv, hipStream_t st) {
  const int slot = ctx->tab_ring_next;
  ctx->tab_ring_next = (slot + 1) % vpgs_ctx::kTabRing;
  HIP_TRY(hipEventSynchronize(ctx->tab_ring_ev[slot]));  // the copy that last read this slot is done
  std::memcpy(&ctx->tab_ring[slot], sv->h_tab, sizeof(CallTables));
  HIP_TRY(hipMemcpyAsync(sv->tab.p, &ctx->tab_ring[slot], sizeof(CallTables), hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(ctx->tab_ring_ev[slot], st));
  return VPGS_OK;
}

ProjBuffers proj_of(vpgs_saved* s) {
  ProjBuffers pb;
  pb.rec = static_cast<float4*>(s->rec.p);
  pb.zkey = static_cast<uint32_t*>(s->zkey.p);
  pb.count = static_cast<uint32_t*>(s->count.p);
  pb.rect = static_cast<uint2*>(s->rect.p);
  return pb;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int validate_forward(vpgs_ctx* ctx, int n_sets, const vpgs_gaussians* sets, int n_views, const int32_t* view_set,
                     const vpgs_camera* cams, const vpgs_images* out, const vpgs_render_opts* opts) {
  if (n_sets < 1 || n_sets > VPGS_MAX_SETS) return fail(ctx, VPGS_EINVAL, "n_sets %d outside [1, %d]", n_sets, VPGS_MAX_SETS);
  if (n_views < 1 || n_views > VPGS_MAX_VIEWS)
    return fail(ctx, VPGS_EINVAL, "n_views %d outside [1, %d]", n_views, VPGS_MAX_VIEWS);
  if (!sets || !view_set || !cams || !out) return fail(ctx, VPGS_EINVAL, "NULL argument array");
  for (int s = 0; s < n_sets; ++s) {
    const vpgs_gaussians& g = sets[s];
    if (g.n < 0 || g.n > 0x7fffffffLL) return fail(ctx, VPGS_EINVAL, "set %d: n = %lld out of range", s, (long long)g.n);
    if (g.n > 0 && (!g.means || !g.log_scales || !g.quats || !g.opacities || !g.colors))
      return fail(ctx, VPGS_EINVAL, "set %d: NULL parameter pointer", s);
    if (g.n > 0 && !aligned16(g.quats)) return fail(ctx, VPGS_EINVAL, "set %d: quats must be 16-byte aligned", s);
  }
  for (int v = 0; v < n_views; ++v) {
    if (view_set[v] < 0 || view_set[v] >= n_sets)
      return fail(ctx, VPGS_EINVAL, "view %d: set index %d outside [0, %d)", v, view_set[v], n_sets);
    int rc = check_camera(ctx, cams[v], v);
    if (rc) return rc;
    if (!out[v].rgb || !out[v].depth || !out[v].alpha) return fail(ctx, VPGS_EINVAL, "view %d: NULL output plane", v);
  }
  if (opts) {
    const int tw = opts->tile_w ? opts->tile_w : 16, th = opts->tile_h ? opts->tile_h : 16;
    if (!tile_shape_supported(tw, th)) return fail(ctx, VPGS_EUNSUPPORTED, "tile shape %dx%d not built", tw, th);
    if (opts->lds_batch != 0 && !lds_batch_supported(tw, th, opts->lds_batch))
      return fail(ctx, VPGS_EUNSUPPORTED, "LDS batch of %d entries not built for %dx%d tiles", opts->lds_batch, tw, th);
    if (opts->grid_ctas < 0 || opts->grid_ctas > kMaxGridCtas)
      return fail(ctx, VPGS_EINVAL, "grid_ctas %d out of range [0, %d]", opts->grid_ctas, kMaxGridCtas);
    if (opts->pair_capacity < 0 || opts->pair_capacity > 0x7fffffffLL)
      return fail(ctx, VPGS_EINVAL, "pair_capacity %lld out of range", (long long)opts->pair_capacity);
  }
  return VPGS_OK;
}

}  // namespace vpgs

namespace vpgs {

int read_pair_count(vpgs_ctx* ctx, vpgs_saved* sv, hipStream_t st, uint32_t* out) {
  Counters* cnt = static_cast<Counters*>(sv->counters.p);
  uint32_t* hp = static_cast<uint32_t*>(ctx->h_pinned);
  HIP_TRY(hipMemcpyAsync(hp, &cnt->pairs, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *out = *hp;
  return VPGS_OK;
}

int prepare_front(vpgs_ctx* ctx, vpgs_saved* sv) {
  const CallTables& T = *sv->h_tab;
  uint64_t pixels = 0;
  for (int v = 0; v < T.n_views; ++v) pixels += (uint64_t)T.views[v].W * T.views[v].H;
  sv->n_pixels = (uint32_t)pixels;
  sv->key_bits = ilog2_ceil(std::max<uint32_t>(T.n_tiles, 2u));
  const size_t R = T.n_records;
  int rc;
  if ((rc = ensure(ctx, sv->dk, R * 4)) || (rc = ensure(ctx, sv->dk_alt, R * 4)) || (rc = ensure(ctx, sv->dv, R * 4)) ||
      (rc = ensure(ctx, sv->dv_alt, R * 4)) || (rc = ensure(ctx, sv->dcount, R * 4)) ||
      (rc = ensure(ctx, sv->dpoff, R * 4)) || (rc = ensure(ctx, sv->sort_ws, sort_workspace_bytes((uint32_t)R))))
    return rc;
  if ((rc = ensure(ctx, sv->tab, sizeof(CallTables))) || (rc = ensure(ctx, sv->rec, R * kRecSlots * 16)) ||
      (rc = ensure(ctx, sv->count, R * 4)) || (rc = ensure(ctx, sv->zkey, R * 4)) ||
      (rc = ensure(ctx, sv->rect, R * 8)) || (rc = ensure(ctx, sv->drect, R * 8)) ||
      (rc = ensure(ctx, sv->scan_ws, scan_workspace_bytes((uint32_t)R))) ||
      (rc = ensure(ctx, sv->ranges, (size_t)T.n_tiles * 8)) || (rc = ensure(ctx, sv->order, (size_t)T.n_tiles * 4)) ||
      (rc = ensure(ctx, sv->tfinal, pixels * 4)) ||
      (rc = ensure(ctx, sv->ncontrib, pixels * 4)) || (rc = ensure(ctx, sv->counters, sizeof(Counters))))
    return rc;
  return VPGS_OK;
}

int ensure_pairs(vpgs_ctx* ctx, vpgs_saved* sv, uint32_t cap) {
  int rc;
  if ((rc = ensure(ctx, sv->keys, (size_t)cap * 4)) || (rc = ensure(ctx, sv->keys_alt, (size_t)cap * 4)) ||
      (rc = ensure(ctx, sv->vals, (size_t)cap * 4)) || (rc = ensure(ctx, sv->vals_alt, (size_t)cap * 4)) ||
      (rc = ensure(ctx, sv->sort_ws,
                   sort_workspace_bytes(std::max<uint32_t>(cap, sv->h_tab->n_records)))) ||
      (rc = ensure(ctx, sv->hitmask, hit_mask_bytes(cap, sv->h_tab->n_tiles, sv->tile_w, sv->tile_h, sv->lds_batch))))
    return rc;
  sv->capacity = cap;
  return VPGS_OK;
}

// The gradient accumulator is zero between backwards: it is cleared once
// when (re)allocated, and the projection backward clears every row it reads
// (the only rows the compositing backward adds to).
int ensure_backward(vpgs_ctx* ctx, vpgs_saved* sv, hipStream_t st) {
  const CallTables& T = *sv->h_tab;
  const size_t R = T.n_records;
  const uint32_t pblocks = project_blocks(T);
  const void* old_acc = sv->acc.p;
  int rc;
  if ((rc = ensure(ctx, sv->acc, R * kNumAcc * sizeof(float))) ||
      (rc = ensure(ctx, sv->pose_partial,
                   (size_t)T.n_views * std::max<uint32_t>(pblocks, 1u) * kPosePartialsPerBlock * 6 * sizeof(float))))
    return rc;
  if (sv->acc.p != old_acc) HIP_TRY(launch_fill_f32(static_cast<float*>(sv->acc.p), 0.0f, sv->acc.cap / 4, st));
  return VPGS_OK;
}

int bind_backward(vpgs_ctx* ctx, CallTables& T, const vpgs_image_grads* grad_out, const vpgs_gauss_grads* grads) {
  if (!grad_out || !grads) return fail(ctx, VPGS_EINVAL, "NULL argument array");
  for (int s = 0; s < T.n_sets; ++s) {
    const vpgs_gauss_grads& g = grads[s];
    if (T.sets[s].n > 0 && (!g.means || !g.log_scales || !g.quats || !g.opacities || !g.colors))
      return fail(ctx, VPGS_EINVAL, "set %d: NULL gradient pointer", s);
    if (T.sets[s].n > 0 && !aligned16(g.quats)) return fail(ctx, VPGS_EINVAL, "set %d: d_quats must be 16-byte aligned", s);
  }
  T.accum_space = 0;
  for (int s = 0; s < T.n_sets; ++s) {
    T.sets[s].accum = nullptr;
    T.sets[s].d_means = grads[s].means;
    T.sets[s].d_log_scales = grads[s].log_scales;
    T.sets[s].d_quats = grads[s].quats;
    T.sets[s].d_opacities = grads[s].opacities;
    T.sets[s].d_colors = grads[s].colors;
  }
  for (int v = 0; v < T.n_views; ++v) {
    T.views[v].g_rgb = grad_out[v].rgb;
    T.views[v].g_depth = grad_out[v].depth;
    T.views[v].g_alpha = grad_out[v].alpha;
  }
  return VPGS_OK;
}

int bind_accum(vpgs_ctx* ctx, CallTables& T, const vpgs_densify_accum* acc) {
  if (!acc) return VPGS_OK;
  if (acc->grad_space != 0 && acc->grad_space != 1) return fail(ctx, VPGS_EINVAL, "grad_space must be 0 or 1");
  if (!acc->accum) return fail(ctx, VPGS_EINVAL, "NULL accumulator array");
  for (int s = 0; s < T.n_sets; ++s)
    if (acc->accum[s] && T.sets[s].n > 0 && !aligned16(acc->accum[s]))
      return fail(ctx, VPGS_EINVAL, "set %d: accumulators must be 16-byte aligned", s);
  T.accum_space = acc->grad_space;
  for (int s = 0; s < T.n_sets; ++s) T.sets[s].accum = T.sets[s].n > 0 ? acc->accum[s] : nullptr;
  return VPGS_OK;
}

int enqueue_front(vpgs_ctx* ctx, vpgs_saved* sv, hipStream_t st) {
  const CallTables& T = *sv->h_tab;
  const CallTables* d_tab = static_cast<const CallTables*>(sv->tab.p);
  Counters* cnt = static_cast<Counters*>(sv->counters.p);
  const ProjBuffers pb = proj_of(sv);
  {
    // (the projection also zeroes the counters and the tile ranges)
    StageTimer t(ctx, ST_PROJECT, st);
    HIP_TRY(launch_project(d_tab, T, pb, sv->tile_w, sv->tile_h, cnt, static_cast<uint2*>(sv->ranges.p), st));
  }
  {
    // visible records (count != 0), compacted in record order with their depth keys
    StageTimer t(ctx, ST_SCAN, st);
    HIP_TRY(launch_compact_visible(pb.count, pb.zkey, T.n_records, static_cast<uint32_t*>(sv->dk.p),
                                   static_cast<uint32_t*>(sv->dv.p), &cnt->visible, sv->scan_ws.p, st));
  }
  {
    StageTimer t(ctx, ST_DEPTH, st);
    DepthOrder d;
    d.keys = static_cast<uint32_t*>(sv->dk.p);
    d.vals = static_cast<uint32_t*>(sv->dv.p);
    d.keys_alt = static_cast<uint32_t*>(sv->dk_alt.p);
    d.vals_alt = static_cast<uint32_t*>(sv->dv_alt.p);
    d.rects = static_cast<uint2*>(sv->drect.p);
    d.counts = static_cast<uint32_t*>(sv->dcount.p);
    d.pair_off = static_cast<uint32_t*>(sv->dpoff.p);
    d.pair_off_total = &cnt->pairs;
    d.scan_ws = sv->scan_ws.p;
    d.sorted_in_alt = &sv->depth_in_alt;
    HIP_TRY(launch_depth_order(T, pb, &cnt->visible, d, sv->sort_ws.p, st));
  }
  return VPGS_OK;
}

int enqueue_back(vpgs_ctx* ctx, vpgs_saved* sv, hipStream_t st) {
  const CallTables& T = *sv->h_tab;
  const CallTables* d_tab = static_cast<const CallTables*>(sv->tab.p);
  Counters* cnt = static_cast<Counters*>(sv->counters.p);
  const ProjBuffers pb = proj_of(sv);
  const uint32_t cap = sv->capacity;
  uint32_t* keys = static_cast<uint32_t*>(sv->keys.p);
  uint32_t* vals = static_cast<uint32_t*>(sv->vals.p);
  uint32_t* keys_alt = static_cast<uint32_t*>(sv->keys_alt.p);
  uint32_t* vals_alt = static_cast<uint32_t*>(sv->vals_alt.p);
  {
    StageTimer t(ctx, ST_EMIT, st);
    const uint32_t* sorted_rec = static_cast<const uint32_t*>(sv->depth_in_alt ? sv->dv_alt.p : sv->dv.p);
    HIP_TRY(launch_emit(d_tab, T, sorted_rec, static_cast<const uint2*>(sv->drect.p),
                        static_cast<const uint32_t*>(sv->dpoff.p), &cnt->visible, cnt, keys, vals, cap, st));
  }
  {
    StageTimer t(ctx, ST_SORT, st);
    HIP_TRY(launch_sort(keys, vals, keys_alt, vals_alt, cap, sv->key_bits, cnt, sv->sort_ws.p, &sv->result_in_alt,
                        st));
  }
  const uint32_t* skeys = sv->result_in_alt ? keys_alt : keys;
  const uint32_t* svals = sv->result_in_alt ? vals_alt : vals;
  {
    StageTimer t(ctx, ST_RANGES, st);
    HIP_TRY(launch_ranges(skeys, cnt, cap, static_cast<uint2*>(sv->ranges.p), T.n_tiles, st));
    HIP_TRY(launch_tile_order(static_cast<const uint2*>(sv->ranges.p), T.n_tiles, cnt,
                              static_cast<uint32_t*>(sv->order.p), st));
  }
  {
    StageTimer t(ctx, ST_FWD, st);
    HIP_TRY(launch_composite_forward(d_tab, T, pb, static_cast<const uint2*>(sv->ranges.p), svals,
                                     static_cast<const uint32_t*>(sv->order.p), static_cast<float*>(sv->tfinal.p),
                                     static_cast<uint32_t*>(sv->ncontrib.p), static_cast<uint64_t*>(sv->hitmask.p), cnt,
                                     sv->count_work, sv->tile_w, sv->tile_h, sv->lds_batch,
                                     sv->persistent_blocks ? &cnt->queue_fwd : nullptr, sv->persistent_blocks, st));
  }
  return VPGS_OK;
}

int enqueue_backward(vpgs_ctx* ctx, vpgs_saved* sv, float* d_pose, hipStream_t st) {
  const CallTables& T = *sv->h_tab;
  const CallTables* d_tab = static_cast<const CallTables*>(sv->tab.p);
  Counters* cnt = static_cast<Counters*>(sv->counters.p);
  const ProjBuffers pb = proj_of(sv);
  float* acc = static_cast<float*>(sv->acc.p);
  const uint32_t* svals = static_cast<const uint32_t*>(sv->result_in_alt ? sv->vals_alt.p : sv->vals.p);
  if (sv->persistent_blocks) {
    StageTimer t(ctx, ST_FILL, st);
    HIP_TRY(launch_fill_u32(&cnt->queue_bwd, 0u, 1, st));
  }
  {
    StageTimer t(ctx, ST_BWD, st);
    HIP_TRY(launch_composite_backward(d_tab, T, pb, static_cast<const uint2*>(sv->ranges.p), svals,
                                      static_cast<const uint32_t*>(sv->order.p), static_cast<const float*>(sv->tfinal.p),
                                      static_cast<const uint32_t*>(sv->ncontrib.p),
                                      static_cast<const uint64_t*>(sv->hitmask.p), acc, cnt, sv->tile_w,
                                      sv->tile_h, sv->lds_batch, sv->persistent_blocks ? &cnt->queue_bwd : nullptr,
                                      sv->persistent_blocks, st));
  }
  float* partial = d_pose ? static_cast<float*>(sv->pose_partial.p) : nullptr;
  {
    StageTimer t(ctx, ST_PROJ_BWD, st);
    HIP_TRY(launch_project_backward(d_tab, T, pb, acc, partial, st));
  }
  if (d_pose) {
    StageTimer t(ctx, ST_POSE, st);
    HIP_TRY(launch_pose_reduce(d_tab, T, partial, d_pose, st));
  }
  return VPGS_OK;
}

}  // namespace vpgs

extern "C" {

int vpgs_version(void) { return 1; }

const char* vpgs_status_string(int status) {
  switch (status) {
    case VPGS_OK: return "ok";
    case VPGS_EINVAL: return "invalid argument";
    case VPGS_ENOMEM: return "out of memory";
    case VPGS_EHIP: return "HIP runtime error";
    case VPGS_ECAPACITY: return "pair list capacity exceeded";
    case VPGS_EUNSUPPORTED: return "unsupported option";
    default: return "unknown status";
  }
}

const char* vpgs_last_error(const vpgs_ctx* ctx) { return ctx ? ctx->last_error.c_str() : "NULL context"; }

int vpgs_create(vpgs_ctx** out, int device, void* (*alloc)(size_t, void*), void (*free_)(void*, void*),
                void* user) {
  if (!out) return VPGS_EINVAL;
  *out = nullptr;
  if ((alloc == nullptr) != (free_ == nullptr)) return VPGS_EINVAL;  // both callbacks or neither
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return VPGS_EINVAL;
  vpgs_ctx* ctx = new (std::nothrow) vpgs_ctx();
  if (!ctx) return VPGS_ENOMEM;
  ctx->device = device;
  ctx->alloc = alloc;
  ctx->free_ = free_;
  ctx->alloc_user = user;
  if (hipSetDevice(device) != hipSuccess || hipHostMalloc(&ctx->h_pinned, 4096, hipHostMallocDefault) != hipSuccess) {
    delete ctx;
    return VPGS_EHIP;
  }
  bool ring_ok = hipHostMalloc((void**)&ctx->tab_ring, vpgs_ctx::kTabRing * sizeof(CallTables),
                               hipHostMallocDefault) == hipSuccess;
  for (int k = 0; ring_ok && k < vpgs_ctx::kTabRing; ++k)
    ring_ok = hipEventCreateWithFlags(&ctx->tab_ring_ev[k], hipEventDisableTiming) == hipSuccess;
  if (!ring_ok) {
    for (hipEvent_t e : ctx->tab_ring_ev)
      if (e) (void)hipEventDestroy(e);
    if (ctx->tab_ring) (void)hipHostFree(ctx->tab_ring);
    (void)hipHostFree(ctx->h_pinned);
    delete ctx;
    return VPGS_EHIP;
  }
  const int rc = init_scratch(ctx);
  if (rc) {
    for (hipEvent_t e : ctx->tab_ring_ev) (void)hipEventDestroy(e);
    (void)hipHostFree(ctx->tab_ring);
    (void)hipHostFree(ctx->h_pinned);
    delete ctx;
    return rc;
  }
  *out = ctx;
  return VPGS_OK;
}

int vpgs_profile_enable(vpgs_ctx* ctx, int on) {
  if (!ctx) return VPGS_EINVAL;
  for (auto& p : ctx->pending) {
    (void)hipEventSynchronize(p.b);
    ctx->ev_free.push_back(p.a);
    ctx->ev_free.push_back(p.b);
  }
  ctx->pending.clear();
  for (int i = 0; i < VPGS_NUM_STAGES; ++i) {
    ctx->stage_ms[i] = 0.0;
    ctx->stage_calls[i] = 0;
  }
  ctx->profiling = on != 0;
  return VPGS_OK;
}

int vpgs_profile_read(vpgs_ctx* ctx, int stage, const char** name, int64_t* calls, double* total_ms) {
  if (!ctx) return VPGS_EINVAL;
  if (stage < 0 || stage >= VPGS_NUM_STAGES) return fail(ctx, VPGS_EINVAL, "stage %d out of range", stage);
  for (auto& p : ctx->pending) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(p.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.a, p.b);
    if (e != hipSuccess) return fail(ctx, VPGS_EHIP, "event timing: %s", hipGetErrorString(e));
    ctx->stage_ms[p.stage] += ms;
    ctx->stage_calls[p.stage] += 1;
    ctx->ev_free.push_back(p.a);
    ctx->ev_free.push_back(p.b);
  }
  ctx->pending.clear();
  if (name) *name = kStageNames[stage];
  if (calls) *calls = ctx->stage_calls[stage];
  if (total_ms) *total_ms = ctx->stage_ms[stage];
  return VPGS_OK;
}

int vpgs_destroy(vpgs_ctx* ctx) {
  if (!ctx) return VPGS_EINVAL;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (auto& p : ctx->pending) { ctx->ev_free.push_back(p.a); ctx->ev_free.push_back(p.b); }
  for (hipEvent_t e : ctx->ev_free) (void)hipEventDestroy(e);
  for (vpgs_saved* s : ctx->pool) destroy_saved(s);
  free_buf(ctx, ctx->dec_partial);
  free_buf(ctx, ctx->loss_ws);
  free_buf(ctx, ctx->loss_sums);
  free_buf(ctx, ctx->expand_mask);
  free_buf(ctx, ctx->expand_blocks);
  free_buf(ctx, ctx->distill_ws);
  free_buf(ctx, ctx->icp_build);
  free_buf(ctx, ctx->icp_ws);
  free_buf(ctx, ctx->peak_ws);
  if (ctx->h_pinned) (void)hipHostFree(ctx->h_pinned);
  for (hipEvent_t e : ctx->tab_ring_ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->tab_ring) (void)hipHostFree(ctx->tab_ring);
  delete ctx;
  return VPGS_OK;
}

int vpgs_render_forward(vpgs_ctx* ctx, int n_sets, const vpgs_gaussians* sets, int n_views, const int32_t* view_set,
                        const vpgs_camera* cams, const vpgs_images* out, const vpgs_render_opts* opts,
                        vpgs_saved** saved, void* stream) {
  if (!ctx) return VPGS_EINVAL;
  if (saved) *saved = nullptr;
  int rc = validate_forward(ctx, n_sets, sets, n_views, view_set, cams, out, opts);
  if (rc) return rc;
  const int tw = (opts && opts->tile_w) ? opts->tile_w : 16;
  const int th = (opts && opts->tile_h) ? opts->tile_h : 16;
  const int64_t fixed_cap = opts ? opts->pair_capacity : 0;
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));

  vpgs_saved* sv = nullptr;
  rc = acquire_saved(ctx, &sv);
  if (rc) return rc;
  struct Releaser {
    vpgs_saved* s; bool keep = false;
    ~Releaser() { if (!keep) s->in_use = false; }
  } rel{sv};

  rc = build_tables(ctx, *sv->h_tab, n_sets, sets, n_views, view_set, cams, out, tw, th);
  if (rc) return rc;
  sv->tile_w = tw;
  sv->tile_h = th;
  sv->lds_batch = (opts && opts->lds_batch) ? opts->lds_batch : tw * th;
  sv->persistent_blocks = opts ? (uint32_t)opts->grid_ctas : 0u;
  sv->count_work = !(opts && opts->skip_counts);
  if ((rc = prepare_front(ctx, sv)) || (rc = upload_tables(ctx, sv, st)) || (rc = enqueue_front(ctx, sv, st)))
    return rc;
  uint32_t cap;
  if (fixed_cap > 0) {
    cap = (uint32_t)fixed_cap;
  } else {
    rc = read_pair_count(ctx, sv, st, &cap);
    if (rc) return rc;
    cap = std::max<uint32_t>(cap, 1u);
  }
  if ((rc = ensure_pairs(ctx, sv, cap)) || (rc = enqueue_back(ctx, sv, st))) return rc;
  if (saved) {
    rel.keep = true;
    *saved = sv;
  }
  return VPGS_OK;
}

int vpgs_render_backward(vpgs_ctx* ctx, const vpgs_saved* saved_c, const vpgs_image_grads* grad_out,
                         const vpgs_gauss_grads* grads, float* d_pose, void* stream) {
  return vpgs_render_backward_accum(ctx, saved_c, grad_out, grads, d_pose, nullptr, stream);
}

int vpgs_render_backward_accum(vpgs_ctx* ctx, const vpgs_saved* saved_c, const vpgs_image_grads* grad_out,
                               const vpgs_gauss_grads* grads, float* d_pose, const vpgs_densify_accum* acc,
                               void* stream) {
  if (!ctx) return VPGS_EINVAL;
  vpgs_saved* sv = const_cast<vpgs_saved*>(saved_c);
  if (!sv || !sv->in_use) return fail(ctx, VPGS_EINVAL, "invalid saved-state handle");
  bool known = false;
  for (vpgs_saved* s : ctx->pool) known = known || s == sv;
  if (!known) return fail(ctx, VPGS_EINVAL, "saved-state handle of another context");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));
  int rc = bind_backward(ctx, *sv->h_tab, grad_out, grads);
  if (!rc) rc = bind_accum(ctx, *sv->h_tab, acc);
  if (rc) return rc;
  if ((rc = ensure_backward(ctx, sv, st)) || (rc = upload_tables(ctx, sv, st)) ||
      (rc = enqueue_backward(ctx, sv, d_pose, st)))
    return rc;
  return VPGS_OK;
}

int vpgs_saved_stats(vpgs_ctx* ctx, const vpgs_saved* saved, vpgs_stats* out, void* stream) {
  if (!ctx) return VPGS_EINVAL;
  if (!saved || !out) return fail(ctx, VPGS_EINVAL, "NULL argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));
  Counters* hc = static_cast<Counters*>(ctx->h_pinned);
  HIP_TRY(hipMemcpyAsync(hc, saved->counters.p, sizeof(Counters), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  std::memset(out, 0, sizeof(*out));
  const CallTables& T = *saved->h_tab;
  out->n_records = T.n_records;
  out->n_pairs = hc->pairs;
  unsigned long long ev = 0, bl = 0, fh = 0, bh = 0, ba = 0;
  for (int k = 0; k < kCountSlots; ++k) {
    ev += hc->evaluated[k];
    bl += hc->blended[k];
    fh += hc->fwd_hits[k];
    bh += hc->bwd_hits[k];
    ba += hc->bwd_active[k];
  }
  out->n_evaluated = (int64_t)ev;
  out->n_blended = (int64_t)bl;
  out->n_fwd_steps = (int64_t)fh;
  out->n_bwd_steps = (int64_t)bh;
  out->n_bwd_active = (int64_t)ba;
  out->pair_capacity = saved->capacity;
  out->n_tiles = T.n_tiles;
  out->n_pixels = saved->n_pixels;
  out->overflow = hc->overflow || hc->pairs > saved->capacity;
  out->tile_w = saved->tile_w;
  out->tile_h = saved->tile_h;
  out->lds_batch = saved->lds_batch;
  out->n_visible = hc->visible;
  return out->overflow ? fail(ctx, VPGS_ECAPACITY, "pair list overflow: %u pairs, capacity %u", hc->pairs,
                              saved->capacity)
                       : VPGS_OK;
}

int vpgs_saved_export(vpgs_ctx* ctx, const vpgs_saved* saved, int what, void* dst, size_t bytes, size_t* size,
                      void* stream) {
  if (!ctx) return VPGS_EINVAL;
  if (!saved) return fail(ctx, VPGS_EINVAL, "NULL saved handle");
  const CallTables& T = *saved->h_tab;
  const size_t R = T.n_records;
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));
  size_t need = 0;
  switch (what) {
    case VPGS_BUF_PROJ: need = R * 48; break;
    case VPGS_BUF_EXTENT: need = R * 8; break;
    case VPGS_BUF_COUNT: need = R * 4; break;
    case VPGS_BUF_KEYS: need = (size_t)saved->capacity * 8; break;
    case VPGS_BUF_VALUES: need = (size_t)saved->capacity * 4; break;
    case VPGS_BUF_RANGES: need = (size_t)T.n_tiles * 8; break;
    case VPGS_BUF_TFINAL: need = (size_t)saved->n_pixels * 4; break;
    case VPGS_BUF_NCONTRIB: need = (size_t)saved->n_pixels * 4; break;
    default: return fail(ctx, VPGS_EINVAL, "unknown buffer %d", what);
  }
  if (size) *size = need;
  if (!dst) return size ? VPGS_OK : fail(ctx, VPGS_EINVAL, "NULL destination");
  if (bytes < need) return fail(ctx, VPGS_EINVAL, "destination holds %zu bytes, %zu needed", bytes, need);
  if (need == 0) return VPGS_OK;
  const bool alt = saved->result_in_alt != 0;
  switch (what) {
    case VPGS_BUF_PROJ: {
      // the first three slots of every record as rows of 12 floats
      HIP_TRY(hipMemcpy2DAsync(dst, 48, saved->rec.p, kRecSlots * 16, 48, R, hipMemcpyDeviceToDevice, st));
      return VPGS_OK;
    }
    case VPGS_BUF_EXTENT:
      HIP_TRY(launch_export_extent(proj_of(const_cast<vpgs_saved*>(saved)), (uint32_t)R, static_cast<float2*>(dst), st));
      break;
    case VPGS_BUF_COUNT: HIP_TRY(hipMemcpyAsync(dst, saved->count.p, need, hipMemcpyDeviceToDevice, st)); break;
    case VPGS_BUF_KEYS: {
      vpgs_saved* sv = const_cast<vpgs_saved*>(saved);
      int rc = ensure(ctx, sv->key64, need);
      if (rc) return rc;
      HIP_TRY(launch_key64(static_cast<const uint32_t*>(alt ? saved->keys_alt.p : saved->keys.p),
                           static_cast<const uint32_t*>(alt ? saved->vals_alt.p : saved->vals.p),
                           proj_of(sv), static_cast<const Counters*>(saved->counters.p), saved->capacity,
                           static_cast<uint64_t*>(sv->key64.p), st));
      HIP_TRY(hipMemcpyAsync(dst, sv->key64.p, need, hipMemcpyDeviceToDevice, st));
      break;
    }
    case VPGS_BUF_VALUES:
      HIP_TRY(hipMemcpyAsync(dst, alt ? saved->vals_alt.p : saved->vals.p, need, hipMemcpyDeviceToDevice, st));
      break;
    case VPGS_BUF_RANGES: HIP_TRY(hipMemcpyAsync(dst, saved->ranges.p, need, hipMemcpyDeviceToDevice, st)); break;
    case VPGS_BUF_TFINAL: HIP_TRY(hipMemcpyAsync(dst, saved->tfinal.p, need, hipMemcpyDeviceToDevice, st)); break;
    case VPGS_BUF_NCONTRIB: HIP_TRY(hipMemcpyAsync(dst, saved->ncontrib.p, need, hipMemcpyDeviceToDevice, st)); break;
  }
  return VPGS_OK;
}

int vpgs_saved_release(vpgs_ctx* ctx, vpgs_saved* saved) {
  if (!ctx) return VPGS_EINVAL;
  if (!saved) return VPGS_OK;
  for (vpgs_saved* s : ctx->pool)
    if (s == saved) {
      if (!s->in_use) return fail(ctx, VPGS_EINVAL, "saved-state handle released twice");
      s->in_use = false;
      return VPGS_OK;
    }
  return fail(ctx, VPGS_EINVAL, "saved-state handle of another context");
}

}  // extern "C"
