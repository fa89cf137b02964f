// densify.hip -- submap expansion statistics (Section III-A): the anchor
// reduction of the per-Gaussian accumulators (growth by averaged gradient,
// pruning by accumulated opacity) and the expansion sampler (candidate pixels
// where the map does not explain the frame, ranked selection, back-projection
// with the measured depth).  The accumulators themselves are filled by the
// projection backward (project.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "runtime.h"

namespace vpgs {
namespace {

constexpr int kAnchorBlock = 256;

// One thread per anchor; its k accumulator rows are contiguous, so a
// wavefront streams 64 k rows of consecutive memory.  The sums are FP32 in
// index order and the decisions FP32, as the interface defines them.
__global__ void __launch_bounds__(kAnchorBlock) anchor_stats_kernel(const float4* __restrict__ acc, int64_t m,
                                                                   int k, float tau_g, float tau_o,
                                                                   float4* __restrict__ stats,
                                                                   uint8_t* __restrict__ grow,
                                                                   uint8_t* __restrict__ prune) {
#pragma clang fp contract(off)
  const int64_t a = (int64_t)blockIdx.x * kAnchorBlock + threadIdx.x;
  if (a >= m) return;
  const float4* p = acc + a * k;
  float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int j = 0; j < k; ++j) {
    const float4 v = p[j];
    s.x += v.x; s.y += v.y; s.z += v.z; s.w += v.w;
  }
  const float avg = s.y > 0.f ? s.x / s.y : 0.f;
  stats[a] = make_float4(avg, s.y, s.z, s.w);
  if (grow) grow[a] = avg > tau_g ? 1 : 0;
  if (prune) prune[a] = (s.w > 0.f && s.z < tau_o * s.w) ? 1 : 0;
}

// ---- expansion sampling ------------------------------------------------------

constexpr int kExpandBlock = 256;
constexpr int kExpandChunk = 4 * kExpandBlock;  // pixels per mask workgroup
constexpr int kExpandViews = 8;                 // views per launch (arguments by value)

struct ExpandView {
  int32_t W, H, nb, pad;  // nb = chunks of kExpandChunk pixels
  const float* alpha;
  const float* depth;
  const float* t_depth;
  const float* t_rgb;
  uint8_t* mask;
  uint32_t* bcount;  // [nb] candidates per chunk
  uint32_t* boff;    // [nb + 1] exclusive offsets; boff[nb] = candidates of the view
  int32_t* count;
  const float* u;    // [n_samples]
  int32_t* pixel;
  float* points;
  float* colors;
  float fx, fy, cx, cy;
  float R[9], t[3];
};

struct ExpandBatch {
  ExpandView v[kExpandViews];
  float thr_a, thr_d;
  int32_t n_samples, pad;
};

// Candidate mask and per-chunk counts: thread t of chunk b tests pixels
// b*1024 + t + 256q (q = 0..3), so every load and store is coalesced.
__global__ void __launch_bounds__(kExpandBlock) expand_mask_kernel(ExpandBatch B) {
#pragma clang fp contract(off)
  __shared__ uint32_t part[kExpandBlock / 64];
  const ExpandView& V = B.v[blockIdx.y];
  if ((int)blockIdx.x >= V.nb) return;  // workgroup-uniform
  const int64_t HW = (int64_t)V.W * V.H;
  const int64_t base = (int64_t)blockIdx.x * kExpandChunk;
  uint32_t n = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t p = base + q * kExpandBlock + threadIdx.x;
    bool c = false;
    if (p < HW) {
      const float t = V.t_depth[p];
      const float err = fabsf(V.depth[p] - t);
      c = t > 0.0f && (V.alpha[p] < B.thr_a || err > B.thr_d);
      V.mask[p] = c ? 1 : 0;
    }
    n += (uint32_t)__popcll(__ballot(c));
  }
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = n;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
#pragma unroll
    for (int w = 0; w < kExpandBlock / 64; ++w) tot += part[w];
    V.bcount[blockIdx.x] = tot;
  }
}

// Exclusive offsets of the chunk counts, one workgroup per view: each thread
// sums a contiguous run of chunks, the run totals are scanned in LDS, and
// each thread writes its run's offsets.
__global__ void __launch_bounds__(kExpandBlock) expand_scan_kernel(ExpandBatch B) {
  __shared__ uint32_t run[kExpandBlock];
  const ExpandView& V = B.v[blockIdx.x];
  const int per = (V.nb + kExpandBlock - 1) / kExpandBlock;
  const int b0 = threadIdx.x * per;
  const int b1 = min(b0 + per, V.nb);
  uint32_t s = 0;
  for (int b = b0; b < b1; ++b) s += V.bcount[b];
  run[threadIdx.x] = s;
  __syncthreads();
  for (int d = 1; d < kExpandBlock; d <<= 1) {  // Hillis-Steele inclusive scan
    const uint32_t add = threadIdx.x >= (unsigned)d ? run[threadIdx.x - d] : 0u;
    __syncthreads();
    run[threadIdx.x] += add;
    __syncthreads();
  }
  uint32_t off = run[threadIdx.x] - s;
  for (int b = b0; b < b1; ++b) {
    V.boff[b] = off;
    off += V.bcount[b];
  }
  if (threadIdx.x == kExpandBlock - 1) {
    V.boff[V.nb] = run[kExpandBlock - 1];
    *V.count = (int32_t)run[kExpandBlock - 1];
  }
}

// One wavefront per sample: the chunk holding the candidate of rank r by a
// 64-way search over the offsets, then the position inside the chunk by a
// wavefront prefix count of 16 mask bytes per lane (raster order), and the
// back-projection of that pixel centre with the target depth.
__global__ void __launch_bounds__(kExpandBlock) expand_sample_kernel(ExpandBatch B) {
#pragma clang fp contract(off)
  const ExpandView& V = B.v[blockIdx.y];
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (kExpandBlock / 64) + (threadIdx.x >> 6);
  if (i >= B.n_samples) return;  // wavefront-uniform
  const uint32_t c = V.boff[V.nb];
  if (c == 0) {
    if (lane == 0) {
      V.pixel[i] = -1;
      for (int k = 0; k < 3; ++k) { V.points[3 * i + k] = 0.f; V.colors[3 * i + k] = 0.f; }
    }
    return;
  }
  const float prod = V.u[i] * (float)c;
  uint32_t r = 0;  // u in [0, 1); anything else is clamped to the first or last rank
  if (prod >= (float)c) r = c - 1;
  else if (prod > 0.0f) r = min((uint32_t)prod, c - 1);
  // the last chunk whose offset is <= r, by a 64-way search: the lanes probe
  // evenly spaced offsets of the remaining range and keep the last one that
  // is <= r (boff[lo] <= r holds throughout, boff is non-decreasing)
  int lo = 0, len = V.nb;
  while (len > 1) {
    const int step = (len + 63) >> 6;
    const int idx = lo + lane * step;
    const bool ok = idx < lo + len && V.boff[idx] <= r;
    const int last = 63 - __clzll(__ballot(ok));
    const int end = lo + len;
    lo += last * step;
    len = min(step, end - lo);
  }
  const uint32_t within = r - V.boff[lo];
  const int64_t HW = (int64_t)V.W * V.H;
  const int64_t p0 = (int64_t)lo * kExpandChunk + 16 * lane;
  uint32_t bits = 0;  // candidate flags of the lane's 16 pixels
  if (p0 + 16 <= HW && (reinterpret_cast<uintptr_t>(V.mask + p0) & 15u) == 0) {
    const uint4 w = *reinterpret_cast<const uint4*>(V.mask + p0);
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if ((ws[j] >> (8 * b)) & 0xffu) bits |= 1u << (4 * j + b);
  } else {
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (p0 + q < HW && V.mask[p0 + q]) bits |= 1u << q;
  }
  const uint32_t cnt = (uint32_t)__popc(bits);
  uint32_t incl = cnt;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(incl, d, 64);
    if (lane >= d) incl += o;
  }
  const unsigned long long over = __ballot(incl > within);
  const int L = __ffsll(over) - 1;  // the lane that holds the candidate
  if (lane != L) return;
  uint32_t need = within - (incl - cnt);
  int q = 0;
  for (; q < 16; ++q) {
    if (bits & (1u << q)) {
      if (need == 0) break;
      --need;
    }
  }
  if (q == 16) return;  // unreachable: the chunk offsets count exactly these flags
  const int64_t p = p0 + q;
  const int x = (int)(p % V.W), y = (int)(p / V.W);
  const float T = V.t_depth[p];
  const float dx = (((float)x + 0.5f) - V.cx) / V.fx * T - V.t[0];
  const float dy = (((float)y + 0.5f) - V.cy) / V.fy * T - V.t[1];
  const float dz = T - V.t[2];
  V.pixel[i] = (int32_t)p;
  V.points[3 * i + 0] = V.R[0] * dx + V.R[3] * dy + V.R[6] * dz;
  V.points[3 * i + 1] = V.R[1] * dx + V.R[4] * dy + V.R[7] * dz;
  V.points[3 * i + 2] = V.R[2] * dx + V.R[5] * dy + V.R[8] * dz;
  for (int k = 0; k < 3; ++k) V.colors[3 * i + k] = V.t_rgb[(int64_t)k * HW + p];
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace
}  // namespace vpgs

using namespace vpgs;

extern "C" {

int vpgs_anchor_stats(vpgs_ctx* ctx, int64_t m, int32_t k, const float* accum, float tau_g, float tau_o,
                      float* stats, uint8_t* grow, uint8_t* prune, void* stream) {
  if (!ctx) return VPGS_EINVAL;
  if (m < 0) return fail(ctx, VPGS_EINVAL, "negative anchor count");
  if (k < 1 || k > 64) return fail(ctx, VPGS_EINVAL, "k = %d out of range [1, 64]", k);
  if (m == 0) return VPGS_OK;
  if (!accum || !stats) return fail(ctx, VPGS_EINVAL, "NULL accumulators or statistics");
  if (!aligned16(accum) || !aligned16(stats)) return fail(ctx, VPGS_EINVAL, "buffers must be 16-byte aligned");
  if (std::isnan(tau_g) || std::isnan(tau_o)) return fail(ctx, VPGS_EINVAL, "NaN threshold");
  const int64_t blocks = (m + kAnchorBlock - 1) / kAnchorBlock;
  if (blocks > 0x7fffffff) return fail(ctx, VPGS_EINVAL, "too many anchors");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));
  StageTimer timer(ctx, ST_ANCHOR, st);
  hipLaunchKernelGGL(anchor_stats_kernel, dim3((unsigned)blocks), dim3(kAnchorBlock), 0, st,
                     reinterpret_cast<const float4*>(accum), m, k, tau_g, tau_o, reinterpret_cast<float4*>(stats),
                     grow, prune);
  HIP_TRY(hipGetLastError());
  return VPGS_OK;
}

int vpgs_expansion_sample(vpgs_ctx* ctx, int n_views, const vpgs_camera* cams, const vpgs_images* rendered,
                          const vpgs_targets* targets, const vpgs_expand_opts* opts, const float* uniforms,
                          int32_t* counts, const vpgs_expand_out* out, void* stream) {
  if (!ctx) return VPGS_EINVAL;
  if (n_views < 0 || n_views > VPGS_MAX_VIEWS) return fail(ctx, VPGS_EINVAL, "n_views %d out of range", n_views);
  if (n_views == 0) return VPGS_OK;
  if (!cams || !rendered || !targets || !opts || !counts) return fail(ctx, VPGS_EINVAL, "NULL argument");
  if (std::isnan(opts->alpha_threshold) || std::isnan(opts->depth_threshold))
    return fail(ctx, VPGS_EINVAL, "NaN threshold");
  const int M = opts->n_samples;
  if (M < 0) return fail(ctx, VPGS_EINVAL, "negative sample count");
  if (M > 0 && (!uniforms || !out)) return fail(ctx, VPGS_EINVAL, "samples need uniforms and outputs");
  size_t mask_bytes = 0, block_words = 0;
  for (int v = 0; v < n_views; ++v) {
    const int W = cams[v].width, H = cams[v].height;
    if (W <= 0 || H <= 0 || W > VPGS_MAX_DIM || H > VPGS_MAX_DIM)
      return fail(ctx, VPGS_EINVAL, "view %d: size %dx%d out of range", v, W, H);
    if (!rendered[v].alpha || !rendered[v].depth || !targets[v].depth)
      return fail(ctx, VPGS_EINVAL, "view %d: NULL alpha or depth plane", v);
    if (M > 0 && (!targets[v].rgb || !out[v].pixel || !out[v].points || !out[v].colors))
      return fail(ctx, VPGS_EINVAL, "view %d: NULL sample output or target colour", v);
    const size_t HW = (size_t)W * H;
    if (!out || !out[v].mask) mask_bytes += (HW + 255) / 256 * 256;
    const size_t nb = (HW + kExpandChunk - 1) / kExpandChunk;
    block_words += 2 * nb + 1;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));
  int rc;
  if ((rc = ensure(ctx, ctx->expand_mask, mask_bytes)) ||
      (rc = ensure(ctx, ctx->expand_blocks, block_words * sizeof(uint32_t))))
    return rc;
  StageTimer timer(ctx, ST_EXPAND, st);
  uint8_t* mask_ws = static_cast<uint8_t*>(ctx->expand_mask.p);
  uint32_t* blk_ws = static_cast<uint32_t*>(ctx->expand_blocks.p);
  size_t mask_off = 0, blk_off = 0;
  for (int v0 = 0; v0 < n_views; v0 += kExpandViews) {
    const int nv = std::min(kExpandViews, n_views - v0);
    ExpandBatch B{};
    B.thr_a = opts->alpha_threshold;
    B.thr_d = opts->depth_threshold;
    B.n_samples = M;
    int max_nb = 1;
    for (int b = 0; b < nv; ++b) {
      const int v = v0 + b;
      ExpandView& E = B.v[b];
      const vpgs_camera& c = cams[v];
      E.W = c.width;
      E.H = c.height;
      const size_t HW = (size_t)E.W * E.H;
      E.nb = (int)((HW + kExpandChunk - 1) / kExpandChunk);
      max_nb = std::max(max_nb, E.nb);
      E.alpha = rendered[v].alpha;
      E.depth = rendered[v].depth;
      E.t_depth = targets[v].depth;
      E.t_rgb = targets[v].rgb;
      if (out && out[v].mask) {
        E.mask = out[v].mask;
      } else {
        E.mask = mask_ws + mask_off;
        mask_off += (HW + 255) / 256 * 256;
      }
      E.bcount = blk_ws + blk_off;
      E.boff = E.bcount + E.nb;
      blk_off += 2 * (size_t)E.nb + 1;
      E.count = counts + v;
      if (M > 0) {
        E.u = uniforms + (size_t)v * M;
        E.pixel = out[v].pixel;
        E.points = out[v].points;
        E.colors = out[v].colors;
      }
      E.fx = c.fx; E.fy = c.fy; E.cx = c.cx; E.cy = c.cy;
      for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) E.R[3 * r + k] = c.world_to_cam[4 * r + k];
        E.t[r] = c.world_to_cam[4 * r + 3];
      }
    }
    hipLaunchKernelGGL(expand_mask_kernel, dim3(max_nb, nv), dim3(kExpandBlock), 0, st, B);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(expand_scan_kernel, dim3(nv), dim3(kExpandBlock), 0, st, B);
    HIP_TRY(hipGetLastError());
    if (M > 0) {
      const int gx = (M + kExpandBlock / 64 - 1) / (kExpandBlock / 64);
      hipLaunchKernelGGL(expand_sample_kernel, dim3(gx, nv), dim3(kExpandBlock), 0, st, B);
      HIP_TRY(hipGetLastError());
    }
  }
  return VPGS_OK;
}

}  // extern "C"
