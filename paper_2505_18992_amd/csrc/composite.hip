// composite.hip -- per-tile front-to-back alpha compositing and its
// backward.
//
// One workgroup per (view, tile); one thread per pixel.  Each tile walks its
// depth-sorted slice of the pair list in batches staged in LDS (every pixel
// of the tile reads the same Gaussian, so LDS reads broadcast).  A pixel
// stops at the first Gaussian that would take its transmittance under 1e-4;
// the divergent per-pixel loop retires whole wavefronts once all their lanes
// are done, and the workgroup leaves the batch loop once a barrier count
// shows every pixel done.
//
// The backward walks the same slice in reverse from the last blended entry,
// recovers the transmittance by division and recomputes alpha with the
// forward's exact instruction sequence (nothing per (pixel, Gaussian) is
// stored).  Per-Gaussian gradients are reduced across the wavefront before
// one set of atomic adds per (wavefront, Gaussian).
#include "internal.h"

namespace vpgs {
namespace {

__device__ __forceinline__ int view_of_tile(const CallTables* tab, uint32_t tile) {
  int lo = 0, hi = tab->n_views - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab->views[mid].tile_base <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Gaussian falloff at a pixel centre.  Shared verbatim by the forward and the
// backward (no contraction beyond the explicit fmaf), so the backward
// recomputes bit-identical alpha values.
struct Falloff { float dx, dy, G, raw, alpha; };
__device__ __forceinline__ Falloff falloff(const float4 A, const float4 B, float pxc, float pyc) {
#pragma clang fp contract(off)
  Falloff f;
  f.dx = A.x - pxc;
  f.dy = A.y - pyc;
  const float quad = fmaf(B.z * f.dy, f.dy, (B.x * f.dx) * f.dx);   // Qa dx^2 + Qc dy^2
  const float sigma = fmaf(B.y * f.dx, f.dy, 0.5f * quad);         // + Qb dx dy
  f.G = __expf(-sigma);
  f.raw = A.w * f.G;
  f.alpha = fminf(kAlphaMax, f.raw);
  return f;
}

template <int TW, int TH>
struct FwdShared {
  float4 A[TW * TH], B[TW * TH], C[TW * TH];
};

template <int TW, int TH>
__device__ __forceinline__ void forward_tile(const CallTables* __restrict__ tab, const float4* __restrict__ pa,
                                             const float4* __restrict__ pb, const float4* __restrict__ pc,
                                             const uint2* __restrict__ ranges, const uint32_t* __restrict__ vals,
                                             float* __restrict__ T_final, uint32_t* __restrict__ n_contrib,
                                             uint32_t tile, FwdShared<TW, TH>& sh, uint32_t& ne, uint32_t& nb) {
  constexpr int BS = TW * TH;
  float4* sA = sh.A;
  float4* sB = sh.B;
  float4* sC = sh.C;
  const ViewDesc& V = tab->views[view_of_tile(tab, tile)];
  const uint32_t lt = tile - V.tile_base;
  const int tx = (int)(lt % (uint32_t)V.tiles_x), ty = (int)(lt / (uint32_t)V.tiles_x);
  const int px = tx * TW + (int)(threadIdx.x % TW), py = ty * TH + (int)(threadIdx.x / TW);
  const bool inside = px < V.W && py < V.H;
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  const uint2 rg = ranges[tile];

  float T = 1.0f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f;
  uint32_t last = 0;
  bool done = !inside;

  for (uint32_t start = rg.x; start < rg.y; start += BS) {
    if (__syncthreads_count(done) == BS) break;
    const uint32_t idx = start + threadIdx.x;
    if (idx < rg.y) {
      const uint32_t rec = vals[idx];
      sA[threadIdx.x] = pa[rec];
      sB[threadIdx.x] = pb[rec];
      sC[threadIdx.x] = pc[rec];
    }
    __syncthreads();
    const int nbat = (int)min((uint32_t)BS, rg.y - start);
    for (int j = 0; j < nbat && !done; ++j) {
      const float4 A = sA[j];
      const Falloff f = falloff(A, sB[j], pxc, pyc);
      ++ne;
      if (f.alpha < kAlphaMin) continue;
      const float Tn = T * (1.0f - f.alpha);
      if (Tn < kTransMin) { done = true; break; }
      const float w = f.alpha * T;
      const float4 c = sC[j];
      C0 = fmaf(w, c.x, C0);
      C1 = fmaf(w, c.y, C1);
      C2 = fmaf(w, c.z, C2);
      D = fmaf(w, A.z, D);
      T = Tn;
      last = start + (uint32_t)j + 1u - rg.x;
      ++nb;
    }
  }
  if (inside) {
    const size_t HW = (size_t)V.W * V.H;
    const size_t pix = (size_t)py * V.W + px;
    V.rgb[pix] = C0;
    V.rgb[HW + pix] = C1;
    V.rgb[2 * HW + pix] = C2;
    V.depth[pix] = D;
    V.alpha[pix] = 1.0f - T;
    T_final[V.pix_base + pix] = T;
    n_contrib[V.pix_base + pix] = last;
  }
}

// Evaluation and blend counters: wave sums, one atomic per wave.
__device__ __forceinline__ void flush_counts(uint32_t ne, uint32_t nb, Counters* cnt) {
  unsigned long long e = ne, b = nb;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    e += __shfl_xor(e, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&cnt->evaluated, e);
    atomicAdd(&cnt->blended, b);
  }
}

// Next tile of a persistent workgroup: thread 0 takes a ticket from the
// queue counter and broadcasts it through LDS.
__device__ __forceinline__ uint32_t next_tile(uint32_t* queue, uint32_t* slot) {
  __syncthreads();
  if (threadIdx.x == 0) *slot = atomicAdd(queue, 1u);
  __syncthreads();
  return *slot;
}

// One workgroup per tile (grid = tiles), or, when queue is non-NULL, a
// persistent grid whose workgroups take tiles from the queue until it runs
// past the last tile.
template <int TW, int TH>
__global__ void __launch_bounds__(TW * TH) composite_forward_kernel(
    const CallTables* __restrict__ tab, const float4* __restrict__ pa, const float4* __restrict__ pb,
    const float4* __restrict__ pc, const uint2* __restrict__ ranges, const uint32_t* __restrict__ vals,
    float* __restrict__ T_final, uint32_t* __restrict__ n_contrib, Counters* __restrict__ cnt,
    uint32_t* __restrict__ queue, uint32_t n_tiles) {
  __shared__ FwdShared<TW, TH> sh;
  __shared__ uint32_t slot;
  uint32_t ne = 0, nb = 0;
  if (queue == nullptr) {
    forward_tile<TW, TH>(tab, pa, pb, pc, ranges, vals, T_final, n_contrib, blockIdx.x, sh, ne, nb);
  } else {
    for (uint32_t t = next_tile(queue, &slot); t < n_tiles; t = next_tile(queue, &slot))
      forward_tile<TW, TH>(tab, pa, pb, pc, ranges, vals, T_final, n_contrib, t, sh, ne, nb);
  }
  flush_counts(ne, nb, cnt);
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int TW, int TH>
struct BwdShared {
  float4 A[TW * TH], B[TW * TH], C[TW * TH];
  uint32_t rec[TW * TH];
  uint32_t maxlast[(TW * TH) / 64];
};

template <int TW, int TH>
__device__ __forceinline__ void backward_tile(const CallTables* __restrict__ tab, const float4* __restrict__ pa,
                                              const float4* __restrict__ pb, const float4* __restrict__ pc,
                                              const uint2* __restrict__ ranges, const uint32_t* __restrict__ vals,
                                              const float* __restrict__ T_final,
                                              const uint32_t* __restrict__ n_contrib, float* __restrict__ acc,
                                              uint32_t tile, BwdShared<TW, TH>& sh) {
  constexpr int BS = TW * TH;
  float4* sA = sh.A;
  float4* sB = sh.B;
  float4* sC = sh.C;
  uint32_t* sRec = sh.rec;
  uint32_t* smax = sh.maxlast;
  const ViewDesc& V = tab->views[view_of_tile(tab, tile)];
  const uint32_t lt = tile - V.tile_base;
  const int tx = (int)(lt % (uint32_t)V.tiles_x), ty = (int)(lt / (uint32_t)V.tiles_x);
  const int px = tx * TW + (int)(threadIdx.x % TW), py = ty * TH + (int)(threadIdx.x / TW);
  const bool inside = px < V.W && py < V.H;
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  const uint2 rg = ranges[tile];
  const int lane = threadIdx.x & 63;

  const size_t HW = (size_t)V.W * V.H;
  const size_t pix = inside ? (size_t)py * V.W + px : 0;
  const uint32_t last = inside ? n_contrib[V.pix_base + pix] : 0u;
  float T = inside ? T_final[V.pix_base + pix] : 1.0f;
  float gC0 = 0.f, gC1 = 0.f, gC2 = 0.f, gD = 0.f, gA = 0.f;
  if (inside) {
    if (V.g_rgb) { gC0 = V.g_rgb[pix]; gC1 = V.g_rgb[HW + pix]; gC2 = V.g_rgb[2 * HW + pix]; }
    if (V.g_depth) gD = V.g_depth[pix];
    if (V.g_alpha) gA = V.g_alpha[pix];
  }
  // the walk starts after the last entry any pixel of the tile blended
  uint32_t m = last;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off, 64));
  if (lane == 0) smax[threadIdx.x >> 6] = m;
  __syncthreads();
  uint32_t max_last = 0;
#pragma unroll
  for (int w = 0; w < BS / 64; ++w) max_last = max(max_last, smax[w]);

  float S = 0.f;  // sum over blended entries behind the current one of alpha T f
  for (int end = (int)max_last; end > 0; end -= BS) {
    const int begin = end - BS > 0 ? end - BS : 0;
    __syncthreads();
    {
      const int j = begin + (int)threadIdx.x;
      if (j < end) {
        const uint32_t rec = vals[rg.x + (uint32_t)j];
        sRec[threadIdx.x] = rec;
        sA[threadIdx.x] = pa[rec];
        sB[threadIdx.x] = pb[rec];
        sC[threadIdx.x] = pc[rec];
      }
    }
    __syncthreads();
    for (int j = end - 1; j >= begin; --j) {
      const int slot = j - begin;
      float g[kNumAcc];
#pragma unroll
      for (int k = 0; k < kNumAcc; ++k) g[k] = 0.f;
      bool has = false;
      if ((uint32_t)j < last) {
        const float4 A = sA[slot], B = sB[slot];
        const Falloff f = falloff(A, B, pxc, pyc);
        if (f.alpha >= kAlphaMin) {
          has = true;
          T = T / (1.0f - f.alpha);
          const float4 c = sC[slot];
          const float fj = gC0 * c.x + gC1 * c.y + gC2 * c.z + gD * A.z + gA;
          const float dLda = T * fj - S / (1.0f - f.alpha);
          const float w = f.alpha * T;
          S = fmaf(w, fj, S);
          g[6] = w * gC0;
          g[7] = w * gC1;
          g[8] = w * gC2;
          g[9] = w * gD;
          if (f.raw < kAlphaMax) {
            const float ds = -dLda * f.alpha;  // dL/dsigma
            g[0] = ds * (B.x * f.dx + B.y * f.dy);
            g[1] = ds * (B.y * f.dx + B.z * f.dy);
            g[2] = ds * 0.5f * f.dx * f.dx;
            g[3] = ds * f.dx * f.dy;
            g[4] = ds * 0.5f * f.dy * f.dy;
            g[5] = dLda * f.G;
          }
        }
      }
      if (__ballot(has) != 0ull) {
#pragma unroll
        for (int k = 0; k < kNumAcc; ++k) g[k] = wave_sum(g[k]);
        float mine = g[0];
#pragma unroll
        for (int k = 1; k < kNumAcc; ++k) mine = lane == k ? g[k] : mine;
        if (lane < kNumAcc) unsafeAtomicAdd(acc + (size_t)sRec[slot] * kNumAcc + lane, mine);
      }
    }
  }
}

template <int TW, int TH>
__global__ void __launch_bounds__(TW * TH) composite_backward_kernel(
    const CallTables* __restrict__ tab, const float4* __restrict__ pa, const float4* __restrict__ pb,
    const float4* __restrict__ pc, const uint2* __restrict__ ranges, const uint32_t* __restrict__ vals,
    const float* __restrict__ T_final, const uint32_t* __restrict__ n_contrib, float* __restrict__ acc,
    uint32_t* __restrict__ queue, uint32_t n_tiles) {
  __shared__ BwdShared<TW, TH> sh;
  __shared__ uint32_t slot;
  if (queue == nullptr) {
    backward_tile<TW, TH>(tab, pa, pb, pc, ranges, vals, T_final, n_contrib, acc, blockIdx.x, sh);
  } else {
    for (uint32_t t = next_tile(queue, &slot); t < n_tiles; t = next_tile(queue, &slot))
      backward_tile<TW, TH>(tab, pa, pb, pc, ranges, vals, T_final, n_contrib, acc, t, sh);
  }
}

template <int TW, int TH>
hipError_t launch_fwd_t(const CallTables* d_tab, const CallTables& h, const ProjBuffers pb, const uint2* ranges,
                        const uint32_t* vals, float* T_final, uint32_t* n_contrib, Counters* cnt, uint32_t* queue,
                        uint32_t blocks, hipStream_t s) {
  const uint32_t grid = queue ? blocks : h.n_tiles;
  hipLaunchKernelGGL((composite_forward_kernel<TW, TH>), dim3(grid), dim3(TW * TH), 0, s, d_tab, pb.a, pb.b, pb.c,
                     ranges, vals, T_final, n_contrib, cnt, queue, h.n_tiles);
  return hipGetLastError();
}

template <int TW, int TH>
hipError_t launch_bwd_t(const CallTables* d_tab, const CallTables& h, const ProjBuffers pb, const uint2* ranges,
                        const uint32_t* vals, const float* T_final, const uint32_t* n_contrib, float* acc,
                        uint32_t* queue, uint32_t blocks, hipStream_t s) {
  const uint32_t grid = queue ? blocks : h.n_tiles;
  hipLaunchKernelGGL((composite_backward_kernel<TW, TH>), dim3(grid), dim3(TW * TH), 0, s, d_tab, pb.a, pb.b, pb.c,
                     ranges, vals, T_final, n_contrib, acc, queue, h.n_tiles);
  return hipGetLastError();
}

}  // namespace

bool tile_shape_supported(int tw, int th) {
  return (tw == 16 && th == 16) || (tw == 16 && th == 8) || (tw == 8 && th == 8) || (tw == 32 && th == 8);
}

hipError_t launch_composite_forward(const CallTables* d_tab, const CallTables& h, const ProjBuffers pb,
                                    const uint2* ranges, const uint32_t* vals, float* T_final, uint32_t* n_contrib,
                                    Counters* cnt, int tile_w, int tile_h, uint32_t* queue, uint32_t blocks,
                                    hipStream_t s) {
  if (h.n_tiles == 0) return hipSuccess;
#define VPGS_FWD(TW, TH) \
  if (tile_w == TW && tile_h == TH) \
    return launch_fwd_t<TW, TH>(d_tab, h, pb, ranges, vals, T_final, n_contrib, cnt, queue, blocks, s);
  VPGS_FWD(16, 16) VPGS_FWD(16, 8) VPGS_FWD(8, 8) VPGS_FWD(32, 8)
#undef VPGS_FWD
  return hipErrorInvalidValue;
}

hipError_t launch_composite_backward(const CallTables* d_tab, const CallTables& h, const ProjBuffers pb,
                                     const uint2* ranges, const uint32_t* vals, const float* T_final,
                                     const uint32_t* n_contrib, float* acc, int tile_w, int tile_h, uint32_t* queue,
                                     uint32_t blocks, hipStream_t s) {
  if (h.n_tiles == 0) return hipSuccess;
#define VPGS_BWD(TW, TH) \
  if (tile_w == TW && tile_h == TH) \
    return launch_bwd_t<TW, TH>(d_tab, h, pb, ranges, vals, T_final, n_contrib, acc, queue, blocks, s);
  VPGS_BWD(16, 16) VPGS_BWD(16, 8) VPGS_BWD(8, 8) VPGS_BWD(32, 8)
#undef VPGS_BWD
  return hipErrorInvalidValue;
}

}  // namespace vpgs
