// composite.hip -- per-tile front-to-back alpha compositing and its
// backward.
//
// One workgroup per (view, tile); one thread per pixel, each wavefront an
// 8x8 quadrant of the tile.  Each tile walks its
// depth-sorted slice of the pair list in batches staged in LDS (every pixel
// of the tile reads the same Gaussian, so LDS reads broadcast).  A pixel
// stops at the first Gaussian that would take its transmittance under 1e-4;
// the divergent per-pixel loop retires whole wavefronts once all their lanes
// are done, and the workgroup leaves the batch loop once a barrier count
// shows every pixel done.
//
// The backward walks the same slice in reverse from the last blended entry,
// in the forward's batches, recovers the transmittance by division and
// recomputes alpha with the forward's exact instruction sequence (nothing per
// (pixel, Gaussian) is stored; per (wavefront, batch) the forward leaves the
// bits of the entries that reach the wavefront's quadrant, so the backward
// does not test them again).  Per-Gaussian gradients are reduced across the
// wavefront before one set of atomic adds per (wavefront, Gaussian).
//
// A batch holds NB entries: half, once or twice the tile's pixel count (a
// multiple of 64), so each thread stages at most two entries per batch.
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

// Per-Gaussian constants staged in LDS for the per-pixel loops: the conic
// pre-scaled so that alpha = min(0.99, 2^e) with
//   e = -log2(e) (Qa dx^2 + 2 Qb dx dy + Qc dy^2) / 2 + log2(o),
// i.e. o exp(-sigma) with the constant factors and the opacity folded in.
// Forward and backward stage and evaluate it with the same instructions, so
// the backward recomputes bit-identical alpha values.
__device__ __forceinline__ float4 stage_exponent(const float4 A, const float4 B) {
  return make_float4(B.x * kNegHalfLog2e, B.y * kNegLog2e, B.z * kNegHalfLog2e, __log2f(A.w));
}

struct Falloff { float dx, dy, raw, alpha; };
__device__ __forceinline__ Falloff falloff(const float4 A, const float4 E, float pxc, float pyc) {
#pragma clang fp contract(off)
  Falloff f;
  f.dx = A.x - pxc;
  f.dy = A.y - pyc;
  const float t = fmaf(E.x, f.dx, E.y * f.dy);          // Qa' dx + Qb' dy
  const float e = fmaf(t, f.dx, fmaf(E.z * f.dy, f.dy, E.w));
  f.raw = __builtin_amdgcn_exp2f(e);
  f.alpha = fminf(kAlphaMax, f.raw);
  return f;
}

// Staged entry e lives in slot e + 1 of the LDS arrays; slot 0 is a sentinel
// (staged once per workgroup) whose exponent is -inf, so alpha is 0 there and
// nothing is blended.  Hit lists hold LDS byte offsets (16 x slot) into the
// slot arrays, so a list entry is the address of its Gaussian's data, and are
// padded with the sentinel's offset 0 to a multiple of kGroup entries; the
// per-pixel loops then run whole groups without per-entry bounds tests, and
// the forward checks for early termination between groups.
constexpr int kGroup = 8;
constexpr float kLog2AlphaMin = -7.99435343685885793769f;  // log2(1/255)
constexpr float kNegInf = -__builtin_inff();

template <int TW, int TH, int NB>
struct FwdShared {
  float4 A[NB + 1], E[NB + 1], C[NB + 1];  // by slot
  float2 V[NB];  // the quadrant test's vertex factors (ra, rc) of the record, by entry
  alignas(16) uint32_t hits[(TW * TH) / 64][NB + kGroup];  // per wavefront: offsets of the entries that reach its quadrant
};

// The slot array element at byte offset o (a hit-list entry), and its
// first two components.
__device__ __forceinline__ const float4& at_offset(const float4* a, uint32_t o) {
  return *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(a) + o);
}
__device__ __forceinline__ float2 at_offset2(const float4* a, uint32_t o) {
  return *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(a) + o);
}

// Each wavefront owns an 8x8 quadrant of its tile (lane -> (lane % 8,
// lane / 8)) and keeps in its hit list only the Gaussians that can reach
// alpha >= 1/255 at one of the quadrant's pixel centres.
template <int TW, int TH>
struct Quadrant {
  int px, py;            // this thread's pixel
  float x0, x1, y0, y1;  // pixel-centre bounds of the wavefront's quadrant
  __device__ __forceinline__ Quadrant(int tx, int ty) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int qx = wave % (TW / 8), qy = wave / (TW / 8);
    const int bx = tx * TW + qx * 8, by = ty * TH + qy * 8;
    px = bx + (lane & 7);
    py = by + (lane >> 3);
    x0 = (float)bx + 0.5f;
    x1 = x0 + 7.0f;
    y0 = (float)by + 0.5f;
    y1 = y0 + 7.0f;
  }
  // Whether the staged Gaussian (A, E) can reach alpha >= 1/255 at a pixel
  // centre of the quadrant.  Its exponent is e(d) = E.w - f(d) with
  // f(d) = a dx^2 + b dx dy + c dy^2 (a = -E.x, b = -E.y, c = -E.z, d = mean
  // - pixel centre), a positive-definite form, so alpha >= 1/255 somewhere
  // in the quadrant iff E.w - min f >= log2(1/255) over the rectangle of
  // pixel centres.  f decreases along the segment from any point of the
  // rectangle to the mean, and that segment leaves the rectangle through an
  // edge facing the mean, so the minimum lies on the facing vertical edge
  // (x the mean's x clamped to the rectangle) or the facing horizontal one;
  // along each, f is a 1-D quadratic minimised at its clamped vertex (with
  // the mean inside, both give f = 0).  The margin covers the float32
  // rounding of f here and in the per-pixel evaluation (a few ulps of the
  // largest |term| over the rectangle), so every pixel whose float32 alpha
  // passes the cutoff is kept: the test only removes work.
  __device__ __forceinline__ bool reaches(const float4 A, const float4 E, const float2 V) const {
    const float a = -E.x, b = -E.y, c = -E.z;
    const float dx0 = A.x - x1, dx1 = A.x - x0, dy0 = A.y - y1, dy1 = A.y - y0;
    const float ra = V.x, rc = V.y;  // 1 / (2a), 1 / (2c), from the projection
    auto f = [&](float dx, float dy) { return fmaf(fmaf(b, dy, a * dx), dx, c * dy * dy); };
    const float dxe = fminf(fmaxf(0.0f, dx0), dx1);  // mean - nearest x of the rectangle
    const float dye = fminf(fmaxf(0.0f, dy0), dy1);
    const float ev = f(dxe, fminf(fmaxf(-b * dxe * rc, dy0), dy1));
    const float eh = f(fminf(fmaxf(-b * dye * ra, dx0), dx1), dye);
    const float fmin = fminf(ev, eh);
    const float mx = fmaxf(dx0 * dx0, dx1 * dx1), my = fmaxf(dy0 * dy0, dy1 * dy1);
    // |b dx dy| <= |b| sqrt(mx my) <= |b| (mx + my) / 2
    const float fabs_max = fmaf(a, mx, fmaf(fabsf(b), 0.5f * (mx + my), c * my));
    const float margin = fmaf(16.0f * 1.1920929e-7f, fabs_max + fabsf(E.w), 1e-6f);
    return E.w - fmin >= kLog2AlphaMin - margin;
  }
};

// Compacts the staged entries [0, n) that reach the wavefront's quadrant
// into list[] (as slot offsets), in staging order, pads it with the
// sentinel's offset to a multiple of kGroup and returns the number of hits
// (the same in every lane); lane 0 also stores the batch's hit bits (one
// 64-bit word per 64 entries) in mask_out, from which the backward rebuilds
// the list.  Lane l tests entries l, l + 64, ...; a ballot and a lane-prefix
// count give each hit its place.  All lanes of the wavefront must be active;
// the list is read after the next workgroup barrier.
template <int NB, int TW, int TH>
__device__ __forceinline__ int wave_hits(const float4* A, const float4* E, const float2* V, int n,
                                         const Quadrant<TW, TH>& q, uint32_t* list, uint64_t* mask_out) {
  const int lane = threadIdx.x & 63;
  int count = 0;
#pragma unroll
  for (int k = 0; k < NB / 64; ++k) {
    const int e = k * 64 + lane;
    const bool hit = e < n && q.reaches(A[e + 1], E[e + 1], V[e]);
    const uint64_t m = __ballot(hit);
    const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    if (hit) list[count + below] = (uint32_t)(e + 1) * (uint32_t)sizeof(float4);
    if (lane == 0) mask_out[k] = m;
    count += __popcll(m);
  }
  if (lane < ((count + kGroup - 1) & ~(kGroup - 1)) - count) list[count + lane] = 0u;
  return count;
}

// The backward's list of a batch from the forward's masks: the entries
// below n whose bit is set, in descending order, as slot offsets, padded
// with the sentinel's offset to a multiple of kBwdGroup.  All lanes of the
// wavefront must be active.
constexpr int kBwdGroup = 4;
template <int NB>
__device__ __forceinline__ int mask_hits_desc(const uint64_t* mask, int n, uint32_t* list) {
  const int lane = threadIdx.x & 63;
  int count = 0;
#pragma unroll
  for (int k = NB / 64 - 1; k >= 0; --k) {
    const int lo = k * 64;
    uint64_t m = mask[k];
    if (n <= lo) m = 0ull;
    else if (n < lo + 64) m &= (1ull << (n - lo)) - 1ull;
    const int above = __popcll((m >> lane) >> 1);  // set bits of the higher lanes
    if ((m >> lane) & 1ull) list[count + above] = (uint32_t)(lo + lane + 1) * (uint32_t)sizeof(float4);
    count += __popcll(m);
  }
  if (lane < ((count + kBwdGroup - 1) & ~(kBwdGroup - 1)) - count) list[count + lane] = 0u;
  return count;
}

// The per-wavefront hit masks of every (tile, batch) that the forward
// composites: NB/64 words of 64 bits per wavefront (WV wavefronts per
// tile).  The batches of a tile take consecutive slots from first_slot =
// start / NB + tile (start = the tile's first pair): the slots of
// consecutive tiles do not overlap, and every slot is below capacity / NB +
// n_tiles.
template <int NB, int WV>
__device__ __forceinline__ size_t batch_mask_index(uint32_t start, uint32_t tile, int batch, int wave) {
  const size_t slot = (size_t)(start / NB) + tile + (size_t)batch;
  return (slot * WV + wave) * (NB / 64);
}

template <int TW, int TH, int NB, bool COUNT>
__device__ __forceinline__ void forward_tile(const CallTables* __restrict__ tab, const float4* __restrict__ recs,
                                             const uint2* __restrict__ ranges,
                                             const uint32_t* __restrict__ vals, float* __restrict__ T_final,
                                             uint32_t* __restrict__ n_contrib, uint64_t* __restrict__ masks,
                                             uint32_t tile, FwdShared<TW, TH, NB>& sh, uint32_t& ne, uint32_t& nb,
                                             uint32_t& nsteps) {
  constexpr int BS = TW * TH;     // threads: one per pixel
  constexpr int WV = BS / 64;     // wavefronts per tile
  constexpr int PER = NB > BS ? NB / BS : 1;  // entries each thread stages
  const ViewDesc& V = tab->views[view_of_tile(tab, tile)];
  const uint32_t lt = tile - V.tile_base;
  const int tx = (int)(lt % (uint32_t)V.tiles_x), ty = (int)(lt / (uint32_t)V.tiles_x);
  const Quadrant<TW, TH> q(tx, ty);
  const int px = q.px, py = q.py;
  const bool inside = px < V.W && py < V.H;
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  const uint2 rg = ranges[tile];
  uint32_t* hits = sh.hits[threadIdx.x >> 6];

  float T = 1.0f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f;
  uint32_t last = 0;
  bool done = !inside;

  // batch i + 1 is loaded into registers while batch i is tested and
  // composited, so a long list does not wait on each batch's loads
  float4 pA[PER], pR[PER], pC[PER];
  float2 pV[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    pA[k] = pR[k] = pC[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    pV[k] = make_float2(0.f, 0.f);
    const uint32_t e = (uint32_t)(k * BS) + threadIdx.x;
    if (e < (uint32_t)NB && rg.x + e < rg.y) {
      const float4* r = recs + rec_slot(vals[rg.x + e], 0);
      pA[k] = r[0]; pR[k] = r[1]; pC[k] = r[2]; pV[k] = reinterpret_cast<const float2*>(r + 3)[1];
    }
  }
  for (uint32_t start = rg.x; start < rg.y; start += NB) {
    if (__syncthreads_count(done) == BS) break;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const uint32_t e = (uint32_t)(k * BS) + threadIdx.x;
      if (e < (uint32_t)NB && start + e < rg.y) {
        sh.A[e + 1] = pA[k];
        sh.E[e + 1] = stage_exponent(pA[k], pR[k]);
        sh.C[e + 1] = pC[k];
        sh.V[e] = pV[k];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const uint32_t e = (uint32_t)(k * BS) + threadIdx.x;
      const uint32_t nidx = start + NB + e;
      if (e < (uint32_t)NB && nidx < rg.y) {
        const float4* r = recs + rec_slot(vals[nidx], 0);
        pA[k] = r[0]; pR[k] = r[1]; pC[k] = r[2]; pV[k] = reinterpret_cast<const float2*>(r + 3)[1];
      }
    }
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint64_t* wm = masks + batch_mask_index<NB, WV>(rg.x, tile, (int)((start - rg.x) / NB), wave);
    const int nhit = wave_hits<NB>(sh.A, sh.E, sh.V, (int)min((uint32_t)NB, rg.y - start), q, hits, wm);
    __syncthreads();
    uint32_t lb = 0;  // offset of this pixel's last blended entry of the batch (0: none)
    int g = 0;
    for (; g < nhit && __ballot(!done) != 0ull; g += kGroup) {
      // the group's offsets in two 16-byte reads, so every entry's data
      // reads can issue without waiting on a list read of its own
      uint32_t ho[kGroup];
#pragma unroll
      for (int u = 0; u < kGroup; u += 4) {
        const uint4 h4 = *reinterpret_cast<const uint4*>(hits + g + u);
        ho[u] = h4.x;
        ho[u + 1] = h4.y;
        ho[u + 2] = h4.z;
        ho[u + 3] = h4.w;
      }
#pragma unroll
      for (int u = 0; u < kGroup; ++u) {
        const uint32_t o = ho[u];
        const float2 P = at_offset2(sh.A, o);
        const float4 E = at_offset(sh.E, o);
        const Falloff f = falloff(make_float4(P.x, P.y, 0.f, 0.f), E, pxc, pyc);
        const float4 c = at_offset(sh.C, o);
        const float Az = at_offset(sh.A, o).z;
        if (COUNT) ne += (g + u < nhit && !done) ? 1u : 0u;
        const bool ok = !done && f.alpha >= kAlphaMin;
        // T (1 - alpha) as T - alpha T in one fused operation (rounded once)
        const float Tn = fmaf(-f.alpha, T, T);
        const bool low = Tn < kTransMin;
        const bool blend = ok && !low;
        if (blend) {
          const float w = f.alpha * T;
          C0 = fmaf(w, c.x, C0);
          C1 = fmaf(w, c.y, C1);
          C2 = fmaf(w, c.z, C2);
          D = fmaf(w, Az, D);
          T = Tn;
          lb = o;
          if (COUNT) nb += 1u;
        }
        done = done || (ok && low);
      }
    }
    // the pair index after the blended entry: (start - rg.x) + its entry + 1
    if (lb != 0u) last = start - rg.x + lb / (uint32_t)sizeof(float4);
    nsteps += (uint32_t)min(g, nhit);  // the same in every lane of the wavefront
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

// Work counters: wave sums (the step count is the same in every lane:
// lane 0's is added) summed in LDS (wg[], zeroed by thread 0 before the
// first barrier of the kernel), then one global atomic per counter and
// workgroup, spread over kCountSlots slots.
__device__ __forceinline__ void flush_counts(uint32_t ne, uint32_t nb, uint32_t nsteps, unsigned long long* wg,
                                             Counters* cnt) {
  unsigned long long e = ne, b = nb;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    e += __shfl_xor(e, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&wg[0], e);
    atomicAdd(&wg[1], b);
    atomicAdd(&wg[2], (unsigned long long)nsteps);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int slot = (int)(blockIdx.x % kCountSlots);
    atomicAdd(&cnt->evaluated[slot], wg[0]);
    atomicAdd(&cnt->blended[slot], wg[1]);
    atomicAdd(&cnt->fwd_hits[slot], wg[2]);
  }
}

__device__ __forceinline__ void flush_backward_counts(uint32_t nsteps, uint32_t nactive, unsigned long long* wg,
                                                      Counters* cnt) {
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&wg[0], (unsigned long long)nsteps);
    atomicAdd(&wg[1], (unsigned long long)nactive);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int slot = (int)(blockIdx.x % kCountSlots);
    atomicAdd(&cnt->bwd_hits[slot], wg[0]);
    atomicAdd(&cnt->bwd_active[slot], wg[1]);
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
// (the second bound keeps the forward within 64 VGPRs: eight wavefronts per
// SIMD)
// COUNT: count the evaluations and blends per pixel (instrumentation:
// about four of the step's 27 VALU instructions).
template <int TW, int TH, int NB, bool COUNT>
__global__ void __launch_bounds__(TW * TH, 8) composite_forward_kernel(
    const CallTables* __restrict__ tab, const float4* __restrict__ recs, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ vals, float* __restrict__ T_final, uint32_t* __restrict__ n_contrib,
    uint64_t* __restrict__ masks, const uint32_t* __restrict__ order, Counters* __restrict__ cnt,
    uint32_t* __restrict__ queue, uint32_t n_tiles) {
  __shared__ FwdShared<TW, TH, NB> sh;
  __shared__ uint32_t slot;
  __shared__ unsigned long long wg[3];
  uint32_t ne = 0, nb = 0, nsteps = 0;
  if (threadIdx.x == 0) {  // the sentinel slot (read after the first staging barrier) and the counters
    sh.A[0] = make_float4(0.f, 0.f, 0.f, 0.f);
    sh.E[0] = make_float4(0.f, 0.f, 0.f, kNegInf);
    sh.C[0] = make_float4(0.f, 0.f, 0.f, 0.f);
    wg[0] = wg[1] = wg[2] = 0ull;
  }
  if (queue == nullptr) {
    const uint32_t tile = order[blockIdx.x];
    if (tile < n_tiles)
      forward_tile<TW, TH, NB, COUNT>(tab, recs, ranges, vals, T_final, n_contrib, masks, tile, sh, ne, nb, nsteps);
  } else {
    for (uint32_t t = next_tile(queue, &slot); t < n_tiles; t = next_tile(queue, &slot)) {
      const uint32_t tile = order[t];
      if (tile < n_tiles)
        forward_tile<TW, TH, NB, COUNT>(tab, recs, ranges, vals, T_final, n_contrib, masks, tile, sh, ne, nb, nsteps);
    }
  }
  flush_counts(ne, nb, nsteps, wg, cnt);
}

// ---------------------------------------------------------------------------
// wavefront reduce-scatter of the 10 per-Gaussian gradient values
// ---------------------------------------------------------------------------
// Recursive halving of the 10 values: each step pairs a lane with the one
// that differs in one lane-index bit, keeps half of its values and adds the
// partner's copy of them; a value without a pair is summed in both lanes.
//   bit 5: g[i] with g[5 + i] (v_permlane32_swap exchanges the upper half of
//          one register with the lower half of another, so one swap and one
//          add do a whole pair)                            10 -> 5 values
//   bit 4: (h0, h3) and (h1, h4) by v_permlane16_swap, h2 in both  5 -> 3
//   bit 3: (a, b) by DPP row rotate 8 (lane xor 8), c in both     3 -> 2
//   bit 2: (x, c) by DPP row half-mirror (lane xor 7)             2 -> 1
//   bits 0-1: sums over the quad (DPP quad permutations).
// Lane L ends with the wave total of slot 5 b5 + (b2 ? 2 : 3 b4 + b3) (b =
// bits of L), 25 VALU operations in all.  All lanes of the wavefront must be
// active.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float pair_sum32(float lo, float hi) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float pair_sum16(float lo, float hi) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float wave_reduce_scatter10(const float g[kNumAcc], int lane) {
  const bool b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1;
  float h[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) h[i] = pair_sum32(g[i], g[5 + i]);
  const float a = pair_sum16(h[0], h[3]);
  const float b = pair_sum16(h[1], h[4]);
  float c = pair_sum16(h[2], h[2]);
  const float x = (b3 ? b : a) + dpp<0x128>(b3 ? a : b);  // row_ror:8
  c += dpp<0x128>(c);
  float t = (b2 ? c : x) + dpp<0x141>(b2 ? x : c);        // row_half_mirror
  t += dpp<0xB1>(t);  // quad_perm [1,0,3,2]
  t += dpp<0x4E>(t);  // quad_perm [2,3,0,1]
  return t;
}

__device__ __forceinline__ int scatter_slot(int lane) {
  const int b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1, b4 = (lane >> 4) & 1, b5 = (lane >> 5) & 1;
  return 5 * b5 + (b2 ? 2 : 3 * b4 + b3);
}

// One lane per slot: the first lane of a quad, and for slot 5 b5 + 2 (held
// by every lane with b2 set) only the one with b3 = b4 = 0.
__device__ __forceinline__ bool scatter_writer(int lane) {
  return (lane & 3) == 0 && (((lane >> 2) & 1) == 0 || ((lane >> 3) & 3) == 0);
}

static_assert((uint64_t)VPGS_MAX_RECORDS * kNumAcc * sizeof(float) < (1ull << 32),
              "accumulator rows addressed by 32-bit byte offsets");

template <int TW, int TH, int NB>
struct BwdShared {
  float4 A[NB + 1], E[NB + 1], C[NB + 1];  // by slot; C = (r, g, b, bits of the accumulator row offset)
  alignas(16) uint32_t hits[(TW * TH) / 64][NB + kBwdGroup];  // per wavefront, descending
  uint32_t maxlast[(TW * TH) / 64];
};

template <int TW, int TH, int NB>
__device__ __forceinline__ void backward_tile(const CallTables* __restrict__ tab, const float4* __restrict__ recs,
                                              const uint2* __restrict__ ranges,
                                              const uint32_t* __restrict__ vals, const float* __restrict__ T_final,
                                              const uint32_t* __restrict__ n_contrib, float* __restrict__ acc,
                                              const uint64_t* __restrict__ masks, uint32_t tile,
                                              BwdShared<TW, TH, NB>& sh, uint32_t& nsteps, uint32_t& nactive) {
  constexpr int BS = TW * TH;  // threads: one per pixel
  constexpr int WV = BS / 64;
  const ViewDesc& V = tab->views[view_of_tile(tab, tile)];
  const uint32_t lt = tile - V.tile_base;
  const int tx = (int)(lt % (uint32_t)V.tiles_x), ty = (int)(lt / (uint32_t)V.tiles_x);
  const Quadrant<TW, TH> q(tx, ty);
  const int px = q.px, py = q.py;
  const bool inside = px < V.W && py < V.H;
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  const uint2 rg = ranges[tile];
  const int lane = threadIdx.x & 63;
  const int slot_id = scatter_slot(lane);
  const bool writer = scatter_writer(lane);

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
  // the walk starts after the last entry any pixel of the tile blended; a
  // wavefront skips the entries after its own last one
  uint32_t wave_last = last;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) wave_last = max(wave_last, (uint32_t)__shfl_xor((int)wave_last, off, 64));
  wave_last = __builtin_amdgcn_readfirstlane(wave_last);  // the same in every lane
  if (lane == 0) sh.maxlast[threadIdx.x >> 6] = wave_last;
  __syncthreads();
  uint32_t max_last = 0;
#pragma unroll
  for (int w = 0; w < WV; ++w) max_last = max(max_last, sh.maxlast[w]);

  float S = 0.f;  // sum over blended entries behind the current one of alpha T f
  // the forward's batches, last first (their hit masks are the forward's)
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int b = (int)((max_last + NB - 1) / NB) - 1; b >= 0; --b) {
    const int begin = b * NB;
    const int end = min(begin + NB, (int)max_last);
    __syncthreads();
#pragma unroll
    for (int e = (int)threadIdx.x; e < NB; e += BS) {
      const int j = begin + e;
      if (j < end) {
        const uint32_t rec = vals[rg.x + (uint32_t)j];
        const float4* r = recs + rec_slot(rec, 0);
        const float4 A = r[0];
        const float4 c = r[2];
        sh.A[e + 1] = A;
        sh.E[e + 1] = stage_exponent(A, r[1]);
        // the record's accumulator row as a byte offset (below 2^32: the
        // host bounds the records by VPGS_MAX_RECORDS), carried in the
        // colour's free lane
        sh.C[e + 1] = make_float4(c.x, c.y, c.z, __uint_as_float(rec * (uint32_t)(kNumAcc * sizeof(float))));
      }
    }
    __syncthreads();
    // entries of this wavefront: those before its own last blended one
    uint32_t* hits = sh.hits[wave];
    const int nhit = mask_hits_desc<NB>(masks + batch_mask_index<NB, WV>(rg.x, tile, b, wave),
                                        min(end, (int)wave_last) - begin, hits);
    __syncthreads();
    // this pixel's entries are those before its last blended one: offsets
    // below 16 (last - begin + 1); the padding (offset 0) has alpha 0
    const int lim_slot = min(max((int)last - begin + 1, 0), NB + 1);
    const uint32_t lim = (uint32_t)lim_slot * (uint32_t)sizeof(float4);
    nsteps += (uint32_t)nhit;
    for (int i0 = 0; i0 < nhit; i0 += kBwdGroup) {
    const uint4 h4 = *reinterpret_cast<const uint4*>(hits + i0);
#pragma unroll
    for (int u = 0; u < kBwdGroup; ++u) {
      const uint32_t o = u == 0 ? h4.x : u == 1 ? h4.y : u == 2 ? h4.z : h4.w;
      const float4 A = at_offset(sh.A, o);
      const Falloff f = falloff(A, at_offset(sh.E, o), pxc, pyc);
      const bool valid = o < lim && f.alpha >= kAlphaMin;
      if (__ballot(valid) == 0ull) continue;
      ++nactive;
      const float4 c = at_offset(sh.C, o);
      // invalid lanes take alpha = 0: then 1 / (1 - alpha) = 1 exactly, so
      // they keep T and add nothing, with no further selects
      const float a = valid ? f.alpha : 0.0f;
      const float r1m = __builtin_amdgcn_rcpf(1.0f - a);
      const float Tj = T * r1m;
      const float fj = fmaf(gC0, c.x, fmaf(gC1, c.y, fmaf(gC2, c.z, fmaf(gD, A.z, gA))));
      const float dLda = Tj * fj - S * r1m;
      const float w = a * Tj;
      S = fmaf(w, fj, S);
      T = Tj;
      // s = dL/dalpha * alpha where alpha is not clamped (0 where it is):
      // dL/dsigma = -s and dL/do = s / o (the sum of s is accumulated; the
      // projection backward divides by o).  The conic terms are accumulated
      // as moments of s over the pixel offsets d = mean - pixel centre,
      //   (sum s dx, sum s dy, sum s dx^2, sum s dx dy, sum s dy^2),
      // which the projection backward turns into dL/du, dL/dv = -Q (M0, M1)
      // and dL/d(Qa, Qb, Qc) = -(M2 / 2, M3, M4 / 2).
      const float sg = (valid && f.raw < kAlphaMax) ? dLda * f.raw : 0.0f;
      const float sx = sg * f.dx, sy = sg * f.dy;
      float g[kNumAcc];
      g[0] = sx;
      g[1] = sy;
      g[2] = sx * f.dx;
      g[3] = sx * f.dy;
      g[4] = sy * f.dy;
      g[5] = sg;
      g[6] = w * gC0;
      g[7] = w * gC1;
      g[8] = w * gC2;
      g[9] = w * gD;
      const float mine = wave_reduce_scatter10(g, lane);
      // an empty statement that consumes the sum here, so its last DPP step
      // stays fused into one add instead of moving into the writers' branch
      asm volatile("" ::"v"(mine));
      if (writer)
        unsafeAtomicAdd(reinterpret_cast<float*>(reinterpret_cast<char*>(acc) + (__float_as_uint(c.w) + 4u * slot_id)),
                        mine);
    }
    }
  }
}

template <int TW, int TH, int NB>
__global__ void __launch_bounds__(TW * TH) composite_backward_kernel(
    const CallTables* __restrict__ tab, const float4* __restrict__ recs, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ vals,
    const float* __restrict__ T_final, const uint32_t* __restrict__ n_contrib, float* __restrict__ acc,
    const uint64_t* __restrict__ masks, const uint32_t* __restrict__ order, uint32_t* __restrict__ queue,
    Counters* __restrict__ cnt, uint32_t n_tiles) {
  __shared__ BwdShared<TW, TH, NB> sh;
  __shared__ uint32_t slot;
  __shared__ unsigned long long wg[2];
  uint32_t nsteps = 0, nactive = 0;
  if (threadIdx.x == 0) {  // the sentinel slot (read after the first staging barrier) and the counters
    sh.A[0] = make_float4(0.f, 0.f, 0.f, 0.f);
    sh.E[0] = make_float4(0.f, 0.f, 0.f, kNegInf);
    sh.C[0] = make_float4(0.f, 0.f, 0.f, 0.f);
    wg[0] = wg[1] = 0ull;
  }
  if (queue == nullptr) {
    const uint32_t tile = order[blockIdx.x];
    if (tile < n_tiles)
      backward_tile<TW, TH, NB>(tab, recs, ranges, vals, T_final, n_contrib, acc, masks, tile, sh, nsteps, nactive);
  } else {
    for (uint32_t t = next_tile(queue, &slot); t < n_tiles; t = next_tile(queue, &slot)) {
      const uint32_t tile = order[t];
      if (tile < n_tiles)
        backward_tile<TW, TH, NB>(tab, recs, ranges, vals, T_final, n_contrib, acc, masks, tile, sh, nsteps,
                                  nactive);
    }
  }
  flush_backward_counts(nsteps, nactive, wg, cnt);
}

template <int TW, int TH, int NB>
hipError_t launch_fwd_t(const CallTables* d_tab, const CallTables& h, const ProjBuffers pb, const uint2* ranges,
                        const uint32_t* vals, const uint32_t* order, float* T_final, uint32_t* n_contrib,
                        uint64_t* masks, Counters* cnt, bool count, uint32_t* queue, uint32_t blocks,
                        hipStream_t s) {
  const uint32_t grid = queue ? blocks : h.n_tiles;
  if (count)
    hipLaunchKernelGGL((composite_forward_kernel<TW, TH, NB, true>), dim3(grid), dim3(TW * TH), 0, s, d_tab, pb.rec,
                       ranges, vals, T_final, n_contrib, masks, order, cnt, queue, h.n_tiles);
  else
    hipLaunchKernelGGL((composite_forward_kernel<TW, TH, NB, false>), dim3(grid), dim3(TW * TH), 0, s, d_tab,
                       pb.rec, ranges, vals, T_final, n_contrib, masks, order, cnt, queue, h.n_tiles);
  return hipGetLastError();
}

template <int TW, int TH, int NB>
hipError_t launch_bwd_t(const CallTables* d_tab, const CallTables& h, const ProjBuffers pb, const uint2* ranges,
                        const uint32_t* vals, const uint32_t* order, const float* T_final,
                        const uint32_t* n_contrib, const uint64_t* masks, float* acc, Counters* cnt,
                        uint32_t* queue, uint32_t blocks, hipStream_t s) {
  const uint32_t grid = queue ? blocks : h.n_tiles;
  hipLaunchKernelGGL((composite_backward_kernel<TW, TH, NB>), dim3(grid), dim3(TW * TH), 0, s, d_tab, pb.rec,
                     ranges, vals, T_final, n_contrib, acc, masks, order, queue, cnt, h.n_tiles);
  return hipGetLastError();
}

}  // namespace

bool tile_shape_supported(int tw, int th) {
  return (tw == 16 && th == 16) || (tw == 16 && th == 8) || (tw == 8 && th == 8) || (tw == 32 && th == 8);
}

bool lds_batch_supported(int tw, int th, int nb) {
  const int px = tw * th;
  return tile_shape_supported(tw, th) && nb % 64 == 0 && (2 * nb == px || nb == px || nb == 2 * px);
}

size_t hit_mask_bytes(uint32_t capacity, uint32_t n_tiles, int tile_w, int tile_h, int lds_batch) {
  const size_t nb = (size_t)lds_batch, words = ((size_t)tile_w * tile_h / 64) * (nb / 64);
  return ((size_t)capacity / nb + n_tiles + 1) * words * sizeof(uint64_t);
}

// The built (tile shape, batch) instances: batches of half, once and twice
// the tile's pixels where that is a multiple of 64.
#define VPGS_SHAPES(X)                                                             \
  X(16, 16, 128) X(16, 16, 256) X(16, 16, 512) X(16, 8, 64) X(16, 8, 128) X(16, 8, 256) \
  X(8, 8, 64) X(8, 8, 128) X(32, 8, 128) X(32, 8, 256) X(32, 8, 512)

hipError_t launch_composite_forward(const CallTables* d_tab, const CallTables& h, const ProjBuffers pb,
                                    const uint2* ranges, const uint32_t* vals, const uint32_t* order,
                                    float* T_final, uint32_t* n_contrib, uint64_t* masks, Counters* cnt, bool count,
                                    int tile_w, int tile_h, int lds_batch, uint32_t* queue, uint32_t blocks,
                                    hipStream_t s) {
  if (h.n_tiles == 0) return hipSuccess;
#define VPGS_FWD(TW, TH, NB) \
  if (tile_w == TW && tile_h == TH && lds_batch == NB) \
    return launch_fwd_t<TW, TH, NB>(d_tab, h, pb, ranges, vals, order, T_final, n_contrib, masks, cnt, count, \
                                    queue, blocks, s);
  VPGS_SHAPES(VPGS_FWD)
#undef VPGS_FWD
  return hipErrorInvalidValue;
}

hipError_t launch_composite_backward(const CallTables* d_tab, const CallTables& h, const ProjBuffers pb,
                                     const uint2* ranges, const uint32_t* vals, const uint32_t* order,
                                     const float* T_final, const uint32_t* n_contrib, const uint64_t* masks,
                                     float* acc, Counters* cnt, int tile_w, int tile_h, int lds_batch,
                                     uint32_t* queue, uint32_t blocks, hipStream_t s) {
  if (h.n_tiles == 0) return hipSuccess;
#define VPGS_BWD(TW, TH, NB) \
  if (tile_w == TW && tile_h == TH && lds_batch == NB) \
    return launch_bwd_t<TW, TH, NB>(d_tab, h, pb, ranges, vals, order, T_final, n_contrib, masks, acc, cnt, \
                                    queue, blocks, s);
  VPGS_SHAPES(VPGS_BWD)
#undef VPGS_BWD
  return hipErrorInvalidValue;
}

#undef VPGS_SHAPES

}  // namespace vpgs
