// icp.hip -- the voxel map and frame-to-map registration of the fine
// tracking stage (Section III-B, eq. 10-12).
//
// Voxels: a point p lies in voxel floor(p / v) (FP32 division per axis),
// packed as three 21-bit biased coordinates in a 64-bit key.
//
// Voxel map: the points are sorted by (key, index) -- two stable 32-bit
// radix sorts, low word then high word -- and stored in that order as float4
// (x, y, z, original index).  Each voxel is one run; an open-addressing hash
// table (linear probing, capacity a power of two >= 2 n) maps its key to the
// run's start and min(run length, max_per_voxel), so the stored candidates
// are the voxel's first points by index.
//
// Downsampling: a second hash table takes, per voxel, the minimum index of
// its points (atomicMin); a point is kept iff it is that minimum, and the
// kept indices are compacted in index order.
//
// Registration: a group of lanes per source point (32 for a few thousand
// points, down to one for hundreds of thousands) transforms it (FP32, fixed
// order, no contraction), searches the 27 voxels around it for the nearest
// stored point (squared distance in FP32, ties to the lower index), keeps it
// if d^2 < tau^2, and adds its Geman-McClure-weighted Gauss-Newton terms
// (21 entries of H = sum w J^T J, 6 of g = sum w J^T r, the count and
// sum rho) into a workgroup sum.  One workgroup then adds the workgroup sums
// in FP64, solves H dx = -g by Cholesky and updates T <- Exp(dx) T in FP64.
// The pose lives in device memory between iterations, so a run of
// iterations needs no host round trip; the host checks the stop flag every
// few iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <type_traits>

#include "runtime.h"

namespace vpgs {
namespace {

constexpr uint64_t kEmpty = ~0ull;
constexpr int kVoxBias = 1 << 20;
constexpr int kIcpBlock = 256;
constexpr int kTerms = 29;  // 21 of H (upper triangle, row-major), 6 of g, count, sum rho
constexpr int kItersPerCheck = 8;

struct MapView {
  const float4* pts;       // sorted points (x, y, z, index bits)
  const uint64_t* keys;    // hash keys, kEmpty = free
  const uint2* vals;       // (start, count) of the voxel's run
  uint32_t mask;           // capacity - 1
  float voxel;
};

__device__ __forceinline__ int voxel_coord(float x, float v) {
#pragma clang fp contract(off)
  const float f = fminf(fmaxf(floorf(x / v), -(float)kVoxBias), (float)(kVoxBias - 1));
  return (int)f;
}

__device__ __forceinline__ uint64_t pack_key(int x, int y, int z) {
  return ((uint64_t)(uint32_t)(x + kVoxBias) << 42) | ((uint64_t)(uint32_t)(y + kVoxBias) << 21) |
         (uint64_t)(uint32_t)(z + kVoxBias);
}

__device__ __forceinline__ uint64_t key_of(float x, float y, float z, float v) {
  return pack_key(voxel_coord(x, v), voxel_coord(y, v), voxel_coord(z, v));
}

__device__ __forceinline__ uint32_t hash_slot(uint64_t k, uint32_t mask) {
  k ^= k >> 30;
  k *= 0xbf58476d1ce4e5b9ull;
  k ^= k >> 27;
  k *= 0x94d049bb133111ebull;
  k ^= k >> 31;
  return (uint32_t)k & mask;
}

// Slot holding key k, or -1.  The table is never full, so a free slot ends
// every probe sequence; the bound on the steps is a guard only.
__device__ __forceinline__ int find_slot(const uint64_t* __restrict__ keys, uint32_t mask, uint64_t k) {
  uint32_t s = hash_slot(k, mask);
  for (uint32_t step = 0; step <= mask; ++step) {
    const uint64_t t = keys[s];
    if (t == k) return (int)s;
    if (t == kEmpty) return -1;
    s = (s + 1) & mask;
  }
  return -1;
}

// Slot of key k, inserting it if absent (-1 if the table is full).  A slot's
// key never changes once set, so a (relaxed atomic) read that finds a key is
// final; only a slot read as empty (possibly a stale read) is claimed by
// compare-and-swap.  Points of one voxel mostly find their key already there
// and do not queue on its slot's atomics.
__device__ __forceinline__ int insert_slot(uint64_t* __restrict__ keys, uint32_t mask, uint64_t k) {
  uint32_t s = hash_slot(k, mask);
  for (uint32_t step = 0; step <= mask; ++step) {
    uint64_t cur = __hip_atomic_load(&keys[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cur == kEmpty)
      cur = atomicCAS((unsigned long long*)&keys[s], (unsigned long long)kEmpty, (unsigned long long)k);
    if (cur == kEmpty || cur == k) return (int)s;
    s = (s + 1) & mask;
  }
  return -1;
}

// ---- voxel map build ----------------------------------------------------------

__global__ void vox_key_kernel(const float* __restrict__ p, uint32_t n, float v, uint32_t* __restrict__ lo,
                               uint32_t* __restrict__ hi, uint32_t* __restrict__ idx) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t k = key_of(p[3 * (size_t)i], p[3 * (size_t)i + 1], p[3 * (size_t)i + 2], v);
  lo[i] = (uint32_t)k;
  hi[i] = (uint32_t)(k >> 32);
  idx[i] = i;
}

__global__ void gather_points_kernel(const float* __restrict__ p, const uint32_t* __restrict__ sidx, uint32_t n,
                                     float4* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t s = sidx[i];
  out[i] = make_float4(p[3 * (size_t)s], p[3 * (size_t)s + 1], p[3 * (size_t)s + 2], __uint_as_float(s));
}

__global__ void heads_kernel(const float4* __restrict__ pts, uint32_t n, float v, uint32_t* __restrict__ head) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 a = pts[i];
  bool h = i == 0;
  if (!h) {
    const float4 b = pts[i - 1];
    h = key_of(a.x, a.y, a.z, v) != key_of(b.x, b.y, b.z, v);
  }
  head[i] = h ? 1u : 0u;
}

__global__ void vstart_kernel(const uint32_t* __restrict__ head, const uint32_t* __restrict__ vid, uint32_t n,
                              uint32_t* __restrict__ vstart) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && head[i]) vstart[vid[i]] = i;
}

__global__ void map_insert_kernel(const float4* __restrict__ pts, const uint32_t* __restrict__ vstart,
                                  const uint32_t* __restrict__ nvox, uint32_t n, float v, uint32_t max_per_voxel,
                                  uint64_t* __restrict__ keys, uint2* __restrict__ vals, uint32_t mask) {
  const uint32_t id = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t V = *nvox;
  if (id >= V || id >= n) return;
  const uint32_t start = vstart[id];
  const uint32_t end = id + 1 < V ? vstart[id + 1] : n;
  const float4 a = pts[start];
  const int s = insert_slot(keys, mask, key_of(a.x, a.y, a.z, v));
  if (s >= 0) vals[s] = make_uint2(start, min(end - start, max_per_voxel));
}

// ---- downsampling ------------------------------------------------------------------

// A scan arrives in sweep order, so neighbouring points mostly share a
// voxel: of a run of lanes with one key only the first (the smallest index
// of the run) inserts it and offers its index, and the others, which could
// not win, add no atomics to the same slot.  Runs of one key that are not
// adjacent each insert, which the table and atomicMin resolve.
__global__ void __launch_bounds__(256) ds_insert_kernel(const float* __restrict__ p, uint32_t n, float v,
                                                        uint64_t* __restrict__ keys, uint32_t* __restrict__ first,
                                                        uint32_t mask) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t ii = min(i, n - 1);  // lanes past the end repeat the last point (the same key)
  const uint64_t k = key_of(p[3 * (size_t)ii], p[3 * (size_t)ii + 1], p[3 * (size_t)ii + 2], v);
  const uint32_t klo = (uint32_t)k, khi = (uint32_t)(k >> 32);
  const uint32_t plo = __shfl_up(klo, 1, 64), phi = __shfl_up(khi, 1, 64);
  const bool run_start = (threadIdx.x & 63) == 0 || plo != klo || phi != khi;
  if (i >= n || !run_start) return;
  const int s = insert_slot(keys, mask, k);
  // first[s] only decreases, so a value read at or below i already wins
  if (s >= 0 && __hip_atomic_load(&first[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > i) atomicMin(&first[s], i);
}

__global__ void ds_flag_kernel(const float* __restrict__ p, uint32_t n, float v, const uint64_t* __restrict__ keys,
                               const uint32_t* __restrict__ first, uint32_t mask, uint32_t* __restrict__ flag) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int s = find_slot(keys, mask, key_of(p[3 * (size_t)i], p[3 * (size_t)i + 1], p[3 * (size_t)i + 2], v));
  flag[i] = (s >= 0 && first[s] == i) ? 1u : 0u;
}

__global__ void ds_scatter_kernel(const uint32_t* __restrict__ flag, const uint32_t* __restrict__ pos, uint32_t n,
                                  int32_t* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) out[pos[i]] = (int32_t)i;
}

// ---- registration ----------------------------------------------------------------------

struct Pose32 {
  float R[9], t[3];
};

// Pose and progress of one registration, in device memory.
struct IcpState {
  double T[12];    // sensor-to-map [R | t], row-major
  Pose32 p32;      // T rounded to float32, used by the next correspondence pass
  int32_t done, iterations, count, converged, degenerate, pad;
  float rho;
  float pad2;
};

// Nearest stored point of q among the 27 voxels around it, searched by a
// group of G lanes (lane l takes voxels l, l + G, ..., and each voxel's
// <= max_per_voxel points in order) and reduced across the group by the
// total order (d^2, index).  Every lane of the group returns the result: d^2
// (+inf if no voxel has points), the original index (-1) and the sorted
// position.  Few queries use wide groups (latency), many use narrow ones.
constexpr uint32_t kScan = 4;  // points of a voxel compared per round

template <int G>
__device__ __forceinline__ void group_nearest(const MapView& M, float qx, float qy, float qz, int lane, float& bd,
                                              int32_t& bi, uint32_t& bp) {
#pragma clang fp contract(off)
  bd = __builtin_inff();
  bi = -1;
  bp = 0;
  const int vx = voxel_coord(qx, M.voxel), vy = voxel_coord(qy, M.voxel), vz = voxel_coord(qz, M.voxel);
  for (int nb = lane; nb < 27; nb += G) {
    const int cx = vx + nb / 9 - 1;
    const int cy = vy + (nb / 3) % 3 - 1;
    const int cz = vz + nb % 3 - 1;
    const int s = find_slot(M.keys, M.mask, pack_key(cx, cy, cz));
    if (s >= 0) {
      // kScan points are loaded together; past the end of the run the last
      // point is loaded again, and a point already compared never replaces
      // the best (the comparison is strict in the total order)
      const uint2 run = M.vals[s];
      for (uint32_t j = 0; j < run.y; j += kScan) {
        float4 m[kScan];
        uint32_t at[kScan];
#pragma unroll
        for (int u = 0; u < kScan; ++u) {
          at[u] = run.x + min(j + u, run.y - 1);
          m[u] = M.pts[at[u]];
        }
#pragma unroll
        for (int u = 0; u < kScan; ++u) {
          const float dx = qx - m[u].x, dy = qy - m[u].y, dz = qz - m[u].z;
          const float d2 = (dx * dx + dy * dy) + dz * dz;
          const int32_t id = (int32_t)__float_as_uint(m[u].w);
          const bool take = d2 < bd || (d2 == bd && id < bi);
          bd = take ? d2 : bd;
          bi = take ? id : bi;
          bp = take ? at[u] : bp;
        }
      }
    }
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) {
    const float od = __shfl_xor(bd, off, G);
    const int32_t oi = __shfl_xor(bi, off, G);
    const uint32_t op = __shfl_xor(bp, off, G);
    // an empty lane carries (+inf, -1): it loses to any point
    const bool take = od < bd || (od == bd && oi >= 0 && (bi < 0 || oi < bi));
    bd = take ? od : bd;
    bi = take ? oi : bi;
    bp = take ? op : bp;
  }
}

__device__ __forceinline__ float3 transform(const Pose32& P, float x, float y, float z) {
#pragma clang fp contract(off)
  float3 q;
  q.x = ((P.R[0] * x + P.R[1] * y) + P.R[2] * z) + P.t[0];
  q.y = ((P.R[3] * x + P.R[4] * y) + P.R[5] * z) + P.t[1];
  q.z = ((P.R[6] * x + P.R[7] * y) + P.R[8] * z) + P.t[2];
  return q;
}

template <int G>
__global__ void __launch_bounds__(kIcpBlock) correspond_kernel(MapView M, const float* __restrict__ src, uint32_t n,
                                                               Pose32 P, float tau2, int32_t* __restrict__ nn,
                                                               float* __restrict__ d2out) {
  const uint32_t i = blockIdx.x * (kIcpBlock / G) + threadIdx.x / G;  // uniform over the group
  const int lane = threadIdx.x % G;
  if (i >= n) return;
  const float3 q = transform(P, src[3 * (size_t)i], src[3 * (size_t)i + 1], src[3 * (size_t)i + 2]);
  float bd;
  int32_t bi;
  uint32_t bp;
  group_nearest<G>(M, q.x, q.y, q.z, lane, bd, bi, bp);
  if (lane == 0) {
    if (nn) nn[i] = bd < tau2 ? bi : -1;
    if (d2out) d2out[i] = bd;
  }
}

// Wavefront sum of values held only by the first lane of each G-lane group
// (the other lanes hold zero): the butterfly levels below G would only add
// zeros, so they are skipped; the result (in lane 0) is the same.
template <int G>
__device__ __forceinline__ float wave_sum_groups(float v) {
#pragma unroll
  for (int d = 32; d >= G; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Gauss-Newton terms of the accepted correspondences.  Each lane group
// takes queries group, group + total groups, ... and its lane 0 accumulates
// their terms; the workgroup sum goes to partials[blockIdx.x][kTerms].
// With st non-NULL the pose is read from it and the pass is skipped once the
// registration has stopped.
template <int G>
__global__ void __launch_bounds__(kIcpBlock) linearize_kernel(MapView M, const float* __restrict__ src, uint32_t n,
                                                              Pose32 P, const IcpState* __restrict__ st, float tau2,
                                                              float kappa, float* __restrict__ partials) {
#pragma clang fp contract(off)
  __shared__ float red[kIcpBlock / 64][kTerms];
  if (st != nullptr) {
    if (st->done) return;  // uniform over the grid
    P = st->p32;
  }
  const int lane = threadIdx.x % G;
  float t[kTerms];
#pragma unroll
  for (int k = 0; k < kTerms; ++k) t[k] = 0.f;
  const uint32_t stride = gridDim.x * (kIcpBlock / G);
  for (uint32_t i = blockIdx.x * (kIcpBlock / G) + threadIdx.x / G; i < n; i += stride) {
    const float3 q = transform(P, src[3 * (size_t)i], src[3 * (size_t)i + 1], src[3 * (size_t)i + 2]);
    float bd;
    int32_t bi;
    uint32_t bp;
    group_nearest<G>(M, q.x, q.y, q.z, lane, bd, bi, bp);
    if (lane == 0 && bd < tau2) {
      const float4 m = M.pts[bp];
      const float r[3] = {q.x - m.x, q.y - m.y, q.z - m.z};
      const float e2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
      const float den = kappa + e2;
      const float w = kappa / (den * den);
      // rows of J = [I, -[q]x]
      const float J[3][6] = {{1.f, 0.f, 0.f, 0.f, q.z, -q.y}, {0.f, 1.f, 0.f, -q.z, 0.f, q.x},
                             {0.f, 0.f, 1.f, q.y, -q.x, 0.f}};
      int k = 0;
#pragma unroll
      for (int a = 0; a < 6; ++a)
#pragma unroll
        for (int b = a; b < 6; ++b) t[k++] += w * ((J[0][a] * J[0][b] + J[1][a] * J[1][b]) + J[2][a] * J[2][b]);
#pragma unroll
      for (int a = 0; a < 6; ++a) t[21 + a] += w * ((J[0][a] * r[0] + J[1][a] * r[1]) + J[2][a] * r[2]);
      t[27] += 1.f;
      t[28] += 0.5f * e2 / den;
    }
  }
#pragma unroll
  for (int k = 0; k < kTerms; ++k) {
    const float s = wave_sum_groups<G>(t[k]);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < kTerms) {
    float s = 0.f;
#pragma unroll
    for (int w = 0; w < kIcpBlock / 64; ++w) s += red[w][threadIdx.x];
    partials[(size_t)blockIdx.x * kTerms + threadIdx.x] = s;
  }
}

// FP64 sums of the workgroup partials by one workgroup: kSumSplit threads
// per term each add every kSumSplit-th row in row order (four rows in
// flight), then one thread per term adds its kSumSplit partial sums in
// order.  The order is fixed, so the sums are deterministic.
constexpr int kSumSplit = 8;
static_assert(kSumSplit * kTerms <= kIcpBlock, "one thread per (term, split)");

__device__ void sum_partials(const float* __restrict__ partials, uint32_t nblocks, double* tot) {
  __shared__ double part[kSumSplit][kTerms];
  const int t = threadIdx.x;
  if (t < kSumSplit * kTerms) {
    const int k = t % kTerms, p = t / kTerms;
    double acc = 0.0;
    uint32_t b = (uint32_t)p;
    for (; b + 3 * kSumSplit < nblocks; b += 4 * kSumSplit) {
      const float v0 = partials[(size_t)b * kTerms + k];
      const float v1 = partials[(size_t)(b + kSumSplit) * kTerms + k];
      const float v2 = partials[(size_t)(b + 2 * kSumSplit) * kTerms + k];
      const float v3 = partials[(size_t)(b + 3 * kSumSplit) * kTerms + k];
      acc += (double)v0;
      acc += (double)v1;
      acc += (double)v2;
      acc += (double)v3;
    }
    for (; b < nblocks; b += kSumSplit) acc += (double)partials[(size_t)b * kTerms + k];
    part[p][k] = acc;
  }
  __syncthreads();
  if (t < kTerms) {
    double s = 0.0;
#pragma unroll
    for (int p = 0; p < kSumSplit; ++p) s += part[p][t];
    tot[t] = s;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kIcpBlock) reduce_terms_kernel(const float* __restrict__ partials, uint32_t nblocks, double* __restrict__ out) {
  __shared__ double tot[kTerms];
  sum_partials(partials, nblocks, tot);
  if (threadIdx.x < kTerms) out[threadIdx.x] = tot[threadIdx.x];
}

__device__ __forceinline__ void exp_se3(const double xi[6], double E[12]) {
  const double px = xi[3], py = xi[4], pz = xi[5];
  const double th = sqrt(px * px + py * py + pz * pz);
  const double K[9] = {0.0, -pz, py, pz, 0.0, -px, -py, px, 0.0};
  double K2[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) K2[3 * r + c] = K[3 * r] * K[c] + K[3 * r + 1] * K[3 + c] + K[3 * r + 2] * K[6 + c];
  double a, b, cc;
  if (th < 1e-8) {
    a = 1.0; b = 0.5; cc = 1.0 / 6.0;
  } else {
    double sn, cs;
    sincos(th, &sn, &cs);
    a = sn / th;
    b = (1.0 - cs) / (th * th);
    cc = (th - sn) / (th * th * th);
  }
  double V[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const double I = (k % 4 == 0) ? 1.0 : 0.0;
    E[4 * (k / 3) + k % 3] = I + a * K[k] + b * K2[k];
    V[k] = I + b * K[k] + cc * K2[k];
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) E[4 * r + 3] = V[3 * r] * xi[0] + V[3 * r + 1] * xi[1] + V[3 * r + 2] * xi[2];
}

__device__ __forceinline__ void round_pose(const double T[12], Pose32& p) {
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) p.R[3 * r + c] = (float)T[4 * r + c];
    p.t[r] = (float)T[4 * r + 3];
  }
}

// One Gauss-Newton step from the summed terms (single workgroup).
__global__ void __launch_bounds__(kIcpBlock) solve_kernel(const float* __restrict__ partials, uint32_t nblocks, IcpState* __restrict__ st,
                             double eps, int32_t max_iter) {
  __shared__ double tot[kTerms];
  // the state is read while the partial sums are loaded (they are read even
  // after the registration has stopped, and then not used)
  const int32_t done = st->done;
  double T0[12];
  int32_t iters = 0;
  if (threadIdx.x == 0) {
    for (int q = 0; q < 12; ++q) T0[q] = st->T[q];
    iters = st->iterations;
  }
  sum_partials(partials, nblocks, tot);
  if (done || threadIdx.x != 0) return;
  st->count = (int32_t)tot[27];
  st->rho = (float)tot[28];
  // Every loop below has constant bounds and is unrolled, so that the
  // matrices stay in registers (indexed arrays would live in scratch memory,
  // one memory round trip per dependent access).
  double H[36], g[6];
  int k = 0;
#pragma unroll
  for (int a = 0; a < 6; ++a)
#pragma unroll
    for (int b = a; b < 6; ++b) {
      H[6 * a + b] = tot[k];
      H[6 * b + a] = tot[k];
      ++k;
    }
#pragma unroll
  for (int a = 0; a < 6; ++a) g[a] = tot[21 + a];
  bool ok = st->count >= 6;
  double L[36], inv[6];  // inv[j] = 1 / L[j][j]; only the lower triangle is used
#pragma unroll
  for (int j = 0; j < 6; ++j) {  // Cholesky H = L L^T (not used once a pivot is not positive)
    double d = H[6 * j + j];
#pragma unroll
    for (int q = 0; q < j; ++q) d -= L[6 * j + q] * L[6 * j + q];
    ok = ok && d > 0.0;
    L[6 * j + j] = sqrt(d);
    inv[j] = 1.0 / L[6 * j + j];
#pragma unroll
    for (int r = j + 1; r < 6; ++r) {
      double s = H[6 * r + j];
#pragma unroll
      for (int q = 0; q < j; ++q) s -= L[6 * r + q] * L[6 * j + q];
      L[6 * r + j] = s * inv[j];
    }
  }
  if (!ok) {
    st->degenerate = 1;
    st->done = 1;
    return;
  }
  double y[6], dx[6];
#pragma unroll
  for (int r = 0; r < 6; ++r) {  // L y = -g
    double s = -g[r];
#pragma unroll
    for (int q = 0; q < r; ++q) s -= L[6 * r + q] * y[q];
    y[r] = s * inv[r];
  }
#pragma unroll
  for (int r = 5; r >= 0; --r) {  // L^T dx = y
    double s = y[r];
#pragma unroll
    for (int q = r + 1; q < 6; ++q) s -= L[6 * q + r] * dx[q];
    dx[r] = s * inv[r];
  }
  double E[12], T[12];
  exp_se3(dx, E);
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c)
      T[4 * r + c] = E[4 * r] * T0[c] + E[4 * r + 1] * T0[4 + c] + E[4 * r + 2] * T0[8 + c];
    T[4 * r + 3] = E[4 * r] * T0[3] + E[4 * r + 1] * T0[7] + E[4 * r + 2] * T0[11] + E[4 * r + 3];
  }
  for (int q = 0; q < 12; ++q) st->T[q] = T[q];
  round_pose(T, st->p32);
  st->iterations = ++iters;
  double nrm = 0.0;
  for (int q = 0; q < 6; ++q) nrm += dx[q] * dx[q];
  if (sqrt(nrm) < eps) {
    st->converged = 1;
    st->done = 1;
  } else if (iters >= max_iter) {
    st->done = 1;
  }
}

inline uint32_t blocks_of(uint32_t n, uint32_t b) { return (n + b - 1) / b; }

// Lanes per query: enough lane groups to fill the chip (about 512 k lanes)
// when the queries are few, one lane per query when they are many.
inline int group_lanes(uint32_t n) {
  if (n <= 16384) return 32;
  if (n <= 65536) return 8;
  if (n <= 262144) return 4;
  return 1;
}

// Workgroups of a linearisation pass: one lane group per query up to a cap
// that bounds the partial sums the step adds up.
constexpr uint32_t kMaxLinBlocks = 512;
inline uint32_t linearize_blocks(uint32_t n) {
  return std::max<uint32_t>(1, std::min(blocks_of(n, kIcpBlock / group_lanes(n)), kMaxLinBlocks));
}

template <class F>
void with_group(uint32_t n, F&& f) {
  switch (group_lanes(n)) {
    case 32: f(std::integral_constant<int, 32>()); break;
    case 8: f(std::integral_constant<int, 8>()); break;
    case 4: f(std::integral_constant<int, 4>()); break;
    default: f(std::integral_constant<int, 1>()); break;
  }
}

uint32_t pow2_at_least(uint64_t x) {
  uint64_t c = 1;
  while (c < x) c <<= 1;
  return (uint32_t)c;
}

bool finite_pose(const double* P) {
  for (int k = 0; k < 12; ++k)
    if (!std::isfinite(P[k])) return false;
  return true;
}

void compose(const double* A, const double* B, double* out) {  // [A] [B] as 3x4 rigid maps
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) out[4 * r + c] = A[4 * r] * B[c] + A[4 * r + 1] * B[4 + c] + A[4 * r + 2] * B[8 + c];
    out[4 * r + 3] = A[4 * r] * B[3] + A[4 * r + 1] * B[7] + A[4 * r + 2] * B[11] + A[4 * r + 3];
  }
}

Pose32 pose32_of(const double* P) {
  Pose32 p;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) p.R[3 * r + c] = (float)P[4 * r + c];
    p.t[r] = (float)P[4 * r + 3];
  }
  return p;
}

}  // namespace
}  // namespace vpgs

// Scratch of the allocation-free linearisation (vpgs_icp_linearize_noalloc):
// the workgroup partial sums of one pass, at most kMaxLinBlocks rows of
// kTerms floats (58 KiB).  Every device holds its own copy for the life of
// the process.  Host code never passes this name: it uses the device address
// that hipGetSymbolAddress returned on that device.
constexpr size_t kLinScratchFloats = (size_t)512 * 29;
static_assert(kLinScratchFloats == (size_t)vpgs::kMaxLinBlocks * vpgs::kTerms, "one row per linearisation workgroup");
static __device__ __align__(256) float scratch[kLinScratchFloats];

namespace vpgs {
namespace {
std::mutex g_scratch_mu;
float* g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device ordinal
}  // namespace

int init_scratch(vpgs_ctx* ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices) return fail(ctx, VPGS_EUNSUPPORTED, "device %d", ctx->device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[ctx->device]) return VPGS_OK;
  void* p = nullptr;
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  g_scratch[ctx->device] = static_cast<float*>(p);
  return VPGS_OK;
}

namespace {
float* scratch_of(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (device >= 0 && device < kMaxDevices) ? g_scratch[device] : nullptr;
}
}  // namespace
}  // namespace vpgs

using namespace vpgs;

struct vpgs_voxel_map {
  vpgs_ctx* ctx = nullptr;
  float voxel = 1.0f;
  int32_t max_per_voxel = 1;
  uint32_t n = 0;
  uint32_t mask = 0;
  DevBuf pts, keys, vals, nvox;
};

namespace {

MapView view_of(const vpgs_voxel_map* m) {
  MapView v;
  v.pts = static_cast<const float4*>(m->pts.p);
  v.keys = static_cast<const uint64_t*>(m->keys.p);
  v.vals = static_cast<const uint2*>(m->vals.p);
  v.mask = m->mask;
  v.voxel = m->voxel;
  return v;
}

int check_points(vpgs_ctx* ctx, const float* p, int64_t n, float voxel) {
  if (n < 0 || n > 0x7fffffff) return fail(ctx, VPGS_EINVAL, "point count %lld out of range", (long long)n);
  if (n > 0 && !p) return fail(ctx, VPGS_EINVAL, "NULL points");
  if (!(voxel > 0.0f) || !std::isfinite(voxel)) return fail(ctx, VPGS_EINVAL, "voxel size must be positive");
  return VPGS_OK;
}

int check_map(vpgs_ctx* ctx, const vpgs_voxel_map* m) {
  if (!m || m->ctx != ctx) return fail(ctx, VPGS_EINVAL, "voxel map of another context or NULL");
  return VPGS_OK;
}

int check_linearize(vpgs_ctx* ctx, const vpgs_voxel_map* map, const float* src, int64_t n, const double* pose,
                    float tau, float sigma, const double* terms) {
  if (!ctx) return VPGS_EINVAL;
  int rc = check_map(ctx, map);
  if (rc) return rc;
  if (n < 0 || n > 0x7fffffff) return fail(ctx, VPGS_EINVAL, "source count out of range");
  if ((n > 0 && !src) || !terms) return fail(ctx, VPGS_EINVAL, "NULL source or output");
  if (!pose || !finite_pose(pose)) return fail(ctx, VPGS_EINVAL, "NULL or non-finite pose");
  if (!(tau > 0.0f) || !std::isfinite(tau) || !(sigma > 0.0f) || !std::isfinite(sigma))
    return fail(ctx, VPGS_EINVAL, "tau and sigma must be positive");
  return VPGS_OK;
}

// One linearisation pass and the FP64 sum of its workgroup partials
// (partials: linearize_blocks(n) rows of kTerms floats).
int launch_linearize(vpgs_ctx* ctx, const vpgs_voxel_map* map, const float* src, uint32_t n, const double* pose,
                     float tau, float sigma, float* partials, double* terms, hipStream_t st) {
  const uint32_t nb = linearize_blocks(n);
  with_group(n, [&](auto g) {
    constexpr int G = decltype(g)::value;
    hipLaunchKernelGGL(linearize_kernel<G>, dim3(nb), dim3(kIcpBlock), 0, st, view_of(map), src, n,
                       pose32_of(pose), (const IcpState*)nullptr, tau * tau, sigma / 3.0f, partials);
  });
  hipLaunchKernelGGL(reduce_terms_kernel, dim3(1), dim3(kIcpBlock), 0, st, partials, nb, terms);
  HIP_TRY(hipGetLastError());
  return VPGS_OK;
}

}  // namespace

extern "C" {

int vpgs_voxel_map_create(vpgs_ctx* ctx, const float* points, int64_t n, float voxel, int32_t max_per_voxel,
                          vpgs_voxel_map** out, void* stream) {
  if (!ctx) return VPGS_EINVAL;
  if (!out) return fail(ctx, VPGS_EINVAL, "NULL output");
  int rc = check_points(ctx, points, n, voxel);
  if (rc) return rc;
  if (max_per_voxel < 1) return fail(ctx, VPGS_EINVAL, "max_per_voxel must be >= 1");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));
  vpgs_voxel_map* m = new (std::nothrow) vpgs_voxel_map();
  if (!m) return fail(ctx, VPGS_ENOMEM, "out of host memory");
  m->ctx = ctx;
  m->voxel = voxel;
  m->max_per_voxel = max_per_voxel;
  m->n = (uint32_t)n;
  const uint32_t cap = pow2_at_least(std::max<uint64_t>(2 * (uint64_t)n, 64));
  m->mask = cap - 1;
  auto cleanup = [&](int code) {
    free_buf(m->ctx, m->pts); free_buf(m->ctx, m->keys); free_buf(m->ctx, m->vals); free_buf(m->ctx, m->nvox);
    delete m;
    return code;
  };
  if ((rc = ensure(ctx, m->pts, (size_t)std::max<uint32_t>(m->n, 1) * 16)) ||
      (rc = ensure(ctx, m->keys, (size_t)cap * 8)) || (rc = ensure(ctx, m->vals, (size_t)cap * 8)) ||
      (rc = ensure(ctx, m->nvox, 256)))
    return cleanup(rc);
  StageTimer timer(ctx, ST_VOXEL, st);
  hipError_t e = launch_fill_u32(static_cast<uint32_t*>(m->keys.p), 0xffffffffu, 2 * (size_t)cap, st);
  if (e == hipSuccess) e = launch_fill_u32(static_cast<uint32_t*>(m->nvox.p), 0u, 1, st);
  if (e != hipSuccess) return cleanup(fail(ctx, VPGS_EHIP, "fill: %s", hipGetErrorString(e)));
  if (n == 0) {
    *out = m;
    return VPGS_OK;
  }
  // workspace: lo, hi, idx, lo_alt, idx_alt, hi_perm, hi_alt, idx_b_alt (u32 [n] each), the count,
  // then the sort and scan workspaces
  const size_t N = m->n, w = (N * 4 + 255) / 256 * 256;
  const size_t sort_ws = sort_workspace_bytes(m->n), scan_ws = scan_workspace_bytes(m->n);
  if ((rc = ensure(ctx, ctx->icp_build, 8 * w + 256 + sort_ws + scan_ws))) return cleanup(rc);
  char* base = static_cast<char*>(ctx->icp_build.p);
  uint32_t* buf[8];
  for (int k = 0; k < 8; ++k) buf[k] = reinterpret_cast<uint32_t*>(base + k * w);
  uint32_t* ndev = reinterpret_cast<uint32_t*>(base + 8 * w);
  void* sws = base + 8 * w + 256;
  void* cws = static_cast<char*>(sws) + sort_ws;
  uint32_t *lo = buf[0], *hi = buf[1], *idx = buf[2], *lo_alt = buf[3], *idx_alt = buf[4], *hi_perm = buf[5],
           *hi_alt = buf[6], *idx_b_alt = buf[7];
  const dim3 g(blocks_of(m->n, 256)), b(256);
  e = launch_fill_u32(ndev, m->n, 1, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(vox_key_kernel, g, b, 0, st, points, m->n, voxel, lo, hi, idx);
    e = hipGetLastError();
  }
  int alt_a = 0, alt_b = 0;
  if (e == hipSuccess)  // by the low key word, carrying the index; gathers the high word in that order
    e = launch_radix_sort(lo, idx, lo_alt, idx_alt, m->n, 32, ndev, sws, &alt_a, st, hi, hi_perm);
  uint32_t* idx_a = alt_a ? idx_alt : idx;
  if (e == hipSuccess)  // stably by the high word (bits 32..62 of the key)
    e = launch_radix_sort(hi_perm, idx_a, hi_alt, idx_b_alt, m->n, 31, ndev, sws, &alt_b, st, nullptr, nullptr);
  const uint32_t* sidx = alt_b ? idx_b_alt : idx_a;
  float4* pts = static_cast<float4*>(m->pts.p);
  // run heads and voxel ids reuse lo / lo_alt / hi (no longer needed)
  uint32_t* head = lo;
  uint32_t* vid = lo_alt;
  uint32_t* vstart = hi;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(gather_points_kernel, g, b, 0, st, points, sidx, m->n, pts);
    hipLaunchKernelGGL(heads_kernel, g, b, 0, st, pts, m->n, voxel, head);
    e = hipGetLastError();
  }
  uint32_t* nvox = static_cast<uint32_t*>(m->nvox.p);
  if (e == hipSuccess) e = launch_scan(head, vid, m->n, nvox, cws, st, true);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(vstart_kernel, g, b, 0, st, head, vid, m->n, vstart);
    hipLaunchKernelGGL(map_insert_kernel, g, b, 0, st, pts, vstart, nvox, m->n, voxel, (uint32_t)max_per_voxel,
                       static_cast<uint64_t*>(m->keys.p), static_cast<uint2*>(m->vals.p), m->mask);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return cleanup(fail(ctx, VPGS_EHIP, "voxel map build: %s", hipGetErrorString(e)));
  *out = m;
  return VPGS_OK;
}

int vpgs_voxel_map_info(vpgs_voxel_map* m, int64_t* n_points, int64_t* n_voxels, void* stream) {
  if (!m) return VPGS_EINVAL;
  vpgs_ctx* ctx = m->ctx;
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));
  uint32_t* h = static_cast<uint32_t*>(ctx->h_pinned);
  HIP_TRY(hipMemcpyAsync(h, m->nvox.p, 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (n_points) *n_points = m->n;
  if (n_voxels) *n_voxels = m->n ? h[0] : 0;
  return VPGS_OK;
}

int vpgs_voxel_map_destroy(vpgs_voxel_map* m) {
  if (!m) return VPGS_EINVAL;
  (void)hipSetDevice(m->ctx->device);
  free_buf(m->ctx, m->pts); free_buf(m->ctx, m->keys); free_buf(m->ctx, m->vals); free_buf(m->ctx, m->nvox);
  delete m;
  return VPGS_OK;
}

int vpgs_voxel_downsample(vpgs_ctx* ctx, const float* points, int64_t n, float voxel, int32_t* out_idx,
                          int32_t* out_count, void* stream) {
  if (!ctx) return VPGS_EINVAL;
  int rc = check_points(ctx, points, n, voxel);
  if (rc) return rc;
  if (!out_count || (n > 0 && !out_idx)) return fail(ctx, VPGS_EINVAL, "NULL output");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));
  StageTimer timer(ctx, ST_VOXEL, st);
  if (n == 0) {
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(out_count), 0u, 1, st));
    return VPGS_OK;
  }
  const uint32_t N = (uint32_t)n;
  const uint32_t cap = pow2_at_least(std::max<uint64_t>(2 * (uint64_t)N, 64));
  const size_t w = ((size_t)N * 4 + 255) / 256 * 256;
  const size_t scan_ws = scan_workspace_bytes(N);
  if ((rc = ensure(ctx, ctx->icp_build, (size_t)cap * 12 + 2 * w + scan_ws + 256))) return rc;
  char* base = static_cast<char*>(ctx->icp_build.p);
  uint64_t* keys = reinterpret_cast<uint64_t*>(base);
  uint32_t* first = reinterpret_cast<uint32_t*>(base + (size_t)cap * 8);
  uint32_t* flag = reinterpret_cast<uint32_t*>(base + (size_t)cap * 12);
  uint32_t* pos = reinterpret_cast<uint32_t*>(base + (size_t)cap * 12 + w);
  void* cws = base + (size_t)cap * 12 + 2 * w;
  HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(keys), 0xffffffffu, 3 * (size_t)cap, st));  // keys and first
  const dim3 g(blocks_of(N, 256)), b(256);
  hipLaunchKernelGGL(ds_insert_kernel, g, b, 0, st, points, N, voxel, keys, first, cap - 1);
  hipLaunchKernelGGL(ds_flag_kernel, g, b, 0, st, points, N, voxel, keys, first, cap - 1, flag);
  HIP_TRY(hipGetLastError());
  HIP_TRY(launch_scan(flag, pos, N, reinterpret_cast<uint32_t*>(out_count), cws, st, true));
  hipLaunchKernelGGL(ds_scatter_kernel, g, b, 0, st, flag, pos, N, out_idx);
  HIP_TRY(hipGetLastError());
  return VPGS_OK;
}

int vpgs_icp_correspond(vpgs_ctx* ctx, const vpgs_voxel_map* map, const float* src, int64_t n, const double* pose,
                        float tau, int32_t* nn, float* d2, void* stream) {
  if (!ctx) return VPGS_EINVAL;
  int rc = check_map(ctx, map);
  if (rc) return rc;
  if (n < 0 || n > 0x7fffffff) return fail(ctx, VPGS_EINVAL, "source count out of range");
  if (n > 0 && (!src || (!nn && !d2))) return fail(ctx, VPGS_EINVAL, "NULL source or outputs");
  if (!pose || !finite_pose(pose)) return fail(ctx, VPGS_EINVAL, "NULL or non-finite pose");
  if (!(tau > 0.0f) || !std::isfinite(tau)) return fail(ctx, VPGS_EINVAL, "tau must be positive");
  if (n == 0) return VPGS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));
  StageTimer timer(ctx, ST_ICP, st);
  with_group((uint32_t)n, [&](auto g) {
    constexpr int G = decltype(g)::value;
    hipLaunchKernelGGL(correspond_kernel<G>, dim3(blocks_of((uint32_t)n, kIcpBlock / G)), dim3(kIcpBlock), 0, st,
                       view_of(map), src, (uint32_t)n, pose32_of(pose), tau * tau, nn, d2);
  });
  HIP_TRY(hipGetLastError());
  return VPGS_OK;
}

int vpgs_icp_linearize(vpgs_ctx* ctx, const vpgs_voxel_map* map, const float* src, int64_t n, const double* pose,
                       float tau, float sigma, double* terms, void* stream) {
  int rc = check_linearize(ctx, map, src, n, pose, tau, sigma, terms);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));
  const uint32_t nb = linearize_blocks((uint32_t)n);
  if ((rc = ensure(ctx, ctx->icp_ws, (size_t)nb * kTerms * 4 + 512))) return rc;
  StageTimer timer(ctx, ST_ICP, st);
  return launch_linearize(ctx, map, src, (uint32_t)n, pose, tau, sigma, static_cast<float*>(ctx->icp_ws.p), terms, st);
}

int vpgs_icp_linearize_noalloc(vpgs_ctx* ctx, const vpgs_voxel_map* map, const float* src, int64_t n,
                               const double* pose, float tau, float sigma, double* terms, void* stream) {
  int rc = check_linearize(ctx, map, src, n, pose, tau, sigma, terms);
  if (rc) return rc;
  const uint32_t nb = linearize_blocks((uint32_t)n);
  if ((size_t)nb * kTerms > kLinScratchFloats)
    return fail(ctx, VPGS_EINVAL, "%u workgroup partials exceed the %zu-float scratch", nb, kLinScratchFloats);
  float* partials = scratch_of(ctx->device);
  if (!partials) return fail(ctx, VPGS_EHIP, "scratch of device %d not initialised", ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));
  // every workgroup writes its whole row before the reduction reads it: the
  // scratch needs no clearing
  return launch_linearize(ctx, map, src, (uint32_t)n, pose, tau, sigma, partials, terms, st);
}

int vpgs_icp_register(vpgs_ctx* ctx, const vpgs_voxel_map* map, const float* src, int64_t n,
                      const double* prev_pose, const double* pred_pose, const vpgs_icp_opts* opts, double* pose_out,
                      vpgs_icp_result* result, void* stream) {
  if (!ctx) return VPGS_EINVAL;
  int rc = check_map(ctx, map);
  if (rc) return rc;
  if (n < 0 || n > 0x7fffffff) return fail(ctx, VPGS_EINVAL, "source count out of range");
  if ((n > 0 && !src) || !opts || !pose_out) return fail(ctx, VPGS_EINVAL, "NULL argument");
  if (!prev_pose || !finite_pose(prev_pose) || (pred_pose && !finite_pose(pred_pose)))
    return fail(ctx, VPGS_EINVAL, "NULL or non-finite pose");
  const float tau = opts->tau, sigma = opts->sigma;
  if (!(tau > 0.0f) || !std::isfinite(tau) || !(sigma > 0.0f) || !std::isfinite(sigma))
    return fail(ctx, VPGS_EINVAL, "tau and sigma must be positive");
  if (opts->max_iterations < 0 || !(opts->eps >= 0.0)) return fail(ctx, VPGS_EINVAL, "bad iteration options");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));
  // eq. 10: the source points are the scan under T_{i-1} T_pred
  double init[12];
  if (pred_pose) compose(prev_pose, pred_pose, init);
  else std::memcpy(init, prev_pose, sizeof(init));
  const uint32_t nb = linearize_blocks((uint32_t)n);
  const size_t state_off = ((size_t)nb * kTerms * 4 + 255) / 256 * 256;
  if ((rc = ensure(ctx, ctx->icp_ws, state_off + sizeof(IcpState)))) return rc;
  float* partials = static_cast<float*>(ctx->icp_ws.p);
  IcpState* dst = reinterpret_cast<IcpState*>(static_cast<char*>(ctx->icp_ws.p) + state_off);
  static_assert(sizeof(IcpState) <= 4096, "the state is read back through the 4 KiB pinned buffer");
  IcpState* h = static_cast<IcpState*>(ctx->h_pinned);
  HIP_TRY(hipStreamSynchronize(st));  // the pinned buffer may still feed an earlier copy
  std::memset(h, 0, sizeof(IcpState));
  std::memcpy(h->T, init, sizeof(init));
  h->p32 = pose32_of(init);
  h->done = (opts->max_iterations == 0 || n == 0) ? 1 : 0;
  StageTimer timer(ctx, ST_ICP, st);
  HIP_TRY(hipMemcpyAsync(dst, h, sizeof(IcpState), hipMemcpyHostToDevice, st));
  const MapView mv = view_of(map);
  const Pose32 ignored = h->p32;  // the kernels read the pose from the device state
  for (int it = 0; it < opts->max_iterations; it += kItersPerCheck) {
    const int k = std::min(kItersPerCheck, opts->max_iterations - it);
    for (int q = 0; q < k; ++q) {
      with_group((uint32_t)n, [&](auto g) {
        constexpr int G = decltype(g)::value;
        hipLaunchKernelGGL(linearize_kernel<G>, dim3(nb), dim3(kIcpBlock), 0, st, mv, src, (uint32_t)n, ignored,
                           (const IcpState*)dst, tau * tau, sigma / 3.0f, partials);
      });
      hipLaunchKernelGGL(solve_kernel, dim3(1), dim3(kIcpBlock), 0, st, partials, nb, dst, opts->eps,
                         opts->max_iterations);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(h, dst, sizeof(IcpState), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h->done) break;
  }
  if (opts->max_iterations == 0 || n == 0) {
    HIP_TRY(hipMemcpyAsync(h, dst, sizeof(IcpState), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  std::memcpy(pose_out, h->T, sizeof(h->T));
  if (result) {
    result->iterations = h->iterations;
    result->converged = h->converged;
    result->count = h->count;
    result->degenerate = h->degenerate;
    result->rho = h->rho;
    result->reserved = 0;
  }
  return VPGS_OK;
}

}  // extern "C"
