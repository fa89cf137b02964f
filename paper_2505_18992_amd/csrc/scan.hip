// scan.hip -- exclusive prefix sum of uint32 counts (reduce, scan of the
// block sums, downsweep), the same scan fused with stream compaction of the
// visible records, and small fill kernels.
//
// A scan may take its length from a device counter (n_dev, clamped to the
// allocated n): values at or past it count as zero and their outputs are not
// written, so no host round trip is needed.
#include "internal.h"

namespace vpgs {
namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;
constexpr uint32_t kScanTile = kScanBlock * kScanItems;  // 4096 values per block

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(v, off, 64);
    if (lane >= off) v += t;
  }
  return v;
}

// Exclusive scan of one value per thread across the block; returns the
// exclusive prefix and writes the block total to *total.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* lds, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t incl = wave_incl_scan(v);
  if (lane == 63) lds[wave] = incl;
  __syncthreads();
  uint32_t wbase = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kScanBlock / 64; ++w) {
    const uint32_t x = lds[w];
    if (w < wave) wbase += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return wbase + incl - v;
}

// flags != 0: scan the indicator (value != 0) instead of the values.
__device__ __forceinline__ uint32_t scan_value(uint32_t x, int flags) { return flags ? (x != 0u) : x; }

__device__ __forceinline__ uint32_t scan_length(uint32_t n, const uint32_t* n_dev) {
  if (n_dev == nullptr) return n;
  const uint32_t m = *n_dev;
  return m < n ? m : n;
}

__global__ void __launch_bounds__(kScanBlock) scan_reduce_kernel(const uint32_t* __restrict__ in, uint32_t n_alloc,
                                                                 const uint32_t* __restrict__ n_dev,
                                                                 uint32_t* __restrict__ sums, int flags) {
  __shared__ uint32_t lds[kScanBlock / 64];
  const uint32_t n = scan_length(n_alloc, n_dev);
  const size_t base = (size_t)blockIdx.x * kScanTile;
  if (base >= n) {  // a tile past the end (the length may come from the device)
    if (threadIdx.x == 0) sums[blockIdx.x] = 0u;
    return;
  }
  // every item is loaded before any is summed, so the loads are in flight
  // together (positions past the end read an allocated value and add 0)
  uint32_t x[kScanItems];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) x[k] = in[min(base + (size_t)k * kScanBlock + threadIdx.x, (size_t)n_alloc - 1)];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const size_t idx = base + (size_t)k * kScanBlock + threadIdx.x;
    s += idx < n ? scan_value(x[k], flags) : 0u;
  }
  uint32_t tot;
  block_excl_scan(s, lds, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Down-sweeps.  Each wavefront owns kWaveItems consecutive values of its
// block's tile and walks them in rounds of 64 (coalesced loads and stores):
// its offset within the block comes from the other wavefronts' totals (one
// barrier), each round is a wavefront scan carried by a running sum.
constexpr int kWaveItems = kScanTile / (kScanBlock / 64);  // 1024
constexpr int kWaveRounds = kWaveItems / 64;                // 16

// Sum of one value per lane over the wavefront (every lane gets it).
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Exclusive prefix of this wavefront within its block from the wavefront
// totals; the last wavefront's end is the block total.
__device__ __forceinline__ uint32_t wave_offset(uint32_t wave_total, uint32_t* lds, uint32_t* block_total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) lds[wave] = wave_total;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kScanBlock / 64; ++w) {
    const uint32_t x = lds[w];
    if (w < wave) off += x;
    tot += x;
  }
  *block_total = tot;
  return off;
}

// Exclusive scan of each block's tile, offset by block_offsets[block]
// (NULL = 0).  If total is non-NULL the last block writes the grand total.
__global__ void __launch_bounds__(kScanBlock) scan_down_kernel(const uint32_t* __restrict__ in, uint32_t n_alloc,
                                                               const uint32_t* __restrict__ n_dev,
                                                               const uint32_t* __restrict__ block_offsets,
                                                               uint32_t* __restrict__ out, uint32_t* __restrict__ total,
                                                               int flags) {
  __shared__ uint32_t lds[kScanBlock / 64];
  const uint32_t n = scan_length(n_alloc, n_dev);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if ((size_t)blockIdx.x * kScanTile >= n) {  // a tile past the end: nothing to write but the grand total
    if (total != nullptr && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
      *total = block_offsets ? block_offsets[blockIdx.x] : 0u;
    return;
  }
  const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)wave * kWaveItems + lane;
  uint32_t v[kWaveRounds];
#pragma unroll
  for (int k = 0; k < kWaveRounds; ++k) v[k] = in[min(base + (size_t)k * 64, (size_t)n_alloc - 1)];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kWaveRounds; ++k) {
    const size_t idx = base + (size_t)k * 64;
    v[k] = idx < n ? scan_value(v[k], flags) : 0u;
    s += v[k];
  }
  uint32_t tot;
  const uint32_t off = block_offsets ? block_offsets[blockIdx.x] : 0u;
  uint32_t run = off + wave_offset(wave_sum(s), lds, &tot);
#pragma unroll
  for (int k = 0; k < kWaveRounds; ++k) {
    const size_t idx = base + (size_t)k * 64;
    const uint32_t incl = wave_incl_scan(v[k]);
    if (idx < n) out[idx] = run + incl - v[k];
    run += __shfl(incl, 63, 64);
  }
  if (total != nullptr && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = off + tot;
}

// Down-sweep of the indicator scan (count != 0) that scatters instead of
// storing offsets: visible record r goes to position (number of visible
// records before r), with key = its depth key and value r.  Record order is
// kept, so equal depths stay in index order.
__global__ void __launch_bounds__(kScanBlock) compact_down_kernel(const uint32_t* __restrict__ count, uint32_t n,
                                                                  const uint32_t* __restrict__ block_offsets,
                                                                  const uint32_t* __restrict__ zkey,
                                                                  uint32_t* __restrict__ keys,
                                                                  uint32_t* __restrict__ vals,
                                                                  uint32_t* __restrict__ total) {
  __shared__ uint32_t lds[kScanBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)wave * kWaveItems + lane;
  // counts and depth keys of every round are loaded up front, so the loads
  // are in flight together (positions past the end read allocated values
  // that are not used)
  uint32_t c[kWaveRounds], z[kWaveRounds];
#pragma unroll
  for (int k = 0; k < kWaveRounds; ++k) {
    const size_t ci = min(base + (size_t)k * 64, (size_t)n - 1);
    c[k] = count[ci];
    z[k] = zkey[ci];
  }
  uint32_t flags = 0;  // bit k: this lane's value of round k is visible
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kWaveRounds; ++k) {
    const size_t idx = base + (size_t)k * 64;
    const bool vis = idx < n && c[k] != 0u;
    flags |= (vis ? 1u : 0u) << k;
    s += __popcll(__ballot(vis));
  }
  uint32_t tot;
  const uint32_t off = block_offsets ? block_offsets[blockIdx.x] : 0u;
  uint32_t run = off + wave_offset(s, lds, &tot);
#pragma unroll
  for (int k = 0; k < kWaveRounds; ++k) {
    const bool vis = (flags >> k) & 1u;
    const uint64_t m = __ballot(vis);
    if (vis) {
      const size_t idx = base + (size_t)k * 64;
      const uint32_t pos =
          run + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
      keys[pos] = z[k];
      vals[pos] = (uint32_t)idx;
    }
    run += __popcll(m);
  }
  if (total != nullptr && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = off + tot;
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t value, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}
__global__ void fill_f32_kernel(float* p, float value, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

inline uint32_t div_up(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

}  // namespace

// Workspace: block sums of every level, recursively.
size_t scan_workspace_bytes(uint32_t n) {
  size_t bytes = 0;
  uint32_t m = n;
  while (m > kScanTile) {
    m = div_up(m, kScanTile);
    bytes += 2 * ((size_t)m * sizeof(uint32_t) + 256);
  }
  return bytes + 256;
}

hipError_t launch_scan(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* total, void* ws, hipStream_t s,
                       bool flags, const uint32_t* n_dev) {
  const int fl = flags ? 1 : 0;
  if (n == 0) return total ? launch_fill_u32(total, 0u, 1, s) : hipSuccess;
  const uint32_t blocks = div_up(n, kScanTile);
  if (blocks == 1) {
    hipLaunchKernelGGL(scan_down_kernel, dim3(1), dim3(kScanBlock), 0, s, in, n, n_dev, nullptr, out, total, fl);
    return hipGetLastError();
  }
  char* w = static_cast<char*>(ws);
  uint32_t* sums = reinterpret_cast<uint32_t*>(w);
  const size_t sum_bytes = ((size_t)blocks * sizeof(uint32_t) + 255) / 256 * 256;
  uint32_t* sums_scanned = reinterpret_cast<uint32_t*>(w + sum_bytes);
  hipLaunchKernelGGL(scan_reduce_kernel, dim3(blocks), dim3(kScanBlock), 0, s, in, n, n_dev, sums, fl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_scan(sums, sums_scanned, blocks, total, w + 2 * sum_bytes, s, false, nullptr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scan_down_kernel, dim3(blocks), dim3(kScanBlock), 0, s, in, n, n_dev, sums_scanned, out, nullptr,
                     fl);
  return hipGetLastError();
}

hipError_t launch_compact_visible(const uint32_t* count, const uint32_t* zkey, uint32_t n, uint32_t* keys, uint32_t* vals,
                                  uint32_t* total, void* ws, hipStream_t s) {
  if (n == 0) return total ? launch_fill_u32(total, 0u, 1, s) : hipSuccess;
  const uint32_t blocks = div_up(n, kScanTile);
  if (blocks == 1) {
    hipLaunchKernelGGL(compact_down_kernel, dim3(1), dim3(kScanBlock), 0, s, count, n, nullptr, zkey, keys, vals, total);
    return hipGetLastError();
  }
  char* w = static_cast<char*>(ws);
  uint32_t* sums = reinterpret_cast<uint32_t*>(w);
  const size_t sum_bytes = ((size_t)blocks * sizeof(uint32_t) + 255) / 256 * 256;
  uint32_t* sums_scanned = reinterpret_cast<uint32_t*>(w + sum_bytes);
  hipLaunchKernelGGL(scan_reduce_kernel, dim3(blocks), dim3(kScanBlock), 0, s, count, n, nullptr, sums, 1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_scan(sums, sums_scanned, blocks, total, w + 2 * sum_bytes, s, false, nullptr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(compact_down_kernel, dim3(blocks), dim3(kScanBlock), 0, s, count, n, sums_scanned, zkey, keys, vals,
                     nullptr);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, value, n);
  return hipGetLastError();
}
hipError_t launch_fill_f32(float* p, float value, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, value, n);
  return hipGetLastError();
}

}  // namespace vpgs
