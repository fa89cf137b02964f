// sort.hip -- tile binning: key emission, a stable LSD radix sort of
// (tile id << 32 | depth bits, record index) pairs, and per-tile ranges.
//
// The pair count lives on the device (written by the count scan), so no host
// round trip is needed between projection and compositing; every kernel
// clamps it to the allocated capacity.
#include "internal.h"

namespace vpgs {
namespace {

// ---------------------------------------------------------------------------
// key emission
// ---------------------------------------------------------------------------

__device__ __forceinline__ int view_of_record(const CallTables* tab, uint32_t rec) {
  int lo = 0, hi = tab->n_views - 1;
  while (lo < hi) {  // last view whose rec_base <= rec
    const int mid = (lo + hi + 1) >> 1;
    if (tab->views[mid].rec_base <= rec) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void __launch_bounds__(256) emit_kernel(const CallTables* __restrict__ tab, const uint2* __restrict__ rect,
                                                   const uint32_t* __restrict__ count, const float4* __restrict__ pa,
                                                   const uint32_t* __restrict__ offsets, Counters* __restrict__ cnt,
                                                   uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                   uint32_t n_records, uint32_t capacity) {
  const uint32_t rec = blockIdx.x * blockDim.x + threadIdx.x;
  if (rec >= n_records) return;
  const uint32_t c = count[rec];
  if (c == 0) return;
  const ViewDesc& V = tab->views[view_of_record(tab, rec)];
  const uint2 r = rect[rec];
  const uint32_t tx0 = r.x & 0xffffu, tx1 = r.x >> 16, ty0 = r.y & 0xffffu, ty1 = r.y >> 16;
  const uint32_t zbits = __float_as_uint(pa[rec].z);
  uint32_t off = offsets[rec];
  if (off + c > capacity || off + c < off) cnt->overflow = 1u;
  for (uint32_t ty = ty0; ty <= ty1; ++ty)
    for (uint32_t tx = tx0; tx <= tx1; ++tx) {
      if (off < capacity) {
        const uint64_t tile = (uint64_t)(V.tile_base + ty * (uint32_t)V.tiles_x + tx);
        keys[off] = (tile << 32) | zbits;
        vals[off] = rec;
      }
      ++off;
    }
}

// ---------------------------------------------------------------------------
// radix sort: 8-bit digits, 4096 pairs per block (4 waves x 1024 contiguous)
// ---------------------------------------------------------------------------

constexpr int kSortBlock = 256;
constexpr int kWaves = kSortBlock / 64;
constexpr int kRounds = 16;                              // 64-key rounds per wave
constexpr uint32_t kSortTile = kSortBlock * kRounds;     // 4096
constexpr int kRadix = 256;

__device__ __forceinline__ uint32_t pair_count(const Counters* cnt, uint32_t capacity) {
  const uint32_t p = cnt->pairs;
  return p < capacity ? p : capacity;
}

// Lanes of the wave holding the same 8-bit digit (among the active lanes).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t active) {
  uint64_t peers = active;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint64_t m = __ballot((d >> b) & 1u);
    peers &= ((d >> b) & 1u) ? m : ~m;
  }
  return peers;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__global__ void __launch_bounds__(kSortBlock) radix_hist_kernel(const uint64_t* __restrict__ keys,
                                                                const Counters* __restrict__ cnt, uint32_t capacity,
                                                                int shift, uint32_t* __restrict__ hist) {
  __shared__ uint32_t wcnt[kWaves][kRadix];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int d = threadIdx.x; d < kWaves * kRadix; d += kSortBlock) (&wcnt[0][0])[d] = 0;
  __syncthreads();
  const uint32_t n = pair_count(cnt, capacity);
  const uint32_t base = blockIdx.x * kSortTile + wave * (kSortTile / kWaves);
  if (blockIdx.x * kSortTile < n) {
    for (int r = 0; r < kRounds; ++r) {
      const uint32_t idx = base + r * 64 + lane;
      const bool ok = idx < n;
      const uint32_t d = ok ? (uint32_t)(keys[idx] >> shift) & 0xffu : 0u;
      const uint64_t active = __ballot(ok);
      if (active == 0) break;
      const uint64_t peers = match_digit(d, active);
      if (ok && (peers & lanemask_lt()) == 0) wcnt[wave][d] += (uint32_t)__popcll(peers);
    }
  }
  __syncthreads();
  const int d = threadIdx.x;
  uint32_t s = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) s += wcnt[w][d];
  hist[(size_t)d * gridDim.x + blockIdx.x] = s;
}

__global__ void __launch_bounds__(kSortBlock) radix_scatter_kernel(const uint64_t* __restrict__ keys_in,
                                                                   const uint32_t* __restrict__ vals_in,
                                                                   uint64_t* __restrict__ keys_out,
                                                                   uint32_t* __restrict__ vals_out,
                                                                   const Counters* __restrict__ cnt, uint32_t capacity,
                                                                   int shift, const uint32_t* __restrict__ hist_scan) {
  __shared__ uint32_t wcnt[kWaves][kRadix];   // per-wave digit counts, then per-wave prefixes
  __shared__ uint32_t dstart[kRadix];         // block-local first position of each digit
  __shared__ uint32_t gbase[kRadix];          // global first position of each digit for this block
  __shared__ uint64_t skeys[kSortTile];
  __shared__ uint32_t svals[kSortTile];
  const uint32_t n = pair_count(cnt, capacity);
  if (blockIdx.x * kSortTile >= n) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int d = threadIdx.x; d < kWaves * kRadix; d += kSortBlock) (&wcnt[0][0])[d] = 0;
  __syncthreads();

  const uint32_t base = blockIdx.x * kSortTile + wave * (kSortTile / kWaves);
  uint64_t k[kRounds];
  uint32_t v[kRounds];
  uint32_t loc[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const uint32_t idx = base + r * 64 + lane;
    const bool ok = idx < n;
    k[r] = ok ? keys_in[idx] : 0ull;
    v[r] = ok ? vals_in[idx] : 0u;
    const uint32_t d = (uint32_t)(k[r] >> shift) & 0xffu;
    const uint64_t active = __ballot(ok);
    const uint64_t peers = match_digit(d, active);
    const uint32_t before = wcnt[wave][d];
    loc[r] = before + (uint32_t)__popcll(peers & lanemask_lt());
    if (ok && (peers & lanemask_lt()) == 0) wcnt[wave][d] = before + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  {
    // per-digit: prefix over waves, block total; then exclusive scan over digits
    const int d = threadIdx.x;
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = wcnt[w][d];
      wcnt[w][d] = run;
      run += c;
    }
    // block-wide exclusive scan of run over the 256 digits
    uint32_t incl = run;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t t = __shfl_up(incl, off, 64);
      if (lane >= off) incl += t;
    }
    __shared__ uint32_t wsum[kWaves];
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t wb = 0;
    for (int w = 0; w < wave; ++w) wb += wsum[w];
    dstart[d] = wb + incl - run;
    gbase[d] = hist_scan[(size_t)d * gridDim.x + blockIdx.x];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const uint32_t idx = base + r * 64 + lane;
    if (idx < n) {
      const uint32_t d = (uint32_t)(k[r] >> shift) & 0xffu;
      const uint32_t pos = dstart[d] + wcnt[wave][d] + loc[r];
      skeys[pos] = k[r];
      svals[pos] = v[r];
    }
  }
  __syncthreads();
  const uint32_t tile_n = min(kSortTile, n - blockIdx.x * kSortTile);
  for (uint32_t p = threadIdx.x; p < tile_n; p += kSortBlock) {
    const uint64_t key = skeys[p];
    const uint32_t d = (uint32_t)(key >> shift) & 0xffu;
    const uint32_t g = gbase[d] + (p - dstart[d]);
    keys_out[g] = key;
    vals_out[g] = svals[p];
  }
}

// ---------------------------------------------------------------------------
// ranges
// ---------------------------------------------------------------------------

__global__ void ranges_kernel(const uint64_t* __restrict__ keys, const Counters* __restrict__ cnt, uint32_t capacity,
                              uint2* __restrict__ ranges, uint32_t n_tiles) {
  const uint32_t n = pair_count(cnt, capacity);
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint32_t t = (uint32_t)(keys[k] >> 32);
  if (t >= n_tiles) return;
  if (k == 0 || (uint32_t)(keys[k - 1] >> 32) != t) ranges[t].x = k;
  if (k == n - 1 || (uint32_t)(keys[k + 1] >> 32) != t) ranges[t].y = k + 1;
}

inline uint32_t div_up(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

}  // namespace

hipError_t launch_emit(const CallTables* d_tab, const CallTables& h_tab, const ProjBuffers pb, const uint32_t* offsets,
                       Counters* cnt, uint64_t* keys, uint32_t* vals, uint32_t capacity, int tile_w, int tile_h,
                       hipStream_t s) {
  (void)tile_w; (void)tile_h;
  if (h_tab.n_records == 0) return hipSuccess;
  hipLaunchKernelGGL(emit_kernel, dim3(div_up(h_tab.n_records, 256)), dim3(256), 0, s, d_tab, pb.rect, pb.count, pb.a,
                     offsets, cnt, keys, vals, h_tab.n_records, capacity);
  return hipGetLastError();
}

size_t sort_workspace_bytes(uint32_t capacity) {
  const uint32_t blocks = div_up(capacity > 0 ? capacity : 1, kSortTile);
  const size_t hist = (size_t)blocks * kRadix * sizeof(uint32_t);
  const size_t h = (hist + 255) / 256 * 256;
  return 2 * h + scan_workspace_bytes(blocks * kRadix) + 256;
}

hipError_t launch_sort(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt, uint32_t capacity,
                       int key_bits, const Counters* cnt, void* ws, int* result_in_alt, hipStream_t s) {
  *result_in_alt = 0;
  if (capacity == 0) return hipSuccess;
  const uint32_t blocks = div_up(capacity, kSortTile);
  const size_t hist_bytes = ((size_t)blocks * kRadix * sizeof(uint32_t) + 255) / 256 * 256;
  uint32_t* hist = static_cast<uint32_t*>(ws);
  uint32_t* hist_scan = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + hist_bytes);
  void* scan_ws = static_cast<char*>(ws) + 2 * hist_bytes;
  uint64_t* kin = keys; uint32_t* vin = vals;
  uint64_t* kout = keys_alt; uint32_t* vout = vals_alt;
  int alt = 0;
  for (int shift = 0; shift < key_bits; shift += 8) {
    hipLaunchKernelGGL(radix_hist_kernel, dim3(blocks), dim3(kSortBlock), 0, s, kin, cnt, capacity, shift, hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_scan(hist, hist_scan, blocks * kRadix, nullptr, scan_ws, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(radix_scatter_kernel, dim3(blocks), dim3(kSortBlock), 0, s, kin, vin, kout, vout, cnt, capacity,
                       shift, hist_scan);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint64_t* tk = kin; kin = kout; kout = tk;
    uint32_t* tv = vin; vin = vout; vout = tv;
    alt ^= 1;
  }
  *result_in_alt = alt;
  return hipSuccess;
}

hipError_t launch_ranges(const uint64_t* keys, const Counters* cnt, uint32_t capacity, uint2* ranges, uint32_t n_tiles,
                         hipStream_t s) {
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(ranges), 0u, 2 * (size_t)n_tiles, s);
  if (e != hipSuccess || capacity == 0) return e;
  hipLaunchKernelGGL(ranges_kernel, dim3(div_up(capacity, 256)), dim3(256), 0, s, keys, cnt, capacity, ranges, n_tiles);
  return hipGetLastError();
}

}  // namespace vpgs
