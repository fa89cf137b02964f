// sort.hip -- tile binning.
//
// The per-tile order is (tile, FP32 depth bits, record index).  Instead of
// one wide sort of every (tile, Gaussian) pair, binning runs in two narrow
// stable sorts:
//   1. visible records are compacted in record order and stably sorted by
//      their 32-bit depth bits (so ties keep record order);
//   2. pairs are emitted in that depth order, one 32-bit tile id per
//      overlapped tile, and stably sorted by tile id.
// Stability makes the result the (tile, depth, index) order.  The depth sort
// touches each visible record once instead of every pair, and the tile sort
// needs only ceil(log2(tiles) / 8) passes.
//
// Counts (visible records, pairs) stay on the device; every kernel clamps
// them to the allocated capacity, so no host round trip is needed.
//
// Each radix pass is three kernels: per-workgroup digit histograms, a scan
// of every digit's row of histograms (one workgroup per digit), and the
// scatter, which adds the digit's global base (a scan of the row totals it
// redoes itself) to its row offset.
#include "internal.h"

namespace vpgs {
namespace {

constexpr int kSortBlock = 256;
constexpr int kWaves = kSortBlock / 64;
// A workgroup sorts kSortBlock * R keys, R 64-key rounds per wavefront: 16
// (4096 keys) for large sorts, 4 (1024 keys) for sorts of at most
// kSmallSortKeys, which then spread over four times the workgroups.
constexpr int kRoundsLarge = 16, kRoundsSmall = 4;
constexpr uint32_t kSmallSortKeys = 1u << 20;
inline int sort_rounds(uint32_t capacity) { return capacity <= kSmallSortKeys ? kRoundsSmall : kRoundsLarge; }
constexpr int kRadix = 256;
static_assert(kRadix == kSortBlock, "one digit per thread in the histogram and offset kernels");

__device__ __forceinline__ uint32_t clamped(const uint32_t* n, uint32_t capacity) {
  const uint32_t v = *n;
  return v < capacity ? v : capacity;
}

// Tiles of an inclusive tile rectangle (x0 | x1 << 16, y0 | y1 << 16).
__device__ __forceinline__ uint32_t rect_count(uint2 r) {
  return ((r.x >> 16) - (r.x & 0xffffu) + 1u) * ((r.y >> 16) - (r.y & 0xffffu) + 1u);
}

// ---------------------------------------------------------------------------
// pair emission in depth order
// ---------------------------------------------------------------------------
// One thread per visible record in depth order; a record's pairs are its
// tiles in row-major order.  The 64 records of a wavefront own one
// contiguous run of the pair list.  When the run fits the wavefront's LDS
// stage, the pairs are built there (small rectangles by their own lane,
// larger ones by the whole wavefront, lanes over tiles) and the run is then
// copied out 64 consecutive pairs at a time; otherwise they are written to
// the pair list directly in the same way.
//
// A lane walks its record's tiles with a running (column, tile) pair; the
// wavefront takes tile k of a large record from its row k / w, computed as
// ((float)k + 1/2) (1/w): (k + 1/2) / w lies at least 1 / (2w) from an
// integer and the product errs by under (k + 1/2) / w 2^-23, so the
// truncation is exact for k < 2^22 (a rectangle holds at most 2^20 tiles:
// 8192 / 8 on a side).
template <class Out>
__device__ __forceinline__ void emit_lane(uint32_t c, uint32_t pos, uint32_t rec, uint32_t tile0, uint32_t w,
                                          uint32_t tiles_x, Out out) {
  uint32_t x = 0, t = tile0;
  for (uint32_t k = 0; k < c; ++k) {
    out(pos + k, t, rec);
    ++t;
    if (++x == w) {
      x = 0;
      t += tiles_x - w;
    }
  }
}
template <class Out>
__device__ __forceinline__ void emit_wave(uint32_t lane, uint32_t c, uint32_t pos, uint32_t rec, uint32_t tile0,
                                          uint32_t w, uint32_t tiles_x, Out out) {
  const float inv_w = 1.0f / (float)w;
  for (uint32_t k = lane; k < c; k += 64) {
    const uint32_t row = (uint32_t)(((float)k + 0.5f) * inv_w);
    out(pos + k, tile0 + row * tiles_x + (k - row * w), rec);
  }
}

constexpr uint32_t kSmallFootprint = 8;  // records with more tiles are emitted by the whole wavefront
constexpr int kEmitBlock = 256;
constexpr uint32_t kEmitStage = 512;     // staged pairs per wavefront

__global__ void __launch_bounds__(kEmitBlock) emit_kernel(const CallTables* __restrict__ tab,
                                                          const uint32_t* __restrict__ sorted_rec,
                                                          const uint2* __restrict__ sorted_rect,
                                                          const uint32_t* __restrict__ pair_off,
                                                          const uint32_t* __restrict__ n_visible,
                                                          Counters* __restrict__ cnt, uint32_t n_records,
                                                          uint32_t capacity, uint32_t* __restrict__ keys,
                                                          uint32_t* __restrict__ vals) {
  __shared__ uint32_t stage_key[kEmitBlock / 64][kEmitStage], stage_val[kEmitBlock / 64][kEmitStage];
  const uint32_t nv = clamped(n_visible, n_records);
  if (blockIdx.x * kEmitBlock >= nv) return;
  const uint32_t i = blockIdx.x * kEmitBlock + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t rec = 0, c = 0, off = 0, tile0 = 0, w = 1, tiles_x = 1;
  if (i < nv) {
    rec = sorted_rec[i];
    off = pair_off[i];
    const uint2 rr = sorted_rect[i];
    // the record's view: the last whose first record is <= rec (the table
    // reads are the same for every lane)
    uint32_t tile_base = tab->views[0].tile_base;
    tiles_x = (uint32_t)tab->views[0].tiles_x;
    for (int v = 1; v < tab->n_views; ++v) {
      const uint32_t rb = tab->views[v].rec_base, tb = tab->views[v].tile_base, tx = (uint32_t)tab->views[v].tiles_x;
      const bool in = rec >= rb;
      tile_base = in ? tb : tile_base;
      tiles_x = in ? tx : tiles_x;
    }
    const uint32_t tx0 = rr.x & 0xffffu, tx1 = rr.x >> 16, ty0 = rr.y & 0xffffu, ty1 = rr.y >> 16;
    w = tx1 - tx0 + 1u;
    c = w * (ty1 - ty0 + 1u);  // the record's count
    tile0 = tile_base + ty0 * tiles_x + tx0;
    if (off + c > capacity || off + c < off) cnt->overflow = 1u;
  }
  // the wavefront's run: active lanes are a prefix of the wavefront
  const uint64_t active = __ballot(i < nv);
  if (active == 0ull) return;  // the whole wavefront is past the end (no barrier follows)
  const int last = 63 - __clzll((long long)active);
  const uint32_t begin = __shfl(off, 0, 64), end = __shfl(off + c, last, 64);
  const bool staged = end >= begin && end - begin <= kEmitStage && end <= capacity;  // the same in every lane
  uint32_t* sk = stage_key[wave];
  uint32_t* sv = stage_val[wave];
  auto to_stage = [&](uint32_t p, uint32_t key, uint32_t val) {
    sk[p - begin] = key;
    sv[p - begin] = val;
  };
  auto to_list = [&](uint32_t p, uint32_t key, uint32_t val) {
    if (p < capacity) {
      keys[p] = key;
      vals[p] = val;
    }
  };
  if (c <= kSmallFootprint) {
    if (staged) emit_lane(c, off, rec, tile0, w, tiles_x, to_stage);
    else emit_lane(c, off, rec, tile0, w, tiles_x, to_list);
  }
  uint64_t big = __ballot(c > kSmallFootprint);
  while (big != 0ull) {
    const int src = __ffsll((unsigned long long)big) - 1;
    big &= big - 1ull;
    const uint32_t bc = __shfl(c, src, 64), boff = __shfl(off, src, 64), brec = __shfl(rec, src, 64);
    const uint32_t bt0 = __shfl(tile0, src, 64), bw = __shfl(w, src, 64), btx = __shfl(tiles_x, src, 64);
    if (staged) emit_wave((uint32_t)lane, bc, boff, brec, bt0, bw, btx, to_stage);
    else emit_wave((uint32_t)lane, bc, boff, brec, bt0, bw, btx, to_list);
  }
  if (staged) {
    // LDS accesses of a wavefront complete in order: the reads see every
    // lane's writes above
    __builtin_amdgcn_wave_barrier();
    for (uint32_t q = (uint32_t)lane; q < end - begin; q += 64) {
      keys[begin + q] = sk[q];
      vals[begin + q] = sv[q];
    }
  }
}

// ---------------------------------------------------------------------------
// stable LSD radix sort, 8-bit digits, 4096 keys per workgroup
// ---------------------------------------------------------------------------

// Lanes of the wavefront holding the same 8-bit digit (among active lanes).
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

template <class K, int R>
__global__ void __launch_bounds__(kSortBlock) radix_hist_kernel(const K* __restrict__ keys, const uint32_t* __restrict__ n_ptr,
                                                                uint32_t capacity, int shift, uint32_t mask,
                                                                uint32_t* __restrict__ hist) {
  constexpr uint32_t kTile = kSortBlock * R;
  __shared__ uint32_t cnt[kRadix];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t n = clamped(n_ptr, capacity);
  if (blockIdx.x * kTile >= n) return;  // a tile past the end (its row entries are not read)
  cnt[threadIdx.x] = 0u;
  const uint32_t base = blockIdx.x * kTile + wave * (kTile / kWaves);
  // every round's digit is loaded before any is counted, so the loads are in
  // flight together; positions past the end read the last key and are not
  // counted
  uint32_t dig[R];
#pragma unroll
  for (int r = 0; r < R; ++r) dig[r] = (uint32_t)(keys[min(base + r * 64 + lane, n - 1)] >> shift) & mask;
  __syncthreads();
  // LDS atomic increments (integer counts: the order does not matter); a
  // round whose keys share one digit (the high byte of nearby depths) adds
  // its count once instead of serialising 64 increments of one address
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const bool ok = base + r * 64 + lane < n;
    const uint32_t d0 = __builtin_amdgcn_readfirstlane(dig[r]);
    const uint64_t act = __ballot(ok);
    if (__ballot(ok && dig[r] == d0) == act) {
      if (lane == 0 && act != 0ull) atomicAdd(&cnt[d0], (uint32_t)__popcll(act));
    } else if (ok) {
      atomicAdd(&cnt[dig[r]], 1u);
    }
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan of one value per thread over the 256-thread workgroup;
// *total receives the workgroup sum.
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t v, uint32_t* wsum, uint32_t* total = nullptr) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(incl, off, 64);
    if (lane >= off) incl += t;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t wb = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    wb += w < wave ? wsum[w] : 0u;
    all += wsum[w];
  }
  __syncthreads();
  if (total) *total = all;
  return wb + incl - v;
}

// One workgroup per digit d: exclusive scan of hist[d][0, used) into
// hist_scan and the row total into row_total[d], where used is the number of
// tiles that hold keys (the rest of the grid has no keys and writes nothing).
// The row is read in coalesced chunks of 256, eight chunks in flight.
constexpr int kScanChunks = 8;
__global__ void __launch_bounds__(kSortBlock) radix_offsets_kernel(const uint32_t* __restrict__ hist, uint32_t blocks,
                                                                   uint32_t tile, const uint32_t* __restrict__ n_ptr,
                                                                   uint32_t capacity,
                                                                   uint32_t* __restrict__ hist_scan,
                                                                   uint32_t* __restrict__ row_total) {
  __shared__ uint32_t wsum[kWaves];
  const uint32_t d = blockIdx.x;
  const uint32_t used = min(blocks, (clamped(n_ptr, capacity) + tile - 1) / tile);
  const uint32_t* row = hist + (size_t)d * blocks;
  uint32_t* out = hist_scan + (size_t)d * blocks;
  uint32_t carry = 0;
  for (uint32_t c0 = 0; c0 < used; c0 += kSortBlock * kScanChunks) {
    uint32_t v[kScanChunks];
#pragma unroll
    for (int j = 0; j < kScanChunks; ++j) {
      const uint32_t b = c0 + j * kSortBlock + threadIdx.x;
      const uint32_t x = row[min(b, used - 1)];
      v[j] = b < used ? x : 0u;
    }
#pragma unroll
    for (int j = 0; j < kScanChunks; ++j) {
      const uint32_t b = c0 + j * kSortBlock + threadIdx.x;
      uint32_t total;
      const uint32_t excl = block_excl_scan256(v[j], wsum, &total);
      if (b < used) out[b] = carry + excl;
      carry += total;
    }
  }
  if (threadIdx.x == 0) row_total[d] = carry;
}

// With few workgroups (at most kFusedOffsetsMax), the scatter forms its
// digit offsets itself from the raw histogram (hist_scan then holds it and
// row_total is unused): thread d adds row d over the tiles that hold keys,
// which saves the offsets kernel's launch on small inputs.
constexpr uint32_t kFusedOffsetsMax = 64;

template <class K, int R, bool FUSED>
__global__ void __launch_bounds__(kSortBlock) radix_scatter_kernel(const K* __restrict__ keys_in,
                                                                   const uint32_t* __restrict__ vals_in,
                                                                   K* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
                                                                   const uint32_t* __restrict__ n_ptr, uint32_t capacity,
                                                                   int shift, uint32_t mask,
                                                                   const uint32_t* __restrict__ hist_scan,
                                                                   const uint32_t* __restrict__ row_total,
                                                                   const uint32_t* __restrict__ gather_src,
                                                                   uint32_t* __restrict__ gather_dst,
                                                                   const uint2* __restrict__ rect_src,
                                                                   uint2* __restrict__ rect_dst,
                                                                   uint32_t* __restrict__ count_dst) {
  constexpr uint32_t kTile = kSortBlock * R;
  __shared__ uint32_t wcnt[kWaves][kRadix];   // per-wave digit counts, then per-wave prefixes
  __shared__ uint32_t dstart[kRadix];         // block-local first position of each digit
  __shared__ uint32_t gbase[kRadix];          // global first position of each digit for this block
  __shared__ uint32_t wsum[kWaves];
  __shared__ K skeys[kTile];
  __shared__ uint32_t svals[kTile];
  const uint32_t n = clamped(n_ptr, capacity);
  if (blockIdx.x * kTile >= n) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // this thread's digit: its total and this tile's row offset (read early)
  uint32_t my_total, my_row_off;
  if constexpr (FUSED) {
    const uint32_t used = min(gridDim.x, (n + kTile - 1) / kTile);
    const uint32_t* row = hist_scan + (size_t)threadIdx.x * gridDim.x;
    my_total = 0u;
    my_row_off = 0u;
    for (uint32_t b0 = 0; b0 < used; b0 += 16) {
      uint32_t c[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) c[u] = row[min(b0 + u, used - 1)];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const uint32_t b = b0 + u;
        my_total += b < used ? c[u] : 0u;
        my_row_off += b < blockIdx.x ? c[u] : 0u;
      }
    }
  } else {
    my_total = row_total[threadIdx.x];
    my_row_off = hist_scan[(size_t)threadIdx.x * gridDim.x + blockIdx.x];
  }
  for (int d = threadIdx.x; d < kWaves * kRadix; d += kSortBlock) (&wcnt[0][0])[d] = 0;
  __syncthreads();

  const uint32_t base = blockIdx.x * kTile + wave * (kTile / kWaves);
  K k[R];
  uint32_t v[R];
  uint32_t loc[R];
  // all rounds are loaded before any is ranked (positions past the end read
  // the last pair and take no part in the ranking)
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t ci = min(base + r * 64 + lane, n - 1);
    k[r] = keys_in[ci];
    v[r] = vals_in[ci];
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t idx = base + r * 64 + lane;
    const bool ok = idx < n;
    const uint32_t d = (uint32_t)(k[r] >> shift) & mask;
    const uint64_t active = __ballot(ok);
    const uint64_t peers = match_digit(d, active);
    const uint32_t before = wcnt[wave][d];
    loc[r] = before + (uint32_t)__popcll(peers & lanemask_lt());
    if (ok && (peers & lanemask_lt()) == 0) wcnt[wave][d] = before + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  {
    // per digit: prefix over waves and block total, then a scan over digits
    const int d = threadIdx.x;
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = wcnt[w][d];
      wcnt[w][d] = run;
      run += c;
    }
    uint32_t incl = run;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t t = __shfl_up(incl, off, 64);
      if (lane >= off) incl += t;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t wb = 0;
    for (int w = 0; w < wave; ++w) wb += wsum[w];
    dstart[d] = wb + incl - run;
    __syncthreads();
    // global base of digit d: the totals of the smaller digits
    const uint32_t digit_base = block_excl_scan256(my_total, wsum);
    gbase[d] = digit_base + my_row_off;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t idx = base + r * 64 + lane;
    if (idx < n) {
      const uint32_t d = (uint32_t)(k[r] >> shift) & mask;
      const uint32_t pos = dstart[d] + wcnt[wave][d] + loc[r];
      skeys[pos] = k[r];
      svals[pos] = v[r];
    }
  }
  __syncthreads();
  const uint32_t tile_n = min(kTile, n - blockIdx.x * kTile);
  if (tile_n == kTile) {
    // a full tile: straight-line code, so the gathers are in flight together
    uint32_t gpos[R], gval[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t p = r * kSortBlock + threadIdx.x;
      const K key = skeys[p];
      const uint32_t d = (uint32_t)(key >> shift) & mask;
      const uint32_t g = gbase[d] + (p - dstart[d]);
      const uint32_t val = svals[p];
      keys_out[g] = key;
      vals_out[g] = val;
      gpos[r] = g;
      gval[r] = val;
    }
    if (gather_dst != nullptr) {
      uint32_t gv[R];
#pragma unroll
      for (int r = 0; r < R; ++r) gv[r] = gather_src[gval[r]];
#pragma unroll
      for (int r = 0; r < R; ++r) gather_dst[gpos[r]] = gv[r];
    }
    if (rect_dst != nullptr) {
      uint2 rv[R];
#pragma unroll
      for (int r = 0; r < R; ++r) rv[r] = rect_src[gval[r]];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        rect_dst[gpos[r]] = rv[r];
        count_dst[gpos[r]] = rect_count(rv[r]);
      }
    }
    return;
  }
  for (uint32_t p = threadIdx.x; p < tile_n; p += kSortBlock) {
    const K key = skeys[p];
    const uint32_t d = (uint32_t)(key >> shift) & mask;
    const uint32_t g = gbase[d] + (p - dstart[d]);
    const uint32_t val = svals[p];
    keys_out[g] = key;
    vals_out[g] = val;
    if (gather_dst != nullptr) gather_dst[g] = gather_src[val];
    if (rect_dst != nullptr) {
      const uint2 rv = rect_src[val];
      rect_dst[g] = rv;
      count_dst[g] = rect_count(rv);
    }
  }
}

inline uint32_t div_up(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

size_t radix_ws_bytes(uint32_t capacity) {
  const uint32_t blocks = div_up(capacity > 0 ? capacity : 1, kSortBlock * sort_rounds(capacity));
  const size_t h = ((size_t)blocks * kRadix * sizeof(uint32_t) + 255) / 256 * 256;
  return 2 * h + kRadix * sizeof(uint32_t);
}

// gather_src/gather_dst (may be NULL): the last pass also writes
// gather_dst[i] = gather_src[value i] for every sorted position i.
// rect_src/rect_dst/count_dst (may be NULL): the last pass also writes
// rect_dst[i] = rect_src[value i] and count_dst[i] = its number of tiles.
// One radix pass with R rounds per wavefront: histogram, digit offsets
// (fused into the scatter when the workgroups are few) and scatter.
template <class K, int R>
hipError_t radix_pass(const K* kin, const uint32_t* vin, K* kout, uint32_t* vout, uint32_t blocks, uint32_t capacity,
                      int shift, uint32_t mask, const uint32_t* n_ptr, uint32_t* hist, uint32_t* hist_scan,
                      uint32_t* row_total, hipStream_t s, const uint32_t* gather_src, uint32_t* gather_dst,
                      const uint2* rect_src, uint2* rect_dst, uint32_t* count_dst) {
  hipLaunchKernelGGL((radix_hist_kernel<K, R>), dim3(blocks), dim3(kSortBlock), 0, s, kin, n_ptr, capacity, shift, mask,
                     hist);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (blocks <= kFusedOffsetsMax) {
    hipLaunchKernelGGL((radix_scatter_kernel<K, R, true>), dim3(blocks), dim3(kSortBlock), 0, s, kin, vin, kout, vout,
                       n_ptr, capacity, shift, mask, hist, row_total, gather_src, gather_dst, rect_src, rect_dst,
                       count_dst);
  } else {
    hipLaunchKernelGGL(radix_offsets_kernel, dim3(kRadix), dim3(kSortBlock), 0, s, hist, blocks,
                       (uint32_t)(kSortBlock * R), n_ptr, capacity, hist_scan, row_total);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((radix_scatter_kernel<K, R, false>), dim3(blocks), dim3(kSortBlock), 0, s, kin, vin, kout, vout,
                       n_ptr, capacity, shift, mask, hist_scan, row_total, gather_src, gather_dst, rect_src, rect_dst,
                       count_dst);
  }
  return hipGetLastError();
}

template <class K>
hipError_t radix_sort(K* keys, uint32_t* vals, K* keys_alt, uint32_t* vals_alt, uint32_t capacity, int key_bits,
                      const uint32_t* n_ptr, void* ws, int* result_in_alt, hipStream_t s,
                      const uint32_t* gather_src = nullptr, uint32_t* gather_dst = nullptr,
                      const uint2* rect_src = nullptr, uint2* rect_dst = nullptr, uint32_t* count_dst = nullptr) {
  *result_in_alt = 0;
  if (capacity == 0) return hipSuccess;
  const int rounds = sort_rounds(capacity);
  const uint32_t blocks = div_up(capacity, kSortBlock * rounds);
  const size_t hist_bytes = ((size_t)blocks * kRadix * sizeof(uint32_t) + 255) / 256 * 256;
  uint32_t* hist = static_cast<uint32_t*>(ws);
  uint32_t* hist_scan = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + hist_bytes);
  uint32_t* row_total = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + 2 * hist_bytes);
  K* kin = keys; uint32_t* vin = vals;
  K* kout = keys_alt; uint32_t* vout = vals_alt;
  int alt = 0;
  // passes of at most 8 bits, the narrower digits first (the first pass
  // scatters into the most runs per tile, so its runs are made longer)
  const int passes = (key_bits + 7) / 8;
  for (int pass = 0, shift = 0; pass < passes; ++pass) {
    const int bits = key_bits / passes + (pass >= passes - key_bits % passes ? 1 : 0);
    const uint32_t mask = (1u << bits) - 1u;
    const bool last = pass == passes - 1;
    const hipError_t e =
        (rounds == kRoundsSmall ? radix_pass<K, kRoundsSmall> : radix_pass<K, kRoundsLarge>)(
            kin, vin, kout, vout, blocks, capacity, shift, mask, n_ptr, hist, hist_scan, row_total, s,
            last ? gather_src : nullptr, last ? gather_dst : nullptr, last ? rect_src : nullptr,
            last ? rect_dst : nullptr, last ? count_dst : nullptr);
    if (e != hipSuccess) return e;
    K* tk = kin; kin = kout; kout = tk;
    uint32_t* tv = vin; vin = vout; vout = tv;
    alt ^= 1;
    shift += bits;
  }
  *result_in_alt = alt;
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// ranges and key export
// ---------------------------------------------------------------------------
// Four sorted keys per thread (one 16-byte load when it lies within the
// buffer) and their two neighbours.
__global__ void ranges_kernel(const uint32_t* __restrict__ tiles, const uint32_t* __restrict__ n_ptr,
                              uint32_t capacity, uint2* __restrict__ ranges, uint32_t n_tiles) {
  const uint32_t n = clamped(n_ptr, capacity);
  const uint32_t k0 = (blockIdx.x * blockDim.x + threadIdx.x) * 4u;
  if (k0 >= n) return;
  uint32_t t[4];
  if (k0 + 4u <= capacity) {
    const uint4 q = *reinterpret_cast<const uint4*>(tiles + k0);
    t[0] = q.x; t[1] = q.y; t[2] = q.z; t[3] = q.w;
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) t[j] = k0 + j < n ? tiles[k0 + j] : 0u;
  }
  const uint32_t prev = k0 > 0 ? tiles[k0 - 1] : 0u;
  const uint32_t next = k0 + 4u < n ? tiles[k0 + 4u] : 0u;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t k = k0 + j;
    if (k >= n || t[j] >= n_tiles) continue;
    const uint32_t before = j > 0 ? t[j - 1] : prev, after = j < 3 ? t[j + 1] : next;
    if (k == 0 || before != t[j]) ranges[t[j]].x = k;
    if (k == n - 1 || after != t[j]) ranges[t[j]].y = k + 1;
  }
}

__global__ void key64_kernel(const uint32_t* __restrict__ tiles, const uint32_t* __restrict__ rec_of,
                             const float4* __restrict__ recs, const uint32_t* __restrict__ n_ptr, uint32_t capacity,
                             uint64_t* __restrict__ out) {
  const uint32_t n = clamped(n_ptr, capacity);
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= capacity) return;
  out[k] = k < n ? ((uint64_t)tiles[k] << 32) | __float_as_uint(recs[rec_slot(rec_of[k], 0)].z) : 0ull;
}

// Half-octave class of a list length: 0 for an empty list, else
// 1 + 2 floor(log2 len) + the bit below the leading one.
__device__ __forceinline__ int length_class(uint32_t len) {
  if (len == 0) return 0;
  const int lg = 31 - __clz((int)len);
  const int sub = lg > 0 ? (int)((len >> (lg - 1)) & 1u) : 0;
  return 1 + 2 * lg + sub;
}

__global__ void __launch_bounds__(256) tile_hist_kernel(const uint2* __restrict__ ranges, uint32_t n_tiles,
                                                        Counters* __restrict__ cnt) {
  __shared__ uint32_t h[kOrderBuckets];
  for (int b = threadIdx.x; b < kOrderBuckets; b += blockDim.x) h[b] = 0;
  __syncthreads();
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  if (t < n_tiles) {
    const uint2 r = ranges[t];
    atomicAdd(&h[length_class(r.y - r.x)], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kOrderBuckets; b += blockDim.x)
    if (h[b]) atomicAdd(&cnt->tile_hist[b], h[b]);
}

// Each workgroup ranks its tiles within their classes in LDS, reserves a run
// of slots per class with one global atomic, and writes its tiles there;
// classes are laid out from the longest down.
__global__ void __launch_bounds__(256) tile_order_kernel(const uint2* __restrict__ ranges, uint32_t n_tiles,
                                                         Counters* __restrict__ cnt, uint32_t* __restrict__ order) {
  __shared__ uint32_t first[kOrderBuckets], local[kOrderBuckets], base[kOrderBuckets];
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int b = kOrderBuckets - 1; b >= 0; --b) {
      first[b] = acc;
      acc += cnt->tile_hist[b];
    }
  }
  for (int b = threadIdx.x; b < kOrderBuckets; b += blockDim.x) local[b] = 0;
  __syncthreads();
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  int cls = 0;
  uint32_t rank = 0;
  if (t < n_tiles) {
    const uint2 r = ranges[t];
    cls = length_class(r.y - r.x);
    rank = atomicAdd(&local[cls], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kOrderBuckets; b += blockDim.x)
    base[b] = local[b] ? atomicAdd(&cnt->tile_cursor[b], local[b]) : 0u;
  __syncthreads();
  if (t < n_tiles) order[first[cls] + base[cls] + rank] = t;
}

}  // namespace

size_t sort_workspace_bytes(uint32_t capacity) { return radix_ws_bytes(capacity); }

hipError_t launch_depth_order(const CallTables& h, const ProjBuffers pb, const uint32_t* n_visible, DepthOrder d,
                              void* ws, hipStream_t s) {
  const uint32_t R = h.n_records;
  if (R == 0) return launch_fill_u32(d.pair_off_total, 0u, 1, s);
  int alt = 0;
  hipError_t e = radix_sort<uint32_t>(d.keys, d.vals, d.keys_alt, d.vals_alt, R, 32, n_visible, ws, &alt, s, nullptr,
                                      nullptr, pb.rect, d.rects, d.counts);
  if (e != hipSuccess) return e;
  *d.sorted_in_alt = alt;
  return launch_scan(d.counts, d.pair_off, R, d.pair_off_total, d.scan_ws, s, false, n_visible);
}

hipError_t launch_emit(const CallTables* d_tab, const CallTables& h, const uint32_t* sorted_rec,
                       const uint2* sorted_rect, const uint32_t* pair_off, const uint32_t* n_visible, Counters* cnt,
                       uint32_t* keys, uint32_t* vals, uint32_t capacity, hipStream_t s) {
  if (h.n_records == 0) return hipSuccess;
  hipLaunchKernelGGL(emit_kernel, dim3(div_up(h.n_records, kEmitBlock)), dim3(kEmitBlock), 0, s, d_tab, sorted_rec,
                     sorted_rect, pair_off, n_visible, cnt, h.n_records, capacity, keys, vals);
  return hipGetLastError();
}

hipError_t launch_radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, uint32_t capacity,
                             int key_bits, const uint32_t* n_dev, void* ws, int* result_in_alt, hipStream_t s,
                             const uint32_t* gather_src, uint32_t* gather_dst) {
  return radix_sort<uint32_t>(keys, vals, keys_alt, vals_alt, capacity, key_bits, n_dev, ws, result_in_alt, s,
                              gather_src, gather_dst);
}

hipError_t launch_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, uint32_t capacity,
                       int key_bits, const Counters* cnt, void* ws, int* result_in_alt, hipStream_t s) {
  return radix_sort<uint32_t>(keys, vals, keys_alt, vals_alt, capacity, key_bits, &cnt->pairs, ws, result_in_alt, s);
}

hipError_t launch_ranges(const uint32_t* tiles, const Counters* cnt, uint32_t capacity, uint2* ranges,
                         uint32_t n_tiles, hipStream_t s) {
  if (capacity == 0) return hipSuccess;  // (the projection left every range empty)
  hipLaunchKernelGGL(ranges_kernel, dim3(div_up(capacity, 1024)), dim3(256), 0, s, tiles, &cnt->pairs, capacity, ranges,
                     n_tiles);
  return hipGetLastError();
}

hipError_t launch_tile_order(const uint2* ranges, uint32_t n_tiles, Counters* cnt, uint32_t* order, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  const dim3 grid(div_up(n_tiles, 256));
  hipLaunchKernelGGL(tile_hist_kernel, grid, dim3(256), 0, s, ranges, n_tiles, cnt);
  hipLaunchKernelGGL(tile_order_kernel, grid, dim3(256), 0, s, ranges, n_tiles, cnt, order);
  return hipGetLastError();
}

hipError_t launch_key64(const uint32_t* tiles, const uint32_t* recs, const ProjBuffers pb, const Counters* cnt,
                        uint32_t capacity, uint64_t* out, hipStream_t s) {
  if (capacity == 0) return hipSuccess;
  hipLaunchKernelGGL(key64_kernel, dim3(div_up(capacity, 256)), dim3(256), 0, s, tiles, recs, pb.rec, &cnt->pairs,
                     capacity, out);
  return hipGetLastError();
}

}  // namespace vpgs
