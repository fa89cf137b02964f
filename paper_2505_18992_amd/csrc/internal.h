// internal.h -- shared definitions of the HIP kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vpgs.h"

namespace vpgs {

// Method constants (FP32): the compositing cutoffs, the EWA low-pass
// dilation and the field-of-view guard of the projection.
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTransMin = 1e-4f;
constexpr float kDilate = 0.3f;
constexpr float kGuardLo = 0.15f;  // guard reaches 15% of the image beyond each edge
constexpr float kGuardHi = 1.15f;
constexpr float kDefaultNear = 0.2f;

// Number of per-record gradient accumulators written by the backward
// compositor.  With s = dL/dalpha * alpha per pixel (0 where alpha is
// clamped) and d = (u, v) - pixel centre they hold
//   sum s dx, sum s dy, sum s dx^2, sum s dx dy, sum s dy^2,   (conic moments)
//   sum s (= o dL/dopacity), dL/d(r, g, b), dL/dz.
constexpr int kNumAcc = 10;

// One view of a render call, as the kernels see it.
struct ViewDesc {
  int32_t W, H, tiles_x, tiles_y;
  uint32_t tile_base;  // first global tile id of the view
  uint32_t rec_base;   // first record of the view
  uint32_t pix_base;   // first pixel of the view in the concatenated per-pixel buffers
  int32_t set;         // Gaussian set rendered by the view
  float fx, fy, cx, cy, near_z;
  float glx, ghx, gly, ghy;  // guard limits on x/z and y/z
  float R[9], t[3];
  float* rgb;
  float* depth;
  float* alpha;
  const float* g_rgb;
  const float* g_depth;
  const float* g_alpha;
};

// One Gaussian set of a render call.
struct SetDesc {
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opacities;
  const float* colors;
  float* d_means;
  float* d_log_scales;
  float* d_quats;
  float* d_opacities;
  float* d_colors;
  float* accum;         // [n,4] expansion accumulators added to by the backward, or NULL
  int64_t n;
  uint32_t block_base;  // first thread block of the set in per-Gaussian launches
  int32_t view_first;   // its views are set_views[view_first .. view_first + view_count)
  int32_t view_count;
  int32_t pad;
};

struct CallTables {
  ViewDesc views[VPGS_MAX_VIEWS];
  SetDesc sets[VPGS_MAX_SETS];
  int32_t set_views[VPGS_MAX_VIEWS];
  int32_t n_views, n_sets;
  uint32_t n_records, n_tiles;
  int32_t accum_space;  // gradient of the accumulators: 0 pixels, 1 normalised device coordinates
  int32_t pad;
};

// Device counters of one forward.
// The evaluation and blend counts are spread over kCountSlots slots (each
// wavefront adds to the slot of its workgroup index) so that thousands of
// workgroups do not serialise on one address; readers sum the slots.
constexpr int kCountSlots = 64;
// Tiles are composited longest list first: their lengths fall into
// kOrderBuckets classes (half-octaves), ordered by descending class.
constexpr int kOrderBuckets = 66;
struct Counters {
  unsigned long long evaluated[kCountSlots];
  unsigned long long blended[kCountSlots];
  unsigned long long fwd_hits[kCountSlots];    // (wavefront, hit-list entry) steps of the forward
  unsigned long long bwd_hits[kCountSlots];    // and of the backward (added over backward calls)
  unsigned long long bwd_active[kCountSlots];  // backward steps in which some lane contributes
  uint32_t pairs;      // pairs requested by the scan
  uint32_t overflow;   // 1 if pairs > capacity
  uint32_t visible;
  uint32_t queue_fwd;  // tile tickets of the persistent forward compositor
  uint32_t queue_bwd;  // and of the persistent backward compositor
  uint32_t pad[3];
  uint32_t tile_hist[kOrderBuckets];    // tiles per list-length class (the compositing order)
  uint32_t tile_cursor[kOrderBuckets];  // slots taken in each class
};
static_assert(sizeof(Counters) <= 4096, "the counters are read back through a 4 KiB pinned buffer");

// Per-record projected data (struct of arrays).
// Per-(view, Gaussian) projection record: four float4 (64 bytes, one
// aligned line), written only for records that overlap a tile (count != 0):
//   [0] (u, v, z, opacity)
//   [1] (Qa, Qb, Qc, 0)            conic
//   [2] (r, g, b, 0)
//   [3] (hx, hy, ra, rc)           box half extents; ra, rc = the
//       reciprocals of 2a and 2c of the compositor's quadrant test (a, c =
//       -Qa, -Qc times kNegHalfLog2e)
// count, the depth key (IEEE bits of the FP32 z) and the inclusive tile
// rectangle (x0 | x1 << 16, y0 | y1 << 16) are separate arrays, read
// contiguously by the scans.
constexpr float kNegHalfLog2e = -0.72134752044448170368f;  // -log2(e) / 2
constexpr float kNegLog2e = -1.44269504088896340736f;
constexpr int kRecSlots = 4;
struct ProjBuffers {
  float4* rec;      // [R * kRecSlots]
  uint32_t* count;  // [R] tiles overlapped, 0 = culled
  uint32_t* zkey;   // [R] depth key of records with count != 0
  uint2* rect;      // [R] tile rectangle of records with count != 0
};
__host__ __device__ __forceinline__ size_t rec_slot(uint32_t r, int k) { return (size_t)r * kRecSlots + k; }

// ---- launch helpers (defined in the .hip files) --------------------------------

// The projection also resets the per-forward state: the counters and the
// tile ranges (every tile empty) before any later kernel of the forward.
hipError_t launch_project(const CallTables* d_tab, const CallTables& h_tab, ProjBuffers pb, int tile_w,
                          int tile_h, Counters* cnt, uint2* ranges, hipStream_t s);
// Blocks of the per-Gaussian launches.  The projection backward leaves one
// 6-float pose partial per (view, block, wavefront): the pose partial buffer
// holds n_views * project_blocks * kPosePartialsPerBlock * 6 floats.
constexpr int kPosePartialsPerBlock = 4;
uint32_t project_blocks(const CallTables& h);
// Reads each visible record's row of acc and leaves it zero.
hipError_t launch_project_backward(const CallTables* d_tab, const CallTables& h_tab, const ProjBuffers pb,
                                   float* acc, float* pose_partial, hipStream_t s);
hipError_t launch_pose_reduce(const CallTables* d_tab, const CallTables& h_tab, const float* pose_partial,
                              float* d_pose, hipStream_t s);

// Exclusive scan of n uint32 values (or, with flags, of value != 0); total
// (device, uint32) receives the sum.  With n_dev the length is the device
// count min(*n_dev, n): later values count as zero and are not written.
size_t scan_workspace_bytes(uint32_t n);
hipError_t launch_scan(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* total, void* ws,
                       hipStream_t s, bool flags = false, const uint32_t* n_dev = nullptr);

// (hx, hy) per record into out[R], zero where count == 0.
hipError_t launch_export_extent(const ProjBuffers pb, uint32_t n, float2* out, hipStream_t s);

// Stream compaction of the visible records (count != 0) in record order:
// keys = depth keys, vals = record index; *total = their number.
hipError_t launch_compact_visible(const uint32_t* count, const uint32_t* zkey, uint32_t n, uint32_t* keys,
                                  uint32_t* vals, uint32_t* total, void* ws, hipStream_t s);

// Depth order of the compacted visible records: stable sort by FP32 depth
// bits, their tile rectangles and counts gathered in that order (by the last
// sort pass) and the exclusive scan of the counts (pair offsets; the total
// goes to *pair_off_total).
struct DepthOrder {
  uint32_t* keys;
  uint32_t* vals;
  uint32_t* keys_alt;
  uint32_t* vals_alt;
  uint2* rects;
  uint32_t* counts;
  uint32_t* pair_off;
  uint32_t* pair_off_total;
  void* scan_ws;
  int* sorted_in_alt;  // host: 1 if the sorted records are in vals_alt
};
hipError_t launch_depth_order(const CallTables& h_tab, const ProjBuffers pb, const uint32_t* n_visible, DepthOrder d,
                              void* sort_ws, hipStream_t s);

// One (tile id, record) pair per overlapped tile, in depth order (records
// and their rectangles in that order, as the depth order leaves them).
hipError_t launch_emit(const CallTables* d_tab, const CallTables& h_tab, const uint32_t* sorted_rec,
                       const uint2* sorted_rect, const uint32_t* pair_off, const uint32_t* n_visible,
                       Counters* cnt, uint32_t* keys, uint32_t* vals, uint32_t capacity, hipStream_t s);

// Stable LSD radix sort of (tile id, record) pairs over key bits [0, key_bits).
// The pair count is read from cnt->pairs (clamped to capacity) on the device.
size_t sort_workspace_bytes(uint32_t capacity);
hipError_t launch_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                       uint32_t capacity, int key_bits, const Counters* cnt, void* ws, int* result_in_alt,
                       hipStream_t s);

// Stable LSD radix sort of (key, value) over key bits [0, key_bits) for the
// first min(*n_dev, capacity) entries; the result is in the alt buffers iff
// *result_in_alt.  The last pass also writes gather_dst[i] =
// gather_src[value of sorted entry i] when both are non-NULL.
hipError_t launch_radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, uint32_t capacity,
                             int key_bits, const uint32_t* n_dev, void* ws, int* result_in_alt, hipStream_t s,
                             const uint32_t* gather_src, uint32_t* gather_dst);

// Per-tile [start, end) of the sorted pairs; ranges must hold zeros on entry
// (empty tiles are not written).
hipError_t launch_ranges(const uint32_t* tiles, const Counters* cnt, uint32_t capacity, uint2* ranges,
                         uint32_t n_tiles, hipStream_t s);
// The compositing order of the tiles: order[i] is the tile the i-th
// workgroup (or queue ticket) takes, by descending half-octave of the list
// length, so that the longest lists start first (the order within a class is
// unspecified; every tile appears once).  Uses the zeroed tile_hist and
// tile_cursor of cnt.
hipError_t launch_tile_order(const uint2* ranges, uint32_t n_tiles, Counters* cnt, uint32_t* order, hipStream_t s);

// Sorted keys in the exported 64-bit form (tile id << 32 | depth bits).
hipError_t launch_key64(const uint32_t* tiles, const uint32_t* recs, const ProjBuffers pb, const Counters* cnt,
                        uint32_t capacity, uint64_t* out, hipStream_t s);

// Compositing: one workgroup per tile, or (queue != NULL) `blocks`
// persistent workgroups taking tiles from the zeroed counter *queue; the
// i-th workgroup or ticket takes tile order[i].
// Each tile's list is staged in LDS in batches of lds_batch entries (half,
// once or twice the tile's pixel count, a multiple of 64:
// lds_batch_supported).  The forward leaves per (tile, batch, wavefront) the
// bits of the batch entries that reach the wavefront's quadrant in masks
// (hit_mask_bytes of them for the pair capacity, tile shape and batch); the
// backward reads them.
bool lds_batch_supported(int tw, int th, int lds_batch);
size_t hit_mask_bytes(uint32_t capacity, uint32_t n_tiles, int tile_w, int tile_h, int lds_batch);
hipError_t launch_composite_forward(const CallTables* d_tab, const CallTables& h_tab, const ProjBuffers pb,
                                    const uint2* ranges, const uint32_t* vals, const uint32_t* order,
                                    float* T_final, uint32_t* n_contrib, uint64_t* masks, Counters* cnt,
                                    bool count, int tile_w, int tile_h, int lds_batch, uint32_t* queue,
                                    uint32_t blocks, hipStream_t s);
hipError_t launch_composite_backward(const CallTables* d_tab, const CallTables& h_tab, const ProjBuffers pb,
                                     const uint2* ranges, const uint32_t* vals, const uint32_t* order,
                                     const float* T_final, const uint32_t* n_contrib, const uint64_t* masks,
                                     float* acc, Counters* cnt, int tile_w, int tile_h, int lds_batch,
                                     uint32_t* queue, uint32_t blocks, hipStream_t s);

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t n, hipStream_t s);
hipError_t launch_fill_f32(float* p, float value, size_t n, hipStream_t s);

bool tile_shape_supported(int tw, int th);

}  // namespace vpgs
