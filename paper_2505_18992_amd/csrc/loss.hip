// loss.hip -- the mapping loss of eq. 7-9 and its gradient planes.
//
// Per view (rendered colour X, depth D; target colour Y, depth T):
//   L_c    = mean |X - Y| over channels and pixels
//   L_SSIM = (1 - ls) mean |X - Y| + ls (1 - mean SSIM(X, Y))     (eq. 8)
//   L_d    = mean |D - T| over pixels with T > 0
//   L      = L_c + L_SSIM + ld L_d                                  (eq. 7)
// SSIM uses an 11x11 Gaussian window (sigma 1.5) with zero padding, C1 =
// 0.01^2, C2 = 0.03^2.  The volume term of eq. 9 (ls, ld, lv the lambdas)
// is a separate per-Gaussian kernel that adds lv prod(exp(l)) to the
// log-scale gradients.
//
// SSIM at pixel p depends on the filtered statistics m1 = G*X, m2 = G*Y,
// e11 = G*X^2, e22 = G*Y^2, e12 = G*XY.  With S_p the map value,
//   dS_p/dX_q = G(p - q) (P1_p + 2 X_q P2_p + Y_q P3_p),
//   P1 = dS/dm1, P2 = dS/de11, P3 = dS/de12 (the others held fixed),
// so the gradient of mean S is (G*P1 + 2 X (G*P2) + Y (G*P3)) / N.  Two
// stencil kernels per view: the first filters the five statistics and
// writes S's partials (and block sums of the loss terms), the second
// filters the partials and writes the gradient planes.  A workgroup walks a
// 32-column strip down a segment of kSeg rows in bands of 32 rows: each band
// stages its new input rows (with a 5-column halo, zero outside the image),
// filters them horizontally once (each thread 4 adjacent outputs from
// registers), appends them to the 42 horizontally filtered rows the band's
// vertical filter needs (the last 10 rows of the previous band stay), and
// filters vertically (each thread 4 outputs down a column).  Only the first
// band of a segment filters 10 rows that another segment also filters.  One
// launch of each covers up to 16 views.
#include <algorithm>
#include <cmath>

#include "runtime.h"

namespace vpgs {
namespace {

constexpr int kRad = 5, kTaps = 2 * kRad + 1;
constexpr int kSW = 32;                   // strip width (output columns)
constexpr int kBand = 32;                 // output rows per band
constexpr int kSeg = 128;                 // output rows per workgroup (whole bands)
constexpr int kSWH = kSW + 2 * kRad;      // staged columns (42)
constexpr int kRows = kBand + 2 * kRad;   // horizontally filtered rows a band's vertical filter reads (42)
constexpr int kLossBlock = 256;
constexpr int kHRun = 4;  // horizontal outputs per thread: kBand rows x kSW / kHRun runs = kLossBlock
constexpr int kVRun = 4;  // vertical outputs per thread: kSW columns x kBand / kVRun runs = kLossBlock
static_assert(kBand * (kSW / kHRun) == kLossBlock && kSW * (kBand / kVRun) == kLossBlock, "filter runs");
static_assert(kSeg % kBand == 0 && 2 * kRad <= kBand, "bands");
constexpr float kC1 = 0.0001f, kC2 = 0.0009f;
constexpr int kSumSlots = 64;   // block sums are spread over slots per view
constexpr int kSums = 4;        // sum S, sum |X - Y|, sum valid |D - T|, valid count

// Normalised Gaussian taps, sigma 1.5: exp(-(k - 5)^2 / 4.5) / their sum,
// rounded to float.
__constant__ float kGauss[kTaps] = {1.028380124e-03f, 7.598758209e-03f, 3.600077331e-02f, 1.093606874e-01f,
                                    2.130055428e-01f, 2.660117149e-01f, 2.130055428e-01f, 1.093606874e-01f,
                                    3.600077331e-02f, 7.598758209e-03f, 1.028380124e-03f};

constexpr int kLossViews = 16;  // views per launch (their arguments travel by value)

struct ViewArgs {
  int W, H;
  const float* x;   // rendered colour [3,H,W]
  const float* d;   // rendered depth [H,W]
  const float* y;   // target colour
  const float* t;   // target depth
  float* gx;        // colour gradient [3,H,W]
  float* gd;        // depth gradient [H,W]
  float* ga;        // alpha gradient [H,W] (zeroed) or NULL
  float* P;         // partials workspace [3 channels][3][H,W]
  double* sums;     // [kSums][kSumSlots] of this view
  int tiles_x, tiles_y;
};

// A launch covers up to kLossViews views: grid = (max tiles_x, max tiles_y,
// 3 channels x views); workgroups past their view's tiles return.
struct LossBatch {
  ViewArgs v[kLossViews];
};

__device__ __forceinline__ float block_sum(float v, float* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  float r = 0.f;
#pragma unroll
  for (int w = 0; w < kLossBlock / 64; ++w) r += red[w];
  return r;  // every thread
}

// Stages input rows [r0, r0 + n) (n <= kBand) of NP planes, columns x0 - 5
// .. x0 + kSW + 4, into lds[q][0, n)[kSWH], zero outside the image.  Every
// load of the thread is issued before its first LDS write (out-of-image
// slots read the plane's first element and are replaced by zero).
constexpr int kStagePer = (kBand * kSWH + kLossBlock - 1) / kLossBlock;
// A thread's share of staging rows r0 .. r0 + n - 1 (columns x0 - kRad ..
// x0 + kSW + kRad - 1) of NP planes: loaded into registers by load(), then
// written to LDS by store() (zero outside the image), so the loads of the
// next rows can be issued while the current ones are still in use.
template <int NP>
struct StageRegs {
  float v[NP][kStagePer];
  bool in[kStagePer];
  int n;
  __device__ __forceinline__ void load(const float* const* src, int W, int H, int x0, int r0, int n_) {
    n = n_;
#pragma unroll
    for (int u = 0; u < kStagePer; ++u) {
      const int k = (int)threadIdx.x + u * kLossBlock;
      const int r = k / kSWH, c = k - r * kSWH;  // constant divisor
      const int gy = r0 + r, gx = x0 - kRad + c;
      in[u] = r < n && gx >= 0 && gx < W && gy >= 0 && gy < H;
      const size_t off = in[u] ? (size_t)gy * W + gx : 0;
#pragma unroll
      for (int q = 0; q < NP; ++q) v[q][u] = src[q][off];
    }
  }
  __device__ __forceinline__ void store(float (*lds)[kBand][kSWH]) const {
#pragma unroll
    for (int u = 0; u < kStagePer; ++u) {
      const int k = (int)threadIdx.x + u * kLossBlock;
      const int r = k / kSWH, c = k - r * kSWH;
      if (r >= n) continue;
#pragma unroll
      for (int q = 0; q < NP; ++q) lds[q][r][c] = in[u] ? v[q][u] : 0.0f;
    }
  }
};

template <int NP>
__device__ __forceinline__ void stage_rows(const float* const* src, int W, int H, int x0, int r0, int n,
                                           float (*lds)[kBand][kSWH]) {
  StageRegs<NP> st;
  st.load(src, W, H, x0, r0, n);
  st.store(lds);
}

// Moves the last 2 kRad horizontally filtered rows to the top of hs (the
// next band's upper halo).
template <int NQ>
__device__ __forceinline__ void keep_halo_rows(float (*hs)[kRows][kSW]) {
  float v[NQ][(2 * kRad * kSW + kLossBlock - 1) / kLossBlock];
#pragma unroll
  for (int u = 0; u < (2 * kRad * kSW + kLossBlock - 1) / kLossBlock; ++u) {
    const int k = (int)threadIdx.x + u * kLossBlock;
    if (k < 2 * kRad * kSW)
#pragma unroll
      for (int q = 0; q < NQ; ++q) v[q][u] = hs[q][kBand + k / kSW][k % kSW];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < (2 * kRad * kSW + kLossBlock - 1) / kLossBlock; ++u) {
    const int k = (int)threadIdx.x + u * kLossBlock;
    if (k < 2 * kRad * kSW)
#pragma unroll
      for (int q = 0; q < NQ; ++q) hs[q][k / kSW][k % kSW] = v[q][u];
  }
}

// Workgroups are dispatched to the eight XCDs round robin by linear id, and
// each XCD has its own L2.  Neighbouring strips share their halo columns, so
// the linear id is renumbered to give every XCD a contiguous run of strips:
// XCD k takes the k-th eighth of the grid in (x, y, z) order.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint3 xcd_block() {
  const uint32_t gx = gridDim.x, gy = gridDim.y;
  const uint32_t n = gx * gy * gridDim.z;
  const uint32_t h = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const uint32_t x = h % kXcds, k = h / kXcds, q = n / kXcds, r = n % kXcds;
  const uint32_t id = x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
  return make_uint3(id % gx, (id / gx) % gy, id / (gx * gy));
}

// ---------------------------------------------------------------------------
// kernel 1: statistics, SSIM partials and the block sums
// ---------------------------------------------------------------------------
// With A1 = 2 m1 m2 + C1, A2 = 2 (e12 - m1 m2) + C2, B1 = m1^2 + m2^2 + C1,
// B2 = (e11 - m1^2) + (e22 - m2^2) + C2 and S = A1 A2 / (B1 B2):
//   dS/dm1  = 2 / (B1 B2) (m2 (A2 - A1) + A1 A2 m1 (1 / B2 - 1 / B1))
//   dS/de11 = -A1 A2 / (B1 B2^2)
//   dS/de12 = 2 A1 / (B1 B2)
// (only B1 >= C1 and B2 >= C2 are divided by; A2 may vanish).
//
// Horizontal filter of the staged rows [0, n) of x and y into hs rows
// [dst, dst + n): the four statistics x, y, x^2 + y^2, xy.  Only the sum of
// the second moments enters SSIM (through sigma_x^2 + sigma_y^2), so the two
// are filtered as one map.
constexpr int kStats = 4;
__device__ __forceinline__ void stats_rows(const float (*sxy)[kBand][kSWH], int n, int dst,
                                           float (*hs)[kRows][kSW]) {
  const int r = threadIdx.x / (kSW / kHRun), j0 = (threadIdx.x % (kSW / kHRun)) * kHRun;
  if (r >= n) return;
  // the run's samples and their products, each formed once (not once per tap)
  float xv[kHRun + 2 * kRad], yv[kHRun + 2 * kRad], ss[kHRun + 2 * kRad], xy[kHRun + 2 * kRad];
#pragma unroll
  for (int t = 0; t < kHRun + 2 * kRad; ++t) {
    xv[t] = sxy[0][r][j0 + t];
    yv[t] = sxy[1][r][j0 + t];
    ss[t] = xv[t] * xv[t] + yv[t] * yv[t];
    xy[t] = xv[t] * yv[t];
  }
#pragma unroll
  for (int o = 0; o < kHRun; ++o) {
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
#pragma unroll
    for (int t = 0; t < kTaps; ++t) {
      const float g = kGauss[t];
      s0 = fmaf(g, xv[o + t], s0);
      s1 = fmaf(g, yv[o + t], s1);
      s2 = fmaf(g, ss[o + t], s2);
      s3 = fmaf(g, xy[o + t], s3);
    }
    hs[0][dst + r][j0 + o] = s0; hs[1][dst + r][j0 + o] = s1; hs[2][dst + r][j0 + o] = s2;
    hs[3][dst + r][j0 + o] = s3;
  }
}

// At most 128 VGPRs (four wavefronts per SIMD): the next band's rows held
// in registers would otherwise cost a wavefront per SIMD.
__global__ void __launch_bounds__(kLossBlock) __attribute__((amdgpu_waves_per_eu(4))) ssim_stats_kernel(LossBatch batch) {
  __shared__ float sxy[2][kBand][kSWH];  // staged x, y rows
  __shared__ float hs[kStats][kRows][kSW];  // horizontal sums of x, y, x^2 + y^2, xy
  __shared__ float red[kLossBlock / 64];
  const uint3 blk = xcd_block();
  const ViewArgs& a = batch.v[blk.z / 3];
  if ((int)blk.x >= a.tiles_x || (int)blk.y >= a.tiles_y) return;
  const int c = blk.z % 3;
  const int x0 = blk.x * kSW, y0 = blk.y * kSeg;
  const size_t HW = (size_t)a.W * a.H;
  const float* planes[2] = {a.x + c * HW, a.y + c * HW};
  float* P = a.P + (size_t)c * 3 * HW;
  float ssum = 0.f, l1sum = 0.f;
  // the segment's upper halo (input rows y0 - 5 .. y0 + 4), with the first
  // band's rows loaded alongside; each band then loads the next band's rows
  // while it filters
  StageRegs<2> nxt;
  {
    StageRegs<2> halo;
    halo.load(planes, a.W, a.H, x0, y0 - kRad, 2 * kRad);
    nxt.load(planes, a.W, a.H, x0, y0 + kRad, kBand);
    halo.store(sxy);
  }
  __syncthreads();
  stats_rows(sxy, 2 * kRad, 0, hs);
  const int seg_end = min(y0 + kSeg, a.H);
  const int vj = threadIdx.x % kSW, vi0 = (threadIdx.x / kSW) * kVRun;
  for (int yb = y0; yb < seg_end; yb += kBand) {
    const int lr = threadIdx.x / kSW, lj = threadIdx.x % kSW;
    // output rows yb .. yb + 4 are still staged from the previous band (its
    // staged rows kBand - 5 ..) or, in the first band, from the upper halo
    // (staged rows 5 .. 9): their |x - y| terms, before the staging below
    // overwrites them
    float lprev = 0.f;
    const bool lhave = lr < kRad && yb + lr < seg_end && x0 + lj < a.W;
    if (lhave) {
      const int rr = (yb == y0 ? kRad : kBand - kRad) + lr;
      lprev = fabsf(sxy[0][rr][lj + kRad] - sxy[1][rr][lj + kRad]);
    }
    __syncthreads();
    // input rows yb + 5 .. yb + kBand + 4 after the 10 already filtered
    nxt.store(sxy);
    __syncthreads();
    stats_rows(sxy, kBand, 2 * kRad, hs);
    {
      // |x - y| of the band's output pixels: rows yb + 5 .. yb + kBand - 1
      // are staged (staged row rr holds row yb + 5 + rr)
#pragma unroll
      for (int rr = lr; rr < kBand - kRad; rr += kLossBlock / kSW) {
        const int py = yb + kRad + rr;
        if (py < seg_end && x0 + lj < a.W) l1sum += fabsf(sxy[0][rr][lj + kRad] - sxy[1][rr][lj + kRad]);
      }
      if (lhave) l1sum += lprev;
    }
    __syncthreads();
    // the next band's input rows, in flight through this band's vertical filter
    if (yb + kBand < seg_end) nxt.load(planes, a.W, a.H, x0, yb + kBand + kRad, kBand);
    float vm[kStats][kVRun];
#pragma unroll
    for (int q = 0; q < kStats; ++q) {
      float col[kVRun + 2 * kRad];
#pragma unroll
      for (int t = 0; t < kVRun + 2 * kRad; ++t) col[t] = hs[q][vi0 + t][vj];
#pragma unroll
      for (int o = 0; o < kVRun; ++o) {
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t < kTaps; ++t) acc = fmaf(kGauss[t], col[o + t], acc);
        vm[q][o] = acc;
      }
    }
#pragma unroll
    for (int o = 0; o < kVRun; ++o) {
      const int px = x0 + vj, py = yb + vi0 + o;
      if (px >= a.W || py >= seg_end) continue;
      const float m1 = vm[0][o], m2 = vm[1][o], es = vm[2][o], e12 = vm[3][o];  // es = E[x^2] + E[y^2]
      const float A1 = 2.f * m1 * m2 + kC1, A2 = 2.f * (e12 - m1 * m2) + kC2;
      const float mm = m1 * m1 + m2 * m2;
      const float B1 = mm + kC1, B2 = (es - mm) + kC2;
      const float rB1 = 1.0f / B1, rB2 = 1.0f / B2;
      const float rr = rB1 * rB2;
      const float S = A1 * A2 * rr;
      const size_t pix = (size_t)py * a.W + px;
      P[pix] = 2.f * rr * (m2 * (A2 - A1) + A1 * A2 * m1 * (rB2 - rB1));  // dS/dm1
      P[HW + pix] = -S * rB2;                                               // dS/de11
      P[2 * HW + pix] = 2.f * A1 * rr;                                      // dS/de12
      ssum += S;
    }
    __syncthreads();
    keep_halo_rows<kStats>(hs);
  }
  const int slot = (int)((blk.y * a.tiles_x + blk.x) % kSumSlots);
  ssum = block_sum(ssum, red);
  l1sum = block_sum(l1sum, red);
  if (threadIdx.x == 0) {
    atomicAdd(&a.sums[0 * kSumSlots + slot], (double)ssum);
    atomicAdd(&a.sums[1 * kSumSlots + slot], (double)l1sum);
  }
  if (c == 0) {  // depth terms once per pixel
    // eight pixels' loads in flight per thread (out-of-range pixels read
    // pixel 0 and count nothing); the sums keep the pixel order
    constexpr int kDU = 8;
    static_assert((kSeg * kSW) % (kLossBlock * kDU) == 0, "whole chunks");
    float dsum = 0.f, nvalid = 0.f;
    for (int k0 = threadIdx.x; k0 < kSeg * kSW; k0 += kLossBlock * kDU) {
      float tv[kDU], dv[kDU];
      bool ok[kDU];
#pragma unroll
      for (int u = 0; u < kDU; ++u) {
        const int k = k0 + u * kLossBlock;
        const int i = k / kSW, j = k - i * kSW;
        const int px = x0 + j, py = y0 + i;
        ok[u] = px < a.W && py < a.H;
        const size_t pix = ok[u] ? (size_t)py * a.W + px : 0;
        tv[u] = a.t[pix];
        dv[u] = a.d[pix];
      }
#pragma unroll
      for (int u = 0; u < kDU; ++u)
        if (ok[u] && tv[u] > 0.0f) {
          dsum += fabsf(dv[u] - tv[u]);
          nvalid += 1.0f;
        }
    }
    dsum = block_sum(dsum, red);
    nvalid = block_sum(nvalid, red);
    if (threadIdx.x == 0) {
      atomicAdd(&a.sums[2 * kSumSlots + slot], (double)dsum);
      atomicAdd(&a.sums[3 * kSumSlots + slot], (double)nvalid);
    }
  }
}

// ---------------------------------------------------------------------------
// kernel 2: gradient planes
// ---------------------------------------------------------------------------
// Loss terms of one view from the block sums: L_c, L_SSIM, L_d, total.
__device__ void view_terms(const ViewArgs& a, float lam_ssim, float lam_d, float* __restrict__ terms) {
  const double* sums = a.sums;
  double s[kSums] = {0, 0, 0, 0};
  for (int q = 0; q < kSums; ++q)
    for (int k = 0; k < kSumSlots; ++k) s[q] += sums[q * kSumSlots + k];
  const double n = 3.0 * a.W * a.H;
  const double l1 = s[1] / n, ssim = s[0] / n;
  const double ld = s[3] > 0 ? s[2] / s[3] : 0.0;
  const double l_ssim = (1.0 - lam_ssim) * l1 + lam_ssim * (1.0 - ssim);
  terms[0] = (float)l1;
  terms[1] = (float)l_ssim;
  terms[2] = (float)ld;
  terms[3] = (float)(l1 + l_ssim + lam_d * ld);
}

__device__ __forceinline__ float sgnf(float v) { return v > 0.f ? 1.f : (v < 0.f ? -1.f : 0.f); }

// Horizontal filter of the staged rows [0, n) of the three partial planes
// into hs rows [dst, dst + n).
__device__ __forceinline__ void partial_rows(const float (*sp)[kBand][kSWH], int n, int dst,
                                             float (*hs)[kRows][kSW]) {
  const int r = threadIdx.x / (kSW / kHRun), j0 = (threadIdx.x % (kSW / kHRun)) * kHRun;
  if (r >= n) return;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    float row[kHRun + 2 * kRad];
#pragma unroll
    for (int t = 0; t < kHRun + 2 * kRad; ++t) row[t] = sp[q][r][j0 + t];
#pragma unroll
    for (int o = 0; o < kHRun; ++o) {
      float acc = 0.f;
#pragma unroll
      for (int t = 0; t < kTaps; ++t) acc = fmaf(kGauss[t], row[o + t], acc);
      hs[q][dst + r][j0 + o] = acc;
    }
  }
}

__global__ void __launch_bounds__(kLossBlock) ssim_grad_kernel(LossBatch batch, float lam_ssim, float lam_d,
                                                                 float* __restrict__ terms) {
  __shared__ float sp[3][kBand][kSWH];
  __shared__ float hs[3][kRows][kSW];
  __shared__ float s_nvalid;
  const uint3 blk = xcd_block();
  const ViewArgs& a = batch.v[blk.z / 3];
  if ((int)blk.x >= a.tiles_x || (int)blk.y >= a.tiles_y) return;
  const int c = blk.z % 3;
  const float n = 3.0f * (float)a.W * (float)a.H;
  const float w_ssim = -lam_ssim / n;
  const float w_l1 = (2.0f - lam_ssim) / n;  // L_c and the (1 - lambda_ssim) L1 part of L_SSIM
  const int x0 = blk.x * kSW, y0 = blk.y * kSeg;
  const size_t HW = (size_t)a.W * a.H;
  const float* P = a.P + (size_t)c * 3 * HW;
  const float* planes[3] = {P, P + HW, P + 2 * HW};
  if (c == 0 && threadIdx.x == 0) {  // valid target-depth pixels of the view (first kernel's sums)
    double nv = 0.0;
    for (int k = 0; k < kSumSlots; ++k) nv += a.sums[3 * kSumSlots + k];
    s_nvalid = (float)nv;
    // the first block of the view also reduces the first kernel's sums to the
    // view's loss terms: L_c, L_SSIM, L_d and the total (eq. 7-8)
    if (blk.x == 0 && blk.y == 0) view_terms(a, lam_ssim, lam_d, terms + 4 * (blk.z / 3));
  }
  stage_rows<3>(planes, a.W, a.H, x0, y0 - kRad, 2 * kRad, sp);
  __syncthreads();
  partial_rows(sp, 2 * kRad, 0, hs);
  const float nvalid = c == 0 ? s_nvalid : 0.f;  // read after the barrier below
  const int seg_end = min(y0 + kSeg, a.H);
  const int vj = threadIdx.x % kSW, vi0 = (threadIdx.x / kSW) * kVRun;
  for (int yb = y0; yb < seg_end; yb += kBand) {
    // the inputs of this thread's output pixels, issued before the staging
    // so their loads overlap it (out-of-range pixels read pixel 0)
    float ox[kVRun], oy[kVRun], ot[kVRun], od[kVRun];
#pragma unroll
    for (int o = 0; o < kVRun; ++o) {
      const int px = x0 + vj, py = yb + vi0 + o;
      const size_t pix = (px < a.W && py < seg_end) ? (size_t)py * a.W + px : 0;
      ox[o] = a.x[c * HW + pix];
      oy[o] = a.y[c * HW + pix];
      if (c == 0) {
        ot[o] = a.t[pix];
        od[o] = a.d[pix];
      } else {
        ot[o] = od[o] = 0.0f;
      }
    }
    __syncthreads();
    stage_rows<3>(planes, a.W, a.H, x0, yb + kRad, kBand, sp);
    __syncthreads();
    partial_rows(sp, kBand, 2 * kRad, hs);
    __syncthreads();
    float vq[3][kVRun];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      float col[kVRun + 2 * kRad];
#pragma unroll
      for (int t = 0; t < kVRun + 2 * kRad; ++t) col[t] = hs[q][vi0 + t][vj];
#pragma unroll
      for (int o = 0; o < kVRun; ++o) {
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t < kTaps; ++t) acc = fmaf(kGauss[t], col[o + t], acc);
        vq[q][o] = acc;
      }
    }
#pragma unroll
    for (int o = 0; o < kVRun; ++o) {
      const int px = x0 + vj, py = yb + vi0 + o;
      if (px >= a.W || py >= seg_end) continue;
      const float q1 = vq[0][o], q2 = vq[1][o], q3 = vq[2][o];
      const size_t pix = (size_t)py * a.W + px;
      const float xv = ox[o], yv = oy[o];
      a.gx[c * HW + pix] = w_ssim * (q1 + 2.f * xv * q2 + yv * q3) + w_l1 * sgnf(xv - yv);
      if (c == 0) {
        const float tv = ot[o];
        a.gd[pix] = (tv > 0.0f && nvalid > 0.f) ? lam_d * sgnf(od[o] - tv) / nvalid : 0.0f;
        if (a.ga) a.ga[pix] = 0.0f;
      }
    }
    __syncthreads();
    keep_halo_rows<3>(hs);
  }
}


// Volume term of eq. 9: loss = lv sum_i prod(exp(l_i)); adds lv prod(exp(l_i))
// to each of the three log-scale gradients of Gaussian i.
__global__ void volume_kernel(const float* __restrict__ ls, int64_t n, float lam_vol, float* __restrict__ dls,
                              double* __restrict__ acc) {
  __shared__ float red[kLossBlock / 64];
  const int64_t i = (int64_t)blockIdx.x * kLossBlock + threadIdx.x;
  float v = 0.f;
  if (i < n) {
    v = lam_vol * expf(ls[3 * i] + ls[3 * i + 1] + ls[3 * i + 2]);
    dls[3 * i] += v;
    dls[3 * i + 1] += v;
    dls[3 * i + 2] += v;
  }
  v = block_sum(v, red);
  if (threadIdx.x == 0) atomicAdd(&acc[blockIdx.x % kSumSlots], (double)v);
}

__global__ void volume_total_kernel(const double* __restrict__ acc, float* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int k = 0; k < kSumSlots; ++k) s += acc[k];
  *out = (float)s;
}

__global__ void zero_f64_kernel(double* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

}  // namespace
}  // namespace vpgs

using namespace vpgs;

int vpgs_mapping_loss(vpgs_ctx* ctx, int n_views, const vpgs_camera* cams, const vpgs_images* rendered,
                      const vpgs_targets* targets, const vpgs_loss_opts* opts, float* terms, const vpgs_images* grad,
                      void* stream) {
  if (!ctx) return VPGS_EINVAL;
  if (n_views < 0 || n_views > VPGS_MAX_VIEWS) return fail(ctx, VPGS_EINVAL, "n_views %d out of range", n_views);
  if (n_views == 0) return VPGS_OK;
  if (!cams || !rendered || !targets || !terms || !grad) return fail(ctx, VPGS_EINVAL, "NULL argument");
  const float lam_ssim = opts ? opts->lambda_ssim : 0.2f;
  const float lam_d = opts ? opts->lambda_depth : 1.0f;
  if (!(lam_ssim >= 0.f && lam_ssim <= 1.f) || !(lam_d >= 0.f) || !std::isfinite(lam_d))
    return fail(ctx, VPGS_EINVAL, "loss weights out of range");
  size_t ws = 0;
  for (int v = 0; v < n_views; ++v) {
    const int W = cams[v].width, H = cams[v].height;
    if (W <= 0 || H <= 0 || W > VPGS_MAX_DIM || H > VPGS_MAX_DIM)
      return fail(ctx, VPGS_EINVAL, "view %d: size %dx%d out of range", v, W, H);
    if (!rendered[v].rgb || !rendered[v].depth || !targets[v].rgb || !targets[v].depth || !grad[v].rgb ||
        !grad[v].depth)
      return fail(ctx, VPGS_EINVAL, "view %d: NULL image plane", v);
    ws += (size_t)9 * W * H * sizeof(float);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));
  int rc;
  const size_t sums_bytes = (size_t)n_views * kSums * kSumSlots * sizeof(double);
  if ((rc = ensure(ctx, ctx->loss_ws, ws)) || (rc = ensure(ctx, ctx->loss_sums, sums_bytes))) return rc;
  StageTimer timer(ctx, ST_LOSS, st);
  const int nz = n_views * kSums * kSumSlots;
  hipLaunchKernelGGL(zero_f64_kernel, dim3((nz + 255) / 256), dim3(256), 0, st,
                     static_cast<double*>(ctx->loss_sums.p), nz);
  HIP_TRY(hipGetLastError());
  size_t off = 0;  // each view's partials workspace
  for (int v0 = 0; v0 < n_views; v0 += kLossViews) {
    const int nb = std::min(kLossViews, n_views - v0);
    LossBatch batch{};
    int gx = 1, gy = 1;
    for (int b = 0; b < nb; ++b) {
      const int v = v0 + b;
      ViewArgs& a = batch.v[b];
      a.W = cams[v].width;
      a.H = cams[v].height;
      a.x = rendered[v].rgb;
      a.d = rendered[v].depth;
      a.y = targets[v].rgb;
      a.t = targets[v].depth;
      a.gx = grad[v].rgb;
      a.gd = grad[v].depth;
      a.ga = grad[v].alpha;
      a.P = static_cast<float*>(ctx->loss_ws.p) + off;
      off += (size_t)9 * a.W * a.H;
      a.sums = static_cast<double*>(ctx->loss_sums.p) + (size_t)v * kSums * kSumSlots;
      a.tiles_x = (a.W + kSW - 1) / kSW;
      a.tiles_y = (a.H + kSeg - 1) / kSeg;
      gx = std::max(gx, a.tiles_x);
      gy = std::max(gy, a.tiles_y);
    }
    const dim3 grid(gx, gy, 3 * nb);
    hipLaunchKernelGGL(ssim_stats_kernel, grid, dim3(kLossBlock), 0, st, batch);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(ssim_grad_kernel, grid, dim3(kLossBlock), 0, st, batch, lam_ssim, lam_d, terms + 4 * v0);
    HIP_TRY(hipGetLastError());
  }
  return VPGS_OK;
}

int vpgs_volume_loss(vpgs_ctx* ctx, int n_sets, const vpgs_gaussians* sets, float lambda_vol, float* loss,
                     const vpgs_gauss_grads* grads, void* stream) {
  if (!ctx) return VPGS_EINVAL;
  if (n_sets < 0 || n_sets > VPGS_MAX_SETS) return fail(ctx, VPGS_EINVAL, "n_sets %d out of range", n_sets);
  if (n_sets == 0) return VPGS_OK;
  if (!sets || !loss || !grads) return fail(ctx, VPGS_EINVAL, "NULL argument");
  if (!(lambda_vol >= 0.f) || !std::isfinite(lambda_vol)) return fail(ctx, VPGS_EINVAL, "lambda_vol out of range");
  for (int s = 0; s < n_sets; ++s) {
    if (sets[s].n < 0) return fail(ctx, VPGS_EINVAL, "set %d: negative size", s);
    if (sets[s].n > 0 && (!sets[s].log_scales || !grads[s].log_scales))
      return fail(ctx, VPGS_EINVAL, "set %d: NULL log-scales", s);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));
  int rc;
  if ((rc = ensure(ctx, ctx->loss_sums, (size_t)n_sets * kSumSlots * sizeof(double)))) return rc;
  StageTimer timer(ctx, ST_VOLUME, st);
  double* acc = static_cast<double*>(ctx->loss_sums.p);
  const int nz = n_sets * kSumSlots;
  hipLaunchKernelGGL(zero_f64_kernel, dim3((nz + 255) / 256), dim3(256), 0, st, acc, nz);
  HIP_TRY(hipGetLastError());
  for (int s = 0; s < n_sets; ++s) {
    const int64_t n = sets[s].n;
    if (n > 0) {
      const int64_t blocks = (n + kLossBlock - 1) / kLossBlock;
      if (blocks > 0x7fffffff) return fail(ctx, VPGS_EINVAL, "set %d too large", s);
      hipLaunchKernelGGL(volume_kernel, dim3((unsigned)blocks), dim3(kLossBlock), 0, st, sets[s].log_scales, n,
                         lambda_vol, grads[s].log_scales, acc + (size_t)s * kSumSlots);
      HIP_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(volume_total_kernel, dim3(1), dim3(64), 0, st, acc + (size_t)s * kSumSlots, loss + s);
    HIP_TRY(hipGetLastError());
  }
  return VPGS_OK;
}
