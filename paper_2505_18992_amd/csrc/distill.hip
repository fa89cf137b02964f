// distill.hip -- the submap-fusion distillation loss of eq. 14 and its
// gradient planes.
//
// Keyframe k of the overlap of submaps alpha and beta is rendered from both
// (colour C_a, C_b [3,H,W], depth D_a, D_b [H,W]):
//   l_k = mean (C_a - C_b)^2 over channels and pixels + mean (D_a - D_b)^2 over pixels
//   L   = (1/m) sum_k l_k
// and both sides get the gradient: dL/dC_a = 2 (C_a - C_b) / (3 m H W) =
// -dL/dC_b, dL/dD_a = 2 (D_a - D_b) / (m H W) = -dL/dD_b.  One streaming
// pass reads the four planes once and writes the gradient planes once; the
// squared differences are reduced per workgroup in FP32 and across
// workgroups in FP64.
#include <algorithm>
#include <cmath>

#include "runtime.h"

namespace vpgs {
namespace {

constexpr int kDistBlock = 256;
constexpr int kDistPix = 4 * kDistBlock;  // pixels per workgroup
constexpr int kDistPairs = 8;             // keyframes per launch (arguments by value)
constexpr int kDistSlots = 64;            // FP64 partial sums spread over slots per keyframe

struct PairArgs {
  int32_t W, H, nb, pad;
  const float* ca;
  const float* da;
  const float* cb;
  const float* db;
  float* gca;  // any gradient plane may be NULL
  float* gda;
  float* gaa;  // alpha gradients: zeroed when given
  float* gcb;
  float* gdb;
  float* gab;
  double* sums;  // [2][kDistSlots]: colour and depth sums of squares
  float sc, sd;  // 2 / (3 m H W) and 2 / (m H W)
};

struct PairBatch {
  PairArgs p[kDistPairs];
};

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__global__ void __launch_bounds__(kDistBlock) distill_kernel(PairBatch B) {
  __shared__ float red[2][kDistBlock / 64];
  const PairArgs& P = B.p[blockIdx.y];
  if ((int)blockIdx.x >= P.nb) return;  // workgroup-uniform
  const int64_t HW = (int64_t)P.W * P.H;
  const int64_t base = (int64_t)blockIdx.x * kDistPix;
  float ssc = 0.f, ssd = 0.f;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t i = base + q * kDistBlock + threadIdx.x;
    if (i >= HW) continue;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float e = P.ca[c * HW + i] - P.cb[c * HW + i];
      ssc = fmaf(e, e, ssc);
      const float g = P.sc * e;
      if (P.gca) P.gca[c * HW + i] = g;
      if (P.gcb) P.gcb[c * HW + i] = -g;
    }
    const float e = P.da[i] - P.db[i];
    ssd = fmaf(e, e, ssd);
    const float g = P.sd * e;
    if (P.gda) P.gda[i] = g;
    if (P.gdb) P.gdb[i] = -g;
    if (P.gaa) P.gaa[i] = 0.f;
    if (P.gab) P.gab[i] = 0.f;
  }
  ssc = wave_sum(ssc);
  ssd = wave_sum(ssd);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = ssc;
    red[1][threadIdx.x >> 6] = ssd;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kDistBlock / 64; ++w) s += (double)red[threadIdx.x][w];
    atomicAdd(P.sums + threadIdx.x * kDistSlots + (blockIdx.x % kDistSlots), s);
  }
}

__global__ void distill_zero_kernel(double* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

struct PairCounts {
  int64_t n[VPGS_MAX_VIEWS];  // pixels of each keyframe
};

// terms[2k + j] = sums / count; loss = (1/m) sum of all terms.
__global__ void distill_terms_kernel(const double* __restrict__ sums, PairCounts counts, int m,
                                     float* __restrict__ terms, float* __restrict__ loss) {
  __shared__ double tot[64];
  double acc = 0.0;
  for (int k = threadIdx.x; k < m; k += blockDim.x) {
    double s[2] = {0.0, 0.0};
    for (int j = 0; j < 2; ++j)
      for (int t = 0; t < kDistSlots; ++t) s[j] += sums[((size_t)k * 2 + j) * kDistSlots + t];
    const double tc = s[0] / (3.0 * (double)counts.n[k]);
    const double td = s[1] / (double)counts.n[k];
    if (terms) {
      terms[2 * k] = (float)tc;
      terms[2 * k + 1] = (float)td;
    }
    acc += tc + td;
  }
  tot[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int t = 0; t < (int)blockDim.x; ++t) a += tot[t];
    if (loss) *loss = (float)(a / m);
  }
}

}  // namespace
}  // namespace vpgs

using namespace vpgs;

extern "C" {

int vpgs_distill_loss(vpgs_ctx* ctx, int m, const vpgs_camera* cams, const vpgs_images* rend_a,
                      const vpgs_images* rend_b, float* terms, float* loss, const vpgs_images* grad_a,
                      const vpgs_images* grad_b, void* stream) {
  if (!ctx) return VPGS_EINVAL;
  if (m < 0 || m > VPGS_MAX_VIEWS) return fail(ctx, VPGS_EINVAL, "m = %d keyframes out of range", m);
  if (m == 0) return VPGS_OK;
  if (!cams || !rend_a || !rend_b) return fail(ctx, VPGS_EINVAL, "NULL argument");
  if (!terms && !loss && !grad_a && !grad_b) return fail(ctx, VPGS_EINVAL, "no output requested");
  for (int k = 0; k < m; ++k) {
    const int W = cams[k].width, H = cams[k].height;
    if (W <= 0 || H <= 0 || W > VPGS_MAX_DIM || H > VPGS_MAX_DIM)
      return fail(ctx, VPGS_EINVAL, "keyframe %d: size %dx%d out of range", k, W, H);
    if (!rend_a[k].rgb || !rend_a[k].depth || !rend_b[k].rgb || !rend_b[k].depth)
      return fail(ctx, VPGS_EINVAL, "keyframe %d: NULL rendered plane", k);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));
  const size_t nsums = (size_t)m * 2 * kDistSlots;
  int rc;
  if ((rc = ensure(ctx, ctx->distill_ws, nsums * sizeof(double)))) return rc;
  double* sums = static_cast<double*>(ctx->distill_ws.p);
  PairCounts counts{};
  for (int k = 0; k < m; ++k) counts.n[k] = (int64_t)cams[k].width * cams[k].height;
  StageTimer timer(ctx, ST_DISTILL, st);
  hipLaunchKernelGGL(distill_zero_kernel, dim3((unsigned)((nsums + 255) / 256)), dim3(256), 0, st, sums, (int)nsums);
  HIP_TRY(hipGetLastError());
  for (int k0 = 0; k0 < m; k0 += kDistPairs) {
    const int np = std::min(kDistPairs, m - k0);
    PairBatch B{};
    int max_nb = 1;
    for (int j = 0; j < np; ++j) {
      const int k = k0 + j;
      PairArgs& P = B.p[j];
      P.W = cams[k].width;
      P.H = cams[k].height;
      const int64_t HW = (int64_t)P.W * P.H;
      P.nb = (int)((HW + kDistPix - 1) / kDistPix);
      max_nb = std::max(max_nb, P.nb);
      P.ca = rend_a[k].rgb; P.da = rend_a[k].depth;
      P.cb = rend_b[k].rgb; P.db = rend_b[k].depth;
      if (grad_a) { P.gca = grad_a[k].rgb; P.gda = grad_a[k].depth; P.gaa = grad_a[k].alpha; }
      if (grad_b) { P.gcb = grad_b[k].rgb; P.gdb = grad_b[k].depth; P.gab = grad_b[k].alpha; }
      P.sums = sums + (size_t)k * 2 * kDistSlots;
      P.sc = (float)(2.0 / (3.0 * (double)m * (double)HW));
      P.sd = (float)(2.0 / ((double)m * (double)HW));
    }
    hipLaunchKernelGGL(distill_kernel, dim3(max_nb, np), dim3(kDistBlock), 0, st, B);
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(distill_terms_kernel, dim3(1), dim3(64), 0, st, sums, counts, m, terms, loss);
  HIP_TRY(hipGetLastError());
  return VPGS_OK;
}

}  // extern "C"
