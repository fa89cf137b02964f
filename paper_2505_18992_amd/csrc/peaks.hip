// peaks.hip -- microbenchmarks of the device rates that bound the kernels
// of this library: LDS read bandwidth (distinct addresses per lane and one
// broadcast address per wavefront, the compositors' pattern), the FP32
// fused-multiply-add rate, the exp2 rate, and HBM copy bandwidth.  The
// roofline fractions reported for the kernels are taken against these
// measured rates as well as against the published ones.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "runtime.h"

namespace vpgs {
namespace {

constexpr int kPeakBlock = 256;
constexpr int kLdsEntries = 2048;  // float4: 32 KiB of LDS per workgroup
constexpr int kLdsUnroll = 16;

// Every lane reads kLdsUnroll float4 per iteration at constant offsets from
// a base that moves by one entry per iteration (so the loads cannot be
// hoisted); BROADCAST reads one address per wavefront.  All indices stay
// below kLdsEntries: base < kLdsEntries / 2 and the offsets stay below
// kLdsUnroll * 64 = kLdsEntries / 2.
template <bool BROADCAST>
__global__ void __launch_bounds__(kPeakBlock) lds_read_kernel(int iters, float* __restrict__ sink) {
  __shared__ float4 buf[kLdsEntries];
  for (int i = threadIdx.x; i < kLdsEntries; i += kPeakBlock) buf[i] = make_float4((float)i, 1.f, 2.f, 3.f);
  __syncthreads();
  const int lane = BROADCAST ? 0 : (int)(threadIdx.x & 63);
  // the four words of every read are summed as integers, two by two (one
  // three-input add each), so the reads stay 16-byte reads and the adds
  // take half the issue slots an LDS read of 64 lanes takes
  uint32_t acc0 = 0u, acc1 = 0u;
  for (int it = 0; it < iters; ++it) {
    const int base = (lane + it) & (kLdsEntries / 2 - 1);
#pragma unroll
    for (int u = 0; u < kLdsUnroll; ++u) {
      const float4 v = buf[base + u * 64];
      acc0 = acc0 + __float_as_uint(v.x) + __float_as_uint(v.y);
      acc1 = acc1 + __float_as_uint(v.z) + __float_as_uint(v.w);
    }
  }
  if (acc0 == 1u && acc1 == 1u) sink[blockIdx.x * kPeakBlock + threadIdx.x] = 1.0f;  // never true; keeps the reads
}

// Eight independent FMA chains per lane.
__global__ void __launch_bounds__(kPeakBlock) fma_kernel(int iters, float b, float c, float* __restrict__ sink) {
  float a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = (float)(threadIdx.x + k);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int k = 0; k < 8; ++k) a[k] = fmaf(a[k], b, c);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += a[k];
  if (s == -1.0f) sink[blockIdx.x * kPeakBlock + threadIdx.x] = s;
}

// Eight independent exp2 chains per lane (the compositors' transcendental).
__global__ void __launch_bounds__(kPeakBlock) exp2_kernel(int iters, float* __restrict__ sink) {
  float a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = -0.001f * (float)(threadIdx.x + k);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int k = 0; k < 8; ++k) a[k] = __builtin_amdgcn_exp2f(a[k]);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += a[k];
  if (s == -1.0f) sink[blockIdx.x * kPeakBlock + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kPeakBlock) copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                          size_t n) {
  const size_t stride = (size_t)gridDim.x * kPeakBlock;
  for (size_t i = (size_t)blockIdx.x * kPeakBlock + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

template <class F>
int time_ms(vpgs_ctx* ctx, hipStream_t st, int reps, F&& launch, double* ms) {
  hipEvent_t a, b;
  HIP_TRY(hipEventCreate(&a));
  HIP_TRY(hipEventCreate(&b));
  launch();  // warm-up
  double best = 1e30;
  for (int r = 0; r < reps; ++r) {
    (void)hipEventRecord(a, st);
    launch();
    (void)hipEventRecord(b, st);
    if (hipEventSynchronize(b) != hipSuccess) break;
    float t = 0.f;
    (void)hipEventElapsedTime(&t, a, b);
    best = std::min(best, (double)t);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  HIP_TRY(hipGetLastError());
  *ms = best;
  return VPGS_OK;
}

}  // namespace
}  // namespace vpgs

using namespace vpgs;

extern "C" {

int vpgs_measure_peaks(vpgs_ctx* ctx, double* out, void* stream) {
  if (!ctx) return VPGS_EINVAL;
  if (!out) return fail(ctx, VPGS_EINVAL, "NULL output");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
  const int blocks = 8 * cus;  // eight workgroups of 256 lanes per compute unit
  const size_t copy_floats4 = (size_t)1 << 24;  // 256 MiB per side
  int rc = ensure(ctx, ctx->peak_ws, 2 * copy_floats4 * sizeof(float4));
  if (rc) return rc;
  float4* src = static_cast<float4*>(ctx->peak_ws.p);
  float4* dst = src + copy_floats4;
  float* sink = reinterpret_cast<float*>(dst);  // never written (see the kernels)
  HIP_TRY(hipMemsetAsync(src, 0, 2 * copy_floats4 * sizeof(float4), st));
  double ms = 0.0;
  const int lds_iters = 2048, fma_iters = 2048, exp_iters = 512;
  // [0] LDS, distinct addresses: 16 bytes per lane per read
  if ((rc = time_ms(ctx, st, 3, [&] {
         hipLaunchKernelGGL(lds_read_kernel<false>, dim3(blocks), dim3(kPeakBlock), 0, st, lds_iters, sink);
       }, &ms)))
    return rc;
  out[0] = (double)blocks * kPeakBlock * lds_iters * kLdsUnroll * 16.0 / (ms * 1e-3) / 1e9;
  // [1] LDS, one address per wavefront
  if ((rc = time_ms(ctx, st, 3, [&] {
         hipLaunchKernelGGL(lds_read_kernel<true>, dim3(blocks), dim3(kPeakBlock), 0, st, lds_iters, sink);
       }, &ms)))
    return rc;
  out[1] = (double)blocks * kPeakBlock * lds_iters * kLdsUnroll * 16.0 / (ms * 1e-3) / 1e9;
  // [2] FP32 FMA
  if ((rc = time_ms(ctx, st, 3, [&] {
         hipLaunchKernelGGL(fma_kernel, dim3(blocks), dim3(kPeakBlock), 0, st, fma_iters, 0.999f, 1e-3f, sink);
       }, &ms)))
    return rc;
  out[2] = (double)blocks * kPeakBlock * fma_iters * 64.0 * 2.0 / (ms * 1e-3) / 1e12;
  // [3] exp2
  if ((rc = time_ms(ctx, st, 3, [&] {
         hipLaunchKernelGGL(exp2_kernel, dim3(blocks), dim3(kPeakBlock), 0, st, exp_iters, sink);
       }, &ms)))
    return rc;
  out[3] = (double)blocks * kPeakBlock * exp_iters * 64.0 / (ms * 1e-3) / 1e12;
  // [4] HBM copy: bytes read + written
  if ((rc = time_ms(ctx, st, 5, [&] {
         hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(kPeakBlock), 0, st, src, dst, copy_floats4);
       }, &ms)))
    return rc;
  out[4] = 2.0 * copy_floats4 * sizeof(float4) / (ms * 1e-3) / 1e9;
  return VPGS_OK;
}

}  // extern "C"
