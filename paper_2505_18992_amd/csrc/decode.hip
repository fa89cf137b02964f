// decode.hip -- neural Gaussians from voxel anchors (Section III-A, eq. 1-5)
// and the backward of that decode.
//
// Forward, one thread per anchor: the 36-vector [feature, view direction,
// distance] (eq. 3) goes through three LINEAR-ReLU-LINEAR heads (eq. 2); the
// k Gaussians of the anchor get mean = anchor + offset * scaling (eq. 1),
// opacity = tanh, colour = sigmoid (eq. 4), log-scale = log sigmoid + log of
// the anchor scaling (eq. 5) and a normalised quaternion.  Weight indices are
// uniform across the wavefront, so the weights stream through scalar loads
// and every lane keeps its hidden layer in a private column of LDS.
//
// Backward: one thread per anchor chains the upstream Gaussian gradients
// through the activations and both layers (feature, scaling and offset
// gradients are written directly) and stores the per-anchor layer inputs and
// output gradients; the weight gradients are then split-K reductions
// (sum over anchors of outer products) written as per-chunk partials and
// summed in a fixed order, so they are deterministic.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "runtime.h"

namespace vpgs {
namespace {

constexpr int kIn = 36;
constexpr int kDecBlock = 64;  // one wavefront per block: LDS holds (width + 7k) floats per thread

struct DecArgs {
  int64_t m;
  int k, width;
  const float* xyz;
  const float* feat;
  const float* scale;
  const float* offsets;
  const float* W1[3];
  const float* b1[3];
  const float* W2[3];
  const float* b2[3];
  float cx, cy, cz;
  // forward outputs
  float* means;
  float* log_scales;
  float* quats;
  float* opac;
  float* colors;
  // backward inputs / outputs
  const float* g_means;
  const float* g_ls;
  const float* g_quats;
  const float* g_opac;
  const float* g_colors;
  float* d_feat;
  float* d_scale;
  float* d_offsets;
  float* ws_h;       // [m, 36]
  float* ws_hid[3];  // [m, width] post-ReLU hidden layer
  float* ws_dpre[3]; // [m, width] gradient at the hidden pre-activation
  float* ws_dy[3];   // [m, out_h] gradient at the head outputs
};

__device__ __forceinline__ float sigmoidf_(float y) { return 1.0f / (1.0f + expf(-y)); }
__device__ __forceinline__ float log_sigmoidf_(float y) { return -(fmaxf(-y, 0.0f) + log1pf(expf(-fabsf(y)))); }

// h = [feat (32), direction (3), distance (1)] of anchor a (eq. 3)
__device__ __forceinline__ void anchor_input(const DecArgs& A, int64_t a, float h[kIn]) {
#pragma unroll
  for (int i = 0; i < 32; ++i) h[i] = A.feat[a * 32 + i];
  const float dx = A.xyz[3 * a] - A.cx, dy = A.xyz[3 * a + 1] - A.cy, dz = A.xyz[3 * a + 2] - A.cz;
  const float delta = sqrtf(dx * dx + dy * dy + dz * dz);
  const float inv = 1.0f / delta;
  h[32] = dx * inv;
  h[33] = dy * inv;
  h[34] = dz * inv;
  h[35] = delta;
}

// Per-thread vectors of the hidden layer live in LDS, column-major over the
// block (element j of thread t at [j * kDecBlock + t]), so loops over the
// hidden units need no unrolling.
__device__ __forceinline__ void hidden_layer(const float* __restrict__ W1, const float* __restrict__ b1, int width,
                                             const float h[kIn], float* hid) {
  for (int j = 0; j < width; ++j) {
    float acc = b1[j];
#pragma unroll
    for (int i = 0; i < kIn; ++i) acc = fmaf(W1[j * kIn + i], h[i], acc);
    hid[j * kDecBlock] = fmaxf(acc, 0.0f);
  }
}

__device__ __forceinline__ float head_out(const float* __restrict__ W2, const float* __restrict__ b2, int width, int row,
                                          const float* hid) {
  float acc = b2[row];
  const float* w = W2 + (size_t)row * width;
#pragma unroll 4
  for (int j = 0; j < width; ++j) acc = fmaf(w[j], hid[j * kDecBlock], acc);
  return acc;
}

__global__ void __launch_bounds__(kDecBlock) decode_forward_kernel(DecArgs A) {
  extern __shared__ float lds[];
  float* hid = lds + threadIdx.x;
  const int64_t a = (int64_t)blockIdx.x * kDecBlock + threadIdx.x;
  if (a >= A.m) return;
  const int k = A.k, width = A.width;
  float h[kIn];
  anchor_input(A, a, h);
  const float l0 = A.scale[3 * a], l1 = A.scale[3 * a + 1], l2 = A.scale[3 * a + 2];
  const float x0 = A.xyz[3 * a], x1 = A.xyz[3 * a + 1], x2 = A.xyz[3 * a + 2];
  for (int m = 0; m < k; ++m) {  // eq. 1
    const int64_t g = a * k + m;
    A.means[3 * g] = x0 + A.offsets[3 * g] * l0;
    A.means[3 * g + 1] = x1 + A.offsets[3 * g + 1] * l1;
    A.means[3 * g + 2] = x2 + A.offsets[3 * g + 2] * l2;
  }
  hidden_layer(A.W1[0], A.b1[0], width, h, hid);
  for (int m = 0; m < k; ++m) A.opac[a * k + m] = tanhf(head_out(A.W2[0], A.b2[0], width, m, hid));
  hidden_layer(A.W1[1], A.b1[1], width, h, hid);
  for (int r = 0; r < 3 * k; ++r) A.colors[a * 3 * k + r] = sigmoidf_(head_out(A.W2[1], A.b2[1], width, r, hid));
  hidden_layer(A.W1[2], A.b1[2], width, h, hid);
  const float ll[3] = {logf(l0), logf(l1), logf(l2)};
  for (int m = 0; m < k; ++m) {
    float y[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) y[j] = head_out(A.W2[2], A.b2[2], width, 7 * m + j, hid);
    const int64_t g = a * k + m;
#pragma unroll
    for (int j = 0; j < 3; ++j) A.log_scales[3 * g + j] = log_sigmoidf_(y[j]) + ll[j];
    const float n = fmaxf(sqrtf(y[3] * y[3] + y[4] * y[4] + y[5] * y[5] + y[6] * y[6]), 1e-12f);
    const float in = 1.0f / n;
#pragma unroll
    for (int j = 0; j < 4; ++j) A.quats[4 * g + j] = y[3 + j] * in;
  }
}

// dhid = W2^T dy, dpre = dhid on active units, dh += W1^T dpre; stores the
// hidden layer and dpre for the weight gradients.
__device__ __forceinline__ void head_backward(const DecArgs& A, int head, int64_t a, int n_out, const float* hid,
                                              const float* dyl, float dh[kIn]) {
  const int width = A.width;
  float* hs = A.ws_hid[head] + a * width;
  float* ds = A.ws_dpre[head] + a * width;
  const float* W1 = A.W1[head];
  const float* W2 = A.W2[head];
  for (int j = 0; j < width; ++j) {
    float dhid = 0.0f;
#pragma unroll 4
    for (int o = 0; o < n_out; ++o) dhid = fmaf(W2[(size_t)o * width + j], dyl[o * kDecBlock], dhid);
    const float hv = hid[j * kDecBlock];
    const float dp = hv > 0.0f ? dhid : 0.0f;
    hs[j] = hv;
    ds[j] = dp;
#pragma unroll
    for (int i = 0; i < kIn; ++i) dh[i] = fmaf(W1[j * kIn + i], dp, dh[i]);
  }
}

__global__ void __launch_bounds__(kDecBlock) decode_backward_kernel(DecArgs A) {
  extern __shared__ float lds[];
  float* hid = lds + threadIdx.x;
  float* dyl = lds + (size_t)A.width * kDecBlock + threadIdx.x;
  const int64_t a = (int64_t)blockIdx.x * kDecBlock + threadIdx.x;
  if (a >= A.m) return;
  const int k = A.k, width = A.width;
  float h[kIn], dh[kIn];
  anchor_input(A, a, h);
#pragma unroll
  for (int i = 0; i < kIn; ++i) {
    A.ws_h[a * kIn + i] = h[i];
    dh[i] = 0.0f;
  }
  const float l[3] = {A.scale[3 * a], A.scale[3 * a + 1], A.scale[3 * a + 2]};
  float dl[3] = {0.f, 0.f, 0.f};
  // eq. 1: mean = anchor + offset * l
  for (int m = 0; m < k; ++m) {
    const int64_t g = a * k + m;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float gm = A.g_means[3 * g + c];
      A.d_offsets[3 * g + c] = gm * l[c];
      dl[c] = fmaf(gm, A.offsets[3 * g + c], dl[c]);
    }
  }
  // opacity head: tanh
  hidden_layer(A.W1[0], A.b1[0], width, h, hid);
  for (int m = 0; m < k; ++m) {
    const float t = tanhf(head_out(A.W2[0], A.b2[0], width, m, hid));
    const float dy = A.g_opac[a * k + m] * (1.0f - t * t);
    A.ws_dy[0][a * k + m] = dy;
    dyl[m * kDecBlock] = dy;
  }
  head_backward(A, 0, a, k, hid, dyl, dh);
  // colour head: sigmoid (eq. 4)
  hidden_layer(A.W1[1], A.b1[1], width, h, hid);
  for (int r = 0; r < 3 * k; ++r) {
    const float s = sigmoidf_(head_out(A.W2[1], A.b2[1], width, r, hid));
    const float dy = A.g_colors[a * 3 * k + r] * s * (1.0f - s);
    A.ws_dy[1][a * 3 * k + r] = dy;
    dyl[r * kDecBlock] = dy;
  }
  head_backward(A, 1, a, 3 * k, hid, dyl, dh);
  // covariance head: [scale (eq. 5) | quaternion]
  hidden_layer(A.W1[2], A.b1[2], width, h, hid);
  for (int m = 0; m < k; ++m) {
    const int64_t g = a * k + m;
    float y[7], dy[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) y[j] = head_out(A.W2[2], A.b2[2], width, 7 * m + j, hid);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const float gl = A.g_ls[3 * g + j];
      dy[j] = gl * (1.0f - sigmoidf_(y[j]));  // d log_sigmoid(y) / dy
      dl[j] += gl / l[j];                      // d log l / dl
    }
    const float nr = sqrtf(y[3] * y[3] + y[4] * y[4] + y[5] * y[5] + y[6] * y[6]);
    const float gq[4] = {A.g_quats[4 * g], A.g_quats[4 * g + 1], A.g_quats[4 * g + 2], A.g_quats[4 * g + 3]};
    if (nr > 1e-12f) {
      const float in = 1.0f / nr;
      const float q0 = y[3] * in, q1 = y[4] * in, q2 = y[5] * in, q3 = y[6] * in;
      const float dot = q0 * gq[0] + q1 * gq[1] + q2 * gq[2] + q3 * gq[3];
      dy[3] = (gq[0] - q0 * dot) * in;
      dy[4] = (gq[1] - q1 * dot) * in;
      dy[5] = (gq[2] - q2 * dot) * in;
      dy[6] = (gq[3] - q3 * dot) * in;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) dy[3 + j] = gq[j] * 1e12f;
    }
#pragma unroll
    for (int j = 0; j < 7; ++j) {
      A.ws_dy[2][a * 7 * k + 7 * m + j] = dy[j];
      dyl[(7 * m + j) * kDecBlock] = dy[j];
    }
  }
  head_backward(A, 2, a, 7 * k, hid, dyl, dh);
#pragma unroll
  for (int i = 0; i < 32; ++i) A.d_feat[a * 32 + i] = dh[i];
#pragma unroll
  for (int c = 0; c < 3; ++c) A.d_scale[3 * a + c] = dl[c];
}

// ---------------------------------------------------------------------------
// split-K products: partial[chunk][p][q] = sum_{a in chunk} X[a][p] Y[a][q],
// partial[chunk][P*Q + p] = sum_{a in chunk} X[a][p]
// ---------------------------------------------------------------------------
constexpr int kChunk = 1024;
constexpr int kTile = 16;
constexpr int kStep = 64;

__global__ void __launch_bounds__(256) outer_partial_kernel(const float* __restrict__ X, int P,
                                                            const float* __restrict__ Y, int Q, int64_t M,
                                                            float* __restrict__ partial) {
  __shared__ float xs[kStep][kTile];
  __shared__ float ys[kStep][kTile];
  const int tp = threadIdx.x / kTile, tq = threadIdx.x % kTile;
  const int p = blockIdx.y * kTile + tp, q = blockIdx.z * kTile + tq;
  const int64_t a0 = (int64_t)blockIdx.x * kChunk;
  const int64_t a1 = a0 + kChunk < M ? a0 + kChunk : M;
  float acc = 0.f, bias = 0.f;
  for (int64_t base = a0; base < a1; base += kStep) {
    __syncthreads();
    for (int e = threadIdx.x; e < kStep * kTile; e += 256) {
      const int r = e / kTile, c = e % kTile;
      const int64_t a = base + r;
      const int pp = blockIdx.y * kTile + c, qq = blockIdx.z * kTile + c;
      xs[r][c] = (a < a1 && pp < P) ? X[a * P + pp] : 0.0f;
      ys[r][c] = (a < a1 && qq < Q) ? Y[a * Q + qq] : 0.0f;
    }
    __syncthreads();
#pragma unroll 8
    for (int r = 0; r < kStep; ++r) {
      acc = fmaf(xs[r][tp], ys[r][tq], acc);
      bias += xs[r][tp];
    }
  }
  const size_t per = (size_t)P * Q + P;
  if (p < P && q < Q) partial[blockIdx.x * per + (size_t)p * Q + q] = acc;
  if (p < P && blockIdx.z == 0 && tq == 0) partial[blockIdx.x * per + (size_t)P * Q + p] = bias;
}

__global__ void reduce_partial_kernel(const float* __restrict__ partial, int chunks, int P, int Q,
                                      float* __restrict__ dW, float* __restrict__ db) {
  const size_t per = (size_t)P * Q + P;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= per) return;
  float s = 0.f;
  for (int c = 0; c < chunks; ++c) s += partial[(size_t)c * per + e];
  if (e < (size_t)P * Q) dW[e] = s;
  else db[e - (size_t)P * Q] = s;
}

hipError_t launch_dec_any(bool backward, const DecArgs& A, hipStream_t s) {
  const unsigned blocks = (unsigned)((A.m + kDecBlock - 1) / kDecBlock);
  if (blocks == 0) return hipSuccess;
  if (backward) {
    const size_t lds = (size_t)(A.width + 7 * A.k) * kDecBlock * sizeof(float);
    hipLaunchKernelGGL(decode_backward_kernel, dim3(blocks), dim3(kDecBlock), lds, s, A);
  } else {
    const size_t lds = (size_t)A.width * kDecBlock * sizeof(float);
    hipLaunchKernelGGL(decode_forward_kernel, dim3(blocks), dim3(kDecBlock), lds, s, A);
  }
  return hipGetLastError();
}

bool finite3(const float* c) { return std::isfinite(c[0]) && std::isfinite(c[1]) && std::isfinite(c[2]); }

int validate(vpgs_ctx* ctx, const vpgs_anchors* an, const vpgs_mlp* mlp, const float* cam) {
  if (!an || !mlp || !cam) return fail(ctx, VPGS_EINVAL, "NULL argument");
  if (an->m < 0 || an->m > (1LL << 26)) return fail(ctx, VPGS_EINVAL, "anchor count %lld out of range", (long long)an->m);
  if (an->k < 1 || an->k > 16) return fail(ctx, VPGS_EINVAL, "k = %d outside [1, 16]", an->k);
  if (mlp->in_dim != kIn) return fail(ctx, VPGS_EINVAL, "in_dim must be 36 (got %d)", mlp->in_dim);
  if (mlp->width < 1 || mlp->width > 128) return fail(ctx, VPGS_EINVAL, "width %d outside [1, 128]", mlp->width);
  if (!finite3(cam)) return fail(ctx, VPGS_EINVAL, "non-finite camera centre");
  for (int h = 0; h < 3; ++h)
    if (!mlp->W1[h] || !mlp->b1[h] || !mlp->W2[h] || !mlp->b2[h]) return fail(ctx, VPGS_EINVAL, "NULL weight of head %d", h);
  if (an->m > 0 && (!an->xyz || !an->feat || !an->scale || !an->offsets))
    return fail(ctx, VPGS_EINVAL, "NULL anchor array");
  return VPGS_OK;
}

DecArgs make_args(const vpgs_anchors* an, const vpgs_mlp* mlp, const float* cam) {
  DecArgs A;
  std::memset(&A, 0, sizeof(A));
  A.m = an->m;
  A.k = an->k;
  A.width = mlp->width;
  A.xyz = an->xyz; A.feat = an->feat; A.scale = an->scale; A.offsets = an->offsets;
  for (int h = 0; h < 3; ++h) {
    A.W1[h] = mlp->W1[h]; A.b1[h] = mlp->b1[h]; A.W2[h] = mlp->W2[h]; A.b2[h] = mlp->b2[h];
  }
  A.cx = cam[0]; A.cy = cam[1]; A.cz = cam[2];
  return A;
}

}  // namespace
}  // namespace vpgs

using namespace vpgs;

extern "C" {

int vpgs_decode_forward(vpgs_ctx* ctx, const vpgs_anchors* an, const vpgs_mlp* mlp, const float* cam_center,
                        const vpgs_gauss_buffers* out, void* stream) {
  if (!ctx) return VPGS_EINVAL;
  int rc = validate(ctx, an, mlp, cam_center);
  if (rc) return rc;
  if (!out || (an->m > 0 && (!out->means || !out->log_scales || !out->quats || !out->opacities || !out->colors)))
    return fail(ctx, VPGS_EINVAL, "NULL output array");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));
  DecArgs A = make_args(an, mlp, cam_center);
  A.means = out->means; A.log_scales = out->log_scales; A.quats = out->quats; A.opac = out->opacities;
  A.colors = out->colors;
  StageTimer t(ctx, ST_DEC_FWD, st);
  HIP_TRY(launch_dec_any(false, A, st));
  return VPGS_OK;
}

int vpgs_decode_backward(vpgs_ctx* ctx, const vpgs_anchors* an, const vpgs_mlp* mlp, const float* cam_center,
                         const vpgs_gauss_grads* up, float* d_feat, float* d_scale, float* d_offsets,
                         const vpgs_mlp_grads* dm, void* stream) {
  if (!ctx) return VPGS_EINVAL;
  int rc = validate(ctx, an, mlp, cam_center);
  if (rc) return rc;
  if (!up || !dm) return fail(ctx, VPGS_EINVAL, "NULL argument");
  if (an->m > 0 && (!up->means || !up->log_scales || !up->quats || !up->opacities || !up->colors || !d_feat ||
                    !d_scale || !d_offsets))
    return fail(ctx, VPGS_EINVAL, "NULL gradient array");
  for (int h = 0; h < 3; ++h)
    if (!dm->W1[h] || !dm->b1[h] || !dm->W2[h] || !dm->b2[h]) return fail(ctx, VPGS_EINVAL, "NULL weight gradient");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));
  const int64_t M = an->m;
  const int k = an->k, width = mlp->width;
  const int outs[3] = {k, 3 * k, 7 * k};
  // workspace: h, hidden x3, dpre x3, dy x3
  const size_t ws_floats = (size_t)M * (kIn + 6 * (size_t)width + 11 * (size_t)k);
  const int chunks = (int)std::max<int64_t>((M + kChunk - 1) / kChunk, 1);
  size_t part_floats = 0;
  for (int h = 0; h < 3; ++h) {
    part_floats = std::max(part_floats, (size_t)chunks * ((size_t)outs[h] * width + outs[h]));
    part_floats = std::max(part_floats, (size_t)chunks * ((size_t)width * kIn + width));
  }
  if ((rc = ensure(ctx, ctx->dec_ws, ws_floats * 4)) || (rc = ensure(ctx, ctx->dec_partial, part_floats * 4)))
    return rc;
  DecArgs A = make_args(an, mlp, cam_center);
  A.g_means = up->means; A.g_ls = up->log_scales; A.g_quats = up->quats; A.g_opac = up->opacities;
  A.g_colors = up->colors;
  A.d_feat = d_feat; A.d_scale = d_scale; A.d_offsets = d_offsets;
  float* w = static_cast<float*>(ctx->dec_ws.p);
  A.ws_h = w; w += (size_t)M * kIn;
  for (int h = 0; h < 3; ++h) { A.ws_hid[h] = w; w += (size_t)M * width; }
  for (int h = 0; h < 3; ++h) { A.ws_dpre[h] = w; w += (size_t)M * width; }
  for (int h = 0; h < 3; ++h) { A.ws_dy[h] = w; w += (size_t)M * outs[h]; }
  StageTimer t(ctx, ST_DEC_BWD, st);
  HIP_TRY(launch_dec_any(true, A, st));
  float* part = static_cast<float*>(ctx->dec_partial.p);
  for (int h = 0; h < 3; ++h) {
    // dW2[h] = DY^T HID, db2 = column sums of DY; dW1[h] = DPRE^T H, db1 = column sums of DPRE
    const float* X[2] = {A.ws_dy[h], A.ws_dpre[h]};
    const float* Y[2] = {A.ws_hid[h], A.ws_h};
    const int P[2] = {outs[h], width}, Q[2] = {width, kIn};
    float* dW[2] = {dm->W2[h], dm->W1[h]};
    float* db[2] = {dm->b2[h], dm->b1[h]};
    for (int g = 0; g < 2; ++g) {
      if (M > 0) {
        dim3 grid(chunks, (P[g] + kTile - 1) / kTile, (Q[g] + kTile - 1) / kTile);
        hipLaunchKernelGGL(outer_partial_kernel, grid, dim3(256), 0, st, X[g], P[g], Y[g], Q[g], M, part);
        HIP_TRY(hipGetLastError());
        const size_t per = (size_t)P[g] * Q[g] + P[g];
        hipLaunchKernelGGL(reduce_partial_kernel, dim3((unsigned)((per + 255) / 256)), dim3(256), 0, st, part,
                           chunks, P[g], Q[g], dW[g], db[g]);
        HIP_TRY(hipGetLastError());
      } else {
        HIP_TRY(launch_fill_f32(dW[g], 0.f, (size_t)P[g] * Q[g], st));
        HIP_TRY(launch_fill_f32(db[g], 0.f, (size_t)P[g], st));
      }
    }
  }
  return VPGS_OK;
}

}  // extern "C"
