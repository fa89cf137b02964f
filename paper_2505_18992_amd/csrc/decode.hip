// decode.hip -- neural Gaussians from voxel anchors (Section III-A, eq. 1-5)
// and the backward of that decode.
//
// Forward: the 36-vector [feature, view direction, distance] of an anchor
// (eq. 3) goes through three LINEAR-ReLU-LINEAR heads (eq. 2); the k
// Gaussians of the anchor get mean = anchor + offset * scaling (eq. 1),
// opacity = tanh, colour = sigmoid (eq. 4), log-scale = log sigmoid + log of
// the anchor scaling (eq. 5) and a normalised quaternion.
//
// The heads are small dense products over a batch of anchors, so they run on
// the matrix cores: one wavefront takes 16 anchors (the M rows of a
// 16x16x4 FP32 MFMA tile) end to end, with its input rows, hidden layer and
// head outputs in a private slice of LDS, and streams the weights (a few tens
// of KB, L2-resident) as the B operands.  The activations then run one lane
// per (anchor, Gaussian) output so that the stores are contiguous.
//
// Backward: the same wavefront recomputes its forward, chains the upstream
// Gaussian gradients through the activations and both layers with the same
// tiles (feature, scaling and offset gradients are written directly), and
// stores each layer's input and output gradient.  The weight gradients are
// sums over anchors of outer products: one launch forms all six of them
// (W2 and W1 of each head, the bias as an extra all-ones column) per chunk of
// anchors on the matrix cores, and a second sums the chunks in a fixed order,
// so they are deterministic.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "runtime.h"

namespace vpgs {
namespace {

constexpr int kIn = 36;
constexpr int kRows = 16;      // anchors per wavefront: the rows of every tile
constexpr int kHP = kIn + 1;   // LDS pitch of the input rows

typedef float f32x4 __attribute__((ext_vector_type(4)));

// D += A B for a 16x4 A and a 4x16 B.  Lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and holds D[4 (l / 16) + i][l % 16] in element i.  The
// contraction index that a (lane group, step) pair stands for is free as long
// as A and B agree on it.
__device__ __forceinline__ f32x4 mma(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

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

__host__ __device__ constexpr int head_outs(int h, int k) { return (h == 0 ? 1 : h == 1 ? 3 : 7) * k; }

// Rows of h = [feat (32), direction (3), distance (1)] (eq. 3) for the
// wavefront's anchors a0 .. a0 + nv - 1; rows past nv are zero.
__device__ __forceinline__ void load_inputs(const DecArgs& A, int64_t a0, int nv, int lane, float* Hs) {
#pragma unroll
  for (int e = lane; e < kRows * 32; e += 64) {
    const int r = e >> 5, i = e & 31;
    Hs[r * kHP + i] = r < nv ? A.feat[(a0 + r) * 32 + i] : 0.0f;
  }
  if (lane < kRows) {
    float d[4] = {0.f, 0.f, 0.f, 0.f};
    if (lane < nv) {
      const int64_t a = a0 + lane;
      const float dx = A.xyz[3 * a] - A.cx, dy = A.xyz[3 * a + 1] - A.cy, dz = A.xyz[3 * a + 2] - A.cz;
      const float delta = sqrtf(dx * dx + dy * dy + dz * dz);
      const float inv = 1.0f / delta;
      d[0] = dx * inv;
      d[1] = dy * inv;
      d[2] = dz * inv;
      d[3] = delta;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) Hs[lane * kHP + 32 + j] = d[j];
  }
}

// hid[r][j] = relu(b1[j] + sum_i W1[j][i] h[r][i]) for the KW column tiles
// of the hidden layer (columns past the width come out zero).  ha holds the
// A operand: lane group g covers inputs 9g .. 9g + 8.
template <int KW>
__device__ __forceinline__ void hidden_tiles(const float* __restrict__ W1, const float* __restrict__ b1, int W,
                                             const float ha[9], float* hid, int lane) {
  constexpr int HP = 16 * KW + 1;
  const int lo = lane & 15, grp = lane >> 4;
#pragma unroll
  for (int ct = 0; ct < KW; ++ct) {
    const int j = 16 * ct + lo;
    const bool jv = j < W;
    float b[9];
#pragma unroll
    for (int ks = 0; ks < 9; ++ks) b[ks] = jv ? W1[j * kIn + 9 * grp + ks] : 0.0f;
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 9; ++ks) c = mma(ha[ks], b[ks], c);
    const float bias = jv ? b1[j] : 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) hid[(4 * grp + i) * HP + j] = fmaxf(c[i] + bias, 0.0f);
  }
}

// y[r][o] = b2[o] + sum_j W2[o][j] hid[r][j] for o < outs, 16 outputs per
// tile; lane group g covers hidden units g KS .. g KS + KS - 1.
template <int KW>
__device__ __forceinline__ void out_tiles(const float* __restrict__ W2, const float* __restrict__ b2, int W, int outs,
                                          const float* hid, float* ys, int yp, int lane) {
  constexpr int HP = 16 * KW + 1, KS = 4 * KW;
  const int lo = lane & 15, grp = lane >> 4;
  float ha[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) ha[ks] = hid[lo * HP + KS * grp + ks];
  for (int o0 = 0; o0 < outs; o0 += 16) {
    const int o = o0 + lo;
    const bool ov = o < outs;
    float b[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int j = KS * grp + ks;
      b[ks] = (ov && j < W) ? W2[(size_t)o * W + j] : 0.0f;
    }
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) c = mma(ha[ks], b[ks], c);
    if (ov) {
      const float bias = b2[o];
#pragma unroll
      for (int i = 0; i < 4; ++i) ys[(4 * grp + i) * yp + o] = c[i] + bias;
    }
  }
}

template <int KW>
__global__ void __launch_bounds__(64) decode_forward_kernel(DecArgs A) {
  extern __shared__ float lds[];
  constexpr int HP = 16 * KW + 1;
  const int lane = threadIdx.x;
  const int k = A.k, W = A.width, yp = 7 * k + 1;
  float* Hs = lds;
  float* hid = Hs + kRows * kHP;
  float* ys = hid + kRows * HP;
  const int64_t a0 = (int64_t)blockIdx.x * kRows;
  const int nv = (int)std::min<int64_t>(A.m - a0, kRows);
  load_inputs(A, a0, nv, lane, Hs);
  const int n3 = nv * 3 * k;
  for (int e = lane; e < n3; e += 64) {  // eq. 1
    const int r = e / (3 * k), c = e % 3;
    const int64_t a = a0 + r, g = a0 * 3 * k + e;
    A.means[g] = A.xyz[3 * a + c] + A.offsets[g] * A.scale[3 * a + c];
  }
  __syncthreads();
  float ha[9];
#pragma unroll
  for (int ks = 0; ks < 9; ++ks) ha[ks] = Hs[(lane & 15) * kHP + 9 * (lane >> 4) + ks];
  for (int h = 0; h < 3; ++h) {
    const int outs = head_outs(h, k);
    hidden_tiles<KW>(A.W1[h], A.b1[h], W, ha, hid, lane);
    __syncthreads();
    out_tiles<KW>(A.W2[h], A.b2[h], W, outs, hid, ys, yp, lane);
    __syncthreads();
    if (h == 0) {
      for (int e = lane; e < nv * k; e += 64) {
        const int r = e / k;
        A.opac[a0 * k + e] = tanhf(ys[r * yp + e - r * k]);
      }
    } else if (h == 1) {
      for (int e = lane; e < nv * 3 * k; e += 64) {  // eq. 4
        const int r = e / (3 * k);
        A.colors[a0 * 3 * k + e] = sigmoidf_(ys[r * yp + e - r * 3 * k]);
      }
    } else {
      for (int e = lane; e < nv * k; e += 64) {
        const int r = e / k;
        const float* y = ys + r * yp + 7 * (e - r * k);
        const int64_t a = a0 + r, g = a0 * k + e;
#pragma unroll
        for (int j = 0; j < 3; ++j) A.log_scales[3 * g + j] = log_sigmoidf_(y[j]) + logf(A.scale[3 * a + j]);  // eq. 5
        const float n = fmaxf(sqrtf(y[3] * y[3] + y[4] * y[4] + y[5] * y[5] + y[6] * y[6]), 1e-12f);
        const float in = 1.0f / n;
#pragma unroll
        for (int j = 0; j < 4; ++j) A.quats[4 * g + j] = y[3 + j] * in;
      }
    }
    __syncthreads();
  }
}

// dhid[r][j] = sum_o dy[r][o] W2[o][j]; dpre = dhid where the hidden unit is
// active.  Writes dpre to LDS and the hidden layer and dpre of the valid rows
// to the workspace.  Lane group g covers outputs o0 + 4g .. o0 + 4g + 3.
template <int KW>
__device__ __forceinline__ void hid_grad_tiles(const float* __restrict__ W2, int W, int outs, const float* dys, int yp,
                                               const float* hid, float* dpre, float* ws_hid, float* ws_dpre,
                                               int64_t a0, int nv, int lane) {
  constexpr int HP = 16 * KW + 1;
  const int lo = lane & 15, grp = lane >> 4;
  f32x4 acc[KW];
#pragma unroll
  for (int ct = 0; ct < KW; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int o0 = 0; o0 < outs; o0 += 16) {
    float a[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int o = o0 + 4 * grp + s;
      a[s] = o < outs ? dys[lo * yp + o] : 0.0f;
    }
#pragma unroll
    for (int ct = 0; ct < KW; ++ct) {
      const int j = 16 * ct + lo;
      float b[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int o = o0 + 4 * grp + s;
        b[s] = (o < outs && j < W) ? W2[(size_t)o * W + j] : 0.0f;
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) acc[ct] = mma(a[s], b[s], acc[ct]);
    }
  }
#pragma unroll
  for (int ct = 0; ct < KW; ++ct) {
    const int j = 16 * ct + lo;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 4 * grp + i;
      const float hv = hid[r * HP + j];
      const float dp = hv > 0.0f ? acc[ct][i] : 0.0f;
      dpre[r * HP + j] = dp;
      if (r < nv && j < W) {
        ws_hid[(a0 + r) * W + j] = hv;
        ws_dpre[(a0 + r) * W + j] = dp;
      }
    }
  }
}

// dh[r][c] += sum_j dpre[r][j] W1[j][c] for the 32 feature inputs (the
// direction and distance inputs have no parameters upstream).
template <int KW>
__device__ __forceinline__ void input_grad_tiles(const float* __restrict__ W1, int W, const float* dpre, f32x4 dh[2],
                                                 int lane) {
  constexpr int HP = 16 * KW + 1, KS = 4 * KW;
  const int lo = lane & 15, grp = lane >> 4;
  float a[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) a[ks] = dpre[lo * HP + KS * grp + ks];
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int c = 16 * ct + lo;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int j = KS * grp + ks;
      dh[ct] = mma(a[ks], j < W ? W1[j * kIn + c] : 0.0f, dh[ct]);
    }
  }
}

template <int KW>
__global__ void __launch_bounds__(64) decode_backward_kernel(DecArgs A) {
  extern __shared__ float lds[];
  constexpr int HP = 16 * KW + 1;
  const int lane = threadIdx.x, lo = lane & 15, grp = lane >> 4;
  const int k = A.k, W = A.width, yp = 7 * k + 1;
  float* Hs = lds;
  float* hid = Hs + kRows * kHP;
  float* dpre = hid + kRows * HP;
  float* ys = dpre + kRows * HP;
  const int64_t a0 = (int64_t)blockIdx.x * kRows;
  const int nv = (int)std::min<int64_t>(A.m - a0, kRows);
  load_inputs(A, a0, nv, lane, Hs);
  // eq. 1: mean = anchor + offset * l
  const int n3 = nv * 3 * k;
  for (int e = lane; e < n3; e += 64) {
    const int r = e / (3 * k), c = e % 3;
    const int64_t g = a0 * 3 * k + e;
    A.d_offsets[g] = A.g_means[g] * A.scale[3 * (a0 + r) + c];
  }
  // scaling: through the means and through eq. 5's log l
  if (lane < 3 * nv) {
    const int r = lane / 3, c = lane - 3 * r;
    const int64_t a = a0 + r;
    const float l = A.scale[3 * a + c];
    float s = 0.0f;
    for (int m = 0; m < k; ++m) s = fmaf(A.g_means[3 * (a * k + m) + c], A.offsets[3 * (a * k + m) + c], s);
    for (int m = 0; m < k; ++m) s += A.g_ls[3 * (a * k + m) + c] / l;
    A.d_scale[3 * a + c] = s;
  }
  __syncthreads();
  for (int e = lane; e < nv * kIn; e += 64) {
    const int r = e / kIn;
    A.ws_h[a0 * kIn + e] = Hs[r * kHP + e - r * kIn];
  }
  float ha[9];
#pragma unroll
  for (int ks = 0; ks < 9; ++ks) ha[ks] = Hs[lo * kHP + 9 * grp + ks];
  f32x4 dh[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
  for (int h = 0; h < 3; ++h) {
    const int outs = head_outs(h, k);
    hidden_tiles<KW>(A.W1[h], A.b1[h], W, ha, hid, lane);
    __syncthreads();
    out_tiles<KW>(A.W2[h], A.b2[h], W, outs, hid, ys, yp, lane);
    __syncthreads();
    // gradient at the head outputs, in place of the outputs
    float* wdy = A.ws_dy[h] + a0 * outs;
    if (h == 0) {  // tanh
      for (int e = lane; e < nv * k; e += 64) {
        const int r = e / k, o = e - r * k;
        const float t = tanhf(ys[r * yp + o]);
        const float dy = A.g_opac[a0 * k + e] * (1.0f - t * t);
        ys[r * yp + o] = dy;
        wdy[e] = dy;
      }
    } else if (h == 1) {  // sigmoid (eq. 4)
      for (int e = lane; e < nv * 3 * k; e += 64) {
        const int r = e / (3 * k), o = e - r * 3 * k;
        const float s = sigmoidf_(ys[r * yp + o]);
        const float dy = A.g_colors[a0 * 3 * k + e] * s * (1.0f - s);
        ys[r * yp + o] = dy;
        wdy[e] = dy;
      }
    } else {  // [scale (eq. 5) | quaternion]
      for (int e = lane; e < nv * k; e += 64) {
        const int r = e / k;
        float* y = ys + r * yp + 7 * (e - r * k);
        const int64_t g = a0 * k + e;
        float dy[7];
#pragma unroll
        for (int j = 0; j < 3; ++j) dy[j] = A.g_ls[3 * g + j] * (1.0f - sigmoidf_(y[j]));  // d log_sigmoid(y) / dy
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
          y[j] = dy[j];
          wdy[7 * e + j] = dy[j];
        }
      }
    }
    __syncthreads();
    hid_grad_tiles<KW>(A.W2[h], W, outs, ys, yp, hid, dpre, A.ws_hid[h], A.ws_dpre[h], a0, nv, lane);
    __syncthreads();
    input_grad_tiles<KW>(A.W1[h], W, dpre, dh, lane);
    __syncthreads();
  }
#pragma unroll
  for (int ct = 0; ct < 2; ++ct)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 4 * grp + i;
      if (r < nv) A.d_feat[(a0 + r) * 32 + 16 * ct + lo] = dh[ct][i];
    }
}

// ---------------------------------------------------------------------------
// Weight gradients: for each of the six products, part[chunk][p][q] =
// sum over the chunk's anchors a of X[a][p] Y'[a][q], where Y' is Y with a
// trailing all-ones column (q = Q gives the bias gradient sum_a X[a][p]).
// One block per (chunk, product); wavefront w owns the p tiles w and w + 4
// and every q tile, so no two wavefronts share an output.
// ---------------------------------------------------------------------------
constexpr int kNumProd = 6;
constexpr int kMaxPT = 2;  // P <= 128: 8 tiles over 4 wavefronts
constexpr int kMaxQT = 9;  // Q + 1 <= 129
constexpr int kOuterBlock = 256;

struct OuterJob {
  const float* X;
  const float* Y;
  int P, Q;
  int64_t off;  // offset of this product in a chunk's partial row
};

struct OuterArgs {
  OuterJob job[kNumProd];
  int64_t M;
  int64_t chunk;
  int64_t per;  // floats per chunk: sum of P (Q + 1)
  float* part;
};

__device__ __forceinline__ OuterJob pick_job(const OuterArgs& O, int j) {
  OuterJob J = O.job[0];
#pragma unroll
  for (int t = 1; t < kNumProd; ++t)
    if (j == t) J = O.job[t];
  return J;
}

__global__ void __launch_bounds__(kOuterBlock) outer_mfma_kernel(OuterArgs O) {
  const OuterJob J = pick_job(O, blockIdx.y);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, lo = lane & 15, grp = lane >> 4;
  const int npt = (J.P + 15) >> 4, nqt = (J.Q + 16) >> 4;
  if (w >= npt) return;
  const int64_t c0 = (int64_t)blockIdx.x * O.chunk;
  const int64_t c1 = std::min<int64_t>(c0 + O.chunk, O.M);
  f32x4 acc[kMaxPT][kMaxQT];
#pragma unroll
  for (int pt = 0; pt < kMaxPT; ++pt)
#pragma unroll
    for (int qt = 0; qt < kMaxQT; ++qt) acc[pt][qt] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int64_t a = c0; a < c1; a += 4) {
    const int64_t ar = a + grp;
    const bool av = ar < c1;
    float xa[kMaxPT], yb[kMaxQT];
#pragma unroll
    for (int pt = 0; pt < kMaxPT; ++pt) {
      const int p = 16 * (w + 4 * pt) + lo;
      xa[pt] = (av && p < J.P) ? J.X[ar * J.P + p] : 0.0f;
    }
#pragma unroll
    for (int qt = 0; qt < kMaxQT; ++qt) {
      const int q = 16 * qt + lo;
      yb[qt] = !av ? 0.0f : q < J.Q ? J.Y[ar * J.Q + q] : (q == J.Q ? 1.0f : 0.0f);
    }
#pragma unroll
    for (int pt = 0; pt < kMaxPT; ++pt)
      if (w + 4 * pt < npt)
#pragma unroll
        for (int qt = 0; qt < kMaxQT; ++qt)
          if (qt < nqt) acc[pt][qt] = mma(xa[pt], yb[qt], acc[pt][qt]);
  }
  float* out = O.part + (int64_t)blockIdx.x * O.per + J.off;
  const int q1 = J.Q + 1;
#pragma unroll
  for (int pt = 0; pt < kMaxPT; ++pt) {
    if (w + 4 * pt >= npt) break;
#pragma unroll
    for (int qt = 0; qt < kMaxQT; ++qt) {
      const int q = 16 * qt + lo;
      if (qt >= nqt || q >= q1) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int p = 16 * (w + 4 * pt) + 4 * grp + i;
        if (p < J.P) out[(int64_t)p * q1 + q] = acc[pt][qt][i];
      }
    }
  }
}

struct ReduceArgs {
  float* dW[kNumProd];
  float* db[kNumProd];
  int Q[kNumProd];
  int64_t off[kNumProd + 1];
  int64_t per;
  int chunks;
  const float* part;
};

// Sums the chunks in a fixed order (four interleaved partial sums).
__global__ void __launch_bounds__(256) reduce_outer_kernel(ReduceArgs R) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= R.per) return;
  int j = 0;
#pragma unroll
  for (int t = 1; t < kNumProd; ++t) j += e >= R.off[t];
  int Q = R.Q[0];
  int64_t off = R.off[0];
  float* dW = R.dW[0];
  float* db = R.db[0];
#pragma unroll
  for (int t = 1; t < kNumProd; ++t)
    if (j == t) {
      Q = R.Q[t];
      off = R.off[t];
      dW = R.dW[t];
      db = R.db[t];
    }
  float s[4] = {0.f, 0.f, 0.f, 0.f};
  const float* p = R.part + e;
  int c = 0;
  for (; c + 4 <= R.chunks; c += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) s[u] += p[(int64_t)(c + u) * R.per];
  }
  for (; c < R.chunks; ++c) s[0] += p[(int64_t)c * R.per];
  const float v = (s[0] + s[1]) + (s[2] + s[3]);
  const int64_t loc = e - off;
  const int64_t row = loc / (Q + 1);
  const int q = (int)(loc - row * (Q + 1));
  if (q < Q) dW[row * Q + q] = v;
  else db[row] = v;
}

size_t dec_lds_bytes(bool backward, int kw, int k) {
  const size_t hp = 16 * (size_t)kw + 1, yp = 7 * (size_t)k + 1;
  return (size_t)kRows * (kHP + (backward ? 2 : 1) * hp + yp) * sizeof(float);
}

template <int KW>
void launch_kw(bool backward, const DecArgs& A, unsigned blocks, size_t lds, hipStream_t s) {
  if (backward) hipLaunchKernelGGL(decode_backward_kernel<KW>, dim3(blocks), dim3(64), lds, s, A);
  else hipLaunchKernelGGL(decode_forward_kernel<KW>, dim3(blocks), dim3(64), lds, s, A);
}

hipError_t launch_dec_any(bool backward, const DecArgs& A, hipStream_t s) {
  const unsigned blocks = (unsigned)((A.m + kRows - 1) / kRows);
  if (blocks == 0) return hipSuccess;
  const int kw = (A.width + 15) / 16;
  const size_t lds = dec_lds_bytes(backward, kw, A.k);
  switch (kw) {
    case 1: launch_kw<1>(backward, A, blocks, lds, s); break;
    case 2: launch_kw<2>(backward, A, blocks, lds, s); break;
    case 3: launch_kw<3>(backward, A, blocks, lds, s); break;
    case 4: launch_kw<4>(backward, A, blocks, lds, s); break;
    case 5: launch_kw<5>(backward, A, blocks, lds, s); break;
    case 6: launch_kw<6>(backward, A, blocks, lds, s); break;
    case 7: launch_kw<7>(backward, A, blocks, lds, s); break;
    case 8: launch_kw<8>(backward, A, blocks, lds, s); break;
    default: return hipErrorInvalidValue;
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
  // chunks of at least 256 anchors, at most 512 chunks
  const int64_t chunk = std::max<int64_t>(256, ((M + 511) / 512 + 15) / 16 * 16);
  const int chunks = (int)std::max<int64_t>((M + chunk - 1) / chunk, 1);
  OuterArgs O;
  ReduceArgs R;
  std::memset(&O, 0, sizeof(O));
  std::memset(&R, 0, sizeof(R));
  int64_t per = 0;
  for (int j = 0; j < kNumProd; ++j) {
    const int h = j / 2;
    // even j: dW2[h] = DY^T HID (+ db2); odd j: dW1[h] = DPRE^T H (+ db1)
    const int P = j % 2 == 0 ? outs[h] : width, Q = j % 2 == 0 ? width : kIn;
    O.job[j].P = P;
    O.job[j].Q = Q;
    O.job[j].off = per;
    R.Q[j] = Q;
    R.off[j] = per;
    R.dW[j] = j % 2 == 0 ? dm->W2[h] : dm->W1[h];
    R.db[j] = j % 2 == 0 ? dm->b2[h] : dm->b1[h];
    per += (int64_t)P * (Q + 1);
  }
  R.off[kNumProd] = per;
  if ((rc = ensure(ctx, ctx->dec_ws, ws_floats * 4)) || (rc = ensure(ctx, ctx->dec_partial, (size_t)chunks * per * 4)))
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
  if (M == 0) {
    for (int j = 0; j < kNumProd; ++j) {
      const int P = O.job[j].P, Q = O.job[j].Q;
      HIP_TRY(launch_fill_f32(R.dW[j], 0.f, (size_t)P * Q, st));
      HIP_TRY(launch_fill_f32(R.db[j], 0.f, (size_t)P, st));
    }
    return VPGS_OK;
  }
  HIP_TRY(launch_dec_any(true, A, st));
  for (int h = 0; h < 3; ++h) {
    O.job[2 * h].X = A.ws_dy[h];
    O.job[2 * h].Y = A.ws_hid[h];
    O.job[2 * h + 1].X = A.ws_dpre[h];
    O.job[2 * h + 1].Y = A.ws_h;
  }
  O.M = M;
  O.chunk = chunk;
  O.per = per;
  O.part = static_cast<float*>(ctx->dec_partial.p);
  hipLaunchKernelGGL(outer_mfma_kernel, dim3(chunks, kNumProd), dim3(kOuterBlock), 0, st, O);
  HIP_TRY(hipGetLastError());
  R.per = per;
  R.chunks = chunks;
  R.part = O.part;
  hipLaunchKernelGGL(reduce_outer_kernel, dim3((unsigned)((per + 255) / 256)), dim3(256), 0, st, R);
  HIP_TRY(hipGetLastError());
  return VPGS_OK;
}

}  // extern "C"
