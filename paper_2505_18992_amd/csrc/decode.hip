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
// the matrix cores: a wavefront takes 16 anchors (one dimension of a 16x16x4
// FP32 MFMA tile) end to end and the block's four wavefronts share one head's
// weights, staged in LDS.  The forward computes both products transposed
// (anchors on the N columns), so the hidden layer never leaves registers and
// each lane applies the activations to the outputs it holds.
//
// Backward: with the anchors on the M rows and each wavefront's input rows,
// hidden layer and head outputs in a private slice of LDS, the blocks
// recompute the forward, chain the upstream Gaussian gradients through the
// activations and both layers with the same tiles (feature, scaling and
// offset gradients are written directly), and, holding every layer's input
// and output gradient for their 64 anchors in LDS, form their share of the six weight-gradient products (W2 and W1 of
// each head, the bias as an extra all-ones column) on the matrix cores as one
// partial row per block.  The rows are summed in a fixed order in two levels,
// so the weight gradients are deterministic.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "runtime.h"

namespace vpgs {
namespace {

constexpr int kIn = 36;
constexpr int kRows = 16;      // anchors per wavefront: the rows of every tile
constexpr int kHP = kIn + 1;   // LDS pitch of the input rows
constexpr int kW1P = kIn + 1;  // LDS pitch of the first-layer weight rows
constexpr int kDecWaves = 4;   // wavefronts per block: they share the staged weights
constexpr int kDecThreads = 64 * kDecWaves;

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
  // per-block weight-gradient partials: the block with blockIdx.x = b (anchors
  // from (block0 + b) 64) writes the row at part + b part_per, product j (W2
  // of head j / 2 for even j, W1 for odd j) at part_off[j] within it
  int64_t block0;
  float* part;
  int64_t part_per;
  int64_t part_off[6];
};

// Activations on the hardware exp2, log2 and reciprocal (each about 1 ulp;
// rounding x log2 e adds about 1e-7 |x| relative error to e^x).
constexpr float kLog2e = 1.44269504088896341f;
constexpr float kLn2 = 0.693147180559945309f;
__device__ __forceinline__ float exp_hw(float x) { return __builtin_amdgcn_exp2f(x * kLog2e); }
__device__ __forceinline__ float sigmoidf_(float y) { return __builtin_amdgcn_rcpf(1.0f + exp_hw(-y)); }
// log sigmoid(y) = -(max(-y, 0) + log(1 + e^-|y|))
__device__ __forceinline__ float log_sigmoidf_(float y) {
  return -(fmaxf(-y, 0.0f) + __builtin_amdgcn_logf(1.0f + exp_hw(-fabsf(y))) * kLn2);
}
// tanh(y) = sign(y) (1 - e) / (1 + e) with e = e^(-2|y|)
__device__ __forceinline__ float tanh_hw(float y) {
  const float e = exp_hw(-2.0f * fabsf(y));
  return copysignf((1.0f - e) * __builtin_amdgcn_rcpf(1.0f + e), y);
}

// Block barrier for data in LDS only.  The kernels' global stores are never
// read back within a launch, so unlike __syncthreads() it does not wait for
// them to complete.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__host__ __device__ constexpr int head_outs(int h, int k) { return (h == 0 ? 1 : h == 1 ? 3 : 7) * k; }
__host__ __device__ constexpr int pad16(int n) { return (n + 15) & ~15; }
// LDS pitch of a wavefront's head outputs: the widest head padded to whole
// tiles, plus one
__host__ __device__ constexpr int out_pitch(int k) { return pad16(7 * k) + 1; }

// floor(e / d) for 0 <= e < 2^20 and d <= 48 given inv = 1 / d in FP32:
// (e + 1/2) / d lies at least 1 / (2 d) from an integer and the product errs
// by under 1e-5, so the truncation is exact
__device__ __forceinline__ int quot(int e, float inv) { return (int)(((float)e + 0.5f) * inv); }

// Runs store(e, load(e)) over the elements e < n of a wavefront, U per
// lane at a time with the U loads issued before any store (the outputs
// may not alias the inputs, but the compiler cannot know that).  Lanes past
// n take element n - 1 and store the same value to it as its own lane, so
// nothing depends on e < n and the loads are all in flight together (a
// store under that condition would let the compiler move each load into
// it, behind its own wait).  store(e, v) must depend only on e and v.
template <int U = 4, class Load, class Store>
__device__ __forceinline__ void blocked(int n, int lane, Load load, Store store) {
  for (int base = 0; base < n; base += 64 * U) {
    decltype(load(0)) v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = load(std::min(base + lane + 64 * u, n - 1));
#pragma unroll
    for (int u = 0; u < U; ++u) store(std::min(base + lane + 64 * u, n - 1), v[u]);
  }
}

// Replaces the NV values at ptr(e) in LDS by f(load(e), values) for the
// elements e < n of a wavefront, U per lane at a time: the U global loads
// and LDS reads are all issued before any arithmetic.  Lanes past n take
// element n - 1 and write the same values to it as its own lane (as in
// blocked), so nothing is conditional.  Distinct elements never share LDS
// values.
template <int U, int NV, class Load, class Ptr, class F>
__device__ __forceinline__ void rmw_blocked(int n, int lane, Load load, Ptr ptr, F f) {
  for (int base = 0; base < n; base += 64 * U) {
    decltype(load(0)) g[U];
    float y[U][NV];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = std::min(base + lane + 64 * u, n - 1);
      g[u] = load(e);
      const float* p = ptr(e);
#pragma unroll
      for (int j = 0; j < NV; ++j) y[u][j] = p[j];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) f(g[u], y[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      float* p = ptr(std::min(base + lane + 64 * u, n - 1));
#pragma unroll
      for (int j = 0; j < NV; ++j) p[j] = y[u][j];
    }
  }
}

// Rows of h = [feat (32), direction (3), distance (1)] (eq. 3) for the
// wavefront's anchors a0 .. a0 + nv - 1 (rows past nv are zero), and the log
// of their scalings (eq. 5).
__device__ __forceinline__ void load_inputs(const DecArgs& A, int64_t a0, int nv, int lane, float* Hs, float* logl) {
  // rows past the anchor count read the last anchor (all loads unconditional)
  const int64_t last = A.m - 1;
  float f[kRows / 2];
#pragma unroll
  for (int u = 0; u < kRows / 2; ++u) {
    const int e = lane + 64 * u, r = e >> 5;
    f[u] = A.feat[std::min(a0 + r, last) * 32 + (e & 31)];
  }
  const int64_t a = std::min(a0 + (lane & (kRows - 1)), last);
  const float px = A.xyz[3 * a], py = A.xyz[3 * a + 1], pz = A.xyz[3 * a + 2];
  const float sl = A.scale[std::min(a0 * 3 + std::min(lane, 3 * kRows - 1), 3 * last + 2)];
#pragma unroll
  for (int u = 0; u < kRows / 2; ++u) {
    const int e = lane + 64 * u, r = e >> 5;
    Hs[r * kHP + (e & 31)] = r < nv ? f[u] : 0.0f;
  }
  if (lane < kRows) {
    float d[4] = {0.f, 0.f, 0.f, 0.f};
    if (lane < nv) {
      const float dx = px - A.cx, dy = py - A.cy, dz = pz - A.cz;
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
  if (lane < 3 * kRows) logl[lane] = lane < 3 * nv ? logf(sl) : 0.0f;
}

// The parameters of head h in LDS, shared by the block's wavefronts, padded
// with zeros to whole tiles (so the tile loops need no bounds tests): W1 as
// [wp][kW1P], W2 as [pad16(outs)][wp + 1], then b1 [wp] and b2 [pad16(outs)],
// wp = pad16(width).  Synchronises before (the previous head's may still be in
// use) and after.
struct HeadLds {
  float* w1;
  float* w2;
  float* b1;
  float* b2;
};

__device__ __forceinline__ HeadLds head_lds(float* lds, int W, int k) {
  const int wp = pad16(W);
  HeadLds p;
  p.w1 = lds;
  p.w2 = p.w1 + wp * kW1P;
  p.b1 = p.w2 + pad16(7 * k) * (wp + 1);
  p.b2 = p.b1 + wp;
  return p;
}

__host__ __device__ constexpr int head_lds_floats(int W, int k) {
  return pad16(W) * kW1P + pad16(7 * k) * (pad16(W) + 1) + pad16(W) + pad16(7 * k);
}

// The staged parameters form one index space [W1 | W2 | b1 | b2] in their
// padded layouts; each thread loads kStageU elements of it (padding reads a
// valid address and is replaced by zero) before it stores any, so a head's
// parameters arrive in one or two load latencies.  src_of(e) is the source
// of element e (null for padding), dst_of(e) its LDS destination.
constexpr int kStageU = 16;

template <class Src, class Dst>
__device__ __forceinline__ void stage_flat(int n, const float* any, Src src_of, Dst dst_of) {
  lds_barrier();
  for (int base = 0; base < n; base += kDecThreads * kStageU) {
    float v[kStageU];
#pragma unroll
    for (int u = 0; u < kStageU; ++u) {
      const int e = base + (int)threadIdx.x + kDecThreads * u;
      const float* q = e < n ? src_of(e) : nullptr;
      const float x = *(q != nullptr ? q : any);
      v[u] = q != nullptr ? x : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kStageU; ++u) {
      const int e = base + (int)threadIdx.x + kDecThreads * u;
      if (e < n) *dst_of(e) = v[u];
    }
  }
  lds_barrier();
}

// Head h's parameters in the backward's layout (HeadLds).  Synchronises
// before (the previous head's may still be in use) and after.
template <int KW>
__device__ __forceinline__ void stage_weights(const DecArgs& A, int h, const HeadLds& p) {
  constexpr int wp = 16 * KW;
  const int W = A.width, outs = head_outs(h, A.k), op = pad16(outs);
  const float* __restrict__ W1 = A.W1[h];
  const float* __restrict__ W2 = A.W2[h];
  const float* __restrict__ b1 = A.b1[h];
  const float* __restrict__ b2 = A.b2[h];
  const int n1 = wp * kIn, n2 = n1 + op * wp, n3 = n2 + wp, n = n3 + op;
  stage_flat(
      n, W1,
      [&](int e) -> const float* {
        if (e < n1) return e / kIn < W ? W1 + e : nullptr;
        if (e < n2) {
          const int f = e - n1, o = f / wp, j = f - o * wp;
          return (o < outs && j < W) ? W2 + o * W + j : nullptr;
        }
        if (e < n3) return e - n2 < W ? b1 + (e - n2) : nullptr;
        return e - n3 < outs ? b2 + (e - n3) : nullptr;
      },
      [&](int e) -> float* {
        if (e < n1) {
          const int j = e / kIn;
          return p.w1 + j * kW1P + (e - j * kIn);
        }
        if (e < n2) {
          const int f = e - n1, o = f / wp;
          return p.w2 + o * (wp + 1) + (f - o * wp);
        }
        if (e < n3) return p.b1 + (e - n2);
        return p.b2 + (e - n3);
      });
}

// The forward's layout of one head, for the transposed products (hidden
// units and head outputs on the M rows, anchors on the N columns): W1 as
// [wp][kIn], W2 as [pad16(outs)][wp + 4] (a pitch of 4 mod 16 words puts
// the 16-byte reads of 16 rows on distinct banks), b1 [wp], b2
// [pad16(outs)].  Head 2's rows are permuted so that a lane holds each
// quaternion whole: row 4m + q is quaternion component q of Gaussian m, row
// 4k + 3m + c scale axis c of Gaussian m.
template <int KW>
struct FwdLds {
  static constexpr int wp = 16 * KW, P2 = wp + 4;
  float* w1;
  float* w2;
  float* b1;
  float* b2;
  __device__ FwdLds(float* lds, int k) {
    w1 = lds;
    w2 = w1 + wp * kIn;
    b1 = w2 + pad16(7 * k) * P2;
    b2 = b1 + wp;
  }
};

__host__ __device__ constexpr int fwd_lds_floats(int KW, int k) {
  return 16 * KW * kIn + pad16(7 * k) * (16 * KW + 4) + 16 * KW + pad16(7 * k);
}

// The W2 (and b2) row of head h held at forward row s < 7k.
__device__ __forceinline__ int fwd_row(int h, int s, int k) {
  if (h < 2) return s;
  if (s < 4 * k) return 7 * (s >> 2) + 3 + (s & 3);
  const int r = s - 4 * k, m = r / 3;
  return 7 * m + (r - 3 * m);
}

template <int KW>
__device__ __forceinline__ void stage_forward(const DecArgs& A, int h, const FwdLds<KW>& p) {
  constexpr int wp = FwdLds<KW>::wp, P2 = FwdLds<KW>::P2;
  const int W = A.width, k = A.k, outs = head_outs(h, k), op = pad16(outs);
  const float* __restrict__ W1 = A.W1[h];
  const float* __restrict__ W2 = A.W2[h];
  const float* __restrict__ b1 = A.b1[h];
  const float* __restrict__ b2 = A.b2[h];
  const int n1 = wp * kIn, n2 = n1 + op * wp, n3 = n2 + wp, n = n3 + op;
  stage_flat(
      n, W1,
      [&](int e) -> const float* {
        if (e < n1) return e < W * kIn ? W1 + e : nullptr;
        if (e < n2) {
          const int f = e - n1, o = f / wp, j = f - o * wp;
          return (o < outs && j < W) ? W2 + fwd_row(h, o, k) * W + j : nullptr;
        }
        if (e < n3) return e - n2 < W ? b1 + (e - n2) : nullptr;
        return e - n3 < outs ? b2 + fwd_row(h, e - n3, k) : nullptr;
      },
      [&](int e) -> float* {
        if (e < n1) return p.w1 + e;
        if (e < n2) {
          const int f = e - n1, o = f / wp;
          return p.w2 + o * P2 + (f - o * wp);
        }
        if (e < n3) return p.b1 + (e - n2);
        return p.b2 + (e - n3);
      });
}

// hid[r][j] = relu(b1[j] + sum_i W1[j][i] h[r][i]) for the KW column tiles
// of the hidden layer (columns past the width come out zero).  ha holds the
// A operand: lane group g covers inputs 9g .. 9g + 8.
template <int KW>
__device__ __forceinline__ void hidden_tiles(const float* w1s, const float* b1, const float ha[9], float* hid,
                                             int lane) {
  constexpr int HP = 16 * KW + 1;
  const int lo = lane & 15, grp = lane >> 4;
#pragma unroll
  for (int ct = 0; ct < KW; ++ct) {
    const int j = 16 * ct + lo;
    const float bias = b1[j];
    float b[9];
#pragma unroll
    for (int ks = 0; ks < 9; ++ks) b[ks] = w1s[j * kW1P + 9 * grp + ks];
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 9; ++ks) c = mma(ha[ks], b[ks], c);
#pragma unroll
    for (int i = 0; i < 4; ++i) hid[(4 * grp + i) * HP + j] = fmaxf(c[i] + bias, 0.0f);
  }
}

// y[r][o] = b2[o] + sum_j W2[o][j] hid[r][j] for the pad16(outs) outputs
// (the padding comes out zero), 16 per tile; lane group g covers hidden units
// g KS .. g KS + KS - 1.
template <int KW>
__device__ __forceinline__ void out_tiles(const float* w2s, const float* b2, int outs, const float* hid, float* ys,
                                          int yp, int lane) {
  constexpr int HP = 16 * KW + 1, KS = 4 * KW;
  const int lo = lane & 15, grp = lane >> 4;
  float ha[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) ha[ks] = hid[lo * HP + KS * grp + ks];
  for (int o0 = 0; o0 < outs; o0 += 16) {
    const int o = o0 + lo;
    const float bias = b2[o];
    float b[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) b[ks] = w2s[o * HP + KS * grp + ks];
    // two interleaved accumulators halve the dependent MFMA chain
    f32x4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ks += 2) {
      c0 = mma(ha[ks], b[ks], c0);
      c1 = mma(ha[ks + 1], b[ks + 1], c1);
    }
    const f32x4 c = c0 + c1;
#pragma unroll
    for (int i = 0; i < 4; ++i) ys[(4 * grp + i) * yp + o] = c[i] + bias;
  }
}

struct MeanIn {
  float off, x, l;
};

// Forward, one wavefront per 16 anchors with everything in registers: the
// hidden layer is computed transposed, hid^T = W1 h^T (hidden units on the
// M rows, the anchors on the N columns), which leaves lane (r, g) holding
// hidden units 16 t + 4 g + i of anchor r: exactly the B operand of the
// second product y^T = W2 hid^T when its contraction step (t, i) stands for
// hidden unit 16 t + 4 g + i in lane group g.  Lane (r, g) then holds
// outputs 16 t + 4 g + i of anchor r, which the activations map and store.
// Only the staging of each head's parameters synchronises the block.
template <int KW>
__global__ void __launch_bounds__(kDecThreads) decode_forward_kernel(DecArgs A) {
  extern __shared__ float lds[];
  constexpr int P2 = FwdLds<KW>::P2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lo = lane & 15, grp = lane >> 4;
  const int k = A.k, k3 = 3 * k;
  const float inv_k3 = 1.0f / k3;
  const FwdLds<KW> P(lds, k);
  const int64_t a0 = ((int64_t)blockIdx.x * kDecWaves + wave) * kRows;
  const int nv = (int)std::max<int64_t>(std::min<int64_t>(A.m - a0, kRows), 0);
  blocked<8>(  // eq. 1
      nv * k3, lane,
      [&](int e) {
        const int64_t a = a0 + quot(e, inv_k3);
        const int c = e % 3;
        return MeanIn{A.offsets[a0 * k3 + e], A.xyz[3 * a + c], A.scale[3 * a + c]};
      },
      [&](int e, MeanIn v) { A.means[a0 * k3 + e] = v.x + v.off * v.l; });
  // this lane's anchor; lanes past the anchor count read the last anchor and
  // store nothing
  const bool row_ok = lo < nv;
  const int64_t a = std::min<int64_t>(a0 + lo, A.m - 1);
  // inputs 9 g .. 9 g + 8 of h = [feat (32), direction (3), distance (1)]
  // (eq. 3): the B operand of the first product
  float hin[9];
#pragma unroll
  for (int s = 0; s < 9; ++s) hin[s] = A.feat[a * 32 + std::min(9 * grp + s, 31)];
  const float px = A.xyz[3 * a], py = A.xyz[3 * a + 1], pz = A.xyz[3 * a + 2];
  const float l0 = A.scale[3 * a], l1 = A.scale[3 * a + 1], l2 = A.scale[3 * a + 2];
  if (grp == 3) {
    const float dx = px - A.cx, dy = py - A.cy, dz = pz - A.cz;
    const float delta = sqrtf(dx * dx + dy * dy + dz * dz);
    const float inv = 1.0f / delta;
    hin[5] = dx * inv;
    hin[6] = dy * inv;
    hin[7] = dz * inv;
    hin[8] = delta;
  }
  const float logl[3] = {logf(l0), logf(l1), logf(l2)};  // eq. 5
  for (int h = 0; h < 3; ++h) {
    stage_forward<KW>(A, h, P);
    // hid^T = relu(W1 h^T + b1); KW independent accumulation chains
    f32x4 acc[KW];
#pragma unroll
    for (int t = 0; t < KW; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 9; ++s)
#pragma unroll
      for (int t = 0; t < KW; ++t) acc[t] = mma(P.w1[(16 * t + lo) * kIn + 9 * grp + s], hin[s], acc[t]);
    float hid[KW][4];
#pragma unroll
    for (int t = 0; t < KW; ++t) {
      const float4 b = *reinterpret_cast<const float4*>(P.b1 + 16 * t + 4 * grp);
      hid[t][0] = fmaxf(acc[t][0] + b.x, 0.0f);
      hid[t][1] = fmaxf(acc[t][1] + b.y, 0.0f);
      hid[t][2] = fmaxf(acc[t][2] + b.z, 0.0f);
      hid[t][3] = fmaxf(acc[t][3] + b.w, 0.0f);
    }
    const int outs = head_outs(h, k);
    for (int o0 = 0; o0 < outs; o0 += 16) {
      // y^T = W2 hid^T + b2 for rows o0 .. o0 + 15; two interleaved
      // accumulators halve the dependent chain
      f32x4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < KW; ++t) {
        const float4 w = *reinterpret_cast<const float4*>(P.w2 + (o0 + lo) * P2 + 16 * t + 4 * grp);
        c0 = mma(w.x, hid[t][0], c0);
        c1 = mma(w.y, hid[t][1], c1);
        c0 = mma(w.z, hid[t][2], c0);
        c1 = mma(w.w, hid[t][3], c1);
      }
      const f32x4 c = c0 + c1;
      const float4 b = *reinterpret_cast<const float4*>(P.b2 + o0 + 4 * grp);
      const float y[4] = {c[0] + b.x, c[1] + b.y, c[2] + b.z, c[3] + b.w};
      const int s0 = o0 + 4 * grp;  // rows s0 .. s0 + 3 of anchor a
      if (!row_ok) continue;
      if (h == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (s0 + i < k) A.opac[a * k + s0 + i] = tanh_hw(y[i]);
      } else if (h == 1) {  // eq. 4
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (s0 + i < k3) A.colors[a * k3 + s0 + i] = sigmoidf_(y[i]);
      } else if (s0 < 4 * k) {  // the quaternion of Gaussian s0 / 4
        const float n = fmaxf(sqrtf(y[0] * y[0] + y[1] * y[1] + y[2] * y[2] + y[3] * y[3]), 1e-12f);
        const float in = 1.0f / n;
        float* q = A.quats + 4 * (a * k + (s0 >> 2));
#pragma unroll
        for (int i = 0; i < 4; ++i) q[i] = y[i] * in;
      } else {  // scale axis (s - 4k) % 3 of Gaussian (s - 4k) / 3 (eq. 5)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = s0 + i - 4 * k;
          if (r < k3) {
            const int c = r % 3;
            A.log_scales[a * k3 + r] = log_sigmoidf_(y[i]) + (c == 0 ? logl[0] : c == 1 ? logl[1] : logl[2]);
          }
        }
      }
    }
  }
}

// dhid[r][j] = sum_o dy[r][o] W2[o][j]; dpre = dhid where the hidden unit is
// active, written over the hidden layer (each lane reads and writes only its
// own elements).  Lane group g covers outputs o0 + 4g .. o0 + 4g + 3; the
// padded outputs hold zero gradients against zero weights.
template <int KW>
__device__ __forceinline__ void hid_grad_tiles(const float* w2s, int outs, const float* dys, int yp, float* hid,
                                               int lane) {
  constexpr int HP = 16 * KW + 1;
  const int lo = lane & 15, grp = lane >> 4;
  f32x4 acc[KW];
#pragma unroll
  for (int ct = 0; ct < KW; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int o0 = 0; o0 < outs; o0 += 16) {
    float a[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) a[s] = dys[lo * yp + o0 + 4 * grp + s];
#pragma unroll
    for (int ct = 0; ct < KW; ++ct) {
      const int j = 16 * ct + lo;
#pragma unroll
      for (int s = 0; s < 4; ++s) acc[ct] = mma(a[s], w2s[(o0 + 4 * grp + s) * HP + j], acc[ct]);
    }
  }
#pragma unroll
  for (int ct = 0; ct < KW; ++ct) {
    const int j = 16 * ct + lo;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 4 * grp + i;
      hid[r * HP + j] = hid[r * HP + j] > 0.0f ? acc[ct][i] : 0.0f;
    }
  }
}

// dh[r][c] += sum_j dpre[r][j] W1[j][c] for the 32 feature inputs (the
// direction and distance inputs have no parameters upstream).
template <int KW>
__device__ __forceinline__ void input_grad_tiles(const float* w1s, const float* dpre, f32x4 dh[2], int lane) {
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
      dh[ct] = mma(a[ks], w1s[j * kW1P + c], dh[ct]);
    }
  }
}

// part[p][q] += sum over the block's anchors a of X[a][p] Y'[a][q], where Y'
// is Y with a trailing all-ones column (q = Q gives the bias gradient).  Row
// a of X and Y lives in the LDS region of wavefront a / 16, at row a % 16;
// anchors past nvb (the block's valid count) contribute nothing.  The 16x16
// tiles, in row-major order, are split into contiguous runs, one per
// wavefront, which keeps its A operand (16 rows of X) in registers while the
// run stays in one tile row; a tile sums the block's anchors in 4 MFMA steps
// per wavefront (lane group g takes anchor 4s + g of step s).
__device__ __forceinline__ void wgrad_tiles(const float* region0, int region_floats, int xoff, int xp, int P,
                                            int yoff, int ypitch, int Q, int nvb, float* __restrict__ out, int wave,
                                            int lane) {
  constexpr int S = 4 * kDecWaves;  // contraction steps: 4 anchors each
  const int lo = lane & 15, grp = lane >> 4;
  const int nqt = (Q + 16) >> 4, nt = ((P + 15) >> 4) * nqt;
  const int t0 = wave * nt / kDecWaves, t1 = (wave + 1) * nt / kDecWaves;
  if (t0 >= t1) return;
  // anchor a = 4 s + g sits in the region of wavefront s / 4, at row
  // 4 (s % 4) + g.  Every read is unconditional (columns past the matrix
  // read its last column; bit masks clear padding and anchors past the
  // count), so a tile's reads are in flight together.
  auto load_x = [&](int pt, float* x) {
    const int p = 16 * pt + lo;
    const float* xs = region0 + xoff + grp * xp + std::min(p, P - 1);
    const uint32_t colm = p < P ? ~0u : 0u;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const float v = xs[(s >> 2) * region_floats + 4 * (s & 3) * xp];
      x[s] = __uint_as_float(__float_as_uint(v) & (4 * s + grp < nvb ? colm : 0u));
    }
  };
  auto load_y = [&](int qt, float* y) {
    const int q = 16 * qt + lo;
    const bool qv = q < Q;
    const float one = q == Q ? 1.0f : 0.0f;
    const float* ys = region0 + yoff + grp * ypitch + std::min(q, Q - 1);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const float v = ys[(s >> 2) * region_floats + 4 * (s & 3) * ypitch];
      y[s] = qv ? v : one;
    }
  };
  int pt = t0 / nqt, qt = t0 - pt * nqt;
  float x[S], y[S];
  load_x(pt, x);
  load_y(qt, y);
  for (int t = t0; t < t1; ++t) {
    // the next tile's operands load while this tile's products run
    int npt = pt, nq = qt + 1;
    if (nq == nqt) {
      nq = 0;
      ++npt;
    }
    const bool more = t + 1 < t1, new_row = more && npt != pt;
    float xn[S], yn[S];
    if (more) load_y(nq, yn);
    if (new_row) load_x(npt, xn);
    // two interleaved accumulators (even and odd steps) halve the dependent
    // MFMA chain
    f32x4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < S; s += 2) {
      c0 = mma(x[s], y[s], c0);
      c1 = mma(x[s + 1], y[s + 1], c1);
    }
    const f32x4 c = c0 + c1;
    const int q = 16 * qt + lo;
    if (q <= Q) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int pp = 16 * pt + 4 * grp + i;
        if (pp < P) out[pp * (Q + 1) + q] = c[i];
      }
    }
    if (more) {
#pragma unroll
      for (int s = 0; s < S; ++s) y[s] = yn[s];
    }
    if (new_row) {
#pragma unroll
      for (int s = 0; s < S; ++s) x[s] = xn[s];
    }
    pt = npt;
    qt = nq;
  }
}

struct ScaleGradIn {
  float gl[3], gq[4];
};

template <int KW>
__global__ void __launch_bounds__(kDecThreads) decode_backward_kernel(DecArgs A) {
  extern __shared__ float lds[];
  constexpr int HP = 16 * KW + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lo = lane & 15, grp = lane >> 4;
  const int k = A.k, W = A.width, yp = out_pitch(k);
  const float inv_k = 1.0f / k, inv_k3 = 1.0f / (3 * k);
  const HeadLds P = head_lds(lds, W, k);
  float* region0 = lds + head_lds_floats(W, k);
  const int region_floats = kRows * (kHP + HP + yp) + 3 * kRows;
  const int hid_off = kRows * kHP, ys_off = hid_off + kRows * HP;
  float* Hs = region0 + wave * region_floats;
  float* hid = Hs + hid_off;  // the hidden layer, then the gradient at its pre-activation
  float* ys = Hs + ys_off;    // the head outputs, then the gradient at them
  float* logl = ys + kRows * yp;
  const int64_t b0 = (A.block0 + blockIdx.x) * kDecWaves * kRows;
  const int nvb = (int)std::min<int64_t>(A.m - b0, kDecWaves * kRows);
  const int64_t a0 = b0 + wave * kRows;
  const int nv = std::max(std::min(nvb - wave * kRows, kRows), 0);
  float* part = A.part + (int64_t)blockIdx.x * A.part_per;
  load_inputs(A, a0, nv, lane, Hs, logl);
  const int k3 = 3 * k;
  // eq. 1: mean = anchor + offset * l
  blocked<8>(
      nv * k3, lane, [&](int e) { return float2{A.g_means[a0 * k3 + e], A.scale[3 * (a0 + quot(e, inv_k3)) + e % 3]}; },
      [&](int e, float2 v) { A.d_offsets[a0 * k3 + e] = v.x * v.y; });
  // scaling: through the means and through eq. 5's log l
  if (lane < 3 * nv) {
    const int r = lane / 3, c = lane - 3 * r;
    const int64_t a = a0 + r;
    const float l = A.scale[3 * a + c];
    float s = 0.0f;
    // eight Gaussians' loads in flight at a time (k <= 16); the sum keeps
    // its order: the mean terms, then the log-scale terms
    for (int m0 = 0; m0 < k; m0 += 8) {
      float gm[8], of[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t i = 3 * (a * k + std::min(m0 + u, k - 1)) + c;
        gm[u] = A.g_means[i];
        of[u] = A.offsets[i];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (m0 + u < k) s = fmaf(gm[u], of[u], s);
    }
    for (int m0 = 0; m0 < k; m0 += 8) {
      float gl[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) gl[u] = A.g_ls[3 * (a * k + std::min(m0 + u, k - 1)) + c];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (m0 + u < k) s += gl[u] / l;
    }
    A.d_scale[3 * a + c] = s;
  }
  lds_barrier();
  float ha[9];
#pragma unroll
  for (int ks = 0; ks < 9; ++ks) ha[ks] = Hs[lo * kHP + 9 * grp + ks];
  f32x4 dh[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
  for (int h = 0; h < 3; ++h) {
    const int outs = head_outs(h, k);
    stage_weights<KW>(A, h, P);
    hidden_tiles<KW>(P.w1, P.b1, ha, hid, lane);
    lds_barrier();
    out_tiles<KW>(P.w2, P.b2, outs, hid, ys, yp, lane);
    lds_barrier();
    // gradient at the head outputs, in place of the outputs
    if (h == 0) {  // tanh
      rmw_blocked<4, 1>(
          nv * k, lane, [&](int e) { return A.g_opac[a0 * k + e]; },
          [&](int e) {
            const int r = quot(e, inv_k);
            return ys + r * yp + e - r * k;
          },
          [&](float go, float* y) {
            const float t = tanh_hw(y[0]);
            y[0] = go * (1.0f - t * t);
          });
    } else if (h == 1) {  // sigmoid (eq. 4)
      rmw_blocked<8, 1>(
          nv * k3, lane, [&](int e) { return A.g_colors[a0 * k3 + e]; },
          [&](int e) {
            const int r = quot(e, inv_k3);
            return ys + r * yp + e - r * k3;
          },
          [&](float gc, float* y) {
            const float s = sigmoidf_(y[0]);
            y[0] = gc * s * (1.0f - s);
          });
    } else {  // [scale (eq. 5) | quaternion]
      rmw_blocked<4, 7>(
          nv * k, lane,
          [&](int e) {
            const int64_t g = a0 * k + e;
            return ScaleGradIn{{A.g_ls[3 * g], A.g_ls[3 * g + 1], A.g_ls[3 * g + 2]},
                               {A.g_quats[4 * g], A.g_quats[4 * g + 1], A.g_quats[4 * g + 2], A.g_quats[4 * g + 3]}};
          },
          [&](int e) {
            const int r = quot(e, inv_k);
            return ys + r * yp + 7 * (e - r * k);
          },
          [&](const ScaleGradIn& v, float* y) {
            float dy[7];
#pragma unroll
            for (int j = 0; j < 3; ++j) dy[j] = v.gl[j] * (1.0f - sigmoidf_(y[j]));  // d log_sigmoid(y) / dy
            const float nr = sqrtf(y[3] * y[3] + y[4] * y[4] + y[5] * y[5] + y[6] * y[6]);
            if (nr > 1e-12f) {
              const float in = 1.0f / nr;
              const float q0 = y[3] * in, q1 = y[4] * in, q2 = y[5] * in, q3 = y[6] * in;
              const float dot = q0 * v.gq[0] + q1 * v.gq[1] + q2 * v.gq[2] + q3 * v.gq[3];
              dy[3] = (v.gq[0] - q0 * dot) * in;
              dy[4] = (v.gq[1] - q1 * dot) * in;
              dy[5] = (v.gq[2] - q2 * dot) * in;
              dy[6] = (v.gq[3] - q3 * dot) * in;
            } else {
#pragma unroll
              for (int j = 0; j < 4; ++j) dy[3 + j] = v.gq[j] * 1e12f;
            }
#pragma unroll
            for (int j = 0; j < 7; ++j) y[j] = dy[j];
          });
    }
    lds_barrier();
    // dW2 = DY^T HID, db2 = column sums of DY
    wgrad_tiles(region0, region_floats, ys_off, yp, outs, hid_off, HP, W, nvb, part + A.part_off[2 * h], wave, lane);
    lds_barrier();
    hid_grad_tiles<KW>(P.w2, outs, ys, yp, hid, lane);
    lds_barrier();
    input_grad_tiles<KW>(P.w1, hid, dh, lane);
    // dW1 = DPRE^T H, db1 = column sums of DPRE
    wgrad_tiles(region0, region_floats, hid_off, HP, W, 0, kHP, kIn, nvb, part + A.part_off[2 * h + 1], wave, lane);
  }
#pragma unroll
  for (int ct = 0; ct < 2; ++ct)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 4 * grp + i;
      if (r < nv) A.d_feat[(a0 + r) * 32 + 16 * ct + lo] = dh[ct][i];
    }
}

// dst[g][e] (+)= sum of src[r][e] over the rows r of group g (group rows
// each, eight interleaved partial sums): the first level of the fixed-order
// sum of the block partials.  Adds to dst when accumulate is set.
__global__ void __launch_bounds__(256) sum_rows_kernel(const float* __restrict__ src, int rows, int64_t per,
                                                       int group, int accumulate, float* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= per) return;
  const int r0 = blockIdx.y * group, r1 = std::min(r0 + group, rows);
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  int r = r0;
  for (; r + 8 <= r1; r += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] += src[(int64_t)(r + u) * per + e];
  }
  for (; r < r1; ++r) s[0] += src[(int64_t)r * per + e];
  const float v = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
  float* d = dst + (int64_t)blockIdx.y * per + e;
  *d = accumulate ? *d + v : v;
}

constexpr int kNumProd = 6;
constexpr int kGroupRows = 32;   // block partials per first-level group
constexpr int kSliceRows = 2048;  // blocks per backward launch (64 group rows)

struct ReduceArgs {
  float* dW[kNumProd];
  float* db[kNumProd];
  int Q[kNumProd];
  int64_t off[kNumProd + 1];
  int64_t per;
  int rows;  // group rows to sum
  const float* part;
};

// Sums the group rows in a fixed order (four interleaved partial sums) into
// the weight and bias gradients.
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
  for (; c + 4 <= R.rows; c += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) s[u] += p[(int64_t)(c + u) * R.per];
  }
  for (; c < R.rows; ++c) s[0] += p[(int64_t)c * R.per];
  const float v = (s[0] + s[1]) + (s[2] + s[3]);
  const int64_t loc = e - off;
  const int64_t row = loc / (Q + 1);
  const int q = (int)(loc - row * (Q + 1));
  if (q < Q) dW[row * Q + q] = v;
  else db[row] = v;
}

size_t dec_lds_bytes(int W, int k) {
  const size_t hp = (size_t)pad16(W) + 1, yp = (size_t)out_pitch(k);
  return ((size_t)head_lds_floats(W, k) + kDecWaves * (kRows * (kHP + hp + yp) + 3 * kRows)) * sizeof(float);
}

template <int KW>
hipError_t launch_kw(bool backward, const DecArgs& A, unsigned blocks, hipStream_t s) {
  const size_t lds = backward ? dec_lds_bytes(A.width, A.k) : (size_t)fwd_lds_floats(KW, A.k) * sizeof(float);
  const void* f = backward ? reinterpret_cast<const void*>(&decode_backward_kernel<KW>)
                           : reinterpret_cast<const void*>(&decode_forward_kernel<KW>);
  hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (backward) hipLaunchKernelGGL(decode_backward_kernel<KW>, dim3(blocks), dim3(kDecThreads), lds, s, A);
  else hipLaunchKernelGGL(decode_forward_kernel<KW>, dim3(blocks), dim3(kDecThreads), lds, s, A);
  return hipGetLastError();
}

// LDS per block: the staged parameters of one head (forward: at most about
// 77 KB, width 128 and k = 16) and, in the backward, per wavefront its input
// rows, hidden layer, head outputs and log scalings (at most about 146 KB).
hipError_t launch_dec_any(bool backward, const DecArgs& A, hipStream_t s, unsigned blocks) {
  if (blocks == 0) return hipSuccess;
  switch ((A.width + 15) / 16) {
    case 1: return launch_kw<1>(backward, A, blocks, s);
    case 2: return launch_kw<2>(backward, A, blocks, s);
    case 3: return launch_kw<3>(backward, A, blocks, s);
    case 4: return launch_kw<4>(backward, A, blocks, s);
    case 5: return launch_kw<5>(backward, A, blocks, s);
    case 6: return launch_kw<6>(backward, A, blocks, s);
    case 7: return launch_kw<7>(backward, A, blocks, s);
    case 8: return launch_kw<8>(backward, A, blocks, s);
    default: return hipErrorInvalidValue;
  }
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
  HIP_TRY(launch_dec_any(false, A, st, (unsigned)((an->m + kRows * kDecWaves - 1) / (kRows * kDecWaves))));
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
  DecArgs A = make_args(an, mlp, cam_center);
  A.g_means = up->means; A.g_ls = up->log_scales; A.g_quats = up->quats; A.g_opac = up->opacities;
  A.g_colors = up->colors;
  A.d_feat = d_feat; A.d_scale = d_scale; A.d_offsets = d_offsets;
  ReduceArgs R;
  std::memset(&R, 0, sizeof(R));
  int64_t per = 0;
  for (int j = 0; j < kNumProd; ++j) {
    const int h = j / 2;
    // even j: dW2[h] = DY^T HID (+ db2); odd j: dW1[h] = DPRE^T H (+ db1)
    const int P = j % 2 == 0 ? outs[h] : width, Q = j % 2 == 0 ? width : kIn;
    A.part_off[j] = per;
    R.Q[j] = Q;
    R.off[j] = per;
    R.dW[j] = j % 2 == 0 ? dm->W2[h] : dm->W1[h];
    R.db[j] = j % 2 == 0 ? dm->b2[h] : dm->b1[h];
    per += (int64_t)P * (Q + 1);
  }
  R.off[kNumProd] = per;
  A.part_per = per;
  StageTimer t(ctx, ST_DEC_BWD, st);
  if (M == 0) {
    for (int j = 0; j < kNumProd; ++j) {
      const int64_t n = R.off[j + 1] - R.off[j];
      HIP_TRY(launch_fill_f32(R.dW[j], 0.f, (size_t)(n / (R.Q[j] + 1) * R.Q[j]), st));
      HIP_TRY(launch_fill_f32(R.db[j], 0.f, (size_t)(n / (R.Q[j] + 1)), st));
    }
    return VPGS_OK;
  }
  // One partial row per block of the per-anchor kernel.  The blocks run in
  // slices of at most kSliceRows; each slice's rows are summed in groups of
  // kGroupRows into the group rows (added to the earlier slices' sums), and
  // the group rows are summed last, all in a fixed order.
  const int64_t rows = (M + kRows * kDecWaves - 1) / (kRows * kDecWaves);
  const int slice = (int)std::min<int64_t>(rows, kSliceRows);
  const int groups = (slice + kGroupRows - 1) / kGroupRows;
  if ((rc = ensure(ctx, ctx->dec_partial, (size_t)(slice + groups) * per * 4))) return rc;
  A.part = static_cast<float*>(ctx->dec_partial.p);
  float* gsum = A.part + (int64_t)slice * per;
  const unsigned eblocks = (unsigned)((per + 255) / 256);
  for (int64_t b = 0; b < rows; b += slice) {
    const int n = (int)std::min<int64_t>(slice, rows - b);
    A.block0 = b;
    HIP_TRY(launch_dec_any(true, A, st, (unsigned)n));
    hipLaunchKernelGGL(sum_rows_kernel, dim3(eblocks, (n + kGroupRows - 1) / kGroupRows), dim3(256), 0, st, A.part,
                       n, per, kGroupRows, b > 0 ? 1 : 0, gsum);
    HIP_TRY(hipGetLastError());
  }
  R.per = per;
  R.rows = groups;
  R.part = gsum;
  hipLaunchKernelGGL(reduce_outer_kernel, dim3(eblocks), dim3(256), 0, st, R);
  HIP_TRY(hipGetLastError());
  return VPGS_OK;
}

}  // extern "C"
