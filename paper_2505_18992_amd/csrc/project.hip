// project.hip -- EWA projection of Gaussians into every view that renders
// them, and its backward (chain to the Gaussian parameters and to the left
// se(3) increment of each view's pose).
//
// One thread per Gaussian of a set loops over the views of that set, so the
// 56 parameter bytes of a Gaussian are read once per call however many views
// share the set.
#include "internal.h"

namespace vpgs {
namespace {

constexpr int kProjBlock = 256;
static_assert(kProjBlock / 64 == kPosePartialsPerBlock, "one pose partial per wavefront");

// Set index of a thread block (sets own contiguous block ranges).
__device__ __forceinline__ int set_of_block(const CallTables* tab, uint32_t blk) {
  int s = 0;
  for (int i = 1; i < tab->n_sets; ++i)
    if (blk >= tab->sets[i].block_base) s = i;
  return s;
}

// Camera-space mean and projected centre in FP32 with a fixed operation
// order and no contraction: these values decide visibility, the sort order
// and the tile rectangle, so they are reproducible bit for bit.
struct SpecPoint { float x, y, z, tx, ty, u, v; };
__device__ __forceinline__ SpecPoint spec_point(const ViewDesc& V, float mx, float my, float mz) {
#pragma clang fp contract(off)
  SpecPoint p;
  p.x = ((V.R[0] * mx + V.R[1] * my) + V.R[2] * mz) + V.t[0];
  p.y = ((V.R[3] * mx + V.R[4] * my) + V.R[5] * mz) + V.t[1];
  p.z = ((V.R[6] * mx + V.R[7] * my) + V.R[8] * mz) + V.t[2];
  p.tx = p.x / p.z;
  p.ty = p.y / p.z;
  p.u = V.fx * p.tx + V.cx;
  p.v = V.fy * p.ty + V.cy;
  return p;
}

// EWA screen-space covariance [[a, b], [b, c]] (with the low-pass dilation)
// and the rows of the projection Jacobian at the guarded centre; 1/z and the
// reciprocal of the determinant come from the hardware reciprocal (the
// forward and the backward form them the same way; the exactly rounded
// centre of SpecPoint is only needed for u and v).
struct ScreenCov { float tx, ty, txc, tyc, iz, J00, J02, J11, J12, a, b, c, idet; };
__device__ __forceinline__ ScreenCov screen_cov(const ViewDesc& V, const SpecPoint& p, const float Sc[9]) {
  ScreenCov s;
  s.iz = __builtin_amdgcn_rcpf(p.z);
  s.tx = p.x * s.iz;
  s.ty = p.y * s.iz;
  s.txc = fminf(fmaxf(s.tx, V.glx), V.ghx);
  s.tyc = fminf(fmaxf(s.ty, V.gly), V.ghy);
  s.J00 = V.fx * s.iz;
  s.J02 = -(V.fx * s.txc) * s.iz;
  s.J11 = V.fy * s.iz;
  s.J12 = -(V.fy * s.tyc) * s.iz;
  s.a = s.J00 * s.J00 * Sc[0] + 2.f * s.J00 * s.J02 * Sc[2] + s.J02 * s.J02 * Sc[8] + kDilate;
  s.b = s.J00 * s.J11 * Sc[1] + s.J00 * s.J12 * Sc[2] + s.J02 * s.J11 * Sc[5] + s.J02 * s.J12 * Sc[8];
  s.c = s.J11 * s.J11 * Sc[4] + 2.f * s.J11 * s.J12 * Sc[5] + s.J12 * s.J12 * Sc[8] + kDilate;
  s.idet = __builtin_amdgcn_rcpf(s.a * s.c - s.b * s.b);
  return s;
}

// Pixel box of the padded opacity-aware ellipse, in FP32 with a fixed
// operation order (pixel centres at +0.5: px is inside iff
// u - hx - 1 <= px + 0.5 <= u + hx + 1).
struct PixBox { int x0, x1, y0, y1; };
__device__ __forceinline__ PixBox pixel_box(float u, float v, float hx, float hy, int W, int H) {
#pragma clang fp contract(off)
  const float lox = fminf(fmaxf((u - hx) - 1.5f, 0.0f), (float)W);
  const float hix = fmaxf(fminf((u + hx) + 0.5f, (float)(W - 1)), -1.0f);
  const float loy = fminf(fmaxf((v - hy) - 1.5f, 0.0f), (float)H);
  const float hiy = fmaxf(fminf((v + hy) + 0.5f, (float)(H - 1)), -1.0f);
  PixBox b;
  b.x0 = (int)ceilf(lox);
  b.x1 = (int)floorf(hix);
  b.y0 = (int)ceilf(loy);
  b.y1 = (int)floorf(hiy);
  return b;
}

struct Quat { float w, x, y, z, inv_norm; bool ok; };
__device__ __forceinline__ Quat unit_quat(float4 q) {
  Quat r;
  const float m = fmaxf(fmaxf(fabsf(q.x), fabsf(q.y)), fmaxf(fabsf(q.z), fabsf(q.w)));
  r.ok = m > 0.0f && m < INFINITY;
  if (!r.ok) { r.w = 1; r.x = r.y = r.z = 0; r.inv_norm = 0; return r; }
  const float w = q.x / m, x = q.y / m, y = q.z / m, z = q.w / m;
  const float n = sqrtf(w * w + x * x + y * y + z * z);
  const float in = 1.0f / n;
  r.w = w * in; r.x = x * in; r.y = y * in; r.z = z * in;
  r.inv_norm = in / m;  // 1 / |q|
  return r;
}

__device__ __forceinline__ void quat_to_rot(const Quat& q, float Rq[9]) {
  const float w = q.w, x = q.x, y = q.y, z = q.z;
  Rq[0] = 1.f - 2.f * (y * y + z * z); Rq[1] = 2.f * (x * y - w * z);       Rq[2] = 2.f * (x * z + w * y);
  Rq[3] = 2.f * (x * y + w * z);       Rq[4] = 1.f - 2.f * (x * x + z * z); Rq[5] = 2.f * (y * z - w * x);
  Rq[6] = 2.f * (x * z - w * y);       Rq[7] = 2.f * (y * z + w * x);       Rq[8] = 1.f - 2.f * (x * x + y * y);
}

// Sigma = M M^T with M = R_q diag(s); returns the 3x3 matrix.
__device__ __forceinline__ void world_cov(const float Rq[9], const float s[3], float Sg[9]) {
  float M[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) M[3 * r + k] = Rq[3 * r + k] * s[k];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) Sg[3 * r + k] = M[3 * r] * M[3 * k] + M[3 * r + 1] * M[3 * k + 1] + M[3 * r + 2] * M[3 * k + 2];
}

// Sc = R Sg R^T
__device__ __forceinline__ void cam_cov(const float R[9], const float Sg[9], float Sc[9]) {
  float RS[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) RS[3 * r + k] = R[3 * r] * Sg[k] + R[3 * r + 1] * Sg[3 + k] + R[3 * r + 2] * Sg[6 + k];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) Sc[3 * r + k] = RS[3 * r] * R[3 * k] + RS[3 * r + 1] * R[3 * k + 1] + RS[3 * r + 2] * R[3 * k + 2];
}

__global__ void __launch_bounds__(kProjBlock) project_kernel(const CallTables* __restrict__ tab, ProjBuffers pb,
                                                             int tile_shift_x, int tile_shift_y,
                                                             Counters* __restrict__ cnt, uint2* __restrict__ ranges) {
  {
    // per-forward reset (no kernel of this forward has touched these yet)
    const uint32_t g = blockIdx.x * kProjBlock + threadIdx.x, stride = gridDim.x * kProjBlock;
    for (uint32_t w = g; w < (uint32_t)(sizeof(Counters) / 4); w += stride) reinterpret_cast<uint32_t*>(cnt)[w] = 0u;
    for (uint32_t t = g; t < tab->n_tiles; t += stride) ranges[t] = make_uint2(0u, 0u);
  }
  const int s = set_of_block(tab, blockIdx.x);
  const SetDesc& S = tab->sets[s];
  const int64_t i = (int64_t)(blockIdx.x - S.block_base) * kProjBlock + threadIdx.x;
  if (i >= S.n) return;
  const float mx = S.means[3 * i], my = S.means[3 * i + 1], mz = S.means[3 * i + 2];
  const float l0 = S.log_scales[3 * i], l1 = S.log_scales[3 * i + 1], l2 = S.log_scales[3 * i + 2];
  const float4 q4 = reinterpret_cast<const float4*>(S.quats)[i];
  const float o = S.opacities[i];
  const float c0 = S.colors[3 * i], c1 = S.colors[3 * i + 1], c2 = S.colors[3 * i + 2];
  const Quat q = unit_quat(q4);
  float Rq[9], Sg[9];
  quat_to_rot(q, Rq);
  const float sc[3] = {expf(l0), expf(l1), expf(l2)};
  world_cov(Rq, sc, Sg);
  const bool opaque = o > kAlphaMin;
  const float kq = 2.0f * logf(o / kAlphaMin);

  for (int vi = 0; vi < S.view_count; ++vi) {
    const int v = tab->set_views[S.view_first + vi];
    const ViewDesc& V = tab->views[v];
    const uint32_t rec = V.rec_base + (uint32_t)i;
    const SpecPoint p = spec_point(V, mx, my, mz);
    bool ok = q.ok && opaque && (p.z > V.near_z);
    float Sc[9];
    cam_cov(V.R, Sg, Sc);
    const ScreenCov sc2 = screen_cov(V, p, Sc);
    const float a = sc2.a, b = sc2.b, c = sc2.c;
    ok = ok && a * c - b * b > 0.0f;
    const float Qa = c * sc2.idet, Qb = -b * sc2.idet, Qc = a * sc2.idet;
    const float hx = __builtin_amdgcn_sqrtf(kq * a), hy = __builtin_amdgcn_sqrtf(kq * c);
    ok = ok && isfinite(p.u) && isfinite(p.v) && isfinite(Qa) && isfinite(Qb) && isfinite(Qc) &&
         isfinite(hx) && isfinite(hy);
    uint32_t count = 0;
    uint2 rect = make_uint2(0, 0);
    if (ok) {
      const PixBox bx = pixel_box(p.u, p.v, hx, hy, V.W, V.H);
      if (bx.x0 <= bx.x1 && bx.y0 <= bx.y1) {
        const uint32_t tx0 = (uint32_t)bx.x0 >> tile_shift_x, tx1 = (uint32_t)bx.x1 >> tile_shift_x;
        const uint32_t ty0 = (uint32_t)bx.y0 >> tile_shift_y, ty1 = (uint32_t)bx.y1 >> tile_shift_y;
        count = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
        rect = make_uint2(tx0 | (tx1 << 16), ty0 | (ty1 << 16));
        float4* out = pb.rec + rec_slot(rec, 0);
        out[0] = make_float4(p.u, p.v, p.z, o);
        out[1] = make_float4(Qa, Qb, Qc, 0.0f);
        out[2] = make_float4(c0, c1, c2, 0.0f);
        // the quadrant test's vertex factors, as the compositor would form
        // them from the staged conic
        const float ra = __builtin_amdgcn_rcpf(2.0f * -(Qa * kNegHalfLog2e));
        const float rc = __builtin_amdgcn_rcpf(2.0f * -(Qc * kNegHalfLog2e));
        out[3] = make_float4(hx, hy, ra, rc);
        pb.zkey[rec] = __float_as_uint(p.z);
        pb.rect[rec] = rect;
      }
    }
    pb.count[rec] = count;
  }
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------

// Wavefront reduce-scatter of the six pose terms: each step pairs a lane
// with the one that differs in one lane-index bit, keeps half of its values
// and adds the partner's copy of them.
//   bit 5: p[i] with p[3 + i] by v_permlane32_swap            6 -> 3 values
//   bit 4: (h0, h1) by v_permlane16_swap, h2 in both            3 -> 2
//   bit 3: (a, c) by DPP row rotate 8 (lane xor 8)              2 -> 1
//   bits 0-2: sums over the 8-lane group (DPP).
// Lane L ends with the wave total of term 3 b5 + (b3 ? 2 : b4) (b = bits of
// L).  All lanes of the wavefront must be active.
template <int CTRL>
__device__ __forceinline__ float pdpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float psum32(float lo, float hi) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float psum16(float lo, float hi) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float pose_reduce_scatter6(const float p[6], int lane) {
  const bool b3 = (lane >> 3) & 1;
  const float h0 = psum32(p[0], p[3]), h1 = psum32(p[1], p[4]), h2 = psum32(p[2], p[5]);
  const float a = psum16(h0, h1);
  const float c = psum16(h2, h2);
  float x = (b3 ? c : a) + pdpp<0x128>(b3 ? a : c);  // row_ror:8
  x += pdpp<0x141>(x);  // row_half_mirror
  x += pdpp<0xB1>(x);   // quad_perm [1,0,3,2]
  x += pdpp<0x4E>(x);   // quad_perm [2,3,0,1]
  return x;
}
__device__ __forceinline__ int pose_slot(int lane) {
  const int b3 = (lane >> 3) & 1, b4 = (lane >> 4) & 1, b5 = (lane >> 5) & 1;
  return 3 * b5 + (b3 ? 2 : b4);
}
// One lane per term: the first of its 8-lane group, and for term 3 b5 + 2
// (held by the groups with b3 set) only the one with b4 = 0.
__device__ __forceinline__ bool pose_writer(int lane) {
  return (lane & 7) == 0 && !(((lane >> 3) & 1) && ((lane >> 4) & 1));
}

__global__ void __launch_bounds__(kProjBlock) project_backward_kernel(const CallTables* __restrict__ tab, ProjBuffers pb,
                                                                      float* __restrict__ acc,
                                                                      float* __restrict__ pose_partial) {
  const int s = set_of_block(tab, blockIdx.x);
  const SetDesc& S = tab->sets[s];
  const int64_t i = (int64_t)(blockIdx.x - S.block_base) * kProjBlock + threadIdx.x;
  const bool live = i < S.n;
  const int64_t ii = live ? i : 0;

  const float mx = S.means[3 * ii], my = S.means[3 * ii + 1], mz = S.means[3 * ii + 2];
  const float ls[3] = {S.log_scales[3 * ii], S.log_scales[3 * ii + 1], S.log_scales[3 * ii + 2]};
  const float4 q4 = reinterpret_cast<const float4*>(S.quats)[ii];
  const Quat q = unit_quat(q4);
  float Rq[9], Sg[9];
  quat_to_rot(q, Rq);
  const float sc[3] = {expf(ls[0]), expf(ls[1]), expf(ls[2])};
  world_cov(Rq, sc, Sg);

  float dmu[3] = {0, 0, 0}, dSg[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  float dop = 0.f, dcol[3] = {0, 0, 0};
  // expansion accumulators: screen-space gradient norm and rendered views,
  // opacity and views whose frustum holds the centre
  const bool track = S.accum != nullptr;
  const float o_par = S.opacities[ii];
  const float inv_o = 1.0f / o_par;
  const float o_acc = track ? fmaxf(o_par, 0.0f) : 0.0f;
  float a_grad = 0.f, a_ren = 0.f, a_op = 0.f, a_seen = 0.f;

  uint32_t vis = 0;  // bit u: the record of view (vi & ~7) + u is visible
  for (int vi = 0; vi < S.view_count; ++vi) {
    if ((vi & 7) == 0) {
      // the tile counts of the next eight views' records, loaded together
      uint32_t c8[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int vj = min(vi + u, S.view_count - 1);
        c8[u] = pb.count[tab->views[tab->set_views[S.view_first + vj]].rec_base + (uint32_t)ii];
      }
      vis = 0;
#pragma unroll
      for (int u = 0; u < 8; ++u) vis |= (live && vi + u < S.view_count && c8[u] != 0) ? (1u << u) : 0u;
    }
    const int v = tab->set_views[S.view_first + vi];
    const ViewDesc& V = tab->views[v];
    const uint32_t rec = V.rec_base + (uint32_t)ii;
    float pose[6] = {0, 0, 0, 0, 0, 0};
    if ((vis >> (vi & 7)) & 1u) {
      // read the record's accumulated gradient and leave its row zero for
      // the next backward (rows of culled records are never touched)
      float* g = acc + (size_t)rec * kNumAcc;
      const float m0 = g[0], m1 = g[1], m2 = g[2], m3 = g[3], m4 = g[4], go = g[5];
      const float gz_direct = g[9];
      const float gc0 = g[6], gc1 = g[7], gc2 = g[8];
#pragma unroll
      for (int k = 0; k < kNumAcc; ++k) g[k] = 0.0f;
      dop += go * inv_o;  // the row holds the sum of s = o dL/do (o > 1/255 for a visible record)
      dcol[0] += gc0; dcol[1] += gc1; dcol[2] += gc2;

      const SpecPoint p = spec_point(V, mx, my, mz);
      float Sc[9];
      cam_cov(V.R, Sg, Sc);
      const ScreenCov sc2 = screen_cov(V, p, Sc);
      const float tx = sc2.tx, ty = sc2.ty, txc = sc2.txc, tyc = sc2.tyc, iz = sc2.iz;
      const float J00 = sc2.J00, J02 = sc2.J02, J11 = sc2.J11, J12 = sc2.J12;
      const float a = sc2.a, b = sc2.b, c = sc2.c;
      const float Qa = c * sc2.idet, Qb = -b * sc2.idet, Qc = a * sc2.idet;
      // the row holds moments of s = dL/dalpha * alpha over the pixel offsets
      // d = (u, v) - pixel centre; dL/dsigma = -s with
      // sigma = (Qa dx^2 + 2 Qb dx dy + Qc dy^2) / 2
      const float gu = -(Qa * m0 + Qb * m1), gv = -(Qb * m0 + Qc * m1);
      const float gQa = -0.5f * m2, gQb = -m3, gQc = -0.5f * m4;
      if (track) {
        const float su = tab->accum_space ? 0.5f * (float)V.W : 1.0f;
        const float sv = tab->accum_space ? 0.5f * (float)V.H : 1.0f;
        const float nu = gu * su, nv = gv * sv;
        a_grad += sqrtf(nu * nu + nv * nv);
        a_ren += 1.0f;
      }

      // conic = Sigma2D^-1:  dL/dSigma2D = -Q G Q, G the symmetric conic gradient
      const float dA = -(Qa * Qa * gQa + Qa * Qb * gQb + Qb * Qb * gQc);
      const float dB = -(2.f * Qa * Qb * gQa + (Qa * Qc + Qb * Qb) * gQb + 2.f * Qb * Qc * gQc);  // scalar b
      const float dC = -(Qb * Qb * gQa + Qb * Qc * gQb + Qc * Qc * gQc);
      const float G00 = dA, G01 = 0.5f * dB, G11 = dC;
      // Sigma2D = J Sc J^T:  dSc = J^T G J,  dJ = 2 G J Sc
      const float Jm[6] = {J00, 0.f, J02, 0.f, J11, J12};
      float GJ[6];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        GJ[k] = G00 * Jm[k] + G01 * Jm[3 + k];
        GJ[3 + k] = G01 * Jm[k] + G11 * Jm[3 + k];
      }
      float dSc[9];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) dSc[3 * r + k] = Jm[r] * GJ[k] + Jm[3 + r] * GJ[3 + k];
      float dJ[6];
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k)
          dJ[3 * r + k] = 2.f * (GJ[3 * r] * Sc[k] + GJ[3 * r + 1] * Sc[3 + k] + GJ[3 * r + 2] * Sc[6 + k]);
      // J and (u, v, z) to the camera-space mean
      float dx = gu * V.fx * iz, dy = gv * V.fy * iz;
      float dz = gz_direct - (gu * V.fx * tx + gv * V.fy * ty) * iz;
      dz += -(dJ[0] * V.fx + dJ[4] * V.fy) * iz * iz;
      dz += (dJ[2] * V.fx * txc + dJ[5] * V.fy * tyc) * iz * iz;
      const float dtxc = -dJ[2] * V.fx * iz, dtyc = -dJ[5] * V.fy * iz;
      if (tx > V.glx && tx < V.ghx) { dx += dtxc * iz; dz -= dtxc * tx * iz; }
      if (ty > V.gly && ty < V.ghy) { dy += dtyc * iz; dz -= dtyc * ty * iz; }
      // camera-space mean to the world mean: dmu = R^T dp
      dmu[0] += V.R[0] * dx + V.R[3] * dy + V.R[6] * dz;
      dmu[1] += V.R[1] * dx + V.R[4] * dy + V.R[7] * dz;
      dmu[2] += V.R[2] * dx + V.R[5] * dy + V.R[8] * dz;
      // Sc = R Sg R^T:  dSg = R^T dSc R (accumulated over views)
      float T1[9];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) T1[3 * r + k] = V.R[r] * dSc[k] + V.R[3 + r] * dSc[3 + k] + V.R[6 + r] * dSc[6 + k];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) dSg[3 * r + k] += T1[3 * r] * V.R[k] + T1[3 * r + 1] * V.R[3 + k] + T1[3 * r + 2] * V.R[6 + k];
      // pose: rho = dp; phi = p x dp + 2 vee-part of A = Sc dSc
      float A[9];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) A[3 * r + k] = Sc[3 * r] * dSc[k] + Sc[3 * r + 1] * dSc[3 + k] + Sc[3 * r + 2] * dSc[6 + k];
      pose[0] = dx; pose[1] = dy; pose[2] = dz;
      pose[3] = p.y * dz - p.z * dy + 2.f * (A[5] - A[7]);
      pose[4] = p.z * dx - p.x * dz + 2.f * (A[6] - A[2]);
      pose[5] = p.x * dy - p.y * dx + 2.f * (A[1] - A[3]);
    }
    if (track && live) {
      const SpecPoint p = spec_point(V, mx, my, mz);
      if (p.z > V.near_z && p.u >= 0.0f && p.u < (float)V.W && p.v >= 0.0f && p.v < (float)V.H) {
        a_op += o_acc;
        a_seen += 1.0f;
      }
    }
    if (pose_partial != nullptr) {
      // wavefront sums (no barrier); the pose reduction adds the wavefronts
      const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
      const float t = pose_reduce_scatter6(pose, lane);
      if (pose_writer(lane)) {
        float* dst = pose_partial + (((size_t)v * gridDim.x + blockIdx.x) * kPosePartialsPerBlock + wave) * 6;
        dst[pose_slot(lane)] = t;
      }
    }
  }
  if (!live) return;
  // Sg = M M^T with M = R_q diag(s):  dM = 2 dSg M
  float M[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) M[3 * r + k] = Rq[3 * r + k] * sc[k];
  float dM[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      dM[3 * r + k] = (dSg[3 * r] + dSg[r]) * M[k] + (dSg[3 * r + 1] + dSg[3 + r]) * M[3 + k] +
                      (dSg[3 * r + 2] + dSg[6 + r]) * M[6 + k];
  // (the symmetrised form (dSg + dSg^T) M equals 2 dSg M for symmetric dSg)
  float ds[3], dR[9];
#pragma unroll
  for (int k = 0; k < 3; ++k) ds[k] = dM[k] * Rq[k] + dM[3 + k] * Rq[3 + k] + dM[6 + k] * Rq[6 + k];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) dR[3 * r + k] = dM[3 * r + k] * sc[k];
  const float w = q.w, x = q.x, y = q.y, z = q.z;
  const float dqw = 2.f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
  const float dqx = 2.f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.f * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] - 2.f * x * dR[8]);
  const float dqy = 2.f * (-2.f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] - 2.f * y * dR[8]);
  const float dqz = 2.f * (-2.f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.f * z * dR[4] + y * dR[5] + x * dR[6] + y * dR[7]);
  const float dot = w * dqw + x * dqx + y * dqy + z * dqz;
  const float in = q.inv_norm;
  S.d_means[3 * i] = dmu[0]; S.d_means[3 * i + 1] = dmu[1]; S.d_means[3 * i + 2] = dmu[2];
  S.d_log_scales[3 * i] = ds[0] * sc[0];
  S.d_log_scales[3 * i + 1] = ds[1] * sc[1];
  S.d_log_scales[3 * i + 2] = ds[2] * sc[2];
  reinterpret_cast<float4*>(S.d_quats)[i] =
      make_float4((dqw - w * dot) * in, (dqx - x * dot) * in, (dqy - y * dot) * in, (dqz - z * dot) * in);
  S.d_opacities[i] = dop;
  S.d_colors[3 * i] = dcol[0]; S.d_colors[3 * i + 1] = dcol[1]; S.d_colors[3 * i + 2] = dcol[2];
  if (track) {
    float4* a = reinterpret_cast<float4*>(S.accum) + i;
    float4 cur = *a;
    cur.x += a_grad; cur.y += a_ren; cur.z += a_op; cur.w += a_seen;
    *a = cur;
  }
}

// One workgroup per view: the sum of the wavefront partials of the blocks of
// the view's set, four rows (of 6 floats) per thread in flight.
__global__ void __launch_bounds__(256) pose_reduce_kernel(const CallTables* __restrict__ tab,
                                                          const float* __restrict__ partial, int total_blocks,
                                                          float* __restrict__ d_pose) {
  __shared__ float red[4][6];
  const int v = blockIdx.x;
  const SetDesc& S = tab->sets[tab->views[v].set];
  const size_t first = ((size_t)v * total_blocks + S.block_base) * kPosePartialsPerBlock;
  const uint32_t rows = (uint32_t)((S.n + kProjBlock - 1) / kProjBlock) * kPosePartialsPerBlock;
  const float2* p = reinterpret_cast<const float2*>(partial + first * 6);  // 3 float2 per row
  float s[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  uint32_t r = threadIdx.x;
  for (; r + 3 * 256 < rows; r += 4 * 256) {
    float2 a[4][3];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int c = 0; c < 3; ++c) a[u][c] = p[3 * (size_t)(r + u * 256) + c];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        s[2 * c] += a[u][c].x;
        s[2 * c + 1] += a[u][c].y;
      }
  }
  for (; r < rows; r += 256)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float2 a = p[3 * (size_t)r + c];
      s[2 * c] += a.x;
      s[2 * c + 1] += a.y;
    }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s[k] += __shfl_xor(s[k], off, 64);
    if (lane == 0) red[wave][k] = s[k];
  }
  __syncthreads();
  const int k = threadIdx.x;
  if (k < 6) d_pose[6 * v + k] = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
}

int ilog2(int x) {
  int r = 0;
  while ((1 << r) < x) ++r;
  return r;
}

}  // namespace

uint32_t project_blocks(const CallTables& h) {
  uint32_t b = 0;
  for (int s = 0; s < h.n_sets; ++s) b += (uint32_t)((h.sets[s].n + kProjBlock - 1) / kProjBlock);
  return b;
}

// Half extents (hx, hy) of every record, zero for culled ones.
__global__ void export_extent_kernel(ProjBuffers pb, uint32_t n, float2* __restrict__ out) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  float2 e = make_float2(0.0f, 0.0f);
  if (pb.count[r] != 0) {
    const float4 x = pb.rec[rec_slot(r, 3)];
    e = make_float2(x.x, x.y);
  }
  out[r] = e;
}

hipError_t launch_export_extent(const ProjBuffers pb, uint32_t n, float2* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(export_extent_kernel, dim3((n + 255) / 256), dim3(256), 0, s, pb, n, out);
  return hipGetLastError();
}

hipError_t launch_project(const CallTables* d_tab, const CallTables& h_tab, ProjBuffers pb, int tile_w, int tile_h,
                          Counters* cnt, uint2* ranges, hipStream_t s) {
  const uint32_t pblocks = project_blocks(h_tab);
  const uint32_t blocks = pblocks > 0 ? pblocks : 1u;  // one block at least, for the reset
  hipLaunchKernelGGL(project_kernel, dim3(blocks), dim3(kProjBlock), 0, s, d_tab, pb, ilog2(tile_w), ilog2(tile_h),
                     cnt, ranges);
  return hipGetLastError();
}

hipError_t launch_project_backward(const CallTables* d_tab, const CallTables& h_tab, const ProjBuffers pb,
                                   float* acc, float* pose_partial, hipStream_t s) {
  const uint32_t blocks = project_blocks(h_tab);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(project_backward_kernel, dim3(blocks), dim3(kProjBlock), 0, s, d_tab, pb, acc, pose_partial);
  return hipGetLastError();
}

hipError_t launch_pose_reduce(const CallTables* d_tab, const CallTables& h_tab, const float* pose_partial,
                              float* d_pose, hipStream_t s) {
  if (h_tab.n_views == 0) return hipSuccess;
  hipLaunchKernelGGL(pose_reduce_kernel, dim3(h_tab.n_views), dim3(256), 0, s, d_tab, pose_partial,
                     (int)project_blocks(h_tab), d_pose);
  return hipGetLastError();
}

}  // namespace vpgs
