// oracle.cpp -- plain, slow FP64 reference of the differentiable Gaussian
// splatting renderer (RGB, depth, alpha; gradients to the Gaussian parameters
// and to a left se(3) camera-pose increment).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
// calls this file; only the tests, the smoke check and the CPU-baseline leg of
// the benchmark do.  It shares no code, header or constant table with the HIP
// path.
//
// What is computed (the paper renders colour and opacity of its Gaussian
// submaps, eq. 6, through the 3D Gaussian splatting rasterisation pipeline it
// cites in Section I and Section II; depth enters the L1 depth loss of eq. 7
// and the photometric tracking of Section III-B).  The paper gives no renderer
// detail, so the definition below is the standard EWA-splatting compositor
// with the readings listed in the design notes:
//
//   F1  q^ = q/|q| (w,x,y,z); R_q the rotation of the unit quaternion.
//   F2  s = exp(l); Sigma = R_q diag(s^2) R_q^T.
//   F3  p = R mu + t; visible iff the FP32 depth z > near (strict).
//   F4  t = (x/z, y/z); guard clamp to the 1.3x field of view in pixel-margin
//       form; J = [[fx/z, 0, -fx tx'/z], [0, fy/z, -fy ty'/z]].
//   F5  Sigma2D = J (R Sigma R^T) J^T + 0.3 I.
//   F6  det = ac - b^2 > 0; conic Q = (c, -b, a)/det.
//   F7  u = fx tx + cx, v = fy ty + cy.
//   F8  pixel (px, py) samples at (px + 0.5, py + 0.5).
//   F9  cull unless o > 1/255; opacity-aware box {d^T Q d <= 2 ln(o / (1/255))}
//       padded by one pixel.
//   F10 order: ascending (bits of the FP32 depth, index).
//   F11 per pixel: alpha = min(0.99, o exp(-sigma)); skip alpha < 1/255; stop
//       before blending when T (1 - alpha) < 1e-4.
//   F12 RGB = sum alpha T c, depth = sum alpha T z, alpha = 1 - T.
//
// Gradients are forward-mode dual numbers over the same templated functions
// (no hand-written adjoint): per pixel a 10-component dual over the blended
// suffix gives d(outputs)/d(u, v, Qa, Qb, Qc, o, c, z) of each blended
// Gaussian; per Gaussian a 20-component dual over the projection gives the
// Jacobian of those 10 quantities with respect to its 14 parameters and the
// 6 pose coordinates.  The chain rule multiplies the two.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

// The scalar every step is evaluated in.  The reference build is FP64; an
// FP32 build of the same source (ORACLE_REAL=float, with single-precision
// literals) measures how far a float32 evaluation of the definition moves
// each result, and is the like-for-like CPU timing of the method.
#ifndef ORACLE_REAL
#define ORACLE_REAL double
#endif
typedef ORACLE_REAL real;

namespace {

// FP32 literals of the method, held in the evaluation scalar so that both
// sides test against the same real numbers.
const real kAlphaMin = (real)(1.0f / 255.0f);
const real kAlphaMax = (real)0.99f;
const real kTmin = (real)1e-4f;
const real kDilate = (real)0.3f;
const real kGuardLo = (real)0.15f;   // guard margin beyond the image, in image widths
const real kGuardHi = (real)1.15f;

// ---------------------------------------------------------------------------
// forward-mode dual numbers
// ---------------------------------------------------------------------------
template <int N>
struct Dual {
  real v;
  real d[N];
  Dual() : v(0) { std::memset(d, 0, sizeof(d)); }
  Dual(real x) : v(x) { std::memset(d, 0, sizeof(d)); }  // NOLINT: implicit constant
};
template <int N> inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) { Dual<N> r(a.v + b.v); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) { Dual<N> r(a.v - b.v); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a) { Dual<N> r(-a.v); for (int i = 0; i < N; ++i) r.d[i] = -a.d[i]; return r; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) { Dual<N> r(a.v * b.v); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) { Dual<N> r(a.v / b.v); for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v); return r; }
template <int N> inline Dual<N> operator+(const Dual<N>& a, real b) { return a + Dual<N>(b); }
template <int N> inline Dual<N> operator+(real a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, real b) { return a - Dual<N>(b); }
template <int N> inline Dual<N> operator-(real a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, real b) { return a * Dual<N>(b); }
template <int N> inline Dual<N> operator*(real a, const Dual<N>& b) { return Dual<N>(a) * b; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, real b) { return a / Dual<N>(b); }
template <int N> inline Dual<N> operator/(real a, const Dual<N>& b) { return Dual<N>(a) / b; }
template <int N> inline Dual<N> exp(const Dual<N>& a) { real e = std::exp(a.v); Dual<N> r(e); for (int i = 0; i < N; ++i) r.d[i] = e * a.d[i]; return r; }
template <int N> inline Dual<N> sqrt(const Dual<N>& a) { real s = std::sqrt(a.v); Dual<N> r(s); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] / (2.0 * s); return r; }
template <int N> inline real val(const Dual<N>& a) { return a.v; }
inline real val(real a) { return a; }
using std::exp;
using std::sqrt;

// ---------------------------------------------------------------------------
// camera
// ---------------------------------------------------------------------------
struct Cam {
  int W, H;
  real fx, fy, cx, cy, nearp;
  real R[9], t[3];
  float fR[9], ft[3], ffx, ffy, fcx, fcy, fnear;  // the same values as float
};

Cam make_cam(int W, int H, const double* intr, const double* w2c) {
  Cam c;
  c.W = W; c.H = H;
  c.fx = intr[0]; c.fy = intr[1]; c.cx = intr[2]; c.cy = intr[3]; c.nearp = intr[4];
  for (int r = 0; r < 3; ++r) {
    for (int k = 0; k < 3; ++k) c.R[3 * r + k] = w2c[4 * r + k];
    c.t[r] = w2c[4 * r + 3];
  }
  for (int i = 0; i < 9; ++i) c.fR[i] = (float)c.R[i];
  for (int i = 0; i < 3; ++i) c.ft[i] = (float)c.t[i];
  c.ffx = (float)c.fx; c.ffy = (float)c.fy; c.fcx = (float)c.cx; c.fcy = (float)c.cy;
  c.fnear = (float)c.nearp;
  return c;
}

// FP32 values that decide integers (visibility, sort order) and that the
// binning keys depend on.  Exp-free, fixed operation order, no contraction
// (this file is compiled with -ffp-contract=off).
struct Spec32 { float x, y, z, u, v; };
Spec32 spec32(const Cam& c, const real* mu) {
  const float mx = (float)mu[0], my = (float)mu[1], mz = (float)mu[2];
  Spec32 s;
  s.x = ((c.fR[0] * mx + c.fR[1] * my) + c.fR[2] * mz) + c.ft[0];
  s.y = ((c.fR[3] * mx + c.fR[4] * my) + c.fR[5] * mz) + c.ft[1];
  s.z = ((c.fR[6] * mx + c.fR[7] * my) + c.fR[8] * mz) + c.ft[2];
  const float tx = s.x / s.z, ty = s.y / s.z;
  s.u = c.ffx * tx + c.fcx;
  s.v = c.ffy * ty + c.fcy;
  return s;
}
inline uint32_t fbits(float f) { uint32_t b; std::memcpy(&b, &f, 4); return b; }

// ---------------------------------------------------------------------------
// projection (F1-F7), templated on the scalar so duals flow through it
// ---------------------------------------------------------------------------
template <class S>
struct Proj { S u, v, z, Qa, Qb, Qc, a, b, c; };

template <class S>
bool project_math(const S mu[3], const S ls[3], const S q[4], const S R[9], const S t[3],
                  const Cam& cam, Proj<S>& out) {
  // F3 camera-space mean
  S p[3];
  for (int r = 0; r < 3; ++r) p[r] = R[3 * r] * mu[0] + R[3 * r + 1] * mu[1] + R[3 * r + 2] * mu[2] + t[r];
  // F1 unit quaternion and its rotation
  S n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  if (!(val(n2) > 0.0)) return false;
  S inv = 1.0 / sqrt(n2);
  S w = q[0] * inv, x = q[1] * inv, y = q[2] * inv, z = q[3] * inv;
  S Rq[9] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y),
             2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x),
             2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)};
  // F2 Sigma = M M^T with M = R_q diag(exp(l))
  S s[3] = {exp(ls[0]), exp(ls[1]), exp(ls[2])};
  S M[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) M[3 * r + k] = Rq[3 * r + k] * s[k];
  S Sig[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) {
      S acc(0.0);
      for (int m = 0; m < 3; ++m) acc = acc + M[3 * r + m] * M[3 * k + m];
      Sig[3 * r + k] = acc;
    }
  // F5 camera-space covariance R Sigma R^T
  S RS[9], Sc[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) {
      S acc(0.0);
      for (int m = 0; m < 3; ++m) acc = acc + R[3 * r + m] * Sig[3 * m + k];
      RS[3 * r + k] = acc;
    }
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) {
      S acc(0.0);
      for (int m = 0; m < 3; ++m) acc = acc + RS[3 * r + m] * R[3 * k + m];
      Sc[3 * r + k] = acc;
    }
  // F4 Jacobian of the pinhole map with the guard clamp
  S tx = p[0] / p[2], ty = p[1] / p[2];
  const real lx = (-kGuardLo * cam.W - cam.cx) / cam.fx, hx = (kGuardHi * cam.W - cam.cx) / cam.fx;
  const real ly = (-kGuardLo * cam.H - cam.cy) / cam.fy, hy = (kGuardHi * cam.H - cam.cy) / cam.fy;
  S txc = tx, tyc = ty;
  if (val(tx) < lx) txc = S(lx);
  if (val(tx) > hx) txc = S(hx);
  if (val(ty) < ly) tyc = S(ly);
  if (val(ty) > hy) tyc = S(hy);
  S J[6] = {cam.fx / p[2], S(0.0), -(cam.fx * txc) / p[2],
            S(0.0), cam.fy / p[2], -(cam.fy * tyc) / p[2]};
  S JS[6];
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 3; ++k) {
      S acc(0.0);
      for (int m = 0; m < 3; ++m) acc = acc + J[3 * r + m] * Sc[3 * m + k];
      JS[3 * r + k] = acc;
    }
  S C2[4];
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 2; ++k) {
      S acc(0.0);
      for (int m = 0; m < 3; ++m) acc = acc + JS[3 * r + m] * J[3 * k + m];
      C2[2 * r + k] = acc;
    }
  out.a = C2[0] + kDilate;
  out.b = C2[1];
  out.c = C2[3] + kDilate;
  // F6 conic
  S det = out.a * out.c - out.b * out.b;
  if (!(val(det) > 0.0)) return false;
  out.Qa = out.c / det;
  out.Qb = -out.b / det;
  out.Qc = out.a / det;
  // F7 projected mean
  out.u = cam.fx * tx + cam.cx;
  out.v = cam.fy * ty + cam.cy;
  out.z = p[2];
  return true;
}

// Primal per-Gaussian record in FP64 plus the FP32 values that decide integers.
struct Prim {
  int valid;
  real u, v, z, Qa, Qb, Qc, a, b, c, o, col[3];
  real hx, hy;
  int x0, x1, y0, y1;
  uint32_t zbits;
  float u32, v32, z32;
  int near_guard;  // 1 if the guard clamp is within a relative 1e-6 of switching
};

bool finite_all(const Prim& p) {
  const real xs[] = {p.u, p.v, p.z, p.Qa, p.Qb, p.Qc, p.a, p.b, p.c};
  for (real x : xs) if (!std::isfinite(x)) return false;
  return true;
}

Prim project_one(const Cam& cam, const real* mu, const real* ls, const real* q, real o,
                 const real* col, int use_box) {
  Prim pr;
  std::memset(&pr, 0, sizeof(pr));
  const Spec32 s32 = spec32(cam, mu);
  pr.u32 = s32.u; pr.v32 = s32.v; pr.z32 = s32.z;
  pr.zbits = fbits(s32.z);
  pr.o = o;
  for (int k = 0; k < 3; ++k) pr.col[k] = col[k];
  // visibility is decided in FP32 (F3) and on the float opacity (F9)
  if (!(s32.z > cam.fnear)) return pr;
  if (!((float)o > 1.0f / 255.0f)) return pr;
  Proj<real> P;
  if (!project_math<real>(mu, ls, q, cam.R, cam.t, cam, P)) return pr;
  pr.u = P.u; pr.v = P.v; pr.z = P.z; pr.Qa = P.Qa; pr.Qb = P.Qb; pr.Qc = P.Qc;
  pr.a = P.a; pr.b = P.b; pr.c = P.c;
  if (!finite_all(pr)) return pr;
  {
    const real tx = (cam.R[0] * mu[0] + cam.R[1] * mu[1] + cam.R[2] * mu[2] + cam.t[0]) / P.z;
    const real ty = (cam.R[3] * mu[0] + cam.R[4] * mu[1] + cam.R[5] * mu[2] + cam.t[1]) / P.z;
    const real lims[4] = {(-kGuardLo * cam.W - cam.cx) / cam.fx, (kGuardHi * cam.W - cam.cx) / cam.fx,
                            (-kGuardLo * cam.H - cam.cy) / cam.fy, (kGuardHi * cam.H - cam.cy) / cam.fy};
    const real vals[4] = {tx, tx, ty, ty};
    for (int i = 0; i < 4; ++i)
      if (std::fabs(vals[i] - lims[i]) <= 1e-6 * std::max(1.0, std::fabs(lims[i]))) pr.near_guard = 1;
  }
  // F9 opacity-aware box, padded by one pixel, pixel centres at +0.5
  const real kq = 2.0 * std::log(o / kAlphaMin);
  pr.hx = std::sqrt(kq * P.a);
  pr.hy = std::sqrt(kq * P.c);
  if (use_box) {
    const real lo_x = std::ceil(P.u - pr.hx - 1.5), hi_x = std::floor(P.u + pr.hx + 0.5);
    const real lo_y = std::ceil(P.v - pr.hy - 1.5), hi_y = std::floor(P.v + pr.hy + 0.5);
    const real x0 = std::max(lo_x, 0.0), x1 = std::min(hi_x, (real)(cam.W - 1));
    const real y0 = std::max(lo_y, 0.0), y1 = std::min(hi_y, (real)(cam.H - 1));
    if (!(x0 <= x1 && y0 <= y1)) return pr;
    pr.x0 = (int)x0; pr.x1 = (int)x1; pr.y0 = (int)y0; pr.y1 = (int)y1;
  } else {
    pr.x0 = 0; pr.x1 = cam.W - 1; pr.y0 = 0; pr.y1 = cam.H - 1;
  }
  pr.valid = 1;
  return pr;
}

struct Inputs {
  int64_t n;
  const real *means, *ls, *quats, *opac, *cols;
};

// The caller's FP64 arrays in the evaluation scalar.
struct InputCopy {
  std::vector<real> m, l, q, o, c;
  Inputs in;
  InputCopy(int64_t n, const double* means, const double* ls, const double* quats, const double* opac,
            const double* cols)
      : m(means, means + 3 * n), l(ls, ls + 3 * n), q(quats, quats + 4 * n), o(opac, opac + n),
        c(cols, cols + 3 * n), in{n, m.data(), l.data(), q.data(), o.data(), c.data()} {}
};

std::vector<Prim> project_all(const Cam& cam, const Inputs& in, int use_box) {
  std::vector<Prim> out((size_t)in.n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < in.n; ++i)
    out[i] = project_one(cam, in.means + 3 * i, in.ls + 3 * i, in.quats + 4 * i, in.opac[i], in.cols + 3 * i, use_box);
  return out;
}

// Candidate lists: Gaussians whose box contains a pixel, in F10 order.  Lists
// are kept per block of pixel rows x 64 columns only to find candidates
// quickly; every pixel still filters by its own box test.
struct Buckets {
  int bw, bh, nbx, nby;
  std::vector<std::vector<int32_t>> lists;
};

Buckets make_buckets(const Cam& cam, const std::vector<Prim>& pr) {
  Buckets b;
  b.bw = 64; b.bh = 4;
  b.nbx = (cam.W + b.bw - 1) / b.bw;
  b.nby = (cam.H + b.bh - 1) / b.bh;
  b.lists.assign((size_t)b.nbx * b.nby, {});
  std::vector<int32_t> order;
  for (size_t i = 0; i < pr.size(); ++i)
    if (pr[i].valid) order.push_back((int32_t)i);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) {
    if (pr[a].zbits != pr[c].zbits) return pr[a].zbits < pr[c].zbits;
    return a < c;
  });
  for (int32_t i : order) {
    const Prim& p = pr[i];
    for (int by = p.y0 / b.bh; by <= p.y1 / b.bh; ++by)
      for (int bx = p.x0 / b.bw; bx <= p.x1 / b.bw; ++bx) b.lists[(size_t)by * b.nbx + bx].push_back(i);
  }
  return b;
}

inline void pixel_candidates(const Buckets& b, const std::vector<Prim>& pr, int px, int py, std::vector<int32_t>& out) {
  out.clear();
  const auto& L = b.lists[(size_t)(py / b.bh) * b.nbx + px / b.bw];
  for (int32_t i : L) {
    const Prim& p = pr[i];
    if (px >= p.x0 && px <= p.x1 && py >= p.y0 && py <= p.y1) out.push_back(i);
  }
}

struct Margins { real alpha, clamp, trans; };

// F11 primal composite of one pixel over its ordered candidates.
struct PixOut {
  real C[3], D, T;
  int nb, ne;
  int flag;
  int32_t last;  // candidate position of the last blended Gaussian, -1 if none
};

PixOut composite_pixel(const std::vector<Prim>& pr, const std::vector<int32_t>& cand, int px, int py,
                       const Margins& m, std::vector<int32_t>* blended, std::vector<real>* bl_alpha,
                       std::vector<real>* bl_T) {
  PixOut r;
  r.C[0] = r.C[1] = r.C[2] = 0.0; r.D = 0.0; r.T = 1.0; r.nb = 0; r.ne = 0; r.flag = 0; r.last = -1;
  const real cxp = px + 0.5, cyp = py + 0.5;
  // A float32 evaluation carries the projected centre to within a few units
  // in the last place of |u|, |v|; that moves sigma by |d sigma/d u| du and
  // alpha by the same relative amount.  The flag margins add this term, and
  // the transmittance margin accumulates the relative errors of (1 - alpha).
  const real ulp_pos = std::ldexp(1.0, -22);
  real T = 1.0, eT = 0.0;
  for (size_t k = 0; k < cand.size(); ++k) {
    const Prim& p = pr[cand[k]];
    if (p.near_guard) r.flag = 1;
    const real dx = p.u - cxp, dy = p.v - cyp;
    const real sigma = 0.5 * (p.Qa * dx * dx + p.Qc * dy * dy) + p.Qb * dx * dy;
    const real raw = p.o * std::exp(-sigma);
    const real drel = std::fabs(p.Qa * dx + p.Qb * dy) * std::fabs(p.u) * ulp_pos +
                        std::fabs(p.Qb * dx + p.Qc * dy) * std::fabs(p.v) * ulp_pos +
                        (1.0 + sigma) * 16.0 * std::ldexp(1.0, -24);  // exp and conic rounding
    if (std::fabs(raw - kAlphaMax) <= m.clamp + raw * drel) r.flag = 1;
    const real alpha = std::min(kAlphaMax, raw);
    r.ne++;
    if (std::fabs(alpha - kAlphaMin) <= (m.alpha + drel) * kAlphaMin) r.flag = 1;
    if (alpha < kAlphaMin) continue;
    const real Tn = T * (1.0 - alpha);
    eT += alpha * drel / (1.0 - alpha);
    if (std::fabs(Tn - kTmin) <= (m.trans + eT) * kTmin) r.flag = 1;
    if (Tn < kTmin) break;
    const real w = alpha * T;
    for (int ch = 0; ch < 3; ++ch) r.C[ch] += w * p.col[ch];
    r.D += w * p.z;
    if (blended) { blended->push_back(cand[k]); bl_alpha->push_back(alpha); bl_T->push_back(T); }
    T = Tn;
    r.nb++;
    r.last = (int32_t)k;
  }
  r.T = T;
  return r;
}

// The 10 per-Gaussian quantities the compositor consumes.
enum { QU = 0, QV, QA, QB, QC, QO, QR, QG, QBL, QZ, NQ };

// d(outputs)/d(quantities of the blended Gaussian at position k) for one
// pixel: the blended sequence is fixed by the primal pass, a 10-component dual
// runs the F11 recurrence over the suffix starting at k.
void pixel_quantity_grads(const std::vector<Prim>& pr, const std::vector<int32_t>& bl,
                          const std::vector<real>& bl_T, size_t k, int px, int py,
                          Dual<NQ> out[5] /* R, G, B, D, A */, Dual<NQ>* alpha_k) {
  typedef Dual<NQ> D;
  const real cxp = px + 0.5, cyp = py + 0.5;
  const Prim& g = pr[bl[k]];
  D q[NQ];
  const real qv[NQ] = {g.u, g.v, g.Qa, g.Qb, g.Qc, g.o, g.col[0], g.col[1], g.col[2], g.z};
  for (int i = 0; i < NQ; ++i) { q[i] = D(qv[i]); q[i].d[i] = 1.0; }
  D C[3] = {D(0.0), D(0.0), D(0.0)};
  D Dp(0.0);
  D T(bl_T[k]);
  for (size_t j = k; j < bl.size(); ++j) {
    const Prim& p = pr[bl[j]];
    D alpha, cc[3], z;
    if (j == k) {
      D dx = q[QU] - cxp, dy = q[QV] - cyp;
      D sigma = 0.5 * (q[QA] * dx * dx + q[QC] * dy * dy) + q[QB] * dx * dy;
      D raw = q[QO] * exp(-sigma);
      alpha = raw.v < kAlphaMax ? raw : D(kAlphaMax);
      if (alpha_k) *alpha_k = alpha;
      cc[0] = q[QR]; cc[1] = q[QG]; cc[2] = q[QBL]; z = q[QZ];
    } else {
      const real dx = p.u - cxp, dy = p.v - cyp;
      const real sigma = 0.5 * (p.Qa * dx * dx + p.Qc * dy * dy) + p.Qb * dx * dy;
      alpha = D(std::min(kAlphaMax, p.o * std::exp(-sigma)));
      cc[0] = D(p.col[0]); cc[1] = D(p.col[1]); cc[2] = D(p.col[2]); z = D(p.z);
    }
    D w = alpha * T;
    for (int ch = 0; ch < 3; ++ch) C[ch] = C[ch] + w * cc[ch];
    Dp = Dp + w * z;
    T = T * (1.0 - alpha);
  }
  out[0] = C[0]; out[1] = C[1]; out[2] = C[2]; out[3] = Dp; out[4] = 1.0 - T;
}

}  // namespace

extern "C" {

// Per-Gaussian projection in FP64 plus the FP32 spec values.
//   intr = (fx, fy, cx, cy, near); w2c = row-major 3x4 [R|t].
//   out_f64[n*11] = (u, v, z, a, b, c, Qa, Qb, Qc, hx, hy); out_f32[n*3] = (u32, v32, z32);
//   valid[n] = 1 if the Gaussian survives culling (box test included).
int oracle_project(int W, int H, const double* intr, const double* w2c, int64_t n,
                   const double* means, const double* ls, const double* quats, const double* opac,
                   const double* cols, double* out_f64, float* out_f32, uint8_t* valid, int32_t* box) {
  const Cam cam = make_cam(W, H, intr, w2c);
  const InputCopy copy(n, means, ls, quats, opac, cols);
  const Inputs& in = copy.in;
  std::vector<Prim> pr = project_all(cam, in, 1);
  for (int64_t i = 0; i < n; ++i) {
    const Prim& p = pr[i];
    double* o = out_f64 + 11 * i;
    o[0] = p.u; o[1] = p.v; o[2] = p.z; o[3] = p.a; o[4] = p.b; o[5] = p.c;
    o[6] = p.Qa; o[7] = p.Qb; o[8] = p.Qc; o[9] = p.hx; o[10] = p.hy;
    out_f32[3 * i] = p.u32; out_f32[3 * i + 1] = p.v32; out_f32[3 * i + 2] = p.z32;
    valid[i] = (uint8_t)p.valid;
    if (box) { box[4 * i] = p.x0; box[4 * i + 1] = p.x1; box[4 * i + 2] = p.y0; box[4 * i + 3] = p.y1; }
  }
  return 0;
}

// FP64 forward render of one view.  brute_force = 1 ignores the boxes and
// tests every visible Gaussian at every pixel.  Margins flag pixels where an
// FP32 evaluation of a threshold test could differ from this one.
int oracle_render(int W, int H, const double* intr, const double* w2c, int64_t n,
                  const double* means, const double* ls, const double* quats, const double* opac,
                  const double* cols, int brute_force, double m_alpha, double m_clamp, double m_trans,
                  double* rgb, double* depth, double* alpha, double* T_final, int32_t* n_blend,
                  int32_t* n_eval, uint8_t* flags) {
  const Cam cam = make_cam(W, H, intr, w2c);
  const InputCopy copy(n, means, ls, quats, opac, cols);
  const Inputs& in = copy.in;
  std::vector<Prim> pr = project_all(cam, in, brute_force ? 0 : 1);
  Buckets b = make_buckets(cam, pr);
  const Margins m{(real)m_alpha, (real)m_clamp, (real)m_trans};
  const size_t HW = (size_t)W * H;
#pragma omp parallel
  {
    std::vector<int32_t> cand;
#pragma omp for schedule(dynamic, 1)
    for (int py = 0; py < H; ++py)
      for (int px = 0; px < W; ++px) {
        pixel_candidates(b, pr, px, py, cand);
        PixOut r = composite_pixel(pr, cand, px, py, m, nullptr, nullptr, nullptr);
        const size_t pi = (size_t)py * W + px;
        for (int ch = 0; ch < 3; ++ch) rgb[ch * HW + pi] = r.C[ch];
        depth[pi] = r.D;
        alpha[pi] = 1.0 - r.T;
        if (T_final) T_final[pi] = r.T;
        if (n_blend) n_blend[pi] = r.nb;
        if (n_eval) n_eval[pi] = r.ne;
        if (flags) flags[pi] = (uint8_t)r.flag;
      }
  }
  return 0;
}

// FP64 gradient of L = sum_p g_rgb . RGB + g_d D + g_a A for one view.
// skip[p] = 1 drops pixel p from the loss.  Outputs are written (not
// accumulated).  s_* are the error scales: sums over pixels and quantities of
// |contribution to d L / d(quantity)| |d(quantity)/d(parameter)|, where the
// contribution through alpha_i counts the magnitudes of the two terms of
// d L / d alpha_i = T_i f_i - S_i / (1 - alpha_i) (f = g . (c, z, 1), S the
// weighted sum of f behind i): a floating-point evaluation of that difference
// errs relative to those magnitudes, not to their (possibly cancelling) sum.
int oracle_grad(int W, int H, const double* intr, const double* w2c, int64_t n,
                const double* means, const double* ls, const double* quats, const double* opac,
                const double* cols, const double* g_rgb, const double* g_depth, const double* g_alpha,
                const uint8_t* skip, double* d_means, double* d_ls, double* d_quats, double* d_opac,
                double* d_cols, double* d_pose, double* s_means, double* s_ls, double* s_quats,
                double* s_opac, double* s_cols, double* s_pose, double* q_grad, double* b_means,
                double* b_ls, double* b_quats, double* b_opac, double* b_cols, double* b_pose,
                double* q_scale, double* q_bound) {
  const Cam cam = make_cam(W, H, intr, w2c);
  const InputCopy copy(n, means, ls, quats, opac, cols);
  const Inputs& in = copy.in;
  std::vector<Prim> pr = project_all(cam, in, 1);
  Buckets b = make_buckets(cam, pr);
  const Margins m{0.0, 0.0, 0.0};
  const size_t HW = (size_t)W * H;
  std::vector<real> G((size_t)n * NQ, 0.0), Gabs((size_t)n * NQ, 0.0), Gfp((size_t)n * NQ, 0.0);
  const real ulp_pos = std::ldexp(1.0, -22);
#pragma omp parallel
  {
    std::vector<int32_t> cand, bl;
    std::vector<real> bla, blT, fbar, drel, eTb;
    Dual<NQ> outs[5], alpha_k;
#pragma omp for schedule(dynamic, 1)
    for (int py = 0; py < H; ++py)
      for (int px = 0; px < W; ++px) {
        const size_t pi = (size_t)py * W + px;
        if (skip && skip[pi]) continue;
        const real gw[5] = {(real)g_rgb[pi], (real)g_rgb[HW + pi], (real)g_rgb[2 * HW + pi], (real)g_depth[pi],
                            (real)g_alpha[pi]};
        if (gw[0] == 0 && gw[1] == 0 && gw[2] == 0 && gw[3] == 0 && gw[4] == 0) continue;
        pixel_candidates(b, pr, px, py, cand);
        bl.clear(); bla.clear(); blT.clear();
        composite_pixel(pr, cand, px, py, m, &bl, &bla, &blT);
        // magnitude of f for every blended Gaussian, and the suffix sums
        fbar.assign(bl.size(), 0.0);
        for (size_t j = 0; j < bl.size(); ++j) {
          const Prim& p = pr[bl[j]];
          fbar[j] = std::fabs(gw[0]) * std::fabs(p.col[0]) + std::fabs(gw[1]) * std::fabs(p.col[1]) +
                    std::fabs(gw[2]) * std::fabs(p.col[2]) + std::fabs(gw[3]) * std::fabs(p.z) + std::fabs(gw[4]);
        }
        // first-order float32 propagation: relative error of each blended
        // alpha from the rounding of the projected centre, and the relative
        // error it leaves in the transmittance of everything behind it
        drel.assign(bl.size(), 0.0);
        eTb.assign(bl.size(), 0.0);
        real eT = 0.0;
        for (size_t j = 0; j < bl.size(); ++j) {
          const Prim& p = pr[bl[j]];
          const real dx = p.u - (px + 0.5), dy = p.v - (py + 0.5);
          const real sigma = 0.5 * (p.Qa * dx * dx + p.Qc * dy * dy) + p.Qb * dx * dy;
          drel[j] = std::fabs(p.Qa * dx + p.Qb * dy) * std::fabs(p.u) * ulp_pos +
                    std::fabs(p.Qb * dx + p.Qc * dy) * std::fabs(p.v) * ulp_pos +
                    (1.0 + sigma) * 16.0 * std::ldexp(1.0, -24);  // exp and conic rounding
          eTb[j] = eT;
          eT += bla[j] * drel[j] / (1.0 - bla[j]) + 2.0 * std::ldexp(1.0, -24);
        }
        real behind = 0.0;  // sum over blended j > k of alpha_j T_j fbar_j
        for (size_t kk = bl.size(); kk-- > 0;) {
          const size_t k = kk;
          pixel_quantity_grads(pr, bl, blT, k, px, py, outs, &alpha_k);
          const int32_t gi = bl[k];
          const real mag = blT[k] * fbar[k] + behind / (1.0 - bla[k]);
          for (int qn = 0; qn < NQ; ++qn) {
            real acc = 0.0;
            for (int o = 0; o < 5; ++o) acc += gw[o] * outs[o].d[qn];
            const real scale = qn <= QO ? mag * std::fabs(alpha_k.d[qn]) : std::fabs(acc);
            const real fp = qn <= QO ? scale * (eT + drel[k]) : scale * (eTb[k] + drel[k]);
#pragma omp atomic
            G[(size_t)gi * NQ + qn] += acc;
#pragma omp atomic
            Gabs[(size_t)gi * NQ + qn] += scale;
#pragma omp atomic
            Gfp[(size_t)gi * NQ + qn] += fp;
          }
          behind += bla[k] * blT[k] * fbar[k];
        }
      }
  }
  if (q_grad)  // d L / d(u, v, Qa, Qb, Qc, o, r, g, b, z) of every Gaussian
    for (size_t i = 0; i < G.size(); ++i) q_grad[i] = G[i];
  if (q_scale)  // and their error scales and float32 bounds
    for (size_t i = 0; i < G.size(); ++i) { q_scale[i] = Gabs[i]; q_bound[i] = Gfp[i]; }
  // chain through the projection: 14 parameter duals + 6 pose duals
  typedef Dual<20> D20;
  real pose[6] = {0, 0, 0, 0, 0, 0}, spose[6] = {0, 0, 0, 0, 0, 0}, bpose[6] = {0, 0, 0, 0, 0, 0};
#pragma omp parallel
  {
    real lpose[6] = {0, 0, 0, 0, 0, 0}, lspose[6] = {0, 0, 0, 0, 0, 0}, lbpose[6] = {0, 0, 0, 0, 0, 0};
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      double* dm = d_means + 3 * i; double* dl = d_ls + 3 * i; double* dq = d_quats + 4 * i;
      double* dc = d_cols + 3 * i;
      double* sm = s_means + 3 * i; double* sl = s_ls + 3 * i; double* sq = s_quats + 4 * i;
      double* sc = s_cols + 3 * i;
      for (int k = 0; k < 3; ++k) dm[k] = dl[k] = dc[k] = sm[k] = sl[k] = sc[k] = 0.0;
      for (int k = 0; k < 4; ++k) dq[k] = sq[k] = 0.0;
      d_opac[i] = s_opac[i] = 0.0;
      double* bm = b_means + 3 * i; double* bl_ = b_ls + 3 * i; double* bq = b_quats + 4 * i;
      double* bc = b_cols + 3 * i;
      for (int k = 0; k < 3; ++k) bm[k] = bl_[k] = bc[k] = 0.0;
      for (int k = 0; k < 4; ++k) bq[k] = 0.0;
      b_opac[i] = 0.0;
      const real* Gi = &G[(size_t)i * NQ];
      const real* Ai = &Gabs[(size_t)i * NQ];
      const real* Fi = &Gfp[(size_t)i * NQ];
      bool any = false;
      for (int qn = 0; qn < NQ; ++qn) any = any || Ai[qn] != 0.0;
      if (!any) continue;
      D20 mu[3], l3[3], q4[4], R[9], t[3];
      for (int k = 0; k < 3; ++k) { mu[k] = D20(means[3 * i + k]); mu[k].d[k] = 1.0; }
      for (int k = 0; k < 3; ++k) { l3[k] = D20(ls[3 * i + k]); l3[k].d[3 + k] = 1.0; }
      for (int k = 0; k < 4; ++k) { q4[k] = D20(quats[4 * i + k]); q4[k].d[6 + k] = 1.0; }
      // left increment at zero: R' = (I + [phi]x) R, t' = (I + [phi]x) t + rho;
      // pose duals occupy slots 14..16 (rho) and 17..19 (phi).
      for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) R[3 * r + c] = D20(cam.R[3 * r + c]);
        t[r] = D20(cam.t[r]);
        t[r].d[14 + r] = 1.0;
      }
      // [e_k]x rows: e_x -> (0,0,0; 0,0,-1; 0,1,0) etc.
      const real E[3][9] = {{0, 0, 0, 0, 0, -1, 0, 1, 0}, {0, 0, 1, 0, 0, 0, -1, 0, 0}, {0, -1, 0, 1, 0, 0, 0, 0, 0}};
      for (int kk = 0; kk < 3; ++kk)
        for (int r = 0; r < 3; ++r) {
          for (int c = 0; c < 3; ++c) {
            real acc = 0.0;
            for (int mm = 0; mm < 3; ++mm) acc += E[kk][3 * r + mm] * cam.R[3 * mm + c];
            R[3 * r + c].d[17 + kk] = acc;
          }
          real acc = 0.0;
          for (int mm = 0; mm < 3; ++mm) acc += E[kk][3 * r + mm] * cam.t[mm];
          t[r].d[17 + kk] += acc;
        }
      Proj<D20> P;
      if (!project_math<D20>(mu, l3, q4, R, t, cam, P)) continue;
      D20 qd[NQ];
      qd[QU] = P.u; qd[QV] = P.v; qd[QA] = P.Qa; qd[QB] = P.Qb; qd[QC] = P.Qc; qd[QZ] = P.z;
      qd[QO] = D20(opac[i]); qd[QO].d[10] = 1.0;
      for (int k = 0; k < 3; ++k) { qd[QR + k] = D20(cols[3 * i + k]); qd[QR + k].d[11 + k] = 1.0; }
      real dv[20], sv[20], bv[20];
      for (int j = 0; j < 20; ++j) {
        real acc = 0.0, sacc = 0.0, bacc = 0.0;
        for (int qn = 0; qn < NQ; ++qn) {
          acc += Gi[qn] * qd[qn].d[j];
          sacc += Ai[qn] * std::fabs(qd[qn].d[j]);
          bacc += Fi[qn] * std::fabs(qd[qn].d[j]);
        }
        dv[j] = acc; sv[j] = sacc; bv[j] = bacc;
      }
      for (int k = 0; k < 3; ++k) { bm[k] = bv[k]; bl_[k] = bv[3 + k]; bc[k] = bv[11 + k]; }
      for (int k = 0; k < 4; ++k) bq[k] = bv[6 + k];
      b_opac[i] = bv[10];
      for (int k = 0; k < 6; ++k) lbpose[k] += bv[14 + k];
      for (int k = 0; k < 3; ++k) { dm[k] = dv[k]; sm[k] = sv[k]; dl[k] = dv[3 + k]; sl[k] = sv[3 + k]; }
      for (int k = 0; k < 4; ++k) { dq[k] = dv[6 + k]; sq[k] = sv[6 + k]; }
      d_opac[i] = dv[10]; s_opac[i] = sv[10];
      for (int k = 0; k < 3; ++k) { dc[k] = dv[11 + k]; sc[k] = sv[11 + k]; }
      for (int k = 0; k < 6; ++k) { lpose[k] += dv[14 + k]; lspose[k] += sv[14 + k]; }
    }
#pragma omp critical
    for (int k = 0; k < 6; ++k) { pose[k] += lpose[k]; spose[k] += lspose[k]; bpose[k] += lbpose[k]; }
  }
  for (int k = 0; k < 6; ++k) { d_pose[k] = pose[k]; s_pose[k] = spose[k]; b_pose[k] = bpose[k]; }
  return 0;
}

// Tile binning on given FP32 per-Gaussian values (the integer part of the
// path): pixel box from (u, v, hx, hy) in FP32 with a fixed operation order,
// tile rectangle, one (tile << 32 | depth bits, index) pair per overlapped
// tile, a stable sort, and the [start, end) range of every tile (empty tiles
// get (0, 0)).  Returns the pair count, or -1 if it exceeds cap.
int64_t oracle_binning(int64_t n, const uint8_t* valid, const float* u, const float* v, const float* hx,
                       const float* hy, const uint32_t* zbits, int W, int H, int tw, int th,
                       uint32_t tile_base, uint32_t index_base, int64_t cap, uint64_t* keys,
                       uint32_t* vals, uint32_t* ranges) {
  const int tiles_x = (W + tw - 1) / tw, tiles_y = (H + th - 1) / th;
  std::vector<std::pair<uint64_t, uint32_t>> pairs;
  for (int64_t i = 0; i < n; ++i) {
    if (!valid[i]) continue;
    const float lox = std::fmin(std::fmax((u[i] - hx[i]) - 1.5f, 0.0f), (float)W);
    const float hix = std::fmax(std::fmin((u[i] + hx[i]) + 0.5f, (float)(W - 1)), -1.0f);
    const float loy = std::fmin(std::fmax((v[i] - hy[i]) - 1.5f, 0.0f), (float)H);
    const float hiy = std::fmax(std::fmin((v[i] + hy[i]) + 0.5f, (float)(H - 1)), -1.0f);
    const int x0 = (int)std::ceil(lox), x1 = (int)std::floor(hix);
    const int y0 = (int)std::ceil(loy), y1 = (int)std::floor(hiy);
    if (x0 > x1 || y0 > y1) continue;
    for (int ty = y0 / th; ty <= y1 / th; ++ty)
      for (int tx = x0 / tw; tx <= x1 / tw; ++tx) {
        const uint64_t tile = (uint64_t)tile_base + (uint64_t)ty * tiles_x + tx;
        pairs.push_back({(tile << 32) | zbits[i], (uint32_t)(index_base + i)});
      }
  }
  std::stable_sort(pairs.begin(), pairs.end(),
                   [](const std::pair<uint64_t, uint32_t>& a, const std::pair<uint64_t, uint32_t>& c) {
                     return a.first < c.first;
                   });
  const int64_t P = (int64_t)pairs.size();
  if (P > cap) return -1;
  for (int64_t k = 0; k < P; ++k) { keys[k] = pairs[k].first; vals[k] = pairs[k].second; }
  const int ntiles = tiles_x * tiles_y;
  for (int t = 0; t < 2 * ntiles; ++t) ranges[t] = 0;
  for (int64_t k = 0; k < P; ++k) {
    const int t = (int)((pairs[k].first >> 32) - tile_base);
    if (k == 0 || (pairs[k - 1].first >> 32) != (pairs[k].first >> 32)) ranges[2 * t] = (uint32_t)k;
    ranges[2 * t + 1] = (uint32_t)(k + 1);
  }
  return P;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
