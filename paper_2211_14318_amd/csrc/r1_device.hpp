// Device-side building blocks of the rank-one lamination path (gfx950, wave64).
//
// Method: arXiv 2211.14318 (Balzani et al.).  W is the condensed incremental
// potential of eq. 2.9 with the neo-Hooke psi0 of eq. 2.3; lamination follows
// eq. 3.3 along the discrete rank-one lines of Section 4.1; each line is
// convexified (the lower hull of Algorithm 1) and read at its centre.
//
// Layout of one line on a wavefront: a line of n_t = 2c+1 samples is owned by
// a segment of S lanes.  Lane sl of the segment holds the K/2 sample pairs at
// offsets m = 1 + sl + S*h (h < K/2) on both sides of the centre: w[h] is the
// sample at t = -m*h_t (left), w[K/2+h] the one at t = +m*h_t (right).  The
// centre sample is the same for every direction and is passed in.  Offsets
// m > c are padding: their abscissa is NaN, so their samples are NaN, which
// every hull comparison treats as absent.  64/S lines are processed side by side.
//
// Hull at the centre: the centre is a hull vertex iff every left sample's slope
// towards it is strictly smaller than every right sample's slope from it (one
// pass, fused with sampling).  Otherwise the hull segment over the centre is
// the lower common tangent ("bridge") of the left and right sample sets, found
// by slope iteration (hull_centre), with the alternating tangent search as a
// fallback.  Ties prefer the outermost sample, matching the strict-vertex
// reading of Algorithm 1.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "r1.h"
#include "r1_math.hpp"

namespace r1d {

constexpr int kWave = 64;
constexpr int kBridgeCap = 256;   // tangent rounds before giving up (never reached in practice)

template <typename T> __device__ __forceinline__ T inf_v();
template <> __device__ __forceinline__ float inf_v<float>() { return __builtin_inff(); }
template <> __device__ __forceinline__ double inf_v<double>() { return __builtin_inf(); }

// Logarithm used by W: FP32 takes the hardware log2 (v_log_f32) and carries
// ln 2 in the coefficients; FP64 takes the natural log of r1_math.hpp.
__device__ __forceinline__ float lg_t(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ double lg_t(double x) { return r1x::log_f64(x); }
// Exponential of an argument pre-scaled by the per-point constant kexp:
// FP32 uses the hardware exp2 (kexp carries log2 e), FP64 the exp of r1_math.hpp.
__device__ __forceinline__ float expk(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ double expk(double x) { return r1x::exp_f64(x); }

struct Material {
  int dim, model;        // model: 0 neo-Hooke damage, 1 double-well test energy, 2 St. Venant-Kirchhoff damage
  double mu, lambda, D_inf, D0;
};

struct Level {           // one lamination level on the device
  const double* a;       // n_dir x dim
  const double* b;
  int n_dir, n_t;
  double tau;
  double ab2;            // |a|^2 |b|^2 when equal for every direction (to rounding), else NaN
  const void* lay;       // nullable: the level's lane-layout table (layout_table), else formed in place
};

// Offsets m = 1 .. kLayoutMax cover the widest lane layout (S K / 2 = 64 x 32 / 2)
// and every offset of the largest grid.
constexpr int kLayoutMax = 1024;
static_assert(kLayoutMax >= (R1_MAX_NT - 1) / 2, "layout table shorter than the largest grid");
constexpr size_t kLayoutBytes = size_t(kLayoutMax) * (2 * sizeof(double) + 2 * sizeof(float));

// Host side: the lane-layout table of a level with n_t samples on [-tau, tau]:
// for m = 1 .. kLayoutMax the abscissa t_m = tau 2m / (n_t - 1) (NaN beyond the
// grid) and 1/m, both in FP64, then both rounded to FP32 -- the same expressions,
// evaluated in the same order, as make_layout forms in place, so either way the
// kernels see identical values.
inline void layout_table(int n_t, double tau, void* out) {
  double* t64 = static_cast<double*>(out);
  double* i64 = t64 + kLayoutMax;
  float* t32 = reinterpret_cast<float*>(i64 + kLayoutMax);
  float* i32 = t32 + kLayoutMax;
  const int c = (n_t - 1) / 2;
  for (int m = 1; m <= kLayoutMax; ++m) {
    t64[m - 1] = m <= c ? tau * double(2 * m) / double(n_t - 1) : __builtin_nan("");
    i64[m - 1] = 1.0 / double(m);
    t32[m - 1] = float(t64[m - 1]);
    i32[m - 1] = float(i64[m - 1]);
  }
}

// Model families, a compile-time parameter M of the sampling code: kFamNH is the
// neo-Hooke damage model with the double-well test energy (told apart at run
// time by Point::model), kFamSTVK the St. Venant-Kirchhoff damage model.  Each
// family gets its own kernels, so neither pays registers for the other's paths.
constexpr int kFamNH = 0;
constexpr int kFamSTVK = 2;

// Per-point constants of W (eq. 2.9 written as a function of psi0).  With
// D_n = D(beta_n):
//   psi0 <= beta_n :  W = (1 - D_n) psi0
//   psi0 >  beta_n :  W = psi0 - D_n beta_n - D_inf[(psi0 - beta_n) + D0 (e^{-psi0/D0} - e^{-beta_n/D0})]
// Both branches are  W = E1 psi0 + h(max(psi0, beta_n))  with E1 = 1 - D_n and
//   h(m) = (D_n - D_inf) m + B - C e^{-m/D0},  B = D_inf e^{-beta_n/D0}(beta_n + D0),  C = D_inf D0,
// because h(beta_n) = 0: one formula, no branch.
//
// Samples are evaluated in the scaled variable u = k psi0 with k = -1/D0 (FP64)
// or -log2(e)/D0 (FP32, whose exponential is exp2), so that e^{-m/D0} is
// exp_k(min(u, k beta_n)) with no extra multiply:
//   W = (E1/k) u + ((D_n - D_inf)/k) v + B - C exp_k(v),   v = min(u, k beta_n).
// psi0 = mu/2 (|G|^2 - d) - mu L + lambda/2 L^2 (L = ln J; FP32 takes log2, so
// its L coefficients carry ln2 factors); the polynomial part k mu/2 (|G|^2 - d)
// comes pre-scaled in the line coefficients (line_scale).  St. Venant-Kirchhoff
// psi0 is a quartic along a rank-one line, pre-scaled by k as a whole.
//
// Hull form: lower hulls (and their vertices, bridges and the minimum over
// directions) are unchanged by a positive scale and a shift, and E1/k < 0, so
// the lamination works on Ws = (W - B)/sc with sc = -E1/k:
//   Ws = -u + A2 v + C2 exp_k(v),  A2 = (D_inf - D_n)/(1 - D_n),  C2 = -C/sc,
// two FMAs after the exponential instead of three; W = sc Ws + B is formed
// once per envelope.  Every sample is taken in this form.
template <typename T>
struct Point {
  T klk, kmk;            // k lambda/2 (ln2^2), k mu (ln2)
  T ub, B;               // k beta_n; B
  T sc, A2, C2;          // hull form (above)
  double kq;             // scale of the line polynomial, applied in double (line_scale)
  double lam, mu;        // Lame parameters (St. Venant-Kirchhoff line coefficients)
  int model;
};

// Factor of the line polynomial in the sampling form: k mu/2 for the neo-Hooke
// |G|^2 part, k for the St. Venant-Kirchhoff quartic.
template <typename T, int M = kFamNH>
__device__ __forceinline__ double line_scale(const Material& m) {
  const double k = (sizeof(T) == 4 ? -1.4426950408889634 : -1.0) * (1.0 / m.D0);   // as in make_point
  if constexpr (M == kFamSTVK) return k;
  return k * 0.5 * m.mu;
}

template <typename T, int M = kFamNH>
__device__ __forceinline__ Point<T> make_point(const Material& m, double bn) {
  Point<T> q;
  const bool f32 = sizeof(T) == 4;
  const double ln2 = 0.6931471805599453094;
  // two divisions per point: 1/D0 and 1/(1 - D_n); 1/k = -D0 ln2 (FP32) or -D0
  const double iD0 = 1.0 / m.D0;
  const double k = (f32 ? -1.4426950408889634 : -1.0) * iD0;
  const double ik = f32 ? -m.D0 * ln2 : -m.D0;
  double e = r1x::exp_f64(-bn * iD0);
  double Dn = m.D_inf * (1.0 - e);
  const double i1D = 1.0 / (1.0 - Dn);
  q.kmk = T(k * (f32 ? m.mu * ln2 : m.mu));
  q.klk = T(k * (f32 ? 0.5 * m.lambda * ln2 * ln2 : 0.5 * m.lambda));
  q.ub = T(k * bn);
  q.B = T(m.D_inf * e * (bn + m.D0));
  q.sc = T(-(1.0 - Dn) * ik);
  q.A2 = T((m.D_inf - Dn) * i1D);
  q.C2 = T(m.D_inf * m.D0 * k * i1D);
  q.kq = line_scale<T, M>(m);
  q.lam = m.lambda;
  q.mu = m.mu;
  q.model = m.model;
  return q;
}

// Same, for code whose model is known at run time only.
template <typename T>
__device__ __forceinline__ Point<T> make_point_any(const Material& m, double bn) {
  return m.model == 2 ? make_point<T, kFamSTVK>(m, bn) : make_point<T, kFamNH>(m, bn);
}

// Coefficients of W along G + t a(x)b.  det is affine along rank-one lines:
// det(G + t a(x)b) = det G + t a.cof(G) b; |G + t a(x)b|^2 = |G|^2 + 2t a.Gb + t^2 |a|^2|b|^2.
// For the double-well test energy: g(t) = G11 + t a1 b1 and the quadratic rest.
// St. Venant-Kirchhoff: k psi0(t) = c0 + c1 t + c2 t^2 + c3 t^3 + c4 t^4 (J0, J1 unused).
template <typename T>
struct Line { T J0, J1, c0, c1, c2, c3, c4; };

template <int D>
__device__ __forceinline__ void cofactor(const double* G, double* cof) {
  if (D == 2) {
    cof[0] = G[3]; cof[1] = -G[2]; cof[2] = -G[1]; cof[3] = G[0];
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
        cof[i * 3 + j] = G[i1 * 3 + j1] * G[i2 * 3 + j2] - G[i1 * 3 + j2] * G[i2 * 3 + j1];
      }
  }
}

template <int D>
__device__ __forceinline__ double det_of(const double* G, const double* cof) {
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < D; ++j) s += G[j] * cof[j];
  return s;
}

// St. Venant-Kirchhoff (eq. 2.2) along G + t a(x)b, from the Green-Lagrange strain
// E(t) = E0 + t E1 + t^2 E2 with E0 = (G^T G - I)/2, E1 = sym(G^T a (x) b) and
// E2 = |a|^2 b (x) b / 2 (plane strain: the in-plane block, E33 = 0):
// psi0 = lambda/2 (tr E)^2 + mu E:E.  With e1 = a.Gb and e2 = |a|^2 |b|^2 / 2
// (= tr E1, tr E2; E1:E2 = e1 e2, E2:E2 = e2^2):
//   p0 = lambda/2 e0^2 + mu E0:E0,               e0 = tr E0
//   p1 = lambda e0 e1 + 2 mu a.G E0 b
//   p2 = lambda/2 (e1^2 + 2 e0 e2) + mu (|G^T a|^2 |b|^2 / 2 + e1^2 / 2 + |a|^2 b.E0 b)
//   p3 = (lambda + 2 mu) e1 e2,   p4 = (lambda/2 + mu) e2^2.
// Coefficients are formed in double and scaled by k.
// Per-point part of the St. Venant-Kirchhoff line coefficients: G, E0, G E0,
// tr E0 and E0:E0 (shared by every line through the point).
template <int D>
struct StvkGeom {
  double G[D * D], E0[D * D], GE0[D * D];
  double e0, ee;
};

template <int D>
__device__ __forceinline__ StvkGeom<D> make_stvk_geom(const double* G) {
  StvkGeom<D> g;
  g.e0 = 0.0;
  g.ee = 0.0;
#pragma unroll
  for (int k = 0; k < D * D; ++k) g.G[k] = G[k];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double c = 0.0;
#pragma unroll
      for (int r = 0; r < D; ++r) c += G[r * D + i] * G[r * D + j];
      g.E0[i * D + j] = 0.5 * (c - (i == j ? 1.0 : 0.0));
    }
#pragma unroll
  for (int i = 0; i < D; ++i) g.e0 += g.E0[i * D + i];
#pragma unroll
  for (int i = 0; i < D * D; ++i) g.ee += g.E0[i] * g.E0[i];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double c = 0.0;
#pragma unroll
      for (int r = 0; r < D; ++r) c += G[i * D + r] * g.E0[r * D + j];
      g.GE0[i * D + j] = c;
    }
  return g;
}

template <typename T, int D>
__device__ __forceinline__ Line<T> stvk_line_g(double lam, double mu, double k, const StvkGeom<D>& g,
                                               const double* a, const double* b) {
  double e1 = 0.0, ge0b = 0.0, beb = 0.0, gta2 = 0.0, aa = 0.0, bb = 0.0;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    double gta = 0.0, e0b = 0.0, ge = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      gta += g.G[i * D + j] * a[i];
      e0b += g.E0[j * D + i] * b[i];
      ge += g.GE0[i * D + j] * a[i];
    }
    e1 += gta * b[j];
    ge0b += ge * b[j];
    beb += b[j] * e0b;
    gta2 += gta * gta;
    aa += a[j] * a[j];
    bb += b[j] * b[j];
  }
  const double e0 = g.e0, e2 = 0.5 * aa * bb;
  Line<T> L;
  L.J0 = T(0);
  L.J1 = T(0);
  L.c0 = T(k * (0.5 * lam * e0 * e0 + mu * g.ee));
  L.c1 = T(k * (lam * e0 * e1 + 2.0 * mu * ge0b));
  L.c2 = T(k * (0.5 * lam * (e1 * e1 + 2.0 * e0 * e2) + mu * (0.5 * gta2 * bb + 0.5 * e1 * e1 + aa * beb)));
  L.c3 = T(k * ((lam + 2.0 * mu) * e1 * e2));
  L.c4 = T(k * ((0.5 * lam + mu) * e2 * e2));
  return L;
}

template <typename T, int D>
__device__ __forceinline__ Line<T> stvk_line(double lam, double mu, double k, const double* G, const double* a,
                                             const double* b) {
  return stvk_line_g<T, D>(lam, mu, k, make_stvk_geom<D>(G), a, b);
}

template <typename T, int D, int M = kFamNH>
__device__ __forceinline__ Line<T> line_setup(const Point<T>& q, const double* G, const double* cof,
                                              const double* a, const double* b) {
  if constexpr (M == kFamSTVK) return stvk_line<T, D>(q.lam, q.mu, q.kq, G, a, b);
  const int model = q.model;
  const double kq = q.kq;
  Line<T> L;
  L.c3 = T(0);
  L.c4 = T(0);
  if (model == 0) {
    double J1 = 0.0, gab = 0.0, n2 = 0.0, aa = 0.0, bb = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      aa += a[i] * a[i];
      bb += b[i] * b[i];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        J1 += a[i] * cof[i * D + j] * b[j];
        gab += a[i] * G[i * D + j] * b[j];
        n2 += G[i * D + j] * G[i * D + j];
      }
    }
    L.J0 = T(det_of<D>(G, cof));
    L.J1 = T(J1);
    L.c0 = T(kq * (n2 - double(D)));
    L.c1 = T(kq * 2.0 * gab);
    L.c2 = T(kq * aa * bb);
  } else {
    double r0 = 0.0, r1 = 0.0, r2 = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        if (i == 0 && j == 0) continue;
        double e = G[i * D + j] - (i == j ? 1.0 : 0.0);
        double r = a[i] * b[j];
        r0 += e * e; r1 += 2.0 * e * r; r2 += r * r;
      }
    L.J0 = T(G[0]); L.J1 = T(a[0] * b[0]);
    L.c0 = T(r0); L.c1 = T(r1); L.c2 = T(r2);
  }
  return L;
}

// One sample of W on a line in the hull form Ws = (W - B)/sc (see Point): 8
// VALU + 2 transcendental, 7 + 2 when the part of the line polynomial common to
// every line through the point comes per sample (base = c0 + c2 t^2), 6 + 1 for
// St. Venant-Kirchhoff (the quartic k psi0(t), then the damage part).  The
// line's c0, c1, c2 are the scaled polynomial k mu/2 |G(t)|^2 - d (see Point).
// det <= 0 gives NaN (J < 0) or NaN/+inf (J = 0): such samples lie outside the
// admissible interval and every hull comparison below treats NaN as absent.
template <typename T>
__device__ __forceinline__ T ws_sample(T t, const Line<T>& L, const Point<T>& q) {
  T J = fma(t, L.J1, L.J0);
  T u = fma(t, fma(t, L.c2, L.c1), L.c0);
  T lj = lg_t(J);
  u = fma(lj, fma(q.klk, lj, -q.kmk), u);
  T v = fmin(u, q.ub);
  return fma(q.C2, expk(v), fma(q.A2, v, -u));
}

template <typename T>
__device__ __forceinline__ T ws_sample_base(T t, T base, const Line<T>& L, const Point<T>& q) {
  T J = fma(t, L.J1, L.J0);
  T u = fma(t, L.c1, base);
  T lj = lg_t(J);
  u = fma(lj, fma(q.klk, lj, -q.kmk), u);
  T v = fmin(u, q.ub);
  return fma(q.C2, expk(v), fma(q.A2, v, -u));
}

template <typename T>
__device__ __forceinline__ T ws_sample_stvk(T t, const Line<T>& L, const Point<T>& q) {
  T u = fma(t, fma(t, fma(t, fma(t, L.c4, L.c3), L.c2), L.c1), L.c0);
  T v = fmin(u, q.ub);
  return fma(q.C2, expk(v), fma(q.A2, v, -u));
}

template <typename T>
__device__ __forceinline__ T w_sample_doublewell(T t, const Line<T>& L) {
  T g = fma(t, L.J1, L.J0);
  T g2 = fma(g, g, T(-1));
  return fma(g2, g2, fma(t, fma(t, L.c2, L.c1), L.c0));
}

// W at a point (the centre sample of every line through it), in the path's precision,
// through the hull form for the damage energies (the value the envelope returns
// where the point does not laminate).
template <typename T, int D, int M = kFamNH>
__device__ __forceinline__ T w_point(const Point<T>& q, const double* G, const double* cof) {
  double a0[3] = {0, 0, 0};
  Line<T> L = line_setup<T, D, M>(q, G, cof, a0, a0);
  if constexpr (M == kFamSTVK) return fma(ws_sample_stvk<T>(T(0), L, q), q.sc, q.B);
  return q.model == 0 ? fma(ws_sample<T>(T(0), L, q), q.sc, q.B) : w_sample_doublewell<T>(T(0), L);
}

// Same, for code whose model is known at run time only.
template <typename T, int D>
__device__ __forceinline__ T w_point_any(const Point<T>& q, const double* G, const double* cof) {
  return q.model == 2 ? w_point<T, D, kFamSTVK>(q, G, cof) : w_point<T, D, kFamNH>(q, G, cof);
}

// ---- segment reductions ------------------------------------------------------
//
// Reductions over a segment of S lanes run as butterflies.  Steps 1 and 2 use
// DPP quad permutations, steps 4 and 8 the DPP half-row / row mirrors (valid for
// idempotent reductions once the previous steps have made each quad / half-row
// uniform), steps 16 and 32 a lane shuffle.

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}

template <int STEP>
__device__ __forceinline__ int partner_i(int v) {
  if constexpr (STEP == 1) return dpp_i<0xB1>(v);          // quad_perm [1,0,3,2]
  else if constexpr (STEP == 2) return dpp_i<0x4E>(v);     // quad_perm [2,3,0,1]
  else if constexpr (STEP == 4) return dpp_i<0x141>(v);    // row_half_mirror
  else if constexpr (STEP == 8) return dpp_i<0x140>(v);    // row_mirror
  else return __shfl_xor(v, STEP, kWave);
}

template <int STEP>
__device__ __forceinline__ float partner(float v) { return __int_as_float(partner_i<STEP>(__float_as_int(v))); }
template <int STEP>
__device__ __forceinline__ int partner(int v) { return partner_i<STEP>(v); }
template <int STEP>
__device__ __forceinline__ double partner(double v) {
  long long b = __double_as_longlong(v);
  int lo = partner_i<STEP>(int(b & 0xffffffffll));
  int hi = partner_i<STEP>(int(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

template <int S, int STEP = 1, typename T>
__device__ __forceinline__ T seg_max(T v) {
  if constexpr (STEP < S) return seg_max<S, 2 * STEP>(fmax(v, partner<STEP>(v)));
  else return v;
}
template <int S, int STEP = 1, typename T>
__device__ __forceinline__ T seg_min(T v) {
  if constexpr (STEP < S) return seg_min<S, 2 * STEP>(fmin(v, partner<STEP>(v)));
  else return v;
}

// Integer reductions: the DPP move fuses into v_min_i32 / v_max_i32 (one
// instruction per butterfly step).
template <int S, int STEP = 1>
__device__ __forceinline__ int seg_min_i(int v) {
  if constexpr (STEP < S) return seg_min_i<S, 2 * STEP>(min(v, partner_i<STEP>(v)));
  else return v;
}
template <int S, int STEP = 1>
__device__ __forceinline__ int seg_max_i(int v) {
  if constexpr (STEP < S) return seg_max_i<S, 2 * STEP>(max(v, partner_i<STEP>(v)));
  else return v;
}

// Order-preserving map of non-NaN floats to int (an involution): float min/max
// across lanes run as integer min/max of the keys, which fuse with DPP, while a
// float min/max of a DPP result needs extra canonicalizing instructions.
__device__ __forceinline__ int ord_key(float x) {
  int i = __float_as_int(x);
  return i ^ ((i >> 31) & 0x7fffffff);
}
__device__ __forceinline__ float ord_val(int k) { return __int_as_float(k ^ ((k >> 31) & 0x7fffffff)); }

// Slope keys only order candidates across lanes: FP32 uses the hardware reciprocal.
__device__ __forceinline__ float key_div(float n, float d) { return n * __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double key_div(double n, double d) { return n / d; }

template <typename T>
struct Cand {      // a hull candidate: key (a slope), offset magnitude m, sample value w
  T key;
  int m;
  T w;
};

// argmax (MAX) or argmin of key over the segment; ties -> larger m (outermost sample)
template <int S, bool MAX, int STEP = 1, typename T>
__device__ __forceinline__ Cand<T> seg_arg(Cand<T> c) {
  if constexpr (STEP < S) {
    Cand<T> o = {partner<STEP>(c.key), partner<STEP>(c.m), partner<STEP>(c.w)};
    bool better = MAX ? (o.key > c.key) : (o.key < c.key);
    bool take = better || (o.key == c.key && o.m > c.m);
    c.key = take ? o.key : c.key;
    c.m = take ? o.m : c.m;
    c.w = take ? o.w : c.w;
    return seg_arg<S, MAX, 2 * STEP>(c);
  } else {
    return c;
  }
}

// Result of one line: hull value at the centre and the bracketing vertices as
// offset magnitudes (mp on the left, mq on the right; 0/0 = centre is a vertex).
template <typename T>
struct LineHull {
  T h;
  int mp, mq;
  int capped;
};

// Per-lane constants of a line layout: offsets m_h = 1 + sl + S*h and t_h = tau*2m/(n_t-1)
// of the lane's sample pairs, 1/m_h and m_h as T.
template <typename T, int S, int K>
struct Layout {
  T t[K / 2];
  T inv_m[K / 2];
  T mf[K / 2];
  int c;
};

template <typename T, int S, int K>
__device__ __forceinline__ Layout<T, S, K> make_layout(int n_t, double tau) {
  Layout<T, S, K> lay;
  int sl = threadIdx.x & (S - 1);
  lay.c = (n_t - 1) / 2;
#pragma unroll
  for (int h = 0; h < K / 2; ++h) {
    int m = 1 + sl + S * h;
    lay.mf[h] = T(m);
    lay.inv_m[h] = T(1.0 / double(m));
    // offsets beyond the grid are padding: a NaN abscissa makes the sample NaN,
    // which every hull comparison treats as absent (no per-sample select)
    lay.t[h] = m <= lay.c ? T(tau * double(2 * m) / double(n_t - 1)) : T(__builtin_nan(""));
  }
  return lay;
}

// Same, from the level's table when it has one (loads instead of two FP64
// divisions per sample pair).
template <typename T, int S, int K>
__device__ __forceinline__ Layout<T, S, K> make_layout(const Level& lv) {
  static_assert(S * K / 2 <= kLayoutMax, "lane layout wider than the table");
  if (!lv.lay) return make_layout<T, S, K>(lv.n_t, lv.tau);
  const T* tab = sizeof(T) == 8 ? static_cast<const T*>(lv.lay)
                                : reinterpret_cast<const T*>(static_cast<const double*>(lv.lay) + 2 * kLayoutMax);
  Layout<T, S, K> lay;
  const int sl = threadIdx.x & (S - 1);
  lay.c = (lv.n_t - 1) / 2;
#pragma unroll
  for (int h = 0; h < K / 2; ++h) {
    const int m = 1 + sl + S * h;
    lay.mf[h] = T(m);
    lay.t[h] = tab[m - 1];
    lay.inv_m[h] = tab[kLayoutMax + m - 1];
  }
  return lay;
}

// Segment minimum of the lanes' candidate keys e with the offset m of the
// minimizer, ties to the larger m (the outermost sample).  A lane without a
// candidate passes e = +inf and m <= 0.
template <int S>
__device__ __forceinline__ void seg_argmin_outer(float e, int m, int& m_out, float& e_out) {
  const int k = ord_key(e);
  const int kmin = seg_min_i<S>(k);
  m_out = seg_max_i<S>(k == kmin ? m : -1);
  e_out = ord_val(kmin);
}
template <int S>
__device__ __forceinline__ void seg_argmin_outer(double e, int m, int& m_out, double& e_out) {
  Cand<double> c = {e, m, 0.0};
  c = seg_arg<S, false>(c);
  m_out = c.m;
  e_out = c.key;
}

// Slope pass budget of the bridge search before it hands over to the
// alternating tangent search (which always terminates).
constexpr int kSlopePasses = 12;

// Alternating tangent search for the bridge over the centre: p starts as the
// tangent point on the left seen from the centre; then q = tangent point on
// the right seen from p, p = tangent point on the left seen from q, until p
// repeats.  Segments with todo unset are left alone.  Every lane of the wave
// must call it.
template <typename T, int S, int K>
__device__ __forceinline__ void bridge_alternating(const T (&w)[K], const T (&wci)[K / 2],
                                                   const Layout<T, S, K>& lay, bool todo,
                                                   int& p_m, T& p_w, int& q_m, T& q_w, int& capped) {
  constexpr int H = K / 2;
  Cand<T> p = {-inf_v<T>(), 0, T(0)};
#pragma unroll
  for (int h = 0; h < H; ++h) {
    T key = fma(-w[h], lay.inv_m[h], wci[h]);
    bool take = key >= p.key;
    p.key = take ? key : p.key;
    p.m = take ? int(lay.mf[h]) : p.m;
    p.w = take ? w[h] : p.w;
  }
  p = seg_arg<S, true>(p);
  Cand<T> q = {inf_v<T>(), 0, T(0)};
  int it = 0;
  while (__any(todo)) {
    // q: argmin over right samples of (w_j - w_p)/(m_j + m_p)  (cross-multiplied)
    T nb = inf_v<T>(), db = T(1), wb = T(0), mb = T(0);
    const T mpf = T(p.m);
#pragma unroll
    for (int h = 0; h < H; ++h) {
      T num = w[H + h] - p.w;
      T den = lay.mf[h] + mpf;
      bool take = num * db <= nb * den;
      nb = take ? num : nb; db = take ? den : db; mb = take ? lay.mf[h] : mb; wb = take ? w[H + h] : wb;
    }
    Cand<T> qc = {key_div(nb, db), int(mb), wb};
    qc = seg_arg<S, false>(qc);
    // p': argmax over left samples of (w_q - w_i)/(m_q + m_i)
    const T qmf = T(qc.m);
    nb = -inf_v<T>(); db = T(1); mb = T(0); wb = T(0);
#pragma unroll
    for (int h = 0; h < H; ++h) {
      T num = qc.w - w[h];
      T den = qmf + lay.mf[h];
      bool take = num * db >= nb * den;
      nb = take ? num : nb; db = take ? den : db; mb = take ? lay.mf[h] : mb; wb = take ? w[h] : wb;
    }
    Cand<T> pc = {key_div(nb, db), int(mb), wb};
    pc = seg_arg<S, true>(pc);
    if (todo) {
      q = qc;
      if (pc.m == p.m) {
        todo = false;
        p_m = p.m; p_w = p.w; q_m = q.m; q_w = q.w;
      } else {
        p = pc;
      }
    }
    if (++it >= kBridgeCap) {
      if (todo) {
        capped = 1;
        p_m = p.m; p_w = p.w; q_m = q.m; q_w = q.w;
      }
      break;
    }
  }
}

// Slope iteration for the bridge over the centre (see hull_centre) on the
// segments with todo set, from slope s: on return those that converged have
// todo cleared, the pair (mp, mq), the tilted minima (ep, eq) and the slope s
// of the last pass.  A pass at any slope bounds the hull value at the centre
// from below by min(ep, eq, wc) (the line of that slope through the lowest
// tilted sample lies under every sample); a segment whose bound exceeds thr
// stops there too, with the pair and tilted minima of that pass, whose chord
// value at the centre is then an upper bound.  Every lane of the wave must call
// it.
template <typename T, int S, int K>
__device__ __forceinline__ void slope_bridge(const T (&w)[K], const Layout<T, S, K>& lay, bool& todo,
                                             T& s, int& mp, int& mq, T& ep, T& eq, T wc, T thr) {
  constexpr int H = K / 2;
  const int sl = threadIdx.x & (S - 1);
  for (int pass = 0; pass < kSlopePasses && __any(todo); ++pass) {
    T eL = inf_v<T>(), eR = inf_v<T>();
    int hL = -1, hR = -1;
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const T e = fma(s, lay.mf[h], w[h]);           // left sample at -m
      const bool tl = e <= eL;
      eL = tl ? e : eL; hL = tl ? h : hL;
      const T f = fma(-s, lay.mf[h], w[H + h]);      // right sample at +m
      const bool tr = f <= eR;
      eR = tr ? f : eR; hR = tr ? h : hR;
    }
    int mpn, mqn;
    T epn, eqn;
    seg_argmin_outer<S>(eL, 1 + sl + S * hL, mpn, epn);
    seg_argmin_outer<S>(eR, 1 + sl + S * hR, mqn, eqn);
    if (todo) {
      if (pass > 0 && mpn == mp && mqn == mq) {
        todo = false;
        ep = epn; eq = eqn;
      } else if (fmin(fmin(epn, eqn), wc) > thr) {
        todo = false;
        mp = mpn; mq = mqn;
        ep = epn; eq = eqn;
      } else {
        mp = mpn; mq = mqn;
        s = s + key_div(eqn - epn, T(mq + mp));
      }
    }
  }
}

// Hull of the segment's line at its centre.  w: this lane's samples (layout
// above; NaN = absent); wc: centre sample; wci[h] = wc / m_h.  sig: on entry a
// slope to start the bridge search from (NaN: none), on exit the bridge slope
// (NaN when the centre is a vertex).  Every lane of the wave must call this
// together (cross-lane operations).
//
// Vertex test: the centre is a strict hull vertex iff the steepest slope from
// a left sample up to the centre is below the shallowest slope from the centre
// to a right sample.  Otherwise the hull over the centre is the bridge (lower
// common tangent) of the two sides, found by slope iteration: at slope s the
// lowest left and right samples under the tilt, p = argmin w + s m and
// q = argmin w - s m (ties to the outermost sample), are the points where lines
// of slope s support the two sides; s <- slope(p, q) until (p, q) repeats, when
// every sample lies on or above the line through p and q.  The tilted minima
// e_p = w_p + s m_p and e_q = w_q - s m_q give both the next slope,
// s + (e_q - e_p)/(m_p + m_q), and the hull value at the centre,
// (m_q e_p + m_p e_q)/(m_p + m_q), in which the rounding of s cancels.  The
// bridge slope is bracketed by the two vertex-test slopes, which give the cold
// start; a warm start (the previous point's slope on a nearby line) usually
// needs two passes.
//
// thr: a line whose hull value at the centre is shown to exceed it may return
// an upper bound above thr instead (see slope_bridge); +inf: exact for every
// line.
//
// hot (wave-uniform): every line of the wave has a warm start.  The vertex
// test is then skipped: the centre is a vertex exactly when the bridge of the
// other samples passes above it.  If any line of the wave ends without a
// bridge (no sample on one side, or no convergence), the wave takes the
// standard path instead.
template <typename T, int S, int K>
__device__ __forceinline__ LineHull<T> hull_centre(const T (&w)[K], T wc, const T (&wci)[K / 2],
                                                   const Layout<T, S, K>& lay, T& sig, bool hot,
                                                   T thr = inf_v<T>()) {
  constexpr int H = K / 2;
  LineHull<T> r;
  r.h = wc; r.mp = 0; r.mq = 0; r.capped = 0;
  const T nan = T(__builtin_nan(""));
  if (hot) {
    bool todo = true;
    T s = sig;
    int mp = 0, mq = 0;
    T ep = T(0), eq = T(0);
    slope_bridge<T, S, K>(w, lay, todo, s, mp, mq, ep, eq, wc, thr);
    if (!__any(todo || !(mp >= 1 && mq >= 1))) {
      const T mpf = T(mp), mqf = T(mq);
      const T hb = (mqf * ep + mpf * eq) / (mqf + mpf);
      if (hb <= wc) {
        r.h = hb; r.mp = mp; r.mq = mq;
        sig = s;
      } else {
        sig = nan;
      }
      return r;
    }
  }
  T maxL = -inf_v<T>(), minR = inf_v<T>();
#pragma unroll
  for (int h = 0; h < H; ++h) {
    maxL = fmax(maxL, fma(-w[h], lay.inv_m[h], wci[h]));
    minR = fmin(minR, fma(w[H + h], lay.inv_m[h], -wci[h]));
  }
  bool todo;
  if constexpr (sizeof(T) == 4) {
    const int kl = seg_max_i<S>(ord_key(maxL));
    const int kr = seg_min_i<S>(ord_key(minR));
    todo = kl >= kr;
    maxL = ord_val(kl);
    minR = ord_val(kr);
  } else {
    maxL = seg_max<S>(maxL);
    minR = seg_min<S>(minR);
    todo = maxL >= minR;
  }
  if (!__any(todo)) {
    sig = nan;
    return r;
  }
  const bool bridged = todo;
  T s = sig == sig ? fmin(fmax(sig, minR), maxL) : T(0.5) * (maxL + minR);
  int mp = 0, mq = 0;
  T ep = T(0), eq = T(0);
  slope_bridge<T, S, K>(w, lay, todo, s, mp, mq, ep, eq, wc, thr);
  if (__any(todo)) {
    // slope budget spent (not seen in practice): finish with the alternating search
    T wp = T(0), wq = T(0);
    bridge_alternating<T, S, K>(w, wci, lay, todo, mp, wp, mq, wq, r.capped);
    if (todo) {       // express its result in the tilted form used below
      s = key_div(wq - wp, T(mq + mp));
      ep = fma(s, T(mp), wp);
      eq = fma(-s, T(mq), wq);
    }
  }
  if (bridged) {
    const T mpf = T(mp), mqf = T(mq);
    r.h = (mqf * ep + mpf * eq) / (mqf + mpf);
    r.mp = mp;
    r.mq = mq;
    sig = s;
  } else {
    sig = nan;
  }
  return r;
}

// Geometry of a point shared by all lines through it.
template <int D>
struct PointGeom {
  double G[D * D];
  double cof[D * D];
  double det, n2;
};

template <int D>
__device__ __forceinline__ PointGeom<D> make_geom(const double* G) {
  PointGeom<D> g;
#pragma unroll
  for (int k = 0; k < D * D; ++k) g.G[k] = G[k];
  cofactor<D>(G, g.cof);
  g.det = det_of<D>(G, g.cof);
  double n2 = 0.0;
#pragma unroll
  for (int k = 0; k < D * D; ++k) n2 += G[k] * G[k];
  g.n2 = n2;
  return g;
}

// Geometry of a point by model family.
template <int D, int M>
struct GeomOf { using type = PointGeom<D>; };
template <int D>
struct GeomOf<D, kFamSTVK> { using type = StvkGeom<D>; };

template <int D, int M>
__device__ __forceinline__ typename GeomOf<D, M>::type make_geom_m(const double* G) {
  if constexpr (M == kFamSTVK)
    return make_stvk_geom<D>(G);
  else
    return make_geom<D>(G);
}

template <typename T, int D, int M = kFamNH>
__device__ __forceinline__ Line<T> line_of(const Point<T>& q, const typename GeomOf<D, M>::type& g,
                                           const double* a, const double* b) {
  if constexpr (M == kFamSTVK) {
    return stvk_line_g<T, D>(q.lam, q.mu, q.kq, g, a, b);
  } else {
    if (q.model != 0) return line_setup<T, D, M>(q, g.G, g.cof, a, b);
    const double kq = q.kq;
    Line<T> L;
    L.c3 = T(0);
    L.c4 = T(0);
    double J1 = 0.0, gab = 0.0, aa = 0.0, bb = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      aa += a[i] * a[i];
      bb += b[i] * b[i];
      double ca = 0.0, ga = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        ca += g.cof[i * D + j] * b[j];
        ga += g.G[i * D + j] * b[j];
      }
      J1 += a[i] * ca;
      gab += a[i] * ga;
    }
    L.J0 = T(g.det);
    L.J1 = T(J1);
    L.c0 = T(kq * (g.n2 - double(D)));
    L.c1 = T(kq * 2.0 * gab);
    L.c2 = T(kq * aa * bb);
    return L;
  }
}

template <typename T>
struct Env {            // W^1 at a point: value, direction, bracketing offsets
  T h;
  int dir, mp, mq;
  int capped;
  T second;             // runner-up over directions (the smallest value of another direction)
};

// A point's laminate is ambiguous when its winning direction laminates and
// another direction's value is within the tie margin: 1e-10 (FP64) or 1e-5
// (FP32) of max(|W|, 1e-3 / 1e-2).
template <typename T>
__device__ __forceinline__ T tie_margin() { return sizeof(T) == 4 ? T(1e-5) : T(1e-10); }
template <typename T>
__device__ __forceinline__ T tie_floor() { return sizeof(T) == 4 ? T(1e-2) : T(1e-3); }
template <typename T>
__device__ __forceinline__ bool near_tie(const Env<T>& e) {
  return (e.mp + e.mq) > 0 && e.second - e.h <= tie_margin<T>() * fmax(fabs(e.h), tie_floor<T>());
}

// One lamination level at a point (wave-uniform): min over the level's n_dir
// directions of the line hulls at the centre.  wc = W at the point;
// line_fn(dir) returns the coefficients of W along direction dir.  warm
// (optional, 2 n_dir entries owned by this wave) carries each direction's
// bridge slope at the last call (warm[dir]) and at the call before
// (warm[n_dir + dir]) to the next, whose bridge search starts from their linear
// extrapolation (from the last slope alone when the one before is absent): NaN
// for none; callers whose successive points are close and evenly spaced pass
// it.  c2u: when every
// line has the same c2 (and, being lines through one point, the same c0), that
// c2; the polynomial part c0 + c2 t^2 is then formed once per point (NaN: not
// uniform).  order (optional with warm, n_dir entries owned by this wave): the
// directions are visited with those that had a bridge last time first, so that
// lines needing a bridge search share wavefronts; ties in the minimum go to the
// smaller direction index whatever the visiting order.  centre (optional): the
// coefficients of the lines at t = 0 (J0, c0; the rest unused), when the caller
// has them at hand; else line_fn(0) is taken.  Every lane of the wave must call
// it.
template <typename T, int S, int K, int M = kFamNH, typename LineFn>
__device__ Env<T> envelope_lines(const Point<T>& q, T wc, int n_dir, const Layout<T, S, K>& lay,
                                 LineFn line_fn, T* warm = nullptr, T c2u = T(__builtin_nan("")),
                                 int* order = nullptr, const Line<T>* centre = nullptr) {
  constexpr int NSEG = kWave / S;
  constexpr int H = K / 2;
  const int lane = threadIdx.x & (kWave - 1);
  const int seg = lane / S;
  // the damage energies are hulled in the hull form Ws (see Point); every line
  // through the point has the same J0 and c0, so its centre is any line's t = 0
  const bool scaled = M == kFamSTVK || q.model == 0;
  const bool shared = M == kFamNH && q.model == 0 && c2u == c2u;
  T wcs = wc;
  T base[H];
  if (scaled) {
    const Line<T> L0 = centre ? *centre : line_fn(0);
    if constexpr (M == kFamSTVK) {
      wcs = ws_sample_stvk<T>(T(0), L0, q);
    } else {
      wcs = ws_sample<T>(T(0), L0, q);
      if (shared) {
#pragma unroll
        for (int h = 0; h < H; ++h) base[h] = fma(c2u, lay.t[h] * lay.t[h], L0.c0);
      }
    }
  }
  T wci[H];
#pragma unroll
  for (int h = 0; h < H; ++h) wci[h] = wcs * lay.inv_m[h];
  const T isc = scaled ? T(1) / q.sc : T(1);
  if (order) {
    // stable partition of the directions: warm (bridged last time) first
    int n_warm = 0;
    for (int c0 = 0; c0 < n_dir; c0 += kWave)
      n_warm += __popcll(__ballot(c0 + lane < n_dir && warm[c0 + lane] == warm[c0 + lane]));
    int seen_warm = 0, seen_cold = 0;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int c0 = 0; c0 < n_dir; c0 += kWave) {
      const int i = c0 + lane;
      const bool valid = i < n_dir;
      const bool hot = valid && warm[i] == warm[i];
      const unsigned long long mh = __ballot(hot), mc = __ballot(valid && !hot);
      if (valid)
        order[hot ? seen_warm + __popcll(mh & below) : n_warm + seen_cold + __popcll(mc & below)] = i;
      seen_warm += __popcll(mh);
      seen_cold += __popcll(mc);
    }
  }
  Env<T> best = {inf_v<T>(), 0, 0, 0, 0, inf_v<T>()};
  for (int m0 = 0; m0 < n_dir; m0 += NSEG) {
    const bool act = m0 + seg < n_dir;
    const int dir = order ? order[act ? m0 + seg : n_dir - 1] : (act ? m0 + seg : n_dir - 1);
    Line<T> L = line_fn(dir);
    T w[K];
    if constexpr (M == kFamSTVK) {
#pragma unroll
      for (int h = 0; h < H; ++h) {
        w[h] = ws_sample_stvk<T>(-lay.t[h], L, q);
        w[H + h] = ws_sample_stvk<T>(lay.t[h], L, q);
      }
    } else if (shared) {
#pragma unroll
      for (int h = 0; h < H; ++h) {
        w[h] = ws_sample_base<T>(-lay.t[h], base[h], L, q);
        w[H + h] = ws_sample_base<T>(lay.t[h], base[h], L, q);
      }
    } else if (q.model == 0) {
#pragma unroll
      for (int h = 0; h < H; ++h) {
        w[h] = ws_sample<T>(-lay.t[h], L, q);
        w[H + h] = ws_sample<T>(lay.t[h], L, q);
      }
    } else {
#pragma unroll
      for (int h = 0; h < H; ++h) {
        w[h] = w_sample_doublewell<T>(-lay.t[h], L);
        w[H + h] = w_sample_doublewell<T>(lay.t[h], L);
      }
    }
    // lines that cannot come within twice the tie margin of the wave's best so
    // far may stop their bridge search early: the minimum is unchanged and so
    // is the tie flag (their value only enters the runner-up, beyond the
    // margin).  Only for cold searches: warm-started lines come first in their
    // visiting order and rarely meet a lower value already found.
    T thr = inf_v<T>();
    if (!warm) {
      T bw = best.h;
#pragma unroll
      for (int off = S; off < kWave; off <<= 1) bw = fmin(bw, __shfl_xor(bw, off, kWave));
      if (bw < inf_v<T>()) {
        const T bW = scaled ? fma(bw, q.sc, q.B) : bw;
        const T mW = T(2) * tie_margin<T>() * fmax(fabs(bW), tie_floor<T>());
        thr = bw + (scaled ? mW * isc : mW);
      }
    }
    T sg = T(__builtin_nan("")), s1 = sg;
    if (warm && act) {
      s1 = warm[dir];
      const T s2 = warm[n_dir + dir];
      // start from the slope extrapolated linearly from the last two points
      sg = s2 == s2 ? fma(T(2), s1, -s2) : s1;
    }
    const bool hot = warm && __all(act && s1 == s1);
    LineHull<T> lh = hull_centre<T, S, K>(w, wcs, wci, lay, sg, hot, thr);
    if (warm && act && (lane & (S - 1)) == 0) {
      warm[n_dir + dir] = sg == sg ? s1 : sg;
      warm[dir] = sg;
    }
    if (act) {
      if (lh.h < best.h || (lh.h == best.h && dir < best.dir)) {
        best.second = best.h;
        best.h = lh.h; best.dir = dir; best.mp = lh.mp; best.mq = lh.mq;
      } else {
        best.second = fmin(best.second, lh.h);
      }
    }
    best.capped |= lh.capped;
  }
  // across segments: lexicographic (value, direction)
#pragma unroll
  for (int off = S; off < kWave; off <<= 1) {
    T oh = __shfl_xor(best.h, off, kWave);
    int od = __shfl_xor(best.dir, off, kWave);
    int op = __shfl_xor(best.mp, off, kWave);
    int oq = __shfl_xor(best.mq, off, kWave);
    int oc = __shfl_xor(best.capped, off, kWave);
    T os = __shfl_xor(best.second, off, kWave);
    bool take = oh < best.h || (oh == best.h && od < best.dir);
    best.second = take ? fmin(os, best.h) : fmin(best.second, oh);
    best.h = take ? oh : best.h;
    best.dir = take ? od : best.dir;
    best.mp = take ? op : best.mp;
    best.mq = take ? oq : best.mq;
    best.capped |= oc;
  }
  if (scaled) {   // back from the hull form; a centre that is a vertex is W there, exactly
    best.h = (best.mp + best.mq) ? fma(best.h, q.sc, q.B) : wc;
    best.second = fma(best.second, q.sc, q.B);
  }
  return best;
}

// One lamination level at a point with the lines set up from its geometry g
// (make_geom_m).
template <typename T, int D, int S, int K, int M = kFamNH>
__device__ Env<T> envelope_geom(const Point<T>& q, const typename GeomOf<D, M>::type& g, T wc, const Level& lv,
                                const Layout<T, S, K>& lay) {
  // neo-Hooke: every line through G starts at J0 = det G, c0 = kq (|G|^2 - d) (line_of)
  Line<T> c{};
  if constexpr (M != kFamSTVK) {
    c.J0 = T(g.det);
    c.c0 = T(q.kq * (g.n2 - double(D)));
  }
  return envelope_lines<T, S, K, M>(q, wc, lv.n_dir, lay, [&](int dd) {
    double a[D], b[D];
#pragma unroll
    for (int i = 0; i < D; ++i) { a[i] = lv.a[dd * D + i]; b[i] = lv.b[dd * D + i]; }
    return line_of<T, D, M>(q, g, a, b);
  }, nullptr, T(q.kq * lv.ab2), nullptr, (M != kFamSTVK && q.model == 0) ? &c : nullptr);
}

// The same at point G.
template <typename T, int D, int S, int K, int M = kFamNH>
__device__ Env<T> envelope_at(const Point<T>& q, const double* G, T wc, const Level& lv,
                              const Layout<T, S, K>& lay) {
  return envelope_geom<T, D, S, K, M>(q, make_geom_m<D, M>(G), wc, lv, lay);
}

// Lines of an inner level along an outer line G(t_o) = F + t_o R_o, R_o rank one.
// det and |.|^2 are affine / quadratic in t_o, and cof(F + t_o R_o) = cof F + t_o C1
// because cof(R_o) = 0, so every inner coefficient is affine in t_o:
//   J1_i = al_i + t_o be_i,  c1_i = ga_i + t_o de_i,  c2_i = |a_i|^2 |b_i|^2.
// coef[5*i .. 5*i+4] = (al, be, ga, de, c2) of inner direction i, the last three
// times kq (the sampling form of the neo-Hooke polynomial, see Point).
template <int D>
__device__ __forceinline__ void cof_derivative(const double* F, const double* R, double* C1) {
  if (D == 2) {
    C1[0] = R[3]; C1[1] = -R[2]; C1[2] = -R[1]; C1[3] = R[0];
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
        C1[i * 3 + j] = R[i1 * 3 + j1] * F[i2 * 3 + j2] + F[i1 * 3 + j1] * R[i2 * 3 + j2]
                      - R[i1 * 3 + j2] * F[i2 * 3 + j1] - F[i1 * 3 + j2] * R[i2 * 3 + j1];
      }
  }
}

template <typename T, int D>
__device__ __forceinline__ void inner_line_coef(int model, double kq, const double* F, const double* cofF,
                                                const double* R, const double* C1, const double* a,
                                                const double* b, T* coef) {
  double al = 0, be = 0, ga = 0, de = 0, aa = 0, bb = 0;
  if (model == 0) {
#pragma unroll
    for (int i = 0; i < D; ++i) {
      aa += a[i] * a[i];
      bb += b[i] * b[i];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        al += a[i] * cofF[i * D + j] * b[j];
        be += a[i] * C1[i * D + j] * b[j];
        ga += 2.0 * a[i] * F[i * D + j] * b[j];
        de += 2.0 * a[i] * R[i * D + j] * b[j];
      }
    }
    coef[0] = T(al); coef[1] = T(be); coef[2] = T(kq * ga); coef[3] = T(kq * de); coef[4] = T(kq * aa * bb);
  } else {
    // double-well test energy: g = G11 + t a1 b1, rest = sum_{(i,j)!=(1,1)} (G_ij - delta_ij + t a_i b_j)^2
    double r2 = 0, e1 = 0, e1r = 0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        if (i == 0 && j == 0) continue;
        double r = a[i] * b[j];
        r2 += r * r;
        e1 += 2.0 * (F[i * D + j] - (i == j ? 1.0 : 0.0)) * r;
        e1r += 2.0 * R[i * D + j] * r;
      }
    coef[0] = T(a[0] * b[0]); coef[1] = T(0); coef[2] = T(e1); coef[3] = T(e1r); coef[4] = T(r2);
  }
}

// St. Venant-Kirchhoff: psi0 = lambda/2 (tr E)^2 + mu E:E with E = (G^T G - I)/2
// (eq. 2.2; plane strain: in-plane block, E33 = 0), dpsi0/dG = G (lambda tr E I + 2 mu E).
template <int D>
__device__ __forceinline__ double stvk_strain(const double* G, double* E) {
  double tr = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double c = 0.0;
#pragma unroll
      for (int r = 0; r < D; ++r) c += G[r * D + i] * G[r * D + j];
      E[i * D + j] = 0.5 * (c - (i == j ? 1.0 : 0.0));
    }
#pragma unroll
  for (int i = 0; i < D; ++i) tr += E[i * D + i];
  return tr;
}

template <int D>
__device__ __forceinline__ double stvk_psi_stress(const Material& m, const double* G, double* S) {
  double E[D * D];
  double tr = stvk_strain<D>(G, E), ee = 0.0;
#pragma unroll
  for (int i = 0; i < D * D; ++i) ee += E[i] * E[i];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double ge = 0.0;
#pragma unroll
      for (int r = 0; r < D; ++r) ge += G[i * D + r] * E[r * D + j];
      S[i * D + j] = m.lambda * tr * G[i * D + j] + 2.0 * m.mu * ge;
    }
  return 0.5 * m.lambda * tr * tr + m.mu * ee;
}

// P0 = dW/dF = (1 - D(max(beta_n, psi0))) (mu G + (lambda ln J - mu) G^{-T}) in double
// (eq. 2.12) for neo-Hooke, (1 - D(max(beta_n, psi0))) dpsi0/dG for St. Venant-Kirchhoff;
// the double-well test energy has its own gradient.
template <int D, int M = kFamNH>
__device__ __forceinline__ void stress0(const Material& m, double bn, const double* G, double* P) {
  if constexpr (M == kFamSTVK) {
    double S[D * D];
    double psi = stvk_psi_stress<D>(m, G, S);
    double g = 1.0 - m.D_inf * (1.0 - exp(-(psi > bn ? psi : bn) / m.D0));
#pragma unroll
    for (int i = 0; i < D * D; ++i) P[i] = g * S[i];
    return;
  }
  if (m.model != 0) {
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        double e = G[i * D + j] - (i == j ? 1.0 : 0.0);
        P[i * D + j] = (i == 0 && j == 0) ? 4.0 * G[0] * (G[0] * G[0] - 1.0) : 2.0 * e;
      }
    return;
  }
  double cof[D * D];
  cofactor<D>(G, cof);
  double J = det_of<D>(G, cof);
  if (!(J > 0.0)) {
#pragma unroll
    for (int i = 0; i < D * D; ++i) P[i] = __builtin_nan("");
    return;
  }
  double lnJ = log(J), n2 = 0.0;
#pragma unroll
  for (int i = 0; i < D * D; ++i) n2 += G[i] * G[i];
  double psi = 0.5 * m.mu * (n2 - double(D)) - m.mu * lnJ + 0.5 * m.lambda * lnJ * lnJ;
  double beta = psi > bn ? psi : bn;
  double g = 1.0 - m.D_inf * (1.0 - exp(-beta / m.D0));
  double f = (m.lambda * lnJ - m.mu) / J;
#pragma unroll
  for (int i = 0; i < D * D; ++i) P[i] = g * (m.mu * G[i] + f * cof[i]);
}

// stress0 for code whose model is known at run time only.
template <int D>
__device__ __forceinline__ void stress0_any(const Material& m, double bn, const double* G, double* P) {
  if (m.model == 2)
    stress0<D, kFamSTVK>(m, bn, G, P);
  else
    stress0<D, kFamNH>(m, bn, G, P);
}

// Laminate endpoint stress in the path's precision.  FP64: stress0.  FP32: the
// same first Piola-Kirchhoff stress, with cof G, det G and |G|^2 still formed in
// FP64 but ln J and the damage exponential taken, as for the samples, from the
// FP32 log2 / exp2 in the point's scaled constants (k psi0 as in ws_sample, then
// e^{-beta/D0} = exp_k(min(k psi0, k beta_n))) and 1/J from the FP32 reciprocal.
template <typename T, int D, int M>
__device__ __forceinline__ void stress_at(const Point<T>& q, const Material& m, double bn, const double* G,
                                          double* P) {
  if constexpr (sizeof(T) == 8) {
    stress0<D, M>(m, bn, G, P);
  } else if constexpr (M == kFamSTVK) {
    double S[D * D];
    const double psi = stvk_psi_stress<D>(m, G, S);
    const float g = float(1.0 - m.D_inf) + float(m.D_inf) * expk(fminf(float(q.kq * psi), q.ub));
#pragma unroll
    for (int i = 0; i < D * D; ++i) P[i] = double(g) * S[i];
  } else {
    if (m.model != 0) {               // double-well test energy: a polynomial
      stress0<D, M>(m, bn, G, P);
      return;
    }
    double cof[D * D];
    cofactor<D>(G, cof);
    const double J = det_of<D>(G, cof);
    if (!(J > 0.0)) {
#pragma unroll
      for (int i = 0; i < D * D; ++i) P[i] = __builtin_nan("");
      return;
    }
    double n2 = 0.0;
#pragma unroll
    for (int i = 0; i < D * D; ++i) n2 += G[i] * G[i];
    const float lj = lg_t(float(J));                    // log2 J
    const float u = fmaf(lj, fmaf(q.klk, lj, -q.kmk), float(q.kq * (n2 - double(D))));
    const float g = float(1.0 - m.D_inf) + float(m.D_inf) * expk(fminf(u, q.ub));
    const float f = (float(m.lambda) * (lj * 0.693147180559945309f) - float(m.mu)) *
                    __builtin_amdgcn_rcpf(float(J));
#pragma unroll
    for (int i = 0; i < D * D; ++i) P[i] = double(g * fmaf(float(m.mu), float(G[i]), f * float(cof[i])));
  }
}

// The per-point factors of the leaf moduli, formed once and shared by its rows.
template <int D>
struct Leaf0 {
  int kind;          // 0 neo-Hooke, 1 double-well, 2 St. Venant-Kirchhoff, -1 det G <= 0 (NaN)
  double g1, g2;     // damage factors g', g''
  double c, iJ, tr;  // neo-Hooke: lambda ln J - mu, 1/J; St. Venant-Kirchhoff: tr E
  double X[D * D];   // neo-Hooke: cof G (H = cof G / J); St. Venant-Kirchhoff: E
  double S[D * D];   // d psi0 / dG
};

template <int D>
__device__ __forceinline__ Leaf0<D> leaf0(const Material& m, double bn, const double* G) {
  Leaf0<D> f;
  f.kind = m.model == 2 ? 2 : (m.model != 0 ? 1 : 0);
  f.g1 = f.g2 = f.c = f.iJ = f.tr = 0.0;
  if (f.kind == 1) return f;
  double psi;
  if (f.kind == 2) {
    f.tr = stvk_strain<D>(G, f.X);
    psi = stvk_psi_stress<D>(m, G, f.S);
  } else {
    cofactor<D>(G, f.X);
    const double J = det_of<D>(G, f.X);
    if (!(J > 0.0)) {
      f.kind = -1;
      return f;
    }
    const double lnJ = log(J);
    double n2 = 0.0;
#pragma unroll
    for (int r = 0; r < D * D; ++r) n2 += G[r] * G[r];
    psi = 0.5 * m.mu * (n2 - double(D)) - m.mu * lnJ + 0.5 * m.lambda * lnJ * lnJ;
    f.c = m.lambda * lnJ - m.mu;
    f.iJ = 1.0 / J;
#pragma unroll
    for (int r = 0; r < D * D; ++r) f.S[r] = m.mu * G[r] + f.c * (f.X[r] * f.iJ);
  }
  // on the loading branch max(psi, beta_n) = psi: one exponential serves both factors
  const double e = exp(-(psi > bn ? psi : bn) / m.D0);
  f.g1 = 1.0 - m.D_inf * (1.0 - e);
  f.g2 = psi > bn ? -m.D_inf / m.D0 * e : 0.0;
  return f;
}

// Row ij of d^2 W / dG dG (the leaf moduli of Algorithm 3) at one point G, weighted and added:
// acc[kl] += w d^2 W / dG_ij dG_kl (ij = i*D + j, kl = k*D + l), from the point's
// factors f = leaf0(G).
// Neo-Hooke damage (eqs. 2.3, 2.9):
//   A0 = g' [mu d_ik d_jl + lambda H_ij H_kl - (lambda ln J - mu) H_il H_kj] + g'' S_ij S_kl
// with H = G^{-T}, S = d psi0 / dG = mu G + (lambda ln J - mu) H, g' = 1 - D(max(psi0, beta_n))
// and g'' = -(D_inf / D0) e^{-psi0/D0} on the loading branch psi0 > beta_n, 0 otherwise.
// In 2D (plane strain) G is the in-plane block; G^{-T} of the embedding keeps
// that block as the 2x2 inverse-transpose.  NaN where det G <= 0.
// St. Venant-Kirchhoff (eq. 2.2), with E = (G^T G - I)/2, B = G G^T and
// S = dpsi0/dG = G (lambda tr E I + 2 mu E):
//   d^2psi0/dG_ij dG_kl = lambda G_ij G_kl + lambda tr E d_ik d_jl + 2 mu d_ik E_lj
//                         + mu (G_il G_kj + B_ik d_jl),
// with the same damage factors g', g''.  Double-well test energy: 2 on the
// diagonal, 12 G_11^2 - 4 at (11, 11).
template <int D, int IJ>
__device__ __forceinline__ void leaf0_row(const Leaf0<D>& f, const Material& m, const double* G, double w,
                                          double* acc) {
  constexpr int ij = IJ, i = IJ / D, j = IJ % D;
  if (f.kind == 2) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      double Bik = 0.0;
#pragma unroll
      for (int r = 0; r < D; ++r) Bik += G[i * D + r] * G[k * D + r];
#pragma unroll
      for (int l = 0; l < D; ++l) {
        const int kl = k * D + l;
        double h = m.lambda * G[ij] * G[kl] + m.mu * G[i * D + l] * G[k * D + j];
        if (i == k) h += (j == l ? m.lambda * f.tr : 0.0) + 2.0 * m.mu * f.X[l * D + j];
        if (j == l) h += m.mu * Bik;
        acc[kl] += w * (f.g1 * h + f.g2 * f.S[ij] * f.S[kl]);
      }
    }
    return;
  }
  if (f.kind == 1) {
#pragma unroll
    for (int kl = 0; kl < D * D; ++kl)
      acc[kl] += w * (kl != ij ? 0.0 : ij == 0 ? 12.0 * G[0] * G[0] - 4.0 : 2.0);
    return;
  }
  if (f.kind < 0) {
#pragma unroll
    for (int kl = 0; kl < D * D; ++kl) acc[kl] = __builtin_nan("");
    return;
  }
  const double Hij = f.X[ij] * f.iJ;
#pragma unroll
  for (int k = 0; k < D; ++k)
#pragma unroll
    for (int l = 0; l < D; ++l) {
      const int kl = k * D + l;
      const double Hkl = f.X[kl] * f.iJ, Hil = f.X[i * D + l] * f.iJ, Hkj = f.X[k * D + j] * f.iJ;
      const double h = (ij == kl ? m.mu : 0.0) + m.lambda * Hij * Hkl - f.c * Hil * Hkj;
      acc[kl] += w * (f.g1 * h + f.g2 * f.S[ij] * f.S[kl]);
    }
}

// Rows IJ .. END - 1 of the same, row r added to acc + (r - IJ0)*D*D (IJ0 = the
// first row of the range).
template <int D, int IJ = 0, int END = D * D, int IJ0 = IJ>
__device__ __forceinline__ void leaf0_rows(const Leaf0<D>& f, const Material& m, const double* G, double w,
                                           double* acc) {
  if constexpr (IJ < END) {
    leaf0_row<D, IJ>(f, m, G, w, acc + (IJ - IJ0) * D * D);
    leaf0_rows<D, IJ + 1, END, IJ0>(f, m, G, w, acc);
  }
}

// One row at G with the point's factors formed for it alone.
template <int D, int IJ>
__device__ __forceinline__ void tangent0_row(const Material& m, double bn, const double* G, double w, double* acc) {
  leaf0_row<D, IJ>(leaf0<D>(m, bn, G), m, G, w, acc);
}

// All rows of d^2 W / dG dG at G, written to A[(ij*D*D + kl) * stride] (a
// node's column of a component-major array).
template <int D, int IJ = 0, typename T>
__device__ __forceinline__ void tangent0_store_rows(const Leaf0<D>& f, const Material& m, const double* G, T* A,
                                                    int64_t stride) {
  if constexpr (IJ < D * D) {
    double acc[D * D];
#pragma unroll
    for (int kl = 0; kl < D * D; ++kl) acc[kl] = 0.0;
    leaf0_row<D, IJ>(f, m, G, 1.0, acc);
#pragma unroll
    for (int kl = 0; kl < D * D; ++kl) A[int64_t(IJ * D * D + kl) * stride] = T(acc[kl]);
    tangent0_store_rows<D, IJ + 1>(f, m, G, A, stride);
  }
}

template <int D, typename T>
__device__ __forceinline__ void tangent0_store(const Material& m, double bn, const double* G, T* A, int64_t stride) {
  tangent0_store_rows<D>(leaf0<D>(m, bn, G), m, G, A, stride);
}

}  // namespace r1d
