// Kernels of the rank-one lamination path (gfx950), as templates; the
// r1_kernels_<dtype>_<dim>d.hip units instantiate them.
//
//   k_depth1    one wavefront per point: W^1 (and its laminate stress) -- the
//               min over directions of the line hulls at the centre.
//   k_outer     depth 2, one workgroup per (point, outer direction): the outer
//               line's samples are inner envelopes W^1(F + t_i R), computed by
//               the block's waves into LDS; wave 0 then takes the outer hull.
//   k_finalize  depth 2, one wavefront per point: min over outer directions,
//               then the stress through the two-level lamination tree.
//
// Lamination is eq. 3.3 of arXiv 2211.14318 on the lines of Section 4.1; the
// stress is eq. 5.2 (first case) evaluated as Algorithm 3 on a binary tree.
#pragma once
#include "r1_device.hpp"
#include "r1_launch.hpp"

namespace r1k {
using namespace r1d;

template <typename T>
struct OuterRes {       // hull of one outer line at the centre
  T h;
  int mp, mq, capped;
};
static_assert(sizeof(OuterRes<float>) == 16 && sizeof(OuterRes<double>) == 24,
              "r1_outer_res_bytes() must match OuterRes");

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

template <typename T, int D>
__device__ __forceinline__ bool load_point(const KArgs& a, int64_t p, double* G, double& bn) {
  const T* F = static_cast<const T*>(a.F);
  bool fin = true;
#pragma unroll
  for (int k = 0; k < D * D; ++k) {
    G[k] = double(F[int64_t(k) * a.n + p]);
    fin = fin && isfinite(G[k]);
  }
  bn = double(static_cast<const T*>(a.beta_n)[p]);
  return fin && isfinite(bn);
}

template <int D>
__device__ __forceinline__ void line_point(const double* G, const Level& lv, int dir, double t, double* out) {
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) out[i * D + j] = G[i * D + j] + t * lv.a[dir * D + i] * lv.b[dir * D + j];
}

__device__ __forceinline__ double t_of(const Level& lv, int m) {   // t at offset m from the centre
  if (lv.lay && m > 0) return static_cast<const double*>(lv.lay)[m - 1];   // the same value, tabled
  return lv.tau * double(2 * m) / double(lv.n_t - 1);
}

// Inner envelope at G and its laminate stress (P^1 = xi P0(G+) + (1-xi) P0(G-)).
template <typename T, int D, int S, int K, int M>
__device__ Env<T> envelope_with_stress(const KArgs& a, const Level& lv, const Layout<T, S, K>& lay,
                                       double bn, const double* G, double* P) {
  Point<T> q = make_point<T, M>(a.mat, bn);
  double cof[D * D];
  cofactor<D>(G, cof);
  T wc = w_point<T, D, M>(q, G, cof);
  Env<T> e = {wc, 0, 0, 0, 0, inf_v<T>()};
  if (wc < inf_v<T>()) e = envelope_at<T, D, S, K, M>(q, G, wc, lv, lay);
  double Gm[D * D], Gp[D * D], Pm[D * D], Pp[D * D];
  line_point<D>(G, lv, e.dir, -t_of(lv, e.mp), Gm);
  line_point<D>(G, lv, e.dir, t_of(lv, e.mq), Gp);
  stress_at<T, D, M>(q, a.mat, bn, Gm, Pm);
  stress_at<T, D, M>(q, a.mat, bn, Gp, Pp);
  double xi = (e.mp + e.mq) ? double(e.mp) / double(e.mp + e.mq) : 1.0;
#pragma unroll
  for (int k = 0; k < D * D; ++k) P[k] = xi * Pp[k] + (1.0 - xi) * Pm[k];
  return e;
}

template <typename T, int D>
__device__ __forceinline__ void write_bad_point(const KArgs& a, int64_t p, bool nonfinite, bool want_p) {
  T val = nonfinite ? T(__builtin_nan("")) : inf_v<T>();
  static_cast<T*>(a.W)[p] = val;
  if (want_p && a.P)
#pragma unroll
    for (int k = 0; k < D * D; ++k) static_cast<T*>(a.P)[int64_t(k) * a.n + p] = T(__builtin_nan(""));
  if (a.flags) a.flags[p] = nonfinite ? R1_PT_NONFINITE : R1_PT_DETLE0;
  if (a.tree)
    for (int k = 0; k < R1_TREE_NODES; ++k)
      a.tree[p * R1_TREE_NODES + k] = r1_laminate{0, 0, 0, 1.0f};
}

// The one-level laminate's stress at point p (eq. 5.2 on the one-level tree of
// Algorithm 3): P = xi P0(F+) + (1 - xi) P0(F-), F-/+ = G -/+ t a(x)b at offsets
// mp, mq of direction dir, xi = mp / (mp + mq), written to row k of P.  One
// thread's work; the one-level kernels and the batched point work share it, so
// that both give the same bits.
template <typename T, int D, int M>
__device__ __forceinline__ void laminate_stress1(const KArgs& a, int64_t p, const Level& lv, const Point<T>& q,
                                                 const double* G, double bn, int dir, int mp, int mq) {
  double Gm[D * D], Gp[D * D], Pm[D * D], Pp[D * D];
  line_point<D>(G, lv, dir, -t_of(lv, mp), Gm);
  line_point<D>(G, lv, dir, t_of(lv, mq), Gp);
  stress_at<T, D, M>(q, a.mat, bn, Gm, Pm);
  stress_at<T, D, M>(q, a.mat, bn, Gp, Pp);
  const double xi = (mp + mq) ? double(mp) / double(mp + mq) : 1.0;
#pragma unroll
  for (int k = 0; k < D * D; ++k)
    static_cast<T*>(a.P)[int64_t(k) * a.n + p] = T(fma(xi, Pp[k], (1.0 - xi) * Pm[k]));
}

// Per-point constants of a one-level envelope: the geometry (which holds G),
// the constants of W, W at the point, and the point's state (0: finite and
// admissible; 1: non-finite input; 2: W(F) = +inf, det F <= 0).
template <typename T, int D, int M>
struct PointSetup {
  typename GeomOf<D, M>::type g;
  Point<T> q;
  double bn;
  T wc;
  int state;
};

template <typename T, int D, int M>
__device__ __forceinline__ PointSetup<T, D, M> point_setup(const KArgs& a, int64_t p) {
  PointSetup<T, D, M> s;
  double G[D * D];
  const bool fin = load_point<T, D>(a, p, G, s.bn);
  s.q = make_point<T, M>(a.mat, s.bn);
  double cof[D * D];
  cofactor<D>(G, cof);
  s.wc = w_point<T, D, M>(s.q, G, cof);
  s.g = make_geom_m<D, M>(G);
  s.state = !fin ? 1 : (s.wc < inf_v<T>() ? 0 : 2);
  return s;
}

// One-level envelope of point p on level lv from its constants s, with stress,
// tree and flags as requested by a (wave-level: every lane of the wave calls
// it).  kDefer: the stress is left to k_stress1, which finds the point's
// laminate (direction, m_-, m_+) as integers in the first T slot of rows 0, 1,
// 2 of P.
template <typename T, int D, int S, int K, int M, bool kDefer = false>
__device__ __forceinline__ void point_depth1_body(const KArgs& a, int64_t p, const Level& lv,
                                                  const Layout<T, S, K>& lay, const PointSetup<T, D, M>& s) {
  if (s.state != 0) {
    if (lane_id() == 0) write_bad_point<T, D>(a, p, s.state == 1, a.want_stress);
    return;
  }
  const Point<T>& q = s.q;
  const double* G = s.g.G;
  const double bn = s.bn;
  Env<T> e = envelope_geom<T, D, S, K, M>(q, s.g, s.wc, lv, lay);
  const bool stress = a.want_stress && a.P && !kDefer;
  if (lane_id() == 0) {
    static_cast<T*>(a.W)[p] = e.h;
    if (kDefer && a.want_stress && a.P) {
      T* P = static_cast<T*>(a.P);
      *reinterpret_cast<int32_t*>(P + p) = e.dir;
      *reinterpret_cast<int32_t*>(P + a.n + p) = e.mp;
      *reinterpret_cast<int32_t*>(P + 2 * a.n + p) = e.mq;
    }
    const int c = (lv.n_t - 1) / 2;
    if (stress) laminate_stress1<T, D, M>(a, p, lv, q, G, bn, e.dir, e.mp, e.mq);
    if (a.tree) {
      float xi = (e.mp + e.mq) ? float(double(e.mp) / double(e.mp + e.mq)) : 1.0f;
      a.tree[p * R1_TREE_NODES] = r1_laminate{e.dir, c - e.mp, c + e.mq, xi};
      for (int k = 1; k < R1_TREE_NODES; ++k) a.tree[p * R1_TREE_NODES + k] = r1_laminate{0, 0, 0, 1.0f};
    }
    if (a.flags) a.flags[p] = (e.capped ? R1_PT_ITERCAP : 0) | (near_tie(e) ? R1_PT_TIE : 0);
  }
}

// The same with the point's constants formed in place.
template <typename T, int D, int S, int K, int M, bool kDefer = false>
__device__ __forceinline__ void point_depth1(const KArgs& a, int64_t p, const Level& lv) {
  point_depth1_body<T, D, S, K, M, kDefer>(a, p, lv, make_layout<T, S, K>(lv), point_setup<T, D, M>(a, p));
}

// One-level launch: a block of 4 waves takes a.pts_per_wave (<= kPointsPerWave)
// points per wave.  Their constants are formed by one thread per point into LDS
// first (a point's FP64 set-up then costs a lane, not a wavefront), then each
// wave laminates its points one after the other.
constexpr int kPointsPerWave = 8;
constexpr int kPointsPerBlock = 4 * kPointsPerWave;

// Points per wave for n points: kPointsPerWave, or fewer where that would leave
// the launch under 2048 blocks (small batches keep the device filled).
inline int one_level_points_per_wave(int64_t n) {
  const int64_t q = (n + 4 * 2048 - 1) / (4 * 2048);
  return int(q < 1 ? 1 : (q > kPointsPerWave ? kPointsPerWave : q));
}

template <typename T, int D, int S, int K, int M>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? ((D == 2 && M == kFamNH && K <= 14) ? 4 : K <= 16 ? 3 : 1) : 1) void k_depth1(KArgs a) {
  __shared__ PointSetup<T, D, M> ps[kPointsPerBlock];
  const int per_block = 4 * a.pts_per_wave;
  const int64_t p0 = int64_t(blockIdx.x) * per_block;
  if (int(threadIdx.x) < per_block && p0 + threadIdx.x < a.n) ps[threadIdx.x] = point_setup<T, D, M>(a, p0 + threadIdx.x);
  __syncthreads();
  const Layout<T, S, K> lay = make_layout<T, S, K>(a.lv0);
  const int wave = threadIdx.x / kWave;
  for (int i = 0; i < a.pts_per_wave; ++i) {
    const int slot = i * 4 + wave;
    const int64_t p = p0 + slot;
    if (p >= a.n) break;                      // wave-uniform
    point_depth1_body<T, D, S, K, M, true>(a, p, a.lv0, lay, ps[slot]);
  }
}

// Laminate stress of the one-level points (eq. 5.2 on the one-level tree of
// Algorithm 3: P = xi P0(F+) + (1 - xi) P0(F-)), one thread per point, after
// k_depth1: it reads the laminate k_depth1 left in P (see point_depth1) and
// overwrites it with the stress.  Points k_depth1 found bad (W NaN or +inf)
// already hold NaN stresses.
template <typename T, int D, int M>
__global__ __launch_bounds__(256) void k_stress1(KArgs a) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= a.n) return;
  const T w = static_cast<const T*>(a.W)[p];
  if (!(w < inf_v<T>())) return;
  T* P = static_cast<T*>(a.P);
  const int dir = *reinterpret_cast<const int32_t*>(P + p);
  const int mp = *reinterpret_cast<const int32_t*>(P + a.n + p);
  const int mq = *reinterpret_cast<const int32_t*>(P + 2 * a.n + p);
  double G[D * D], bn;
  load_point<T, D>(a, p, G, bn);
  laminate_stress1<T, D, M>(a, p, a.lv0, make_point<T, M>(a.mat, bn), G, bn, dir, mp, mq);
}

// Outer hull of an LDS-resident line (wave-wide, S = 64): wl[m-1] / wr[m-1] are
// the samples at offsets -m / +m, m = 1..c (NaN or +inf = absent).  Same search
// as hull_centre: a values-only vertex test, then alternating tangent queries.
template <typename T>
__device__ LineHull<T> hull_centre_lds(const T* wl, const T* wr, int c, T wc) {
  const int lane = lane_id();
  T maxL = -inf_v<T>(), minR = inf_v<T>();
  for (int m = 1 + lane; m <= c; m += kWave) {
    T inv = T(1.0 / double(m));
    maxL = fmax(maxL, (wc - wl[m - 1]) * inv);
    minR = fmin(minR, (wr[m - 1] - wc) * inv);
  }
  maxL = seg_max<kWave>(maxL);
  minR = seg_min<kWave>(minR);
  LineHull<T> r = {wc, 0, 0, 0};
  if (!(maxL >= minR)) return r;      // wave-uniform
  Cand<T> p = {-inf_v<T>(), 0, T(0)};
  for (int m = 1 + lane; m <= c; m += kWave) {
    T key = (wc - wl[m - 1]) * T(1.0 / double(m));
    bool take = key >= p.key;
    p.key = take ? key : p.key; p.m = take ? m : p.m; p.w = take ? wl[m - 1] : p.w;
  }
  p = seg_arg<kWave, true>(p);
  Cand<T> q = {inf_v<T>(), 0, T(0)};
  for (int it = 0; it < kBridgeCap; ++it) {
    T nb = inf_v<T>(), db = T(1), wb = T(0);
    int mb = 0;
    for (int m = 1 + lane; m <= c; m += kWave) {
      T num = wr[m - 1] - p.w, den = T(m + p.m);
      bool take = num * db <= nb * den;
      nb = take ? num : nb; db = take ? den : db; mb = take ? m : mb; wb = take ? wr[m - 1] : wb;
    }
    Cand<T> qc = {nb / db, mb, wb};
    q = seg_arg<kWave, false>(qc);
    nb = -inf_v<T>(); db = T(1); wb = T(0); mb = 0;
    for (int m = 1 + lane; m <= c; m += kWave) {
      T num = q.w - wl[m - 1], den = T(q.m + m);
      bool take = num * db >= nb * den;
      nb = take ? num : nb; db = take ? den : db; mb = take ? m : mb; wb = take ? wl[m - 1] : wb;
    }
    Cand<T> pc = {nb / db, mb, wb};
    pc = seg_arg<kWave, true>(pc);
    if (pc.m == p.m) {
      r.h = (T(q.m) * p.w + T(p.m) * q.w) / T(q.m + p.m);
      r.mp = p.m; r.mq = q.m;
      return r;
    }
    p = pc;
  }
  r.h = (T(q.m) * p.w + T(p.m) * q.w) / T(q.m + p.m);
  r.mp = p.m; r.mq = q.m; r.capped = 1;
  return r;
}

// Inner directions whose line coefficients are tabulated in LDS per outer line.
constexpr int kMaxTabDirs = 512;

// Waves of an outer-line block (blocks are 256 threads).
constexpr int kOuterWaves = 4;

// Tabulated coefficients per inner direction: 5 for the neo-Hooke family (affine
// in the outer t), 10 for St. Venant-Kirchhoff (p1 cubic, p2 quadratic, p3 affine,
// p4 constant in the outer t).
__host__ __device__ constexpr int tab_coefs(int model) { return model == 2 ? 10 : 5; }

// Bytes of dynamic LDS an outer line needs for samples of elem_bytes bytes:
// the outer line's samples and, when the inner level is tabulated, its
// coefficient table, each wave's warm-start bridge slopes (the last two per
// direction) and each wave's direction visiting order (int).
__host__ __device__ inline size_t outer_lds_bytes(size_t elem_bytes, int n_t_outer, int n_dir_inner, int model) {
  const bool tab = n_dir_inner <= kMaxTabDirs;
  return elem_bytes * (size_t(n_t_outer - 1) +
                       (tab ? size_t(tab_coefs(model) + 2 * kOuterWaves) * size_t(n_dir_inner) : 0)) +
         (tab ? sizeof(int) * size_t(kOuterWaves) * size_t(n_dir_inner) : 0);
}

template <typename T>
__host__ __device__ inline size_t outer_lds_bytes(const Level& lo, const Level& li, int model) {
  return outer_lds_bytes(sizeof(T), lo.n_t, li.n_dir, model);
}

// St. Venant-Kirchhoff inner line along the outer line G(t) = F + t R: its
// coefficients c1 .. c4 (stvk_line) are polynomials in t of degree 3, 2, 1 and 0
// (E(t) of G(t) is quadratic in t).  Their monomial coefficients are fitted in
// double from exact evaluations at t = tau {-1, 0, 1, 2}:
// coef = (c1: t^0..t^3, c2: t^0..t^2, c3: t^0, t^1, c4).
template <typename T, int D>
__device__ __forceinline__ void stvk_inner_coef(double lam, double mu, double k, const double* F, const double* R,
                                                double tau, const double* a, const double* b, T* coef) {
  double y1[4], y2[4], y3[4], c4 = 0.0;
  const double u[4] = {-1.0, 0.0, 1.0, 2.0};
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    double G[D * D];
#pragma unroll
    for (int r = 0; r < D * D; ++r) G[r] = F[r] + u[s] * tau * R[r];
    Line<double> L = stvk_line_g<double, D>(lam, mu, k, make_stvk_geom<D>(G), a, b);
    y1[s] = L.c1; y2[s] = L.c2; y3[s] = L.c3;
    if (s == 1) c4 = L.c4;
  }
  // y(u) = a0 + a1 u + a2 u^2 + a3 u^3 through u = -1, 0, 1, 2; then t = tau u
  const double a0 = y1[1], a2 = 0.5 * (y1[2] + y1[0]) - y1[1], s1 = 0.5 * (y1[2] - y1[0]);
  const double a3 = (y1[3] - a0 - 4.0 * a2 - 2.0 * s1) / 6.0, a1 = s1 - a3;
  const double it = 1.0 / tau;
  coef[0] = T(a0); coef[1] = T(a1 * it); coef[2] = T(a2 * it * it); coef[3] = T(a3 * it * it * it);
  coef[4] = T(y2[1]); coef[5] = T(0.5 * (y2[2] - y2[0]) * it); coef[6] = T((0.5 * (y2[2] + y2[0]) - y2[1]) * it * it);
  coef[7] = T(y3[1]); coef[8] = T(0.5 * (y3[2] - y3[0]) * it);
  coef[9] = T(c4);
}

// One outer line (block-level, every thread calls it): the samples W^1(F + t_i R_mo)
// are inner envelopes computed by the block's waves into LDS; wave 0 takes the
// outer hull at the centre.  w1f = W^1(F) is the centre sample; when
// compute_centre is set it is computed here (by wave 0) instead.  Thread 0
// writes the result to *out.  Returns the centre value used.
template <typename T, int D, int S, int K, int M>
__device__ __forceinline__ T outer_line(const KArgs& a, int64_t p, int mo, const Level& lo, const Level& li, T w1f,
                        bool compute_centre, OuterRes<T>* out, char* smem_raw) {
  const int co = (lo.n_t - 1) / 2;
  // Up to kMaxTabDirs inner directions the waves keep warm-start bridge slopes,
  // visiting orders and the inner lines' coefficients as polynomials in the outer t
  // (tab_coefs) in LDS.
  const bool lds_lines = li.n_dir <= kMaxTabDirs;
  const bool tab = lds_lines;
  constexpr int NC = tab_coefs(M);
  T* coef = reinterpret_cast<T*>(smem_raw);                 // NC * n_dir_i (tab)
  T* warm = coef + (tab ? NC * li.n_dir : 0);                   // 2 kOuterWaves n_dir_i (lds_lines)
  T* wl = warm + (lds_lines ? 2 * kOuterWaves * li.n_dir : 0);  // outer samples at -m
  T* wr = wl + co;                                          // outer samples at +m
  int* order = reinterpret_cast<int*>(wr + co);             // kOuterWaves * n_dir_i (lds_lines)
  __shared__ int capped_any;
  __shared__ T centre;
  double F[D * D], bn;
  load_point<T, D>(a, p, F, bn);
  double R[D * D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) R[i * D + j] = lo.a[mo * D + i] * lo.b[mo * D + j];
  if (threadIdx.x == 0) { capped_any = 0; centre = w1f; }
  if (tab) {
    if constexpr (M == kFamSTVK) {
      const double k = line_scale<T, M>(a.mat);
      for (int i = threadIdx.x; i < li.n_dir; i += blockDim.x)
        stvk_inner_coef<T, D>(a.mat.lambda, a.mat.mu, k, F, R, lo.tau, li.a + i * D, li.b + i * D, coef + NC * i);
    } else {
      double cofF[D * D], C1[D * D];
      cofactor<D>(F, cofF);
      cof_derivative<D>(F, R, C1);
      for (int i = threadIdx.x; i < li.n_dir; i += blockDim.x)
        inner_line_coef<T, D>(a.mat.model, line_scale<T>(a.mat), F, cofF, R, C1, li.a + i * D, li.b + i * D,
                              coef + NC * i);
    }
  }
  if (lds_lines)
    for (int i = threadIdx.x; i < 2 * kOuterWaves * li.n_dir; i += blockDim.x) warm[i] = T(__builtin_nan(""));
  __syncthreads();
  Layout<T, S, K> lay = make_layout<T, S, K>(li);
  Point<T> q = make_point<T, M>(a.mat, bn);
  const int wave = threadIdx.x / kWave, nwave = blockDim.x / kWave;
  int capped = 0;
  if (compute_centre && wave == 0) {
    double cof[D * D];
    cofactor<D>(F, cof);
    T wc = w_point<T, D, M>(q, F, cof);
    T v = wc;
    if (wc < inf_v<T>()) {
      Env<T> e = envelope_at<T, D, S, K, M>(q, F, wc, li, lay);
      v = e.h;
      capped |= e.capped;
    }
    if (lane_id() == 0) centre = v;
  }
  // outer samples, interleaved left/right so the waves share both sides; a
  // wave walks one side outwards in even steps of two samples, so the inner
  // bridge slopes of its last two samples (warm, per inner direction),
  // extrapolated, start the next
  T* warm_w = warm + 2 * wave * li.n_dir;      // blocks have kOuterWaves waves
  int* order_w = order + wave * li.n_dir;
  for (int s = wave; s < 2 * co; s += nwave) {
    int m = 1 + (s >> 1);
    double t = (s & 1) ? t_of(lo, m) : -t_of(lo, m);
    double G[D * D];
#pragma unroll
    for (int k = 0; k < D * D; ++k) G[k] = F[k] + t * R[k];
    T v;
    if (tab) {
      if constexpr (M == kFamSTVK) {
        // W(G) and c0 = k psi0(G), shared by every inner line; c1 .. c4 from the table
        double cof[D * D];
        cofactor<D>(G, cof);
        const double zero[D] = {};
        const Line<T> L0 = line_setup<T, D, M>(q, G, cof, zero, zero);
        T wc = fma(ws_sample_stvk<T>(T(0), L0, q), q.sc, q.B);
        v = wc;
        if (wc < inf_v<T>()) {
          const T tt = T(t);
          Env<T> e = envelope_lines<T, S, K, M>(q, wc, li.n_dir, lay, [&](int dd) {
            const T* cf = coef + NC * dd;
            Line<T> L;
            L.J0 = T(0);
            L.J1 = T(0);
            L.c0 = L0.c0;
            L.c1 = fma(tt, fma(tt, fma(tt, cf[3], cf[2]), cf[1]), cf[0]);
            L.c2 = fma(tt, fma(tt, cf[6], cf[5]), cf[4]);
            L.c3 = fma(tt, cf[8], cf[7]);
            L.c4 = cf[9];
            return L;
          }, warm_w, T(__builtin_nan("")), order_w);
          v = e.h;
          capped |= e.capped;
        }
      } else {
        // W(G) and the per-sample parts of every inner line: J0 = det G, c0 = kq (|G|^2 - d)
        // (neo-Hooke) or G11 and the quadratic rest (double well)
        double cof[D * D];
        cofactor<D>(G, cof);
        double J0, c0 = 0.0;
        if (a.mat.model == 0) {
          J0 = det_of<D>(G, cof);
#pragma unroll
          for (int k = 0; k < D * D; ++k) c0 += G[k] * G[k];
          c0 = q.kq * (c0 - double(D));
        } else {
          J0 = G[0];
#pragma unroll
          for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j)
              if (i || j) c0 += (G[i * D + j] - (i == j ? 1.0 : 0.0)) * (G[i * D + j] - (i == j ? 1.0 : 0.0));
        }
        Line<T> L0 = {T(J0), T(0), T(c0), T(0), T(0)};
        T wc = q.model == 0 ? fma(ws_sample<T>(T(0), L0, q), q.sc, q.B) : w_sample_doublewell<T>(T(0), L0);
        v = wc;
        if (wc < inf_v<T>()) {
          const T tt = T(t);
          Env<T> e = envelope_lines<T, S, K>(q, wc, li.n_dir, lay, [&](int dd) {
            const T* cf = coef + NC * dd;
            return Line<T>{L0.J0, T(fma(tt, cf[1], cf[0])), L0.c0, T(fma(tt, cf[3], cf[2])), cf[4]};
          }, warm_w, T(q.kq * li.ab2), order_w);
          v = e.h;
          capped |= e.capped;
        }
      }
    } else {
      double cof[D * D];
      cofactor<D>(G, cof);
      T wc = w_point<T, D, M>(q, G, cof);
      v = wc;
      if (wc < inf_v<T>()) {
        Env<T> e = envelope_at<T, D, S, K, M>(q, G, wc, li, lay);
        v = e.h;
        capped |= e.capped;
      }
    }
    if (lane_id() == 0) ((s & 1) ? wr : wl)[m - 1] = v;
  }
  if (capped && lane_id() == 0) atomicOr(&capped_any, 1);
  __syncthreads();
  T cv = centre;
  if (wave == 0) {
    LineHull<T> r = hull_centre_lds<T>(wl, wr, co, cv);
    if (threadIdx.x == 0) *out = OuterRes<T>{r.h, r.mp, r.mq, r.capped | capped_any};
  }
  __syncthreads();                            // LDS reused by the caller's next item
  return cv;
}

template <typename T, int D, int S, int K, int M>
__global__ __launch_bounds__(256, (sizeof(T) == 4 && D == 2 && K <= 16) ? 3 : 1) void k_outer(KArgs a) {
  extern __shared__ char smem_raw[];
  const int n_dir_o = a.lv0.n_dir;
  const int64_t p = int64_t(blockIdx.x) / n_dir_o;
  const int mo = int(int64_t(blockIdx.x) % n_dir_o);
  OuterRes<T>* out = static_cast<OuterRes<T>*>(a.scratch_outer) + p * n_dir_o + mo;
  T w1f = static_cast<const T*>(a.scratch_w1f)[p];
  if (!(w1f < inf_v<T>())) {                  // det F <= 0 or non-finite input: block-uniform
    if (threadIdx.x == 0) *out = OuterRes<T>{w1f, 0, 0, 0};
    return;
  }
  outer_line<T, D, S, K, M>(a, p, mo, a.lv0, a.lv1, w1f, false, out, smem_raw);
}

// Two-level result of point p from its outer-line results res[0 .. n_dir_o):
// min over outer directions, then stress and tree through Algorithm 3 on the
// binary tree (wave-level).
template <typename T, int D, int S, int K, int M>
__device__ __forceinline__ void finalize_point(const KArgs& a, int64_t p, const Level& lo, const Level& li,
                               const OuterRes<T>* res) {
  const int n_dir_o = lo.n_dir;
  double F[D * D], bn;
  bool fin = load_point<T, D>(a, p, F, bn);
  Point<T> q0 = make_point<T, M>(a.mat, bn);
  double cof0[D * D];
  cofactor<D>(F, cof0);
  if (!fin || !(w_point<T, D, M>(q0, F, cof0) < inf_v<T>())) {
    if (lane_id() == 0) write_bad_point<T, D>(a, p, !fin, a.want_stress);
    return;
  }
  T bh = inf_v<T>(), bs = inf_v<T>();
  int bd = 0x7fffffff, bp = 0, bq = 0, cap = 0;
  for (int m = lane_id(); m < n_dir_o; m += kWave) {
    OuterRes<T> r = res[m];
    cap |= r.capped;
    if (r.h < bh) { bs = bh; bh = r.h; bd = m; bp = r.mp; bq = r.mq; }
    else bs = fmin(bs, r.h);
  }
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    T oh = __shfl_xor(bh, off), os = __shfl_xor(bs, off);
    int od = __shfl_xor(bd, off), op = __shfl_xor(bp, off), oq = __shfl_xor(bq, off);
    cap |= __shfl_xor(cap, off);
    bool take = oh < bh || (oh == bh && od < bd);
    bs = take ? fmin(os, bh) : fmin(bs, oh);
    bh = take ? oh : bh; bd = take ? od : bd; bp = take ? op : bp; bq = take ? oq : bq;
  }
  bool tie = near_tie(Env<T>{bh, bd, bp, bq, 0, bs});
  const int c = (lo.n_t - 1) / 2, ci = (li.n_t - 1) / 2;
  r1_laminate node[3];
  double Pout[D * D];
  if (a.want_stress || a.tree) {
    Layout<T, S, K> lay = make_layout<T, S, K>(li);
    double Gm[D * D], Gp[D * D], Pm[D * D], Pp[D * D];
    line_point<D>(F, lo, bd, -t_of(lo, bp), Gm);
    line_point<D>(F, lo, bd, t_of(lo, bq), Gp);
    Env<T> em = envelope_with_stress<T, D, S, K, M>(a, li, lay, bn, Gm, Pm);
    cap |= em.capped;
    tie = tie || near_tie(em);
    Env<T> ep = em;
    if (bp + bq) {
      ep = envelope_with_stress<T, D, S, K, M>(a, li, lay, bn, Gp, Pp);
      cap |= ep.capped;
      tie = tie || near_tie(ep);
    } else {
#pragma unroll
      for (int k = 0; k < D * D; ++k) Pp[k] = Pm[k];
    }
    double xi = (bp + bq) ? double(bp) / double(bp + bq) : 1.0;
#pragma unroll
    for (int k = 0; k < D * D; ++k) Pout[k] = xi * Pp[k] + (1.0 - xi) * Pm[k];
    node[0] = r1_laminate{bd, c - bp, c + bq, float(xi)};
    node[1] = r1_laminate{em.dir, ci - em.mp, ci + em.mq,
                          (em.mp + em.mq) ? float(double(em.mp) / double(em.mp + em.mq)) : 1.0f};
    node[2] = r1_laminate{ep.dir, ci - ep.mp, ci + ep.mq,
                          (ep.mp + ep.mq) ? float(double(ep.mp) / double(ep.mp + ep.mq)) : 1.0f};
  }
  if (lane_id() == 0) {
    static_cast<T*>(a.W)[p] = bh;
    if (a.want_stress && a.P)
#pragma unroll
      for (int k = 0; k < D * D; ++k) static_cast<T*>(a.P)[int64_t(k) * a.n + p] = T(Pout[k]);
    if (a.tree)
      for (int k = 0; k < R1_TREE_NODES; ++k) a.tree[p * R1_TREE_NODES + k] = node[k];
    if (a.flags) a.flags[p] = (cap ? R1_PT_ITERCAP : 0) | (tie ? R1_PT_TIE : 0);
  }
}

template <typename T, int D, int S, int K, int M>
__global__ __launch_bounds__(256) void k_finalize(KArgs a) {
  const int64_t p = int64_t(blockIdx.x) * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (p >= a.n) return;
  finalize_point<T, D, S, K, M>(a, p, a.lv0, a.lv1,
                             static_cast<const OuterRes<T>*>(a.scratch_outer) + p * a.lv0.n_dir);
}

// ---- dispatch ------------------------------------------------------------------

template <typename T, int D, int S, int K, int M>
hipError_t launch_T(const KArgs& a, int depth, hipStream_t st, KTimer* tm) {
  dim3 blk(256);
  unsigned per = 256 / kWave;
  const int ppw = one_level_points_per_wave(a.n);
  const dim3 grd1(unsigned((a.n + 4 * ppw - 1) / (4 * ppw)));
  if (depth == 1) {
    KArgs a1 = a;
    a1.pts_per_wave = ppw;
    if (tm) tm->begin("depth1", st);
    hipLaunchKernelGGL((k_depth1<T, D, S, K, M>), grd1, blk, 0, st, a1);
    if (a.want_stress && a.P)
      hipLaunchKernelGGL((k_stress1<T, D, M>), dim3(unsigned((a.n + 255) / 256)), blk, 0, st, a);
    if (tm) tm->end(st);
    return hipGetLastError();
  }
  // depth 2: W^1 at every point (the outer lines' centre), outer lines, finalize
  KArgs pre = a;
  pre.lv0 = a.lv1;
  pre.W = a.scratch_w1f;
  pre.P = nullptr;
  pre.tree = nullptr;
  pre.flags = nullptr;
  pre.want_stress = 0;
  pre.pts_per_wave = ppw;
  dim3 grd(unsigned((a.n + per - 1) / per));
  if (tm) tm->begin("depth2_centre", st);
  hipLaunchKernelGGL((k_depth1<T, D, S, K, M>), grd1, blk, 0, st, pre);
  if (tm) tm->end(st);
  size_t lds = outer_lds_bytes<T>(a.lv0, a.lv1, M);
  dim3 grd_o(unsigned(a.n * a.lv0.n_dir));
  if (tm) tm->begin("outer", st);
  hipLaunchKernelGGL((k_outer<T, D, S, K, M>), grd_o, blk, lds, st, a);
  if (tm) tm->end(st);
  if (tm) tm->begin("finalize", st);
  hipLaunchKernelGGL((k_finalize<T, D, S, K, M>), grd, blk, 0, st, a);
  if (tm) tm->end(st);
  return hipGetLastError();
}

template <typename T, int D, int M>
hipError_t launch_TD(const KArgs& a, int depth, int S, int K, hipStream_t st, KTimer* tm) {
#define R1_CASE(SS, KK) \
  if (S == SS && K == KK) return launch_T<T, D, SS, KK, M>(a, depth, st, tm);
  R1_CASE(8, 2) R1_CASE(8, 4) R1_CASE(8, 8) R1_CASE(8, 16) R1_CASE(8, 32)
  R1_CASE(16, 2) R1_CASE(16, 4) R1_CASE(16, 8) R1_CASE(16, 14) R1_CASE(16, 16) R1_CASE(16, 32)
  R1_CASE(32, 2) R1_CASE(32, 4) R1_CASE(32, 8) R1_CASE(32, 16) R1_CASE(32, 32)
  R1_CASE(64, 2) R1_CASE(64, 4) R1_CASE(64, 8) R1_CASE(64, 16) R1_CASE(64, 32)
#undef R1_CASE
  return hipErrorInvalidValue;
}

}  // namespace r1k
