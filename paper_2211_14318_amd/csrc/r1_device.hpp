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
// m > c are padding and hold +inf.  64/S lines are processed side by side.
//
// Hull at the centre: the centre is a hull vertex iff every left sample's slope
// towards it is strictly smaller than every right sample's slope from it (one
// pass, fused with sampling).  Otherwise the hull segment over the centre is
// the lower common tangent ("bridge") of the left and right sample sets, found
// by alternating tangent queries: q = tangent point on the right seen from p,
// p = tangent point on the left seen from q, until p repeats.  Ties prefer the
// outermost sample, matching the strict-vertex reading of Algorithm 1.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace r1d {

constexpr int kWave = 64;
constexpr int kBridgeCap = 256;   // tangent rounds before giving up (never reached in practice)

template <typename T> __device__ __forceinline__ T inf_v();
template <> __device__ __forceinline__ float inf_v<float>() { return __builtin_inff(); }
template <> __device__ __forceinline__ double inf_v<double>() { return __builtin_inf(); }

// Natural logarithm: hardware log2 for FP32 (v_log_f32), the device library for FP64.
__device__ __forceinline__ float ln_t(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }
__device__ __forceinline__ double ln_t(double x) { return log(x); }
// Exponential of an argument pre-scaled by the per-point constant kexp:
// FP32 uses the hardware exp2 (kexp carries log2 e), FP64 the device library.
__device__ __forceinline__ float expk(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ double expk(double x) { return exp(x); }

struct Material {
  int dim, model;        // model: 0 neo-Hooke damage, 1 double-well test energy
  double mu, lambda, D_inf, D0;
};

struct Level {           // one lamination level on the device
  const double* a;       // n_dir x dim
  const double* b;
  int n_dir, n_t;
  double tau;
};

// Per-point constants of W (eq. 2.9 written as a function of psi0):
//   psi0 <= beta_n :  W = (1 - D_n) psi0
//   psi0 >  beta_n :  W = psi0 - D_n beta_n - D_inf[(psi0 - beta_n) + D0 (e^{-psi0/D0} - e^{-beta_n/D0})]
//                       = A psi0 + B - C e^{-psi0/D0}
// with A = 1 - D_inf, C = D_inf D0, B = D_inf e^{-beta_n/D0} (beta_n + D0).
template <typename T>
struct Point {
  T mu2, mu, lam2;
  T bn, E1, A, B, C, kexp;
  int model;
};

template <typename T>
__device__ __forceinline__ Point<T> make_point(const Material& m, double bn) {
  Point<T> q;
  double e = exp(-bn / m.D0);
  double Dn = m.D_inf * (1.0 - e);
  q.mu2 = T(0.5 * m.mu);
  q.mu = T(m.mu);
  q.lam2 = T(0.5 * m.lambda);
  q.bn = T(bn);
  q.E1 = T(1.0 - Dn);
  q.A = T(1.0 - m.D_inf);
  q.C = T(m.D_inf * m.D0);
  q.B = T(m.D_inf * e * (bn + m.D0));
  q.kexp = (sizeof(T) == 4) ? T(-1.4426950408889634 / m.D0) : T(-1.0 / m.D0);
  q.model = m.model;
  return q;
}

// Coefficients of W along G + t a(x)b.  det is affine along rank-one lines:
// det(G + t a(x)b) = det G + t a.cof(G) b; |G + t a(x)b|^2 = |G|^2 + 2t a.Gb + t^2 |a|^2|b|^2.
// For the double-well test energy: g(t) = G11 + t a1 b1 and the quadratic rest.
template <typename T>
struct Line { T J0, J1, c0, c1, c2; };

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

template <typename T, int D>
__device__ __forceinline__ Line<T> line_setup(int model, const double* G, const double* cof,
                                              const double* a, const double* b) {
  Line<T> L;
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
    L.c0 = T(n2 - double(D));
    L.c1 = T(2.0 * gab);
    L.c2 = T(aa * bb);
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

// One sample of W on a line (the hot loop: 1 log + 1 exp + ~12 VALU).
template <typename T>
__device__ __forceinline__ T w_sample(T t, const Line<T>& L, const Point<T>& q) {
  T J = fma(t, L.J1, L.J0);
  T s = fma(t, fma(t, L.c2, L.c1), L.c0);
  T lnJ = ln_t(J);
  T psi = fma(q.mu2, s, lnJ * fma(q.lam2, lnJ, -q.mu));
  T wd = fma(q.A, psi, q.B) - q.C * expk(psi * q.kexp);
  T w = psi <= q.bn ? q.E1 * psi : wd;
  return J > T(0) ? w : inf_v<T>();
}

template <typename T>
__device__ __forceinline__ T w_sample_doublewell(T t, const Line<T>& L) {
  T g = fma(t, L.J1, L.J0);
  T g2 = fma(g, g, T(-1));
  return fma(g2, g2, fma(t, fma(t, L.c2, L.c1), L.c0));
}

// W at a point (the centre sample of every line through it), in the path's precision.
template <typename T, int D>
__device__ __forceinline__ T w_point(const Point<T>& q, const double* G, const double* cof) {
  double a0[3] = {0, 0, 0};
  Line<T> L = line_setup<T, D>(q.model, G, cof, a0, a0);
  return q.model == 0 ? w_sample<T>(T(0), L, q) : w_sample_doublewell<T>(T(0), L);
}

// ---- segment reductions ------------------------------------------------------

template <typename T>
struct Cand {      // a hull candidate: key (a slope or value), offset magnitude m, sample value w
  T key;
  int m;
  T w;
};

// argmax of key, ties -> larger m (the outermost sample)
template <typename T>
__device__ __forceinline__ bool beats_max(const Cand<T>& x, const Cand<T>& y) {
  return x.key > y.key || (x.key == y.key && x.m > y.m);
}
// argmin of key, ties -> larger m
template <typename T>
__device__ __forceinline__ bool beats_min(const Cand<T>& x, const Cand<T>& y) {
  return x.key < y.key || (x.key == y.key && x.m > y.m);
}

template <int S, bool MAX, typename T>
__device__ __forceinline__ Cand<T> seg_reduce(Cand<T> c) {
#pragma unroll
  for (int off = S / 2; off >= 1; off >>= 1) {
    Cand<T> o;
    o.key = __shfl_xor(c.key, off, S);
    o.m = __shfl_xor(c.m, off, S);
    o.w = __shfl_xor(c.w, off, S);
    bool take = MAX ? beats_max(o, c) : beats_min(o, c);
    c.key = take ? o.key : c.key;
    c.m = take ? o.m : c.m;
    c.w = take ? o.w : c.w;
  }
  return c;
}

template <int S, typename T>
__device__ __forceinline__ T seg_min(T v) {
#pragma unroll
  for (int off = S / 2; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, S));
  return v;
}

// Result of one line: hull value at the centre and the bracketing vertices as
// offset magnitudes (mp on the left, mq on the right; 0/0 = centre is a vertex).
template <typename T>
struct LineHull {
  T h;
  int mp, mq;
  int capped;
};

// Hull of the segment's line at its centre.  w: this lane's samples (layout
// above); wc: centre sample; inv_m[h] = 1/m_h; mf[h] = m_h as T.  Every lane
// of the wave must call this together (it uses cross-lane shuffles).
template <typename T, int S, int K>
__device__ __forceinline__ LineHull<T> hull_centre(const T (&w)[K], T wc, const T (&inv_m)[K / 2],
                                                   const int (&mi)[K / 2]) {
  constexpr int H = K / 2;
  // pass 1: vertex test, and the tangent point on the left seen from the centre
  Cand<T> p = {-inf_v<T>(), 0, T(0)};
  T minR = inf_v<T>();
#pragma unroll
  for (int h = 0; h < H; ++h) {
    Cand<T> c = {(wc - w[h]) * inv_m[h], mi[h], w[h]};
    if (beats_max(c, p)) p = c;
    minR = fmin(minR, (w[H + h] - wc) * inv_m[h]);
  }
  p = seg_reduce<S, true>(p);
  minR = seg_min<S>(minR);
  LineHull<T> r;
  r.h = wc; r.mp = 0; r.mq = 0; r.capped = 0;
  bool todo = p.key >= minR;          // not a strict vertex (NaN -> vertex)
  const bool bridged = todo;          // segment-uniform
  Cand<T> q = {inf_v<T>(), 0, T(0)};
  int it = 0;
  while (__any(todo)) {
    // q: argmin over right samples of (w_j - w_p)/(m_j + m_p)
    T nb = inf_v<T>(), db = T(1);
    int mb = 0;
    T wb = T(0);
    T mpf = T(p.m);
#pragma unroll
    for (int h = 0; h < H; ++h) {
      T num = w[H + h] - p.w;
      T den = T(mi[h]) + mpf;
      bool take = num * db < nb * den || (num * db == nb * den && mi[h] > mb);
      nb = take ? num : nb; db = take ? den : db; mb = take ? mi[h] : mb; wb = take ? w[H + h] : wb;
    }
    Cand<T> qc = {nb / db, mb, wb};
    qc = seg_reduce<S, false>(qc);
    // p': argmax over left samples of (w_q - w_i)/(m_q + m_i)
    T qmf = T(qc.m);
    nb = -inf_v<T>(); db = T(1); mb = 0; wb = T(0);
#pragma unroll
    for (int h = 0; h < H; ++h) {
      T num = qc.w - w[h];
      T den = qmf + T(mi[h]);
      bool take = num * db > nb * den || (num * db == nb * den && mi[h] > mb);
      nb = take ? num : nb; db = take ? den : db; mb = take ? mi[h] : mb; wb = take ? w[h] : wb;
    }
    Cand<T> pc = {nb / db, mb, wb};
    pc = seg_reduce<S, true>(pc);
    bool conv = pc.m == p.m;
    if (todo) {
      q = qc;
      if (conv) {
        todo = false;
      } else {
        p = pc;
      }
    }
    if (++it >= kBridgeCap) {
      if (todo) r.capped = 1;
      break;
    }
  }
  if (bridged) {
    T mpf = T(p.m), mqf = T(q.m);
    r.h = (mqf * p.w + mpf * q.w) / (mqf + mpf);
    r.mp = p.m;
    r.mq = q.m;
  }
  return r;
}

// Per-lane constants of a line layout: offsets m_h = 1 + sl + S*h, t_h = tau*2m/(n_t-1).
template <typename T, int S, int K>
struct Layout {
  T t[K / 2];
  T inv_m[K / 2];
  int mi[K / 2];
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
    lay.mi[h] = m;
    lay.inv_m[h] = T(1.0 / double(m));
    lay.t[h] = T(tau * double(2 * m) / double(n_t - 1));
  }
  return lay;
}

template <typename T>
struct Env {            // W^1 at a point: value, direction, bracketing offsets
  T h;
  int dir, mp, mq;
  int capped;
};

// One lamination level at point G (wave-uniform): min over directions of the
// line hulls at the centre.  wc = W(G).  Every lane of the wave must call it.
template <typename T, int D, int S, int K>
__device__ Env<T> envelope_at(const Point<T>& q, const double* G, T wc, const Level& lv,
                              const Layout<T, S, K>& lay) {
  constexpr int NSEG = kWave / S;
  const int lane = threadIdx.x & (kWave - 1);
  const int seg = lane / S;
  double cof[D * D];
  cofactor<D>(G, cof);
  Env<T> best = {inf_v<T>(), 0, 0, 0, 0};
  for (int m0 = 0; m0 < lv.n_dir; m0 += NSEG) {
    int dir = m0 + seg;
    bool act = dir < lv.n_dir;
    int dd = act ? dir : lv.n_dir - 1;
    double a[D], b[D];
#pragma unroll
    for (int i = 0; i < D; ++i) { a[i] = lv.a[dd * D + i]; b[i] = lv.b[dd * D + i]; }
    Line<T> L = line_setup<T, D>(q.model, G, cof, a, b);
    T w[K];
    if (q.model == 0) {
#pragma unroll
      for (int h = 0; h < K / 2; ++h) {
        bool valid = lay.mi[h] <= lay.c;
        T wl = w_sample<T>(-lay.t[h], L, q);
        T wr = w_sample<T>(lay.t[h], L, q);
        w[h] = valid ? wl : inf_v<T>();
        w[K / 2 + h] = valid ? wr : inf_v<T>();
      }
    } else {
#pragma unroll
      for (int h = 0; h < K / 2; ++h) {
        bool valid = lay.mi[h] <= lay.c;
        T wl = w_sample_doublewell<T>(-lay.t[h], L);
        T wr = w_sample_doublewell<T>(lay.t[h], L);
        w[h] = valid ? wl : inf_v<T>();
        w[K / 2 + h] = valid ? wr : inf_v<T>();
      }
    }
    LineHull<T> lh = hull_centre<T, S, K>(w, wc, lay.inv_m, lay.mi);
    if (act && lh.h < best.h) {
      best.h = lh.h; best.dir = dir; best.mp = lh.mp; best.mq = lh.mq;
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
    bool take = oh < best.h || (oh == best.h && od < best.dir);
    best.h = take ? oh : best.h;
    best.dir = take ? od : best.dir;
    best.mp = take ? op : best.mp;
    best.mq = take ? oq : best.mq;
    best.capped |= oc;
  }
  return best;
}

// P0 = dW/dF = (1 - D(max(beta_n, psi0))) (mu G + (lambda ln J - mu) G^{-T}) in double
// (eq. 2.12); the double-well test energy has its own gradient.
template <int D>
__device__ __forceinline__ void stress0(const Material& m, double bn, const double* G, double* P) {
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

}  // namespace r1d
