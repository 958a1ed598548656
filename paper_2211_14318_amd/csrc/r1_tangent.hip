// Tangent moduli of the laminate: the third output of Algorithm 3 of arXiv
// 2211.14318, A^k = dP^k/dF, evaluated on a lamination tree that the envelope
// kernels (or a caller) wrote.  Along a rank-one line every laminate endpoint
// is a point of W, so A^k is the tree-weighted sum of the leaf moduli
// A^0 = d^2 W / dF dF (eq. 2.9), with the same weights as the stress P^k.
//
// The leaves are rebuilt with the envelope kernels' own line arithmetic, so
// they are the very points whose stress P^k was taken.  One thread per
// (point, component): blockIdx.y is the component (i*d + j)*d*d + k*d + l,
// consecutive threads are consecutive points, and the SoA output
// A[component * n + p] is written coalesced.  The work per thread is a few
// leaves of FP64 scalar algebra.
#include "r1_kernels.hpp"

namespace r1k {

// d^2 W / dG_ij dG_kl at one point of the line set (ij = i*D + j, kl = k*D + l).
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
template <int D>
__device__ __forceinline__ double tangent0_comp(const Material& m, double bn, const double* G, int ij, int kl) {
  const int i = ij / D, j = ij % D, k = kl / D, l = kl % D;
  if (m.model == 2) {
    double E[D * D], S[D * D];
    double tr = stvk_strain<D>(G, E);
    double psi = stvk_psi_stress<D>(m, G, S);
    double Bik = 0.0;
#pragma unroll
    for (int r = 0; r < D; ++r) Bik += G[i * D + r] * G[k * D + r];
    double h = m.lambda * G[ij] * G[kl] + (i == k ? m.lambda * tr * (j == l ? 1.0 : 0.0) + 2.0 * m.mu * E[l * D + j] : 0.0)
             + m.mu * (G[i * D + l] * G[k * D + j] + (j == l ? Bik : 0.0));
    double g1 = 1.0 - m.D_inf * (1.0 - exp(-(psi > bn ? psi : bn) / m.D0));
    double g2 = psi > bn ? -m.D_inf / m.D0 * exp(-psi / m.D0) : 0.0;
    return g1 * h + g2 * S[ij] * S[kl];
  }
  if (m.model != 0) {
    if (ij != kl) return 0.0;
    return ij == 0 ? 12.0 * G[0] * G[0] - 4.0 : 2.0;
  }
  double cof[D * D];
  cofactor<D>(G, cof);
  double J = det_of<D>(G, cof);
  if (!(J > 0.0)) return __builtin_nan("");
  double lnJ = log(J), n2 = 0.0;
#pragma unroll
  for (int i = 0; i < D * D; ++i) n2 += G[i] * G[i];
  double psi = 0.5 * m.mu * (n2 - double(D)) - m.mu * lnJ + 0.5 * m.lambda * lnJ * lnJ;
  double beta = psi > bn ? psi : bn;
  double g1 = 1.0 - m.D_inf * (1.0 - exp(-beta / m.D0));
  double g2 = psi > bn ? -m.D_inf / m.D0 * exp(-psi / m.D0) : 0.0;
  double c = m.lambda * lnJ - m.mu;
  double Hij = cof[ij] / J, Hkl = cof[kl] / J, Hil = cof[i * D + l] / J, Hkj = cof[k * D + j] / J;
  double h = (ij == kl ? m.mu : 0.0) + m.lambda * Hij * Hkl - c * Hil * Hkj;
  double Sij = m.mu * G[ij] + c * Hij, Skl = m.mu * G[kl] + c * Hkl;
  return g1 * h + g2 * Sij * Skl;
}

// Endpoints G-/+ of tree node t on level lv around G, and the volume fraction
// xi of G+.  False when the node does not name a laminate of lv (direction or
// sample index out of range, or not straddling the centre).
template <int D>
__device__ __forceinline__ bool node_split(const Level& lv, const r1_laminate& t, const double* G, double* Gm,
                                           double* Gp, double& xi) {
  const int c = (lv.n_t - 1) / 2;
  if (t.dir < 0 || t.dir >= lv.n_dir || t.i_minus < 0 || t.i_minus > c || t.i_plus < c || t.i_plus >= lv.n_t)
    return false;
  const int mp = c - t.i_minus, mq = t.i_plus - c;
  line_point<D>(G, lv, t.dir, -t_of(lv, mp), Gm);
  line_point<D>(G, lv, t.dir, t_of(lv, mq), Gp);
  xi = (mp + mq) ? double(mp) / double(mp + mq) : 1.0;
  return true;
}

// One node's modulus component over its two leaves: xi A0(G+) + (1 - xi) A0(G-).
template <int D>
__device__ __forceinline__ double node_tangent(const Material& mat, double bn, const Level& lv, const r1_laminate& t,
                                               const double* G, int ij, int kl, bool& ok) {
  double Gm[D * D], Gp[D * D], xi;
  ok = node_split<D>(lv, t, G, Gm, Gp, xi);
  if (!ok) return 0.0;
  double am = tangent0_comp<D>(mat, bn, Gm, ij, kl);
  double ap = tangent0_comp<D>(mat, bn, Gp, ij, kl);
  return xi * ap + (1.0 - xi) * am;
}

template <typename T, int D>
__global__ __launch_bounds__(256) void k_tangent(KArgs a, int depth, const r1_laminate* tree, T* A) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= a.n) return;
  const int comp = blockIdx.y, ij = comp / (D * D), kl = comp % (D * D);
  double F[D * D], bn;
  bool fin = load_point<T, D>(a, p, F, bn);
  double w = double(static_cast<const T*>(a.W)[p]);
  double out = __builtin_nan("");
  if (fin && isfinite(w)) {
    const r1_laminate* t = tree + p * R1_TREE_NODES;
    bool ok = true;
    if (depth == 1) {
      out = node_tangent<D>(a.mat, bn, a.lv0, t[0], F, ij, kl, ok);
    } else {
      double Gm[D * D], Gp[D * D], xi;
      ok = node_split<D>(a.lv0, t[0], F, Gm, Gp, xi);
      if (ok) {
        bool okm, okp;
        double am = node_tangent<D>(a.mat, bn, a.lv1, t[1], Gm, ij, kl, okm);
        double ap = node_tangent<D>(a.mat, bn, a.lv1, t[2], Gp, ij, kl, okp);
        ok = okm && okp;
        out = xi * ap + (1.0 - xi) * am;
      }
    }
    if (!ok) out = __builtin_nan("");
  }
  A[int64_t(comp) * a.n + p] = T(out);
}

template <typename T, int D>
hipError_t launch_tangent_TD(const KArgs& a, int depth, const r1_laminate* tree, void* A, hipStream_t st,
                             KTimer* tm) {
  dim3 blk(256), grd(unsigned((a.n + 255) / 256), D * D * D * D);
  if (tm) tm->begin("tangent", st);
  hipLaunchKernelGGL((k_tangent<T, D>), grd, blk, 0, st, a, depth, tree, static_cast<T*>(A));
  if (tm) tm->end(st);
  return hipGetLastError();
}

}  // namespace r1k

hipError_t r1_launch_tangent(const KArgs& a, int depth, int dtype, const r1_laminate* tree, void* A, hipStream_t st,
                             KTimer* tm) {
  if (dtype == R1_F32)
    return a.mat.dim == 2 ? r1k::launch_tangent_TD<float, 2>(a, depth, tree, A, st, tm)
                          : r1k::launch_tangent_TD<float, 3>(a, depth, tree, A, st, tm);
  return a.mat.dim == 2 ? r1k::launch_tangent_TD<double, 2>(a, depth, tree, A, st, tm)
                        : r1k::launch_tangent_TD<double, 3>(a, depth, tree, A, st, tm);
}
