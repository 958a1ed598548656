// Tangent moduli of the laminate: the third output of Algorithm 3 of arXiv
// 2211.14318, A^k = dP^k/dF, evaluated on a lamination tree that the envelope
// kernels (or a caller) wrote.  Along a rank-one line every laminate endpoint
// is a point of W, so A^k is the tree-weighted sum of the leaf moduli
// A^0 = d^2 W / dF dF (eq. 2.9), with the same weights as the stress P^k.
//
// The leaves are rebuilt with the envelope kernels' own line arithmetic, so
// they are the very points whose stress P^k was taken.  In 2D one thread per
// point forms each leaf's factors (J, ln J, psi0, damage factors) once for all
// 16 moduli; in 3D one thread per (point, row ij of A) forms them once per row.
// Consecutive threads are consecutive points, and the SoA output
// A[((i*d + j)*d*d + k*d + l) * n + p] is written coalesced.
#include "r1_kernels.hpp"

namespace r1k {

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

// Row ij of a node's moduli over its two leaves, weighted by w and added:
// acc += w (xi A0(G+) + (1 - xi) A0(G-)).
template <int D, int IJ>
__device__ __forceinline__ bool node_tangent(const Material& mat, double bn, const Level& lv, const r1_laminate& t,
                                             const double* G, double w, double* acc) {
  double Gm[D * D], Gp[D * D], xi;
  if (!node_split<D>(lv, t, G, Gm, Gp, xi)) return false;
  tangent0_row<D, IJ>(mat, bn, Gp, w * xi, acc);
  tangent0_row<D, IJ>(mat, bn, Gm, w * (1.0 - xi), acc);
  return true;
}

// All rows of a node's moduli over its two leaves, each leaf's factors formed
// once: acc[ij*D*D + kl] += w (xi A0(G+) + (1 - xi) A0(G-)).
template <int D>
__device__ __forceinline__ bool node_tangent_all(const Material& mat, double bn, const Level& lv,
                                                 const r1_laminate& t, const double* G, double w, double* acc) {
  double Gm[D * D], Gp[D * D], xi;
  if (!node_split<D>(lv, t, G, Gm, Gp, xi)) return false;
  leaf0_rows<D>(leaf0<D>(mat, bn, Gp), mat, Gp, w * xi, acc);
  leaf0_rows<D>(leaf0<D>(mat, bn, Gm), mat, Gm, w * (1.0 - xi), acc);
  return true;
}

// All of point p's moduli, A[(ij*d*d + kl) * n + p] (the 2D form: 16 values).
template <typename T, int D>
__device__ __forceinline__ void tangent_point_all(const KArgs& a, int depth, const r1_laminate* tree, T* A,
                                                  int64_t p) {
  constexpr int N4 = D * D * D * D;
  double F[D * D], bn;
  bool fin = load_point<T, D>(a, p, F, bn);
  double w = double(static_cast<const T*>(a.W)[p]);
  double acc[N4];
#pragma unroll
  for (int r = 0; r < N4; ++r) acc[r] = 0.0;
  bool ok = fin && isfinite(w);
  if (ok) {
    const r1_laminate* t = tree + p * R1_TREE_NODES;
    if (depth == 1) {
      ok = node_tangent_all<D>(a.mat, bn, a.lv0, t[0], F, 1.0, acc);
    } else {
      double Gm[D * D], Gp[D * D], xi;
      ok = node_split<D>(a.lv0, t[0], F, Gm, Gp, xi);
      ok = ok && node_tangent_all<D>(a.mat, bn, a.lv1, t[2], Gp, xi, acc);
      ok = ok && node_tangent_all<D>(a.mat, bn, a.lv1, t[1], Gm, 1.0 - xi, acc);
    }
  }
#pragma unroll
  for (int r = 0; r < N4; ++r) A[int64_t(r) * a.n + p] = T(ok ? acc[r] : __builtin_nan(""));
}

// Row IJ of point p's moduli, A[(IJ*d*d + kl) * n + p].
template <typename T, int D, int IJ>
__device__ __forceinline__ void tangent_point_row(const KArgs& a, int depth, const r1_laminate* tree, T* A,
                                                  int64_t p) {
  double F[D * D], bn;
  bool fin = load_point<T, D>(a, p, F, bn);
  double w = double(static_cast<const T*>(a.W)[p]);
  double acc[D * D];
#pragma unroll
  for (int kl = 0; kl < D * D; ++kl) acc[kl] = 0.0;
  bool ok = fin && isfinite(w);
  if (ok) {
    const r1_laminate* t = tree + p * R1_TREE_NODES;
    if (depth == 1) {
      ok = node_tangent<D, IJ>(a.mat, bn, a.lv0, t[0], F, 1.0, acc);
    } else {
      double Gm[D * D], Gp[D * D], xi;
      ok = node_split<D>(a.lv0, t[0], F, Gm, Gp, xi);
      ok = ok && node_tangent<D, IJ>(a.mat, bn, a.lv1, t[2], Gp, xi, acc);
      ok = ok && node_tangent<D, IJ>(a.mat, bn, a.lv1, t[1], Gm, 1.0 - xi, acc);
    }
  }
#pragma unroll
  for (int kl = 0; kl < D * D; ++kl)
    A[int64_t(IJ * D * D + kl) * a.n + p] = T(ok ? acc[kl] : __builtin_nan(""));
}

// 2D: one thread per point, every row.  3D: one thread per (point, row ij of
// A), blockIdx.y = ij (block-uniform; 81 accumulators per thread would not fit
// in registers): the row is a compile-time index, so every array access is
// static.
template <typename T, int D>
__global__ __launch_bounds__(256) void k_tangent(KArgs a, int depth, const r1_laminate* tree, T* A) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= a.n) return;
  if constexpr (D == 2) {
    tangent_point_all<T, D>(a, depth, tree, A, p);
    return;
  }
  switch (blockIdx.y) {
#define R1_ROW(R)                                                                   \
    case R:                                                                         \
      if constexpr (R < D * D) tangent_point_row<T, D, R>(a, depth, tree, A, p);    \
      break;
    R1_ROW(0) R1_ROW(1) R1_ROW(2) R1_ROW(3) R1_ROW(4) R1_ROW(5) R1_ROW(6) R1_ROW(7) R1_ROW(8)
#undef R1_ROW
    default: break;
  }
}

template <typename T, int D>
hipError_t launch_tangent_TD(const KArgs& a, int depth, const r1_laminate* tree, void* A, hipStream_t st,
                             KTimer* tm) {
  dim3 blk(256), grd(unsigned((a.n + 255) / 256), D == 2 ? 1 : D * D);
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
