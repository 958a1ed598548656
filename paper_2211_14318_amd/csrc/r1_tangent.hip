// Tangent moduli of the laminate: the third output of Algorithm 3 of arXiv
// 2211.14318, A^k = dP^k/dF, evaluated on a lamination tree that the envelope
// kernels (or a caller) wrote.  Along a rank-one line every laminate endpoint
// is a point of W, so A^k is the tree-weighted sum of the leaf moduli
// A^0 = d^2 W / dF dF (eq. 2.9), with the same weights as the stress P^k.
//
// The leaves are rebuilt with the envelope kernels' own line arithmetic, so
// they are the very points whose stress P^k was taken.  In 2D one thread per
// point forms each leaf's factors (J, ln J, psi0, damage factors) once for all
// 16 moduli; in 3D one thread per (point, i) forms them once for the 27 moduli
// of rows 3i .. 3i + 2.
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

// Rows R0 .. R1 - 1 of a node's moduli over its two leaves, each leaf's factors
// formed once: acc[(ij - R0)*D*D + kl] += w (xi A0(G+) + (1 - xi) A0(G-)).
template <int D, int R0, int R1>
__device__ __forceinline__ bool node_tangent_rows(const Material& mat, double bn, const Level& lv,
                                                  const r1_laminate& t, const double* G, double w, double* acc) {
  double Gm[D * D], Gp[D * D], xi;
  if (!node_split<D>(lv, t, G, Gm, Gp, xi)) return false;
  leaf0_rows<D, R0, R1>(leaf0<D>(mat, bn, Gp), mat, Gp, w * xi, acc);
  leaf0_rows<D, R0, R1>(leaf0<D>(mat, bn, Gm), mat, Gm, w * (1.0 - xi), acc);
  return true;
}

// Rows R0 .. R1 - 1 of point p's moduli, A[(ij*d*d + kl) * n + p].
template <typename T, int D, int R0, int R1>
__device__ __forceinline__ void tangent_point_rows(const KArgs& a, int depth, const r1_laminate* tree, T* A,
                                                   int64_t p) {
  constexpr int NV = (R1 - R0) * D * D;
  double F[D * D], bn;
  bool fin = load_point<T, D>(a, p, F, bn);
  double w = double(static_cast<const T*>(a.W)[p]);
  double acc[NV];
#pragma unroll
  for (int r = 0; r < NV; ++r) acc[r] = 0.0;
  bool ok = fin && isfinite(w);
  if (ok) {
    const r1_laminate* t = tree + p * R1_TREE_NODES;
    if (depth == 1) {
      ok = node_tangent_rows<D, R0, R1>(a.mat, bn, a.lv0, t[0], F, 1.0, acc);
    } else {
      double Gm[D * D], Gp[D * D], xi;
      ok = node_split<D>(a.lv0, t[0], F, Gm, Gp, xi);
      ok = ok && node_tangent_rows<D, R0, R1>(a.mat, bn, a.lv1, t[2], Gp, xi, acc);
      ok = ok && node_tangent_rows<D, R0, R1>(a.mat, bn, a.lv1, t[1], Gm, 1.0 - xi, acc);
    }
  }
#pragma unroll
  for (int r = 0; r < NV; ++r) A[int64_t(R0 * D * D + r) * a.n + p] = T(ok ? acc[r] : __builtin_nan(""));
}

// 2D: one thread per point, all 16 moduli.  3D: one thread per (point, i), the
// 27 moduli of rows ij = 3i .. 3i + 2, blockIdx.y = i (block-uniform; all 81
// accumulators in one thread would not fit in registers).  The rows are
// compile-time indices, so every array access is static.
template <typename T, int D>
__global__ __launch_bounds__(256) void k_tangent(KArgs a, int depth, const r1_laminate* tree, T* A) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= a.n) return;
  if constexpr (D == 2) {
    tangent_point_rows<T, D, 0, 4>(a, depth, tree, A, p);
  } else {
    switch (blockIdx.y) {
      case 0: tangent_point_rows<T, D, 0, 3>(a, depth, tree, A, p); break;
      case 1: tangent_point_rows<T, D, 3, 6>(a, depth, tree, A, p); break;
      default: tangent_point_rows<T, D, 6, 9>(a, depth, tree, A, p); break;
    }
  }
}

template <typename T, int D>
hipError_t launch_tangent_TD(const KArgs& a, int depth, const r1_laminate* tree, void* A, hipStream_t st,
                             KTimer* tm) {
  dim3 blk(256), grd(unsigned((a.n + 255) / 256), D == 2 ? 1 : D);
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
