// Relax-then-fix driver of quadrature points (r1_path_step): one pseudo-time step
// of the procedure of the biaxial test of arXiv 2211.14318 (Section 6.6) with the
// damage history of Section 2, for a batch of points at once.
//
// The step's relaxed potential is the envelope of the plain lamination kernels,
// taken with the history entering the step as beta_n; this file holds what
// follows it: the state update.  A point whose envelope is not yet fixed and
// whose root laminate is a hull vertex (no lamination: the convex regime) takes
// the history max(beta, psi0(F)); one whose root laminates has reached the
// non-convex regime, and its envelope (the history it was taken with) is fixed
// from then on.  One thread per point; the reads and writes of consecutive
// threads are consecutive words.
#include <hip/hip_runtime.h>

#include "r1_handle.hpp"
#include "r1_kernels.hpp"

namespace {

// psi0 of the damage models in double (neo-Hooke eq. 2.3, plane strain in 2D;
// St. Venant-Kirchhoff eq. 2.2); NaN where neo-Hooke has det G <= 0.
template <int D>
__device__ __forceinline__ double psi0_of(const r1d::Material& m, const double* G) {
  if (m.model == R1_STVK_DAMAGE) {
    double S[D * D];
    return r1d::stvk_psi_stress<D>(m, G, S);
  }
  double cof[D * D];
  r1d::cofactor<D>(G, cof);
  const double J = r1d::det_of<D>(G, cof);
  if (!(J > 0.0)) return __builtin_nan("");
  const double lnJ = log(J);
  double n2 = 0.0;
#pragma unroll
  for (int i = 0; i < D * D; ++i) n2 += G[i] * G[i];
  return 0.5 * m.mu * (n2 - double(D)) - m.mu * lnJ + 0.5 * m.lambda * lnJ * lnJ;
}

template <typename T, int D>
__global__ __launch_bounds__(256) void k_path_update(int64_t n, const T* __restrict__ F, const T* __restrict__ W,
                                                     const r1_laminate* __restrict__ tree, T* __restrict__ beta,
                                                     int32_t* __restrict__ fixed, r1d::Material m) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  if (fixed[p] != 0) return;                           // fixed envelope: the state stays
  const T w = W[p];
  if (!(w < r1d::inf_v<T>())) return;                  // det F <= 0 or non-finite input (NaN fails too)
  const r1_laminate root = tree[p * R1_TREE_NODES];
  if (root.i_minus != root.i_plus) {                   // the non-convex regime is reached
    fixed[p] = 1;
    return;
  }
  if (m.model == R1_TEST_DOUBLEWELL) return;           // no damage, no history
  double G[D * D];
#pragma unroll
  for (int k = 0; k < D * D; ++k) G[k] = double(F[int64_t(k) * n + p]);
  const double psi = psi0_of<D>(m, G);
  const double b = double(beta[p]);
  if (psi > b) beta[p] = T(psi);
}

template <typename T, int D>
hipError_t launch_update(int64_t n, const void* F, const void* W, const r1_laminate* tree, void* beta,
                         int32_t* fixed, const r1d::Material& m, hipStream_t st) {
  const unsigned blocks = unsigned((n + 255) / 256);
  hipLaunchKernelGGL((k_path_update<T, D>), dim3(blocks), dim3(256), 0, st, n, static_cast<const T*>(F),
                     static_cast<const T*>(W), tree, static_cast<T*>(beta), fixed, m);
  return hipGetLastError();
}

}  // namespace

hipError_t r1_launch_path_update(int dtype, int64_t n, const void* F, const void* W, const r1_laminate* tree,
                                 void* beta, int32_t* fixed, const r1d::Material& m, hipStream_t st) {
  if (dtype == R1_F32)
    return m.dim == 2 ? launch_update<float, 2>(n, F, W, tree, beta, fixed, m, st)
                      : launch_update<float, 3>(n, F, W, tree, beta, fixed, m, st);
  return m.dim == 2 ? launch_update<double, 2>(n, F, W, tree, beta, fixed, m, st)
                    : launch_update<double, 3>(n, F, W, tree, beta, fixed, m, st);
}
