// Instantiation of the lamination kernels for double, 2x2 gradients, St. Venant-Kirchhoff
// damage model (eq. 2.2 with eq. 2.9).
#include "r1_batched_kernels.hpp"

hipError_t r1_launch_stvk_f64_2d(const KArgs& a, int depth, int S, int K, hipStream_t st, KTimer* tm) {
  return r1k::launch_TD<double, 2, r1d::kFamSTVK>(a, depth, S, K, st, tm);
}

hipError_t r1_launch_batched_stvk_f64_2d(const BArgs& b, int var, int kind, int grid, size_t lds, int* zero_p,
                                          int zero_n, hipStream_t st) {
  return r1k::launch_batched_TD<double, 2, r1d::kFamSTVK>(b, var, kind, grid, lds, zero_p, zero_n, st);
}

hipError_t r1_occupancy_batched_stvk_f64_2d(int var, int kind, size_t lds, int* blocks_per_cu) {
  return r1k::occupancy_batched_TD<double, 2, r1d::kFamSTVK>(var, kind, lds, blocks_per_cu);
}
