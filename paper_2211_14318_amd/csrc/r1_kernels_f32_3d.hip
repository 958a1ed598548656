// Instantiation of the lamination kernels for float, 3x3 gradients (neo-Hooke damage and
// the double-well test energy).
#include "r1_batched_kernels.hpp"

hipError_t r1_launch_f32_3d(const KArgs& a, int depth, int S, int K, hipStream_t st, KTimer* tm) {
  return r1k::launch_TD<float, 3, r1d::kFamNH>(a, depth, S, K, st, tm);
}

hipError_t r1_launch_batched_f32_3d(const BArgs& b, int var, int kind, int grid, size_t lds, int* zero_p, int zero_n,
                                     hipStream_t st) {
  return r1k::launch_batched_TD<float, 3, r1d::kFamNH>(b, var, kind, grid, lds, zero_p, zero_n, st);
}

hipError_t r1_occupancy_batched_f32_3d(int var, int kind, size_t lds, int* blocks_per_cu) {
  return r1k::occupancy_batched_TD<float, 3, r1d::kFamNH>(var, kind, lds, blocks_per_cu);
}
