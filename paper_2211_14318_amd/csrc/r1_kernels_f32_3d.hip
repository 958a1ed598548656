// Instantiation of the lamination kernels for float, 3x3 gradients.
#include "r1_kernels.hpp"

hipError_t r1_launch_f32_3d(const KArgs& a, int depth, int S, int K, hipStream_t st, KTimer* tm) {
  return r1k::launch_TD<float, 3>(a, depth, S, K, st, tm);
}
