// Instantiation of the lamination kernels for float, 2x2 gradients.
#include "r1_kernels.hpp"

hipError_t r1_launch_f32_2d(const KArgs& a, int depth, int S, int K, hipStream_t st, KTimer* tm) {
  return r1k::launch_TD<float, 2>(a, depth, S, K, st, tm);
}
