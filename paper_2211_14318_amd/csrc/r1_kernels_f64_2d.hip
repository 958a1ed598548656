// Instantiation of the lamination kernels for double, 2x2 gradients.
#include "r1_kernels.hpp"

hipError_t r1_launch_f64_2d(const KArgs& a, int depth, int S, int K, hipStream_t st, KTimer* tm) {
  return r1k::launch_TD<double, 2>(a, depth, S, K, st, tm);
}
