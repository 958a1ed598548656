// Runtime dispatch of the lamination launches over (dtype, dimension).
#include "r1_launch.hpp"

hipError_t r1_launch_f32_2d(const KArgs& a, int depth, int S, int K, hipStream_t st, KTimer* tm);
hipError_t r1_launch_f32_3d(const KArgs& a, int depth, int S, int K, hipStream_t st, KTimer* tm);
hipError_t r1_launch_f64_2d(const KArgs& a, int depth, int S, int K, hipStream_t st, KTimer* tm);
hipError_t r1_launch_f64_3d(const KArgs& a, int depth, int S, int K, hipStream_t st, KTimer* tm);

hipError_t r1_launch_envelope(const KArgs& a, int depth, int dtype, int S, int K, hipStream_t st,
                              KTimer* tm) {
  if (dtype == R1_F32) return a.mat.dim == 2 ? r1_launch_f32_2d(a, depth, S, K, st, tm) : r1_launch_f32_3d(a, depth, S, K, st, tm);
  return a.mat.dim == 2 ? r1_launch_f64_2d(a, depth, S, K, st, tm) : r1_launch_f64_3d(a, depth, S, K, st, tm);
}

size_t r1_outer_res_bytes(int dtype) {
  // OuterRes<T>: {T h; int mp, mq, capped;}
  return dtype == R1_F32 ? 16 : 24;
}
