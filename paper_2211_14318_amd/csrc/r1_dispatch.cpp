// Runtime dispatch of the lamination launches over (dtype, dimension).
#include "r1_launch.hpp"

hipError_t r1_launch_f32_2d(const KArgs& a, int depth, int S, int K, hipStream_t st, KTimer* tm);
hipError_t r1_launch_f32_3d(const KArgs& a, int depth, int S, int K, hipStream_t st, KTimer* tm);
hipError_t r1_launch_f64_2d(const KArgs& a, int depth, int S, int K, hipStream_t st, KTimer* tm);
hipError_t r1_launch_f64_3d(const KArgs& a, int depth, int S, int K, hipStream_t st, KTimer* tm);
hipError_t r1_launch_stvk_f32_2d(const KArgs& a, int depth, int S, int K, hipStream_t st, KTimer* tm);
hipError_t r1_launch_stvk_f32_3d(const KArgs& a, int depth, int S, int K, hipStream_t st, KTimer* tm);
hipError_t r1_launch_stvk_f64_2d(const KArgs& a, int depth, int S, int K, hipStream_t st, KTimer* tm);
hipError_t r1_launch_stvk_f64_3d(const KArgs& a, int depth, int S, int K, hipStream_t st, KTimer* tm);

hipError_t r1_launch_envelope(const KArgs& a, int depth, int dtype, int S, int K, hipStream_t st,
                              KTimer* tm) {
  const bool d2 = a.mat.dim == 2;
  if (a.mat.model == R1_STVK_DAMAGE) {
    if (dtype == R1_F32) return d2 ? r1_launch_stvk_f32_2d(a, depth, S, K, st, tm) : r1_launch_stvk_f32_3d(a, depth, S, K, st, tm);
    return d2 ? r1_launch_stvk_f64_2d(a, depth, S, K, st, tm) : r1_launch_stvk_f64_3d(a, depth, S, K, st, tm);
  }
  if (dtype == R1_F32) return d2 ? r1_launch_f32_2d(a, depth, S, K, st, tm) : r1_launch_f32_3d(a, depth, S, K, st, tm);
  return d2 ? r1_launch_f64_2d(a, depth, S, K, st, tm) : r1_launch_f64_3d(a, depth, S, K, st, tm);
}

size_t r1_outer_res_bytes(int dtype) {
  // OuterRes<T>: {T h; int mp, mq, capped;}
  return dtype == R1_F32 ? 16 : 24;
}

struct BArgs;
hipError_t r1_launch_batched_f32_2d(const BArgs& b, int var, int kind, int grid, size_t lds, int* zero_p,
                                    int zero_n, hipStream_t st);
hipError_t r1_occupancy_batched_f32_2d(int var, int kind, size_t lds, int* blocks_per_cu);
hipError_t r1_launch_batched_f32_3d(const BArgs& b, int var, int kind, int grid, size_t lds, int* zero_p,
                                    int zero_n, hipStream_t st);
hipError_t r1_occupancy_batched_f32_3d(int var, int kind, size_t lds, int* blocks_per_cu);
hipError_t r1_launch_batched_f64_2d(const BArgs& b, int var, int kind, int grid, size_t lds, int* zero_p,
                                    int zero_n, hipStream_t st);
hipError_t r1_occupancy_batched_f64_2d(int var, int kind, size_t lds, int* blocks_per_cu);
hipError_t r1_launch_batched_f64_3d(const BArgs& b, int var, int kind, int grid, size_t lds, int* zero_p,
                                    int zero_n, hipStream_t st);
hipError_t r1_occupancy_batched_f64_3d(int var, int kind, size_t lds, int* blocks_per_cu);
hipError_t r1_launch_batched_stvk_f32_2d(const BArgs& b, int var, int kind, int grid, size_t lds, int* zero_p,
                                    int zero_n, hipStream_t st);
hipError_t r1_occupancy_batched_stvk_f32_2d(int var, int kind, size_t lds, int* blocks_per_cu);
hipError_t r1_launch_batched_stvk_f32_3d(const BArgs& b, int var, int kind, int grid, size_t lds, int* zero_p,
                                    int zero_n, hipStream_t st);
hipError_t r1_occupancy_batched_stvk_f32_3d(int var, int kind, size_t lds, int* blocks_per_cu);
hipError_t r1_launch_batched_stvk_f64_2d(const BArgs& b, int var, int kind, int grid, size_t lds, int* zero_p,
                                    int zero_n, hipStream_t st);
hipError_t r1_occupancy_batched_stvk_f64_2d(int var, int kind, size_t lds, int* blocks_per_cu);
hipError_t r1_launch_batched_stvk_f64_3d(const BArgs& b, int var, int kind, int grid, size_t lds, int* zero_p,
                                    int zero_n, hipStream_t st);
hipError_t r1_occupancy_batched_stvk_f64_3d(int var, int kind, size_t lds, int* blocks_per_cu);

#define R1_BATCHED_CALL(FAM, ...)                                                                  \
  (dtype == R1_F32 ? (dim == 2 ? r1_##FAM##_f32_2d(__VA_ARGS__) : r1_##FAM##_f32_3d(__VA_ARGS__))   \
                   : (dim == 2 ? r1_##FAM##_f64_2d(__VA_ARGS__) : r1_##FAM##_f64_3d(__VA_ARGS__)))

hipError_t r1_launch_batched(const BArgs& b, int dtype, int dim, int model, int var, int kind, int grid, size_t lds,
                             int* zero_p, int zero_n, hipStream_t st) {
  if (model == R1_STVK_DAMAGE) return R1_BATCHED_CALL(launch_batched_stvk, b, var, kind, grid, lds, zero_p, zero_n, st);
  return R1_BATCHED_CALL(launch_batched, b, var, kind, grid, lds, zero_p, zero_n, st);
}

hipError_t r1_occupancy_batched(int dtype, int dim, int model, int var, int kind, size_t lds, int* blocks_per_cu) {
  if (model == R1_STVK_DAMAGE) return R1_BATCHED_CALL(occupancy_batched_stvk, var, kind, lds, blocks_per_cu);
  return R1_BATCHED_CALL(occupancy_batched, var, kind, lds, blocks_per_cu);
}
#undef R1_BATCHED_CALL
