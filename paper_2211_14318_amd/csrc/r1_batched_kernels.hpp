// Persistent kernel for uneven batches: every point carries its own lamination
// (grid size, direction count, depth), all in one launch.
//
// Work items (planned and ordered on the host, largest first):
//   kind 0  up to 4 depth-1 points, one per wavefront of the block;
//   kind 1  one outer line (point, outer direction) of a depth-2 point, taken by
//           the whole block.  The block that finishes the last outer line of a
//           point (per-point counter, device-scope release/acquire) runs the
//           point's finalization: min over outer directions, stress, tree.
// Blocks pop items from a global counter until the list is exhausted, so every
// wave reaches the exit.  The innermost level's layout (lanes per line S,
// samples per lane K) is a per-table-entry variant chosen by the autotuner.
#pragma once
#include "r1_kernels.hpp"

struct BEntry {          // one lamination table entry on the device
  r1d::Level lv0, lv1;   // outermost (or only) level, inner level
  int depth;
  int var;               // layout variant of the innermost level
};

struct BArgs {
  KArgs base;              // n, F, beta_n, W, P, tree, flags, material, want_stress
  const BEntry* table;
  const int32_t* lam_idx;  // caller's per-point table index
  const int4* items;       // {kind, x, y, z}
  int n_items;
  int* counter;            // queue head, zeroed before each launch
  int* pdone;              // per point: finished outer lines, zeroed before each launch
  const int64_t* pbase;    // per point: first outer-result slot
  const int32_t* order;    // depth-1 points, grouped by the kind-0 items
  void* outer;             // per outer line: hull result
};

namespace r1k {

template <typename T, int D>
__device__ void b_point_depth1(int var, const KArgs& a, int64_t p, const Level& lv) {
  switch (var) {
#define X(V, S, K) case V: point_depth1<T, D, S, K>(a, p, lv); break;
    R1_BATCH_VARIANTS(X)
#undef X
    default: break;
  }
}

template <typename T, int D>
__device__ void b_outer_line(int var, const KArgs& a, int64_t p, int mo, const Level& lo,
                             const Level& li, OuterRes<T>* out, char* smem) {
  switch (var) {
#define X(V, S, K) case V: outer_line<T, D, S, K>(a, p, mo, lo, li, T(0), true, out, smem); break;
    R1_BATCH_VARIANTS(X)
#undef X
    default: break;
  }
}

template <typename T, int D>
__device__ void b_finalize(int var, const KArgs& a, int64_t p, const Level& lo, const Level& li,
                           const OuterRes<T>* res) {
  switch (var) {
#define X(V, S, K) case V: finalize_point<T, D, S, K>(a, p, lo, li, res); break;
    R1_BATCH_VARIANTS(X)
#undef X
    default: break;
  }
}

namespace {
__global__ void k_zero_ints(int* p, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0;
}
}  // namespace

template <typename T, int D>
__global__ __launch_bounds__(256) void k_batched(BArgs b) {
  extern __shared__ char smem_raw[];
  __shared__ int s_item, s_last;
  const KArgs& a = b.base;
  for (;;) {
    __syncthreads();                               // previous item done with s_item / LDS
    if (threadIdx.x == 0) s_item = atomicAdd(b.counter, 1);
    __syncthreads();
    const int it = s_item;
    if (it >= b.n_items) return;                   // block-uniform: every wave exits
    const int4 w = b.items[it];
    if (w.x == 0) {
      const int wave = threadIdx.x / kWave;
      if (wave < w.z) {
        const int64_t p = b.order[w.y + wave];
        const BEntry& e = b.table[b.lam_idx[p]];
        b_point_depth1<T, D>(e.var, a, p, e.lv0);
      }
    } else {
      const int64_t p = w.y;
      const int mo = w.z;
      const BEntry& e = b.table[b.lam_idx[p]];
      OuterRes<T>* res = static_cast<OuterRes<T>*>(b.outer) + b.pbase[p];
      // inadmissible or non-finite points skip the outer line; finalization reports them
      double F[D * D], bn;
      bool fin = load_point<T, D>(a, p, F, bn);
      Point<T> q = make_point<T>(a.mat, bn);
      double cof[D * D];
      cofactor<D>(F, cof);
      bool bad = !fin || !(w_point<T, D>(q, F, cof) < inf_v<T>());
      if (bad) {
        if (threadIdx.x == 0) res[mo] = OuterRes<T>{inf_v<T>(), 0, 0, 0};
      } else {
        b_outer_line<T, D>(e.var, a, p, mo, e.lv0, e.lv1, res + mo, smem_raw);
      }
      if (threadIdx.x == 0) {
        __threadfence();                           // release this line's result
        s_last = atomicAdd(&b.pdone[p], 1) == e.lv0.n_dir - 1;
      }
      __syncthreads();
      if (s_last) {
        __threadfence();                           // acquire the other lines' results
        if (threadIdx.x < kWave) b_finalize<T, D>(e.var, a, p, e.lv0, e.lv1, res);
      }
    }
  }
}

template <typename T, int D>
hipError_t launch_batched_TD(const BArgs& b, int grid, size_t lds, int zero_n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_ints, dim3(unsigned((zero_n + 255) / 256 < 1024 ? (zero_n + 255) / 256 : 1024)),
                     dim3(256), 0, st, b.counter, int64_t(zero_n));
  hipLaunchKernelGGL((k_batched<T, D>), dim3(unsigned(grid)), dim3(256), lds, st, b);
  return hipGetLastError();
}

template <typename T, int D>
hipError_t occupancy_batched_TD(size_t lds, int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batched<T, D>, 256, lds);
}

}  // namespace r1k
