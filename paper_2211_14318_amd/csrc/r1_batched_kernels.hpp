// Persistent kernels for uneven batches: every point carries its own
// lamination (grid size, direction count, depth), all in one captured graph.
//
// The innermost level's layout (lanes per line S, samples per lane K) is a
// per-table-entry variant chosen by the autotuner.  For each variant present
// three kernels run in turn:
//   k_bpoint  (persistent) groups of up to 4 points, one per wavefront: the
//             full one-level result of depth-1 points, and W^1 at depth-2
//             points (the centre of their outer lines) into scratch;
//   k_bouter  (persistent) one outer line (point, outer direction) of a
//             depth-2 point per block, as in the plain depth-2 path;
//   k_bfinal  one wavefront per depth-2 point: min over outer directions,
//             stress, tree.
// Work lists are planned and ordered on the host (largest first).  Blocks of a
// persistent kernel pop items from a global counter until the list is
// exhausted, so every wave reaches the exit.  Separate kernels per variant and
// per kind keep each one at the register budget, and occupancy, of the plain
// kernel doing the same work.
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
  const int32_t* lam_idx;  // per-point table index: the plan's own copy
  const int4* items;       // this launch's work list (persistent kernels)
  int n_items;
  int* counter;            // this launch's queue head, zeroed before the launches
  const int32_t* order;    // point ids: groups of point items, depth-2 lists of k_bfinal
  const int64_t* pbase;    // per point: first outer-result slot
  void* outer;             // per outer line: hull result
  void* w1f;               // per point: W^1 at the point (depth-2 points)
};

// Batched launch kinds.
constexpr int kBPoint = 0, kBOuter = 1, kBFinal = 2;

namespace r1k {

namespace {
__global__ __attribute__((unused)) void k_zero_ints(int* p, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0;
}
}  // namespace

// Wave-uniform values as scalars, so the table entries and levels they index are
// loaded into SGPRs (a value read from LDS or memory is not known to be uniform).
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
  const uint64_t u = uint64_t(v);
  return int64_t(uint64_t(uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(u))))) |
                 (uint64_t(uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(u >> 32))))) << 32));
}

// Pops the next item of the block's persistent loop; block-uniform.
__device__ __forceinline__ int next_item(int* counter, int* s_item) {
  __syncthreads();                               // previous item done with s_item / LDS
  if (threadIdx.x == 0) *s_item = atomicAdd(counter, 1);
  __syncthreads();
  return uni(*s_item);
}

// items: {kind, first, count, 0} -- kind 0: depth-1 points order[first ..
// first + count), full result; kind 2: depth-2 points, W^1 into w1f.
template <typename T, int D, int S, int K, int M>
__global__ __launch_bounds__(256, (sizeof(T) == 4 && D == 2) ? 2 : 1) void k_bpoint(BArgs b) {
  __shared__ int s_item;
  for (;;) {
    const int it = next_item(b.counter, &s_item);
    if (it >= b.n_items) return;                 // block-uniform: every wave exits
    const int4 w = b.items[it];
    const int wave = uni(int(threadIdx.x / kWave));
    if (wave < uni(w.z)) {
      const int64_t p = uni(int64_t(b.order[uni(w.y) + wave]));
      const BEntry& e = b.table[uni(b.lam_idx[p])];
      const bool centre = uni(w.x) == 2;
      KArgs x = b.base;
      if (centre) {
        x.W = b.w1f;
        x.P = nullptr;
        x.tree = nullptr;
        x.flags = nullptr;
        x.want_stress = 0;
      }
      point_depth1<T, D, S, K, M>(x, p, centre ? e.lv1 : e.lv0);
    }
  }
}

// items: {1, point, outer direction, 0}.
template <typename T, int D, int S, int K, int M>
__global__ __launch_bounds__(256, (sizeof(T) == 4 && D == 2) ? (K <= 16 && M == kFamNH ? 3 : 2) : 1) void k_bouter(BArgs b) {
  extern __shared__ char smem_raw[];
  __shared__ int s_item;
  for (;;) {
    const int it = next_item(b.counter, &s_item);
    if (it >= b.n_items) return;                 // block-uniform: every wave exits
    const int4 w = b.items[it];
    const int64_t p = uni(w.y);
    const int mo = uni(w.z);
    const BEntry& e = b.table[uni(b.lam_idx[p])];
    OuterRes<T>* res = static_cast<OuterRes<T>*>(b.outer) + b.pbase[p] + mo;
    const T w1f = static_cast<const T*>(b.w1f)[p];
    if (!(w1f < inf_v<T>())) {                   // det F <= 0 or non-finite input: block-uniform
      if (threadIdx.x == 0) *res = OuterRes<T>{w1f, 0, 0, 0};
    } else {
      outer_line<T, D, S, K, M>(b.base, p, mo, e.lv0, e.lv1, w1f, false, res, smem_raw);
    }
  }
}

// One wavefront per depth-2 point order[0 .. n_items).
template <typename T, int D, int S, int K, int M>
__global__ __launch_bounds__(256) void k_bfinal(BArgs b) {
  const int64_t i = int64_t(blockIdx.x) * (blockDim.x / kWave) + uni(int(threadIdx.x / kWave));
  if (i >= b.n_items) return;                    // wave-uniform
  const int64_t p = uni(int64_t(b.order[i]));
  const BEntry& e = b.table[uni(b.lam_idx[p])];
  finalize_point<T, D, S, K, M>(b.base, p, e.lv0, e.lv1, static_cast<const OuterRes<T>*>(b.outer) + b.pbase[p]);
}

// Zeroes zero_n ints at zero_p (when zero_n > 0), then launches the kernel of
// the given kind for layout variant var on grid blocks.
template <typename T, int D, int M>
hipError_t launch_batched_TD(const BArgs& b, int var, int kind, int grid, size_t lds, int* zero_p,
                             int zero_n, hipStream_t st) {
  if (zero_n > 0)
    hipLaunchKernelGGL(k_zero_ints, dim3(unsigned((zero_n + 255) / 256 < 1024 ? (zero_n + 255) / 256 : 1024)),
                       dim3(256), 0, st, zero_p, int64_t(zero_n));
  switch (var) {
#define X(V, S, K)                                                                                   \
  case V:                                                                                            \
    if (kind == kBPoint)                                                                             \
      hipLaunchKernelGGL((k_bpoint<T, D, S, K, M>), dim3(unsigned(grid)), dim3(256), 0, st, b);          \
    else if (kind == kBOuter)                                                                        \
      hipLaunchKernelGGL((k_bouter<T, D, S, K, M>), dim3(unsigned(grid)), dim3(256), lds, st, b);        \
    else                                                                                             \
      hipLaunchKernelGGL((k_bfinal<T, D, S, K, M>), dim3(unsigned(grid)), dim3(256), 0, st, b);          \
    break;
    R1_BATCH_VARIANTS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Resident blocks per CU of a persistent kernel (kind kBPoint or kBOuter).
template <typename T, int D, int M>
hipError_t occupancy_batched_TD(int var, int kind, size_t lds, int* blocks_per_cu) {
  switch (var) {
#define X(V, S, K)                                                                                    \
  case V:                                                                                             \
    return kind == kBOuter                                                                            \
               ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_bouter<T, D, S, K, M>, 256, lds) \
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_bpoint<T, D, S, K, M>, 256, 0);
    R1_BATCH_VARIANTS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

}  // namespace r1k
