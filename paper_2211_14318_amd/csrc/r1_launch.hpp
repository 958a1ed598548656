// Launch interface between the host C-ABI (r1_api.cpp) and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "r1.h"
#include "r1_device.hpp"

struct KArgs {
  int64_t n;
  const void* F;          // T[(d*d) * n], SoA
  const void* beta_n;     // T[n]
  void* W;                // T[n]
  void* P;                // T[(d*d) * n] or null
  r1_laminate* tree;      // [n * R1_TREE_NODES] or null
  int32_t* flags;         // [n] or null
  r1d::Material mat;
  r1d::Level lv0;         // outermost (or only) level
  r1d::Level lv1;         // inner level (depth 2)
  int want_stress;
  void* scratch_w1f;      // depth 2: T[n], W^1 at each point
  void* scratch_outer;    // depth 2: per (point, outer direction) hull result
  int pts_per_wave;       // one-level kernel: points per wave (set by the launcher)
};

// Per-kernel timing with HIP events recorded on the launch stream (off by default).
struct KTimer {
  bool on = false;
  struct Rec {
    const char* name;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  std::map<std::string, std::pair<double, int64_t>> acc;   // name -> (total ms, launches)
  void begin(const char* name, hipStream_t st) {
    if (!on) return;
    Rec r{name, nullptr, nullptr};
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return;
    (void)hipEventRecord(r.a, st);
    pending.push_back(r);
  }
  void end(hipStream_t st) {
    if (!on || pending.empty()) return;
    (void)hipEventRecord(pending.back().b, st);
  }
  hipError_t collect() {
    hipError_t err = hipSuccess;
    for (auto& r : pending) {
      hipError_t e = hipEventSynchronize(r.b);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
      if (e != hipSuccess) err = e;
      auto& x = acc[r.name];
      x.first += ms;
      x.second += 1;
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    pending.clear();
    return err;
  }
};

// depth 1 or 2; S = lanes per line of the innermost level, K = samples per lane.
hipError_t r1_launch_envelope(const KArgs& a, int depth, int dtype, int S, int K, hipStream_t st,
                              KTimer* tm);
size_t r1_outer_res_bytes(int dtype);
// Tangent moduli A (d^4 x n SoA) by Algorithm 3 on tree[n * R1_TREE_NODES] for the
// levels a.lv0 (and a.lv1 at depth 2); reads a.F, a.beta_n and a.W (A is NaN
// where W is not finite or a tree node does not name a laminate of its level).
hipError_t r1_launch_tangent(const KArgs& a, int depth, int dtype, const r1_laminate* tree, void* A, hipStream_t st,
                             KTimer* tm);

// State update of the relax-then-fix driver after the step's envelope (r1_path_step):
// per point, fix the envelope where the root laminate laminates, else raise the
// history beta to psi0(F); points already fixed and points with W not finite keep
// their state.
hipError_t r1_launch_path_update(int dtype, int64_t n, const void* F, const void* W, const r1_laminate* tree,
                                 void* beta, int32_t* fixed, const r1d::Material& m, hipStream_t st);

struct BArgs;
// Uneven-batch kernel of the given kind (kBPoint, kBOuter, kBFinal) for layout
// variant var of the material model's kernels on `grid` blocks with `lds` bytes
// of dynamic LDS, preceded by zeroing zero_n ints at zero_p when zero_n > 0.
hipError_t r1_launch_batched(const BArgs& b, int dtype, int dim, int model, int var, int kind, int grid, size_t lds,
                             int* zero_p, int zero_n, hipStream_t st);
hipError_t r1_occupancy_batched(int dtype, int dim, int model, int var, int kind, size_t lds, int* blocks_per_cu);
// Layout variants of the persistent kernel, (variant, S, K): lanes per line and
// samples per lane of the innermost level.
#define R1_BATCH_VARIANTS(X) \
  X(0, 16, 4) X(1, 16, 8) X(2, 8, 32) X(3, 16, 16) X(4, 32, 8) X(5, 64, 4) \
  X(6, 16, 32) X(7, 32, 16) X(8, 64, 8) X(9, 32, 32) X(10, 64, 16) X(11, 64, 32)

// Number of layout variants.
constexpr int R1_N_BATCH_VARIANTS = 0
#define X(V, SS, KK) + 1
    R1_BATCH_VARIANTS(X)
#undef X
    ;

// Variant index of (S, K), or -1.
inline int r1_batch_variant(int S, int K) {
#define X(V, SS, KK) if (S == SS && K == KK) return V;
  R1_BATCH_VARIANTS(X)
#undef X
  return -1;
}
