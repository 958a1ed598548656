// Handle state and host helpers shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <set>
#include <string>

#include "r1.h"
#include "r1_device.hpp"
#include "r1_launch.hpp"

struct r1_batched_plan_s;

struct r1_handle_s {
  int device = 0;
  std::string err;
  std::map<uint64_t, void*> dirs;          // content hash -> device copy of a level's a, b
  void* scratch = nullptr;                 // grow-only workspace (depth-2 partial results)
  size_t scratch_bytes = 0;
  std::map<int, int> seg_override;         // n_t -> lanes per line (user setting)
  std::map<int64_t, int> seg_tuned;        // (n_t, dtype, dim, role) -> lanes per line (autotuner)
  std::map<uint64_t, r1_batched_plan_s*> plans;  // r1_envelope_batched: plans by content
  std::set<r1_batched_plan_s*> user_plans;        // plans created by r1_batched_plan_create
  KTimer timer;                            // optional per-kernel event timing
  hipStream_t capture_stream = nullptr;    // private stream for graph capture
  uint64_t plan_serial = 0;
  void* noalloc = nullptr;                 // device address of the fixed workspace (r1_envelope_stress_noalloc)
};

namespace r1h {
r1_status fail(r1_handle h, hipError_t e, const char* what);
r1_status check_material(const r1_material* m);
r1_status check_level(const r1_level& lv);
r1_status check_lamination(const r1_lamination* lam);
void level_meta(const r1_level& lv, int dim, r1d::Level* out);
r1_status device_levels(r1_handle h, const r1_level* const* lv, int count, int dim, r1d::Level* out);
r1_status scratch(r1_handle h, size_t bytes, void** p);
int samples_per_lane(int S, int n_t);
int batch_samples_per_lane(int S, int n_t);
// Roles of a level's lines for the segment width: lines of a one-level
// envelope (depth-1 points, and the two extra envelopes of a depth-2 point's
// stress), or the inner level of depth-2 points (sampled along outer lines).
constexpr int kRoleLevel = 0, kRoleInner = 1;
int segment_width(r1_handle h, int n_t, int dtype, int dim, int role = kRoleLevel);
inline int64_t tune_key(int n_t, int dtype, int dim, int role) {
  return (int64_t(n_t) << 8) | (role << 6) | (dtype << 4) | dim;
}
void release_batched(r1_handle h);
// Device address of the fixed workspace on `device` (current), looked up once per
// device; its size in bytes.
r1_status noalloc_scratch(int device, void** ptr);
size_t noalloc_capacity();
r1_status autotune(r1_handle h, const r1_material* mat, int n_t, int dtype, int dim, int role, hipStream_t st,
                   int* lanes);
}  // namespace r1h
