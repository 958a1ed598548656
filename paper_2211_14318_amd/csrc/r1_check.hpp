// Interface of the surrogate's a-posteriori check (r1_check.hip) for the
// surrogate host code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "r1.h"
#include "r1_device.hpp"

constexpr int kCheckMaxOffsets = 32;

struct CheckArgs {
  int64_t n;                   // points of F, beta_n, W (SoA), and rows of pass
  const void* F;
  const void* beta_n;
  const void* W;               // the values to check (served by the network)
  r1d::Material mat;
  r1d::Level lv;               // the fallback's outermost level (device directions)
  float eps;                   // reject when a chord passes eps max(|W|, 0.01) below W
  int n_off;
  int off[kCheckMaxOffsets];   // sample offsets from the centre, on the level's grid
  float off_inv[kCheckMaxOffsets];   // 1 / off[k] (set by r1_launch_check)
  float toff[kCheckMaxOffsets];      // off[k] dt, the offsets' abscissae (set by r1_launch_check)
  const int32_t* list;         // list mode: candidate points list[0 .. *count)
  const int* count;
  int* fb_count;               // list mode: failures appended here
  int32_t* fb_list;
  uint8_t* pass;               // row mode: 1 where row p passes
};

// Offsets of the subset for lines of n_t points (at most kCheckMaxOffsets);
// returns their number.
int r1_check_offsets(int n_t, int* off);
hipError_t r1_launch_check(int dtype, const CheckArgs& a, hipStream_t st);
