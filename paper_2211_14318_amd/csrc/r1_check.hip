// A-posteriori check of the surrogate's served values against lamination on a
// subset of the fallback's line samples.
//
// Every W^0 sample along a line of the fallback's outermost level is a sample of
// the lamination's hull problem, and fewer samples can only raise a hull
// (Algorithm 1 on a subset), so any chord of subset samples that passes below a
// served value w at the centre shows W^k < w there (for depth 2 as well:
// W^1 <= W^0 along the outer lines, so the outer hull over W^1 lies below the
// one over W^0).  A served value is rejected when such a chord passes more than
// eps max(|w|, 0.01) below it.  For a target T and samples at offsets +-o_k
// from the centre the test is O(n) per line (a chord between left sample i and
// right sample j passes below T at the centre iff (w_i - T)/o_i + (w_j - T)/o_j
// < 0), so the check needs only the smallest (w - T)/o on each side.  The
// subset: every sample within 8 of the centre, then offsets growing by about a
// third out to the line's end (bridges from a nearby sample to a far one are the
// laminates the network misses near the lamination boundary).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "r1_check.hpp"
#include "r1_kernels.hpp"

namespace {

// A sample in the form the chords are compared in: the damage energies in the
// hull form (W - B)/sc (sc > 0, so the sign of every chord test is kept when the
// target takes the same form), the double-well energy as it is.
template <typename T, int D, int M>
__device__ __forceinline__ float sample_at(float t, const r1d::Line<float>& L, const r1d::Point<float>& q) {
  if constexpr (M == r1d::kFamSTVK) return r1d::ws_sample_stvk<float>(t, L, q);
  return q.model == 0 ? r1d::ws_sample<float>(t, L, q) : r1d::w_sample_doublewell<float>(t, L);
}

// One direction's chord test for point p: true when a chord of subset samples
// passes below the target at the centre.
template <typename T, int D, int M>
__device__ __forceinline__ bool chord_below(const CheckArgs& a, const r1d::Point<float>& q, const double* G,
                                            const double* cof, float target, int m) {
  const r1d::Line<float> L = r1d::line_setup<float, D, M>(q, G, cof, a.lv.a + m * D, a.lv.b + m * D);
  float lo = __builtin_inff(), hi = __builtin_inff();
  for (int k = 0; k < a.n_off; ++k) {
    const float to = a.toff[k];
    const float inv = a.off_inv[k];
    // NaN samples (det <= 0) are absent: fminf keeps the other operand
    lo = fminf(lo, (sample_at<T, D, M>(-to, L, q) - target) * inv);
    hi = fminf(hi, (sample_at<T, D, M>(to, L, q) - target) * inv);
  }
  return lo + hi < 0.0f;
}

// A point passes when no subset chord of any direction passes below the target.
// NG lanes share a point (NG divides 64, so a group never spans two waves) and
// take its directions m = g, g + NG, ...: a point's direction loop is the chip's
// unit of parallel work, since the candidates are only the points the gates
// serve (a few tens of thousands for 3D workloads of 256 directions).  The loop
// bound is wave-uniform so that the group votes can use the whole wave; a group
// stops once one of its lanes has found a chord.
template <typename T, int D, int M, int NG>
__global__ __launch_bounds__(256) void k_check(CheckArgs a) {
  const int64_t total = a.list ? int64_t(*a.count) : a.n;
  const int lane = int(threadIdx.x) & 63;
  const int g = lane % NG;
  const uint64_t gmask = (NG == 64 ? ~uint64_t(0) : ((uint64_t(1) << NG) - 1)) << (lane - g);
  const int rounds = (a.lv.n_dir + NG - 1) / NG;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t w0 = int64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63u); w0 < total * NG; w0 += stride) {
    const int64_t i = (w0 + lane) / NG;
    const bool valid = i < total;
    const int64_t p = !valid ? 0 : a.list ? int64_t(a.list[i]) : i;
    double G[D * D], cof[D * D];
    r1d::Point<float> q{};
    float target = 0.0f;
    if (valid) {
#pragma unroll
      for (int k = 0; k < D * D; ++k) G[k] = double(static_cast<const T*>(a.F)[int64_t(k) * a.n + p]);
      const double bn = double(static_cast<const T*>(a.beta_n)[p]);
      const float w = float(static_cast<const T*>(a.W)[p]);
      r1d::cofactor<D>(G, cof);
      q = r1d::make_point<float, M>(a.mat, bn);
      target = w - a.eps * fmaxf(fabsf(w), 0.01f);
      if (M == r1d::kFamSTVK || q.model == 0) target = (target - q.B) / q.sc;
    }
    bool found = false, done = !valid;
    for (int r = 0; r < rounds; ++r) {
      const int m = r * NG + g;
      if (!done && m < a.lv.n_dir) found = chord_below<T, D, M>(a, q, G, cof, target, m);
      done = done || (__ballot(found) & gmask) != 0;
      if (__all(done)) break;
    }
    const bool fail = (__ballot(found) & gmask) != 0;
    if (valid && g == 0) {
      if (a.list) {
        if (fail) a.fb_list[atomicAdd(a.fb_count, 1)] = int32_t(p);
      } else {
        a.pass[p] = fail ? 0 : 1;
      }
    }
  }
}

template <typename T, int D, int NG>
hipError_t launch_TDG(const CheckArgs& a, hipStream_t st) {
  // list mode: n bounds the candidate count, which only the device knows
  const unsigned blocks = unsigned(std::min<int64_t>((a.n * NG + 255) / 256, 8192));
  if (a.mat.model == R1_STVK_DAMAGE)
    hipLaunchKernelGGL((k_check<T, D, r1d::kFamSTVK, NG>), dim3(blocks), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_check<T, D, r1d::kFamNH, NG>), dim3(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

// lanes per point: about four directions per lane, at least four lanes
template <typename T, int D>
hipError_t launch_TD(const CheckArgs& a, hipStream_t st) {
  if (a.lv.n_dir >= 256) return launch_TDG<T, D, 64>(a, st);
  if (a.lv.n_dir >= 64) return launch_TDG<T, D, 16>(a, st);
  return launch_TDG<T, D, 4>(a, st);
}

}  // namespace

int r1_check_offsets(int n_t, int* off) {
  const int c = (n_t - 1) / 2;
  int n = 0;
  for (int o = 1; o <= 8 && o <= c; ++o) off[n++] = o;
  int o = 8;
  while (o < c && n < kCheckMaxOffsets - 1) {
    o = std::max(o + 1, int(o * 1.3 + 0.5));
    if (o >= c) break;
    off[n++] = o;
  }
  if (off[n - 1] != c) off[n++] = c;
  return n;
}

hipError_t r1_launch_check(int dtype, const CheckArgs& args, hipStream_t st) {
  if (args.n <= 0) return hipSuccess;
  // the reciprocals of the offsets and their abscissae off[k] dt, once here
  // instead of per sample pair and direction in the kernel (IEEE float division
  // and product on both sides: the same bits)
  CheckArgs a = args;
  const float dt = float(a.lv.tau / double((a.lv.n_t - 1) / 2));
  for (int k = 0; k < a.n_off; ++k) {
    a.off_inv[k] = 1.0f / float(a.off[k]);
    a.toff[k] = float(a.off[k]) * dt;
  }
  if (dtype == R1_F32) return a.mat.dim == 2 ? launch_TD<float, 2>(a, st) : launch_TD<float, 3>(a, st);
  return a.mat.dim == 2 ? launch_TD<double, 2>(a, st) : launch_TD<double, 3>(a, st);
}
