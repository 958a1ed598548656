// r1_envelope_stress_noalloc: the envelope, stress and tree of r1_envelope_stress
// for callers that cannot allocate device memory.  Everything the launch needs
// beyond the caller's buffers -- the levels' directions, W^1 at each point and
// the per (point, outer direction) hull results of depth 2 -- lives in one
// file-scope device array of fixed size, reached through the address the runtime
// reports for it on each device.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>

#include "r1.h"
#include "r1_handle.hpp"
#include "r1_launch.hpp"

namespace {
constexpr size_t kNoAllocBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
}  // namespace

// One copy per device, held until the process ends.  Host code never passes
// this name to a kernel: it uses the device address looked up below.  The array
// has external linkage on purpose: with internal linkage the compiler keeps its
// device symbol local to the code object (absent from the dynamic symbol table),
// where the runtime's lookup by name cannot find it.
__device__ __align__(256) unsigned char r1_noalloc_scratch[kNoAllocBytes];

namespace {
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

// Device address of r1_noalloc_scratch on `device` (which must be current), looked up
// once per device and kept.
r1_status r1h::noalloc_scratch(int device, void** ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= kMaxDevices) return R1_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(r1_noalloc_scratch));
    if (e != hipSuccess || !p) return R1_EDEVICE;
    g_ptr[device] = p;
  }
  *ptr = g_ptr[device];
  return R1_OK;
}

size_t r1h::noalloc_capacity() { return kNoAllocBytes; }

extern "C" r1_status r1_envelope_stress_noalloc(r1_handle h, const r1_material* mat, const r1_lamination* lam,
                                                int64_t n, r1_dtype dtype, const void* F, const void* beta_n,
                                                void* W, void* P, r1_laminate* tree, int32_t* flags,
                                                void* stream) {
  if (!h) return R1_EINVAL;
  r1_status s = r1h::check_material(mat);
  if (s) return s;
  s = r1h::check_lamination(lam);
  if (s) return s;
  if (dtype != R1_F32 && dtype != R1_F64) return R1_EINVAL;
  if (n < 0 || n > (int64_t(1) << 31)) return R1_EINVAL;
  if (n == 0) return R1_OK;
  if (!F || !beta_n || !W) return R1_EINVAL;
  if (lam->depth == 2 && int64_t(n) * lam->level[0].n_dir > int64_t(0x7fffffff)) return R1_EINVAL;
  if (!h->noalloc) {
    h->err = "r1_envelope_stress_noalloc: the device address of the fixed workspace is unknown";
    return R1_EDEVICE;
  }
  const int dim = mat->dim;
  // workspace layout: per level a then b (n_dir x dim doubles each), then at
  // depth 2 W^1 per point and one hull result per (point, outer direction)
  size_t off_dir[R1_MAX_DEPTH], off = 0;
  for (int k = 0; k < lam->depth; ++k) {
    off_dir[k] = off;
    off += align256(2 * sizeof(double) * size_t(lam->level[k].n_dir) * size_t(dim));
  }
  const size_t ts = dtype == R1_F32 ? 4 : 8;
  const size_t off_w1f = off;
  if (lam->depth == 2) off += align256(ts * size_t(n));
  const size_t off_outer = off;
  if (lam->depth == 2) off += r1_outer_res_bytes(dtype) * size_t(n) * size_t(lam->level[0].n_dir);
  if (off > kNoAllocBytes) {
    h->err = "r1_envelope_stress_noalloc: needs " + std::to_string(off) + " bytes of workspace, the fixed limit is " +
             std::to_string(kNoAllocBytes);
    return R1_EINVAL;
  }
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return r1h::fail(h, e, "hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(h->noalloc);
  KArgs a{};
  a.n = n;
  a.F = F;
  a.beta_n = beta_n;
  a.W = W;
  a.P = P;
  a.tree = tree;
  a.flags = flags;
  a.want_stress = P != nullptr;
  a.mat = r1d::Material{mat->dim, mat->model, mat->mu, mat->lambda, mat->D_inf, mat->D0};
  for (int k = 0; k < lam->depth; ++k) {
    const r1_level& lv = lam->level[k];
    r1d::Level& dl = k == 0 ? a.lv0 : a.lv1;
    r1h::level_meta(lv, dim, &dl);
    const size_t bytes = sizeof(double) * size_t(lv.n_dir) * size_t(dim);
    double* da = reinterpret_cast<double*>(base + off_dir[k]);
    e = hipMemcpyAsync(da, lv.a, bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(da + size_t(lv.n_dir) * dim, lv.b, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return r1h::fail(h, e, "hipMemcpyAsync(directions)");
    dl.a = da;
    dl.b = da + size_t(lv.n_dir) * dim;
  }
  if (lam->depth == 2) {
    a.scratch_w1f = base + off_w1f;
    a.scratch_outer = base + off_outer;
  }
  const r1_level& inner = lam->level[lam->depth - 1];
  const int S = r1h::segment_width(h, inner.n_t, dtype, dim, lam->depth == 2 ? r1h::kRoleInner : r1h::kRoleLevel);
  const int K = r1h::samples_per_lane(S, inner.n_t);
  if (K == 0) return R1_EINVAL;
  e = r1_launch_envelope(a, lam->depth, dtype, S, K, st, nullptr);
  if (e != hipSuccess) return r1h::fail(h, e, "kernel launch");
  return R1_OK;
}
