// Host side of the C-ABI declared in include/r1.h: argument checks, the
// per-handle caches (direction tables on the device, scratch workspace,
// segment widths), and the launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "r1.h"
#include "r1_handle.hpp"
#include "r1_launch.hpp"

namespace {

uint64_t fnv1a(const void* p, size_t n, uint64_t h) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

}  // namespace

r1_status r1h::fail(r1_handle h, hipError_t e, const char* what) {
  if (h) {
    h->err = std::string(what) + ": " + hipGetErrorString(e);
  }
  return R1_EDEVICE;
}

r1_status r1h::check_material(const r1_material* m) {
  if (!m) return R1_EINVAL;
  if (m->dim != 2 && m->dim != 3) return R1_EINVAL;
  if (m->model != R1_NEOHOOKE_DAMAGE && m->model != R1_TEST_DOUBLEWELL && m->model != R1_STVK_DAMAGE)
    return R1_EINVAL;
  if (!std::isfinite(m->mu) || !std::isfinite(m->lambda) || !std::isfinite(m->D_inf) ||
      !std::isfinite(m->D0))
    return R1_EINVAL;
  if (m->model != R1_TEST_DOUBLEWELL && (!(m->D0 > 0.0) || m->D_inf < 0.0 || m->D_inf >= 1.0))
    return R1_EINVAL;
  return R1_OK;
}

r1_status r1h::check_level(const r1_level& lv) {
  if (lv.n_dir < 1 || lv.n_dir > R1_MAX_DIRS || !lv.a || !lv.b) return R1_EINVAL;
  if (lv.n_t < 3 || lv.n_t > R1_MAX_NT || (lv.n_t % 2) == 0) return R1_EINVAL;
  if (!std::isfinite(lv.tau) || !(lv.tau > 0.0)) return R1_EINVAL;
  return R1_OK;
}

r1_status r1h::check_lamination(const r1_lamination* lam) {
  if (!lam || lam->depth < 1 || lam->depth > R1_MAX_DEPTH) return R1_EINVAL;
  for (int k = 0; k < lam->depth; ++k) {
    r1_status s = check_level(lam->level[k]);
    if (s) return s;
  }
  return R1_OK;
}

// Host part of a level's device description: sizes, grid and |a|^2 |b|^2
// (the a, b pointers are filled by the caller).
void r1h::level_meta(const r1_level& lv, int dim, r1d::Level* out) {
  out->a = nullptr;
  out->b = nullptr;
  out->lay = nullptr;
  out->n_dir = lv.n_dir;
  out->n_t = lv.n_t;
  out->tau = lv.tau;
  // |a|^2 |b|^2 shared by every direction (unit directions: 1 up to rounding)
  // lets the kernels form the common part of the line polynomial once per point
  double ab0 = 0.0, dev = 0.0;
  for (int32_t m = 0; m < lv.n_dir; ++m) {
    double aa = 0.0, bb = 0.0;
    for (int i = 0; i < dim; ++i) {
      aa += lv.a[size_t(m) * dim + i] * lv.a[size_t(m) * dim + i];
      bb += lv.b[size_t(m) * dim + i] * lv.b[size_t(m) * dim + i];
    }
    if (m == 0) ab0 = aa * bb;
    dev = std::max(dev, std::fabs(aa * bb - ab0));
  }
  out->ab2 = (lv.n_dir > 0 && dev <= 8.0 * 2.220446049250313e-16 * ab0) ? ab0 : std::nan("");
}

namespace {

uint64_t level_key(const r1_level& lv, int dim) {
  size_t bytes = sizeof(double) * size_t(lv.n_dir) * size_t(dim);
  uint64_t key = 1469598103934665603ull;
  int32_t hdr[3] = {lv.n_dir, dim, lv.n_t};
  key = fnv1a(hdr, sizeof(hdr), key);
  key = fnv1a(&lv.tau, sizeof(lv.tau), key);
  key = fnv1a(lv.a, bytes, key);
  return fnv1a(lv.b, bytes, key);
}

}  // namespace

// Device copies of the directions of `count` levels, cached by content.  All
// levels of the call are looked up before anything is evicted, and eviction
// (when the cache would pass 512 entries) spares them, so no pointer handed out
// by this call is freed by it.  Only plain launches use these copies, and
// eviction waits for the device first; batched plans keep their own copies.
r1_status r1h::device_levels(r1_handle h, const r1_level* const* lv, int count, int dim, r1d::Level* out) {
  uint64_t keys[R1_MAX_DEPTH + 2];
  if (count < 1 || count > R1_MAX_DEPTH + 2) return R1_EINVAL;
  int missing = 0;
  for (int k = 0; k < count; ++k) {
    keys[k] = level_key(*lv[k], dim);
    missing += h->dirs.count(keys[k]) == 0;
  }
  if (missing && h->dirs.size() + size_t(missing) > 512) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return fail(h, e, "hipDeviceSynchronize");
    for (auto it = h->dirs.begin(); it != h->dirs.end();) {
      if (std::find(keys, keys + count, it->first) != keys + count) {
        ++it;
        continue;
      }
      (void)hipFree(it->second);
      it = h->dirs.erase(it);
    }
  }
  for (int k = 0; k < count; ++k) {
    const size_t bytes = sizeof(double) * size_t(lv[k]->n_dir) * size_t(dim);
    auto it = h->dirs.find(keys[k]);
    if (it == h->dirs.end()) {
      // a, b, then the lane-layout table of the level's grid
      void* d = nullptr;
      hipError_t e = hipMalloc(&d, 2 * bytes + r1d::kLayoutBytes);
      if (e != hipSuccess) return R1_ENOMEM;
      std::vector<double> host(2 * size_t(lv[k]->n_dir) * size_t(dim) + r1d::kLayoutBytes / sizeof(double));
      std::memcpy(host.data(), lv[k]->a, bytes);
      std::memcpy(host.data() + size_t(lv[k]->n_dir) * dim, lv[k]->b, bytes);
      r1d::layout_table(lv[k]->n_t, lv[k]->tau, host.data() + 2 * size_t(lv[k]->n_dir) * dim);
      e = hipMemcpy(d, host.data(), 2 * bytes + r1d::kLayoutBytes, hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        (void)hipFree(d);
        return fail(h, e, "hipMemcpy(directions)");
      }
      it = h->dirs.emplace(keys[k], d).first;
    }
    level_meta(*lv[k], dim, &out[k]);
    const double* base = static_cast<const double*>(it->second);
    out[k].a = base;
    out[k].b = base + size_t(lv[k]->n_dir) * dim;
    out[k].lay = base + 2 * size_t(lv[k]->n_dir) * dim;
  }
  return R1_OK;
}

r1_status r1h::scratch(r1_handle h, size_t bytes, void** p) {
  if (bytes > h->scratch_bytes) {
    if (h->scratch) {
      hipError_t e = hipDeviceSynchronize();
      if (e != hipSuccess) return fail(h, e, "hipDeviceSynchronize");
      (void)hipFree(h->scratch);
      h->scratch = nullptr;
      h->scratch_bytes = 0;
    }
    size_t sz = bytes + bytes / 4;
    if (hipMalloc(&h->scratch, sz) != hipSuccess) {
      h->scratch = nullptr;
      return R1_ENOMEM;
    }
    h->scratch_bytes = sz;
  }
  *p = h->scratch;
  return R1_OK;
}

// Samples per lane K for a segment of S lanes: the smallest power of two with
// S*K/2 >= c (one sample pair per offset on each side of the centre); for 16
// lanes also 14, which fits lines of 193..225 samples (the 201-sample ones)
// with 11% padding instead of 22%.
int r1h::samples_per_lane(int S, int n_t) {
  int c = (n_t - 1) / 2;
  for (int K = 2; K <= 32; K *= 2)
    if (S * K / 2 >= c) return (S == 16 && K == 16 && S * 14 / 2 >= c) ? 14 : K;
  return 0;
}

int r1h::segment_width(r1_handle h, int n_t, int dtype, int dim, int role) {
  auto it = h->seg_override.find(n_t);
  if (it != h->seg_override.end()) return it->second;
  auto jt = h->seg_tuned.find(r1h::tune_key(n_t, dtype, dim, role));
  if (jt != h->seg_tuned.end()) return jt->second;
  // default: about 16 samples per lane in FP32 and 8 in FP64, whose samples take
  // twice the registers (16 would cost the depth-2 outer kernel half its occupancy)
  const int c = (n_t - 1) / 2;
  const int pairs = dtype == R1_F64 ? 4 : 8;
  int S = 8;
  while (S < 64 && S * pairs < c) S *= 2;
  return S;
}

extern "C" {

r1_status r1_create(r1_handle* handle, int32_t device) {
  if (!handle) return R1_EINVAL;
  *handle = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return R1_EDEVICE;
  if (device < 0 || device >= count) return R1_EINVAL;
  e = hipSetDevice(device);
  if (e != hipSuccess) return R1_EDEVICE;
  r1_handle h = new (std::nothrow) r1_handle_s();
  if (!h) return R1_ENOMEM;
  h->device = device;
  // the fixed workspace of the allocation-free entry point, once per device
  if (r1h::noalloc_scratch(device, &h->noalloc) != R1_OK) {
    h->noalloc = nullptr;
    h->err = "hipGetSymbolAddress(fixed workspace) failed";
  }
  *handle = h;
  return R1_OK;
}

r1_status r1_destroy(r1_handle h) {
  if (!h) return R1_EINVAL;
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  (void)h->timer.collect();
  for (auto& kv : h->dirs) (void)hipFree(kv.second);
  if (h->scratch) (void)hipFree(h->scratch);
  r1h::release_batched(h);
  delete h;
  return R1_OK;
}

const char* r1_status_string(r1_status s) {
  switch (s) {
    case R1_OK: return "ok";
    case R1_EINVAL: return "invalid argument";
    case R1_ENOMEM: return "out of device memory";
    case R1_EDEVICE: return "device error";
    case R1_ENOTTRAINED: return "surrogate not trained";
    case R1_EUNSUPPORTED: return "unsupported";
    case R1_EIO: return "i/o error";
    default: return "unknown status";
  }
}

const char* r1_last_error(r1_handle h) { return h ? h->err.c_str() : ""; }

r1_status r1_set_segment_width(r1_handle h, int32_t n_t, int32_t lanes) {
  if (!h || n_t < 3 || n_t > R1_MAX_NT || (n_t % 2) == 0) return R1_EINVAL;
  if (lanes == 0) {
    h->seg_override.erase(n_t);
    return R1_OK;
  }
  if (lanes != 8 && lanes != 16 && lanes != 32 && lanes != 64) return R1_EINVAL;
  if (r1h::samples_per_lane(lanes, n_t) == 0) return R1_EINVAL;
  h->seg_override[n_t] = lanes;
  return R1_OK;
}

r1_status r1_get_segment_width(r1_handle h, int32_t n_t, r1_dtype dtype, int32_t dim, int32_t* lanes) {
  if (!h || !lanes || n_t < 3 || n_t > R1_MAX_NT || (n_t % 2) == 0) return R1_EINVAL;
  *lanes = r1h::segment_width(h, n_t, dtype, dim);
  return R1_OK;
}

static_assert(R1_TUNE_LEVEL == r1h::kRoleLevel && R1_TUNE_INNER == r1h::kRoleInner, "tuning roles");

r1_status r1_tuning_export(r1_handle h, int32_t* records, int32_t capacity, int32_t* count) {
  if (!h || !count || capacity < 0 || (capacity > 0 && !records)) return R1_EINVAL;
  int32_t k = 0;
  for (const auto& kv : h->seg_tuned) {
    if (k < capacity) {
      int32_t* r = records + 5 * size_t(k);
      r[0] = int32_t(kv.first >> 8);
      r[1] = int32_t((kv.first >> 4) & 3);
      r[2] = int32_t(kv.first & 15);
      r[3] = int32_t((kv.first >> 6) & 3);
      r[4] = kv.second;
    }
    ++k;
  }
  *count = k;
  return R1_OK;
}

r1_status r1_tuning_import(r1_handle h, const int32_t* records, int32_t count) {
  if (!h || count < 0 || (count > 0 && !records)) return R1_EINVAL;
  for (int32_t k = 0; k < count; ++k) {
    const int32_t* r = records + 5 * size_t(k);
    const int n_t = r[0], dtype = r[1], dim = r[2], role = r[3], lanes = r[4];
    if (n_t < 3 || n_t > R1_MAX_NT || n_t % 2 == 0 || (dtype != R1_F32 && dtype != R1_F64) ||
        (dim != 2 && dim != 3) || (role != R1_TUNE_LEVEL && role != R1_TUNE_INNER) ||
        (lanes != 8 && lanes != 16 && lanes != 32 && lanes != 64) || r1h::samples_per_lane(lanes, n_t) == 0)
      return R1_EINVAL;
  }
  for (int32_t k = 0; k < count; ++k) {
    const int32_t* r = records + 5 * size_t(k);
    h->seg_tuned[r1h::tune_key(r[0], r[1], r[2], r[3])] = r[4];
  }
  return R1_OK;
}

r1_status r1_get_inner_segment_width(r1_handle h, int32_t n_t, r1_dtype dtype, int32_t dim, int32_t* lanes) {
  if (!h || !lanes || n_t < 3 || n_t > R1_MAX_NT || (n_t % 2) == 0) return R1_EINVAL;
  *lanes = r1h::segment_width(h, n_t, dtype, dim, r1h::kRoleInner);
  return R1_OK;
}

}  // extern "C"

namespace {

// Kernel arguments shared by the envelope and tangent launches.
r1_status fill_args(r1_handle h, const r1_material* mat, const r1_lamination* lam, int64_t n, r1_dtype dtype,
                    const void* F, const void* beta_n, KArgs* a) {
  r1_status s = r1h::check_material(mat);
  if (s) return s;
  s = r1h::check_lamination(lam);
  if (s) return s;
  if (dtype != R1_F32 && dtype != R1_F64) return R1_EINVAL;
  if (n < 0 || n > (int64_t(1) << 31)) return R1_EINVAL;
  *a = KArgs{};
  a->n = n;
  a->F = F;
  a->beta_n = beta_n;
  a->mat = r1d::Material{mat->dim, mat->model, mat->mu, mat->lambda, mat->D_inf, mat->D0};
  if (n == 0) return R1_OK;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return r1h::fail(h, e, "hipSetDevice");
  const r1_level* lvs[2] = {&lam->level[0], &lam->level[1]};
  r1d::Level out[2];
  s = r1h::device_levels(h, lvs, lam->depth, mat->dim, out);
  if (s) return s;
  a->lv0 = out[0];
  if (lam->depth == 2) a->lv1 = out[1];
  return R1_OK;
}

// Envelope with optional stress, tree, flags and tangent moduli.  When the tree
// is needed (A != nullptr, or need_tree) and the caller passes none, it goes to
// workspace; *tree_used (nullable) receives the tree written.
r1_status envelope_impl(r1_handle h, const r1_material* mat, const r1_lamination* lam, int64_t n,
                        r1_dtype dtype, const void* F, const void* beta_n, void* W, void* P,
                        r1_laminate* tree, int32_t* flags, void* A, void* stream, bool need_tree = false,
                        r1_laminate** tree_used = nullptr) {
  if (!h) return R1_EINVAL;
  KArgs a;
  r1_status s = fill_args(h, mat, lam, n, dtype, F, beta_n, &a);
  if (s) return s;
  if (n == 0) return R1_OK;
  if (!F || !beta_n || !W) return R1_EINVAL;
  a.W = W;
  a.P = P;
  a.tree = tree;
  a.flags = flags;
  a.want_stress = P != nullptr;
  const r1_level& inner = lam->level[lam->depth - 1];
  size_t bytes = 0, w1 = 0;
  if (lam->depth == 2) {
    if (int64_t(n) * lam->level[0].n_dir > int64_t(0x7fffffff)) return R1_EINVAL;
    size_t tsz = dtype == R1_F32 ? 4 : 8;
    w1 = (tsz * size_t(n) + 255) & ~size_t(255);
    bytes = w1 + r1_outer_res_bytes(dtype) * size_t(n) * size_t(lam->level[0].n_dir);
  }
  size_t tree_off = (bytes + 255) & ~size_t(255);
  const bool tree_ws = (A || need_tree) && !tree;
  if (tree_ws) bytes = tree_off + sizeof(r1_laminate) * R1_TREE_NODES * size_t(n);
  if (bytes) {
    void* base = nullptr;
    s = r1h::scratch(h, bytes, &base);
    if (s) return s;
    if (lam->depth == 2) {
      a.scratch_w1f = base;
      a.scratch_outer = static_cast<char*>(base) + w1;
    }
    if (tree_ws) a.tree = reinterpret_cast<r1_laminate*>(static_cast<char*>(base) + tree_off);
  }
  if (tree_used) *tree_used = a.tree;
  int S = r1h::segment_width(h, inner.n_t, dtype, mat->dim, lam->depth == 2 ? r1h::kRoleInner : r1h::kRoleLevel);
  int K = r1h::samples_per_lane(S, inner.n_t);
  if (K == 0) return R1_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  KTimer* tm = h->timer.on ? &h->timer : nullptr;
  hipError_t e = r1_launch_envelope(a, lam->depth, dtype, S, K, st, tm);
  if (e != hipSuccess) return r1h::fail(h, e, "kernel launch");
  if (A) {
    e = r1_launch_tangent(a, lam->depth, dtype, a.tree, A, st, tm);
    if (e != hipSuccess) return r1h::fail(h, e, "kernel launch");
  }
  return R1_OK;
}

}  // namespace

extern "C" {

r1_status r1_envelope_stress(r1_handle h, const r1_material* mat, const r1_lamination* lam,
                             int64_t n, r1_dtype dtype, const void* F, const void* beta_n,
                             void* W, void* P, r1_laminate* tree, int32_t* flags, void* stream) {
  return envelope_impl(h, mat, lam, n, dtype, F, beta_n, W, P, tree, flags, nullptr, stream);
}

r1_status r1_envelope_tangent(r1_handle h, const r1_material* mat, const r1_lamination* lam,
                              int64_t n, r1_dtype dtype, const void* F, const void* beta_n,
                              void* W, void* P, void* A, r1_laminate* tree, int32_t* flags,
                              void* stream) {
  if (!A && n > 0) return R1_EINVAL;
  return envelope_impl(h, mat, lam, n, dtype, F, beta_n, W, P, tree, flags, A, stream);
}

r1_status r1_path_step(r1_handle h, const r1_material* mat, const r1_lamination* lam, int64_t n,
                       r1_dtype dtype, const void* F, void* beta, int32_t* fixed, void* W, void* P,
                       r1_laminate* tree, int32_t* flags, void* stream) {
  if (!h) return R1_EINVAL;
  if (n > 0 && (!beta || !fixed)) return R1_EINVAL;
  r1_laminate* used = nullptr;
  r1_status s = envelope_impl(h, mat, lam, n, dtype, F, beta, W, P, tree, flags, nullptr, stream, true, &used);
  if (s || n == 0) return s;
  const r1d::Material m{mat->dim, mat->model, mat->mu, mat->lambda, mat->D_inf, mat->D0};
  hipError_t e = r1_launch_path_update(dtype, n, F, W, used, beta, fixed, m, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return r1h::fail(h, e, "kernel launch");
  return R1_OK;
}

r1_status r1_laminate_tangent(r1_handle h, const r1_material* mat, const r1_lamination* lam,
                              int64_t n, r1_dtype dtype, const void* F, const void* beta_n,
                              const void* W, const r1_laminate* tree, void* A, void* stream) {
  if (!h) return R1_EINVAL;
  KArgs a;
  r1_status s = fill_args(h, mat, lam, n, dtype, F, beta_n, &a);
  if (s) return s;
  if (n == 0) return R1_OK;
  if (!F || !beta_n || !W || !tree || !A) return R1_EINVAL;
  a.W = const_cast<void*>(W);
  hipError_t e = r1_launch_tangent(a, lam->depth, dtype, tree, A, static_cast<hipStream_t>(stream),
                                   h->timer.on ? &h->timer : nullptr);
  if (e != hipSuccess) return r1h::fail(h, e, "kernel launch");
  return R1_OK;
}

r1_status r1_timing_enable(r1_handle h, int32_t on) {
  if (!h) return R1_EINVAL;
  h->timer.on = on != 0;
  return R1_OK;
}

r1_status r1_timing_reset(r1_handle h) {
  if (!h) return R1_EINVAL;
  hipError_t e = h->timer.collect();
  h->timer.acc.clear();
  return e == hipSuccess ? R1_OK : r1h::fail(h, e, "timing");
}

r1_status r1_timing_query(r1_handle h, const char* kernel, double* total_ms, int64_t* launches) {
  if (!h || !kernel || !total_ms || !launches) return R1_EINVAL;
  hipError_t e = h->timer.collect();
  if (e != hipSuccess) return r1h::fail(h, e, "timing");
  auto it = h->timer.acc.find(kernel);
  *total_ms = it == h->timer.acc.end() ? 0.0 : it->second.first;
  *launches = it == h->timer.acc.end() ? 0 : it->second.second;
  return R1_OK;
}

r1_status r1_envelope(r1_handle h, const r1_material* mat, const r1_lamination* lam, int64_t n,
                      r1_dtype dtype, const void* F, const void* beta_n, void* W, int32_t* flags,
                      void* stream) {
  return r1_envelope_stress(h, mat, lam, n, dtype, F, beta_n, W, nullptr, nullptr, flags, stream);
}

}  // extern "C"
