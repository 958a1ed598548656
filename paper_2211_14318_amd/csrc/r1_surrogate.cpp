// Host side of the learned surrogate (C-ABI in include/r1.h): parameters and
// Adam state on the device, the training loop, the error-gate calibration and
// inference with fallback to plain lamination.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <vector>

#include "r1_check.hpp"
#include "r1_handle.hpp"
#include "r1_mlp.hpp"

struct r1_surrogate_s {
  int device = 0;
  int dim = 2, d_in = 5, d_out = 5, width = 128, n_hidden = 4;
  int64_t n_params = 0;
  std::vector<int64_t> off_w, off_b;        // per layer (n_hidden hidden + output)
  float* params = nullptr;                  // FP32 master weights
  float* grad = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  void* wbf = nullptr;                      // BF16 copies of the width x width layers
  void* wbf_t = nullptr;                    // ... and of their transposes (backward pass)
  void* wfrag = nullptr;                    // ... in MFMA fragment order (inference without LDS weights)
  bool wfrag_ok = false;                    // wfrag matches wbf
  int64_t t = 0;                            // Adam steps taken
  float norm[4 * kMaxCols] = {};            // x_mean, x_std, y_mean, y_std (packed by d_in/d_out)
  float x_lo[kMaxCols] = {}, x_hi[kMaxCols] = {};
  float det_lo = 0.0f;
  double r_max = 1.0, b_lo = 0.0, b_hi = 1.0;
  bool trained = false;
  int bins_on = 0;
  float gate_tau_h[kGateCells] = {};        // per gate cell: accept predicted gaps <= this
  float* gate_tau = nullptr;
  float* norm_dev = nullptr;                // device copy of norm
  void* ws = nullptr;                       // training / inference workspace
  size_t ws_bytes = 0;
  float check_eps = 0.0f;                   // a-posteriori check of served values (0: off)
};

namespace {

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

r1_status grow(r1_surrogate s, size_t bytes) {
  if (bytes <= s->ws_bytes) return R1_OK;
  if (s->ws) {
    if (hipDeviceSynchronize() != hipSuccess) return R1_EDEVICE;
    (void)hipFree(s->ws);
    s->ws = nullptr;
    s->ws_bytes = 0;
  }
  if (hipMalloc(&s->ws, bytes) != hipSuccess) {
    s->ws = nullptr;
    return R1_ENOMEM;
  }
  s->ws_bytes = bytes;
  return R1_OK;
}

void layout(r1_surrogate s) {
  s->off_w.assign(s->n_hidden + 1, 0);
  s->off_b.assign(s->n_hidden + 1, 0);
  int64_t o = 0;
  for (int l = 0; l <= s->n_hidden; ++l) {
    int n_in = l == 0 ? s->d_in : s->width;
    int n_out = l == s->n_hidden ? s->d_out : s->width;
    s->off_w[l] = o;
    o += int64_t(n_out) * n_in;
    s->off_b[l] = o;
    o += n_out;
  }
  s->n_params = o;
}

// BF16 weight block of hidden layer l (1 <= l < n_hidden)
void* wbf_of(r1_surrogate s, int l) {
  return static_cast<char*>(s->wbf) + size_t(l - 1) * s->width * s->width * 2;
}

// Adam step of lr (lr = 0: none) on the gradient in s->grad, which it clears,
// then the BF16 copies of the width x width layers from the master weights.
hipError_t adam_step(r1_surrogate s, float lr, float b1, float b2, float eps, hipStream_t st) {
  AdamArgs a{};
  a.n = s->n_params;
  a.p = s->params;
  a.g = s->grad;
  a.m = s->m;
  a.v = s->v;
  a.lr = lr;
  a.b1 = b1;
  a.b2 = b2;
  a.eps = eps;
  a.c1 = 1.0f - powf(b1, float(s->t));
  a.c2 = 1.0f - powf(b2, float(s->t));
  a.n_hidden = s->n_hidden;
  a.width = s->width;
  for (int l = 0; l <= s->n_hidden; ++l) a.off_w[l] = s->off_w[l];
  a.wbf = s->wbf;
  a.wbf_t = s->wbf_t;
  s->wfrag_ok = false;
  return r1m_train_adam(a, st);
}

// The fragment-order copy of the hidden weights, rebuilt after they changed.
// The rebuild is waited for: the copy is internal state that a later call on
// another stream reads without any ordering the caller could provide.
hipError_t ensure_wfrag(r1_surrogate s, hipStream_t st) {
  if (s->wfrag_ok) return hipSuccess;
  hipError_t e = r1m_wfrag(s->width, s->n_hidden, s->wbf, s->wfrag, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) s->wfrag_ok = true;
  return e;
}

hipError_t refresh_bf16(r1_surrogate s, hipStream_t st) { return adam_step(s, 0.0f, 0.9f, 0.999f, 1e-8f, st); }

r1_status alloc_state(r1_surrogate s) {
  size_t pb = sizeof(float) * size_t(s->n_params);
  if (hipMalloc(&s->params, pb) != hipSuccess || hipMalloc(&s->grad, pb) != hipSuccess ||
      hipMalloc(&s->m, pb) != hipSuccess || hipMalloc(&s->v, pb) != hipSuccess ||
      hipMalloc(&s->wbf, size_t(std::max(1, s->n_hidden - 1)) * s->width * s->width * 2) != hipSuccess ||
      hipMalloc(&s->wbf_t, size_t(std::max(1, s->n_hidden - 1)) * s->width * s->width * 2) != hipSuccess ||
      hipMalloc(&s->wfrag, size_t(std::max(1, s->n_hidden - 1)) * s->width * s->width * 2) != hipSuccess ||
      hipMalloc(&s->gate_tau, sizeof(float) * kGateCells) != hipSuccess ||
      hipMalloc(&s->norm_dev, sizeof(float) * 4 * kMaxCols) != hipSuccess)
    return R1_ENOMEM;
  if (hipMemset(s->m, 0, pb) != hipSuccess || hipMemset(s->v, 0, pb) != hipSuccess ||
      hipMemset(s->gate_tau, 0, sizeof(float) * kGateCells) != hipSuccess)
    return R1_EDEVICE;
  return R1_OK;
}

void free_state(r1_surrogate s) {
  for (void* p : {static_cast<void*>(s->params), static_cast<void*>(s->grad), static_cast<void*>(s->m),
                  static_cast<void*>(s->v), s->wbf, s->wbf_t, s->wfrag, static_cast<void*>(s->gate_tau),
                  static_cast<void*>(s->norm_dev), s->ws})
    if (p) (void)hipFree(p);
}

const float* xm(r1_surrogate s) { return s->norm; }
const float* xsd(r1_surrogate s) { return s->norm + s->d_in; }
const float* ym(r1_surrogate s) { return s->norm + 2 * s->d_in; }
const float* ysd(r1_surrogate s) { return s->norm + 2 * s->d_in + s->d_out; }

// Training workspace for batches of B rows (the buffers of TrainArgs).
struct TrainWs {
  float *Xb, *G, *Z, *loss, *part;
  void *Ht, *Dt;
};

r1_status train_ws(r1_surrogate s, int B, TrainWs* w) {
  const size_t lw = size_t(s->n_hidden) * size_t(B) * s->width;
  const size_t np = size_t(B / 32) * size_t(train_n_small(s->d_in, s->d_out, s->width, s->n_hidden));
  size_t bytes = al(sizeof(float) * size_t(B) * s->d_in) + al(sizeof(float) * size_t(B) * s->d_out) +
                 al(sizeof(float) * lw) + 2 * al(2 * lw) + al(256) + al(sizeof(float) * np);
  r1_status st = grow(s, bytes);
  if (st) return st;
  char* p = static_cast<char*>(s->ws);
  auto take = [&](size_t b) { char* q = p; p += al(b); return q; };
  w->Xb = reinterpret_cast<float*>(take(sizeof(float) * size_t(B) * s->d_in));
  w->G = reinterpret_cast<float*>(take(sizeof(float) * size_t(B) * s->d_out));
  w->Z = reinterpret_cast<float*>(take(sizeof(float) * lw));
  w->Ht = take(2 * lw);
  w->Dt = take(2 * lw);
  w->loss = reinterpret_cast<float*>(take(256));
  w->part = reinterpret_cast<float*>(take(sizeof(float) * np));
  return R1_OK;
}

// Arguments of one batch of B rows with the surrogate's weights and workspace.
TrainArgs batch_args(r1_surrogate s, int B, const TrainWs& w, float z_thr, float ew) {
  TrainArgs a{};
  a.B = B;
  a.d_in = s->d_in;
  a.d_out = s->d_out;
  a.width = s->width;
  a.n_hidden = s->n_hidden;
  a.params = s->params;
  for (int l = 0; l <= s->n_hidden; ++l) {
    a.off_w[l] = s->off_w[l];
    a.off_b[l] = s->off_b[l];
  }
  a.wbf = s->wbf;
  a.wbf_t = s->wbf_t;
  a.grad = s->grad;
  a.norm = s->norm_dev;
  a.z_thr = z_thr;
  a.margin = kHingeMargin;
  a.ew = ew;
  a.loss = w.loss;
  a.store = 1;
  a.Xb = w.Xb;
  a.G = w.G;
  a.Z = w.Z;
  a.Ht = w.Ht;
  a.Dt = w.Dt;
  a.part = w.part;
  return a;
}

uint64_t gcd64(uint64_t a, uint64_t b) {
  while (b) {
    uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

struct Rng {
  uint64_t s;
  uint64_t next() {
    s ^= s << 13;
    s ^= s >> 7;
    s ^= s << 17;
    return s;
  }
  double uni() { return double(next() >> 11) * (1.0 / 9007199254740992.0); }
};

InferParams infer_params(r1_surrogate s, const r1_material* mat, int64_t n) {
  InferParams ip{};
  ip.n = n;
  ip.width = s->width;
  ip.n_hidden = s->n_hidden;
  ip.mat = r1d::Material{mat->dim, mat->model, mat->mu, mat->lambda, mat->D_inf, mat->D0};
  ip.w0 = s->params + s->off_w[0];
  for (int l = 0; l < s->n_hidden; ++l) {
    ip.b[l] = s->params + s->off_b[l];
    ip.wbf[l] = l == 0 ? nullptr : wbf_of(s, l);
  }
  ip.wfrag = s->wfrag;
  ip.wout = s->params + s->off_w[s->n_hidden];
  ip.bout = s->params + s->off_b[s->n_hidden];
  for (int k = 0; k < s->d_in; ++k) {
    ip.x_mean[k] = xm(s)[k];
    ip.x_std[k] = xsd(s)[k];
    ip.x_lo[k] = s->x_lo[k];
    ip.x_hi[k] = s->x_hi[k];
  }
  for (int k = 0; k < s->d_out; ++k) {
    ip.y_mean[k] = ym(s)[k];
    ip.y_std[k] = ysd(s)[k];
  }
  ip.det_lo = s->det_lo;
  ip.r_max = s->r_max;
  ip.b_lo = s->b_lo;
  ip.b_hi = s->b_hi;
  ip.bins_on = s->bins_on;
  ip.gate_tau = s->gate_tau;
  return ip;
}

}  // namespace

extern "C" {

r1_status r1_surrogate_create(r1_handle h, r1_surrogate* out, int32_t dim, int32_t n_hidden,
                              int32_t width, uint64_t seed) {
  if (!h || !out) return R1_EINVAL;
  *out = nullptr;
  if ((dim != 2 && dim != 3) || n_hidden < 2 || n_hidden > kMaxHidden) return R1_EINVAL;
  if (width != 32 && width != 64 && width != 128 && width != 256) return R1_EINVAL;
  if (hipSetDevice(h->device) != hipSuccess) return R1_EDEVICE;
  r1_surrogate s = new (std::nothrow) r1_surrogate_s();
  if (!s) return R1_ENOMEM;
  s->device = h->device;
  s->dim = dim;
  s->d_in = dim * dim + 1;
  s->d_out = dim * dim + 1;
  s->width = width;
  s->n_hidden = n_hidden;
  layout(s);
  r1_status st = alloc_state(s);
  if (st) {
    free_state(s);
    delete s;
    return st;
  }
  // uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases
  std::vector<float> p(size_t(s->n_params), 0.0f);
  Rng rng{seed * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull};
  for (int l = 0; l <= n_hidden; ++l) {
    int n_in = l == 0 ? s->d_in : width;
    double bound = 1.0 / std::sqrt(double(n_in));
    for (int64_t k = s->off_w[l]; k < s->off_b[l]; ++k) p[k] = float((2.0 * rng.uni() - 1.0) * bound);
  }
  for (int k = 0; k < s->d_in; ++k) { s->norm[k] = 0.0f; s->norm[s->d_in + k] = 1.0f; }
  for (int k = 0; k < s->d_out; ++k) { s->norm[2 * s->d_in + k] = 0.0f; s->norm[2 * s->d_in + s->d_out + k] = 1.0f; }
  hipError_t e = hipMemcpy(s->params, p.data(), sizeof(float) * p.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = refresh_bf16(s, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_state(s);
    delete s;
    return R1_EDEVICE;
  }
  *out = s;
  return R1_OK;
}

r1_status r1_surrogate_destroy(r1_surrogate s) {
  if (!s) return R1_EINVAL;
  (void)hipSetDevice(s->device);
  (void)hipDeviceSynchronize();
  free_state(s);
  delete s;
  return R1_OK;
}

r1_status r1_surrogate_param_count(r1_surrogate s, int64_t* count) {
  if (!s || !count) return R1_EINVAL;
  *count = s->n_params;
  return R1_OK;
}

r1_status r1_surrogate_get_params(r1_surrogate s, float* params, int64_t count) {
  if (!s || !params || count != s->n_params) return R1_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return R1_EDEVICE;
  return hipMemcpy(params, s->params, sizeof(float) * size_t(count), hipMemcpyDeviceToHost) == hipSuccess
             ? R1_OK : R1_EDEVICE;
}

r1_status r1_surrogate_set_params(r1_surrogate s, const float* params, int64_t count) {
  if (!s || !params || count != s->n_params) return R1_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return R1_EDEVICE;
  hipError_t e = hipMemcpy(s->params, params, sizeof(float) * size_t(count), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = refresh_bf16(s, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  return e == hipSuccess ? R1_OK : R1_EDEVICE;
}

r1_status r1_surrogate_get_norm(r1_surrogate s, float* x_mean, float* x_std, float* y_mean, float* y_std) {
  if (!s) return R1_EINVAL;
  if (x_mean) std::memcpy(x_mean, xm(s), sizeof(float) * s->d_in);
  if (x_std) std::memcpy(x_std, xsd(s), sizeof(float) * s->d_in);
  if (y_mean) std::memcpy(y_mean, ym(s), sizeof(float) * s->d_out);
  if (y_std) std::memcpy(y_std, ysd(s), sizeof(float) * s->d_out);
  return R1_OK;
}

r1_status r1_surrogate_pack(r1_handle h, int32_t dim, int64_t n, r1_dtype dtype, const void* F,
                            const void* beta_n, const void* W, const void* P, float* X, float* Y,
                            void* stream) {
  if (!h || (dim != 2 && dim != 3) || n < 0 || (dtype != R1_F32 && dtype != R1_F64)) return R1_EINVAL;
  if (n == 0) return R1_OK;
  if (!F || !beta_n || !W || !P || !X || !Y) return R1_EINVAL;
  if (hipSetDevice(h->device) != hipSuccess) return R1_EDEVICE;
  hipError_t e = r1m_pack(dtype, dim, n, F, beta_n, W, P, X, Y, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? R1_OK : r1h::fail(h, e, "pack");
}

r1_status r1_surrogate_loss_grad(r1_handle h, r1_surrogate s, const float* Xn, const float* Yn, int64_t n,
                                 float* grad, float* loss, void* stream) {
  if (!h || !s || !Xn || !Yn || !grad || !loss) return R1_EINVAL;
  if (n < 32 || n % 32 != 0 || n > (1 << 24)) return R1_EINVAL;
  if (hipSetDevice(h->device) != hipSuccess) return R1_EDEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  TrainWs w;
  r1_status rs = train_ws(s, int(n), &w);
  if (rs) return rs;
  TrainArgs a = batch_args(s, int(n), w, -INFINITY, 1.0f);   // plain mean squared error
  a.mode = 0;
  a.Xn = Xn;
  a.Yn = Yn;
  hipError_t e = r1m_fill(s->n_params, s->grad, 0.0f, st);
  if (e == hipSuccess) e = r1m_fill(1, w.loss, 0.0f, st);
  if (e == hipSuccess) e = r1m_train_fwd(a, st);
  if (e == hipSuccess) e = r1m_train_bwd(a, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(grad, s->grad, sizeof(float) * size_t(s->n_params), hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(loss, w.loss, sizeof(float), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e == hipSuccess ? R1_OK : r1h::fail(h, e, "loss_grad");
}

r1_status r1_surrogate_train(r1_handle h, r1_surrogate s, const r1_material* mat, const float* X,
                             const float* Y, int64_t n, const r1_train_cfg* cfg, r1_train_report* report,
                             void* stream) {
  if (!h || !s || !X || !Y || !cfg) return R1_EINVAL;
  r1_status rs = r1h::check_material(mat);
  if (rs) return rs;
  if (mat->dim != s->dim) return R1_EINVAL;
  const int B = cfg->batch;
  if (B < 64 || B % 64 != 0 || B > (1 << 20) || cfg->epochs < 1 || !(cfg->lr > 0.0f)) return R1_EINVAL;
  if (!(cfg->energy_weight > 0.0f)) return R1_EINVAL;
  if (!(cfg->val_fraction >= 0.0f && cfg->val_fraction < 0.5f)) return R1_EINVAL;
  const int64_t n_val = int64_t(double(n) * cfg->val_fraction);
  const int64_t n_train = n - n_val;
  if (n_train < B) return R1_EINVAL;
  if (hipSetDevice(h->device) != hipSuccess) return R1_EDEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int DI = s->d_in, DO = s->d_out;

  // targets in gap form and their statistics, input statistics and box
  float* T = nullptr;
  double* sums = nullptr;
  float* mm = nullptr;
  if (hipMalloc(&T, sizeof(float) * size_t(n) * DO) != hipSuccess) return R1_ENOMEM;
  if (hipMalloc(&sums, sizeof(double) * 4 * kMaxCols) != hipSuccess ||
      hipMalloc(&mm, sizeof(float) * (4 * kMaxCols + 2)) != hipSuccess) {
    (void)hipFree(T);
    if (sums) (void)hipFree(sums);
    return R1_ENOMEM;
  }
  r1d::Material dm{mat->dim, mat->model, mat->mu, mat->lambda, mat->D_inf, mat->D0};
  hipError_t e = r1m_targets(s->dim, n, dm, X, Y, T, st);
  std::vector<float> init(4 * kMaxCols + 2);
  for (int k = 0; k < kMaxCols; ++k) {
    init[k] = INFINITY;                   // x min
    init[kMaxCols + k] = -INFINITY;       // x max
    init[2 * kMaxCols + k] = INFINITY;    // t min (unused)
    init[3 * kMaxCols + k] = -INFINITY;   // t max (unused)
  }
  init[4 * kMaxCols] = INFINITY;          // det min
  init[4 * kMaxCols + 1] = INFINITY;
  if (e == hipSuccess) e = hipMemsetAsync(sums, 0, sizeof(double) * 4 * kMaxCols, st);
  if (e == hipSuccess) e = hipMemcpyAsync(mm, init.data(), sizeof(float) * init.size(), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = r1m_colstats(n_train, DI, s->dim, X, sums, sums + kMaxCols, mm, mm + kMaxCols, mm + 4 * kMaxCols, st);
  if (e == hipSuccess)
    e = r1m_colstats(n_train, DO, 0, T, sums + 2 * kMaxCols, sums + 3 * kMaxCols, mm + 2 * kMaxCols,
                     mm + 3 * kMaxCols, mm + 4 * kMaxCols + 1, st);
  std::vector<double> hs(4 * kMaxCols);
  if (e == hipSuccess) e = hipMemcpyAsync(hs.data(), sums, sizeof(double) * hs.size(), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(init.data(), mm, sizeof(float) * init.size(), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(sums);
  (void)hipFree(mm);
  if (e != hipSuccess) {
    (void)hipFree(T);
    return r1h::fail(h, e, "train statistics");
  }
  auto msd = [&](int base, int k, float* mean, float* sd) {
    double mu = hs[base + k] / double(n_train);
    double var = hs[base + kMaxCols + k] / double(n_train) - mu * mu;
    *mean = float(mu);
    *sd = float(std::sqrt(std::max(var, 0.0)) + 1e-6);
  };
  for (int k = 0; k < DI; ++k) {
    msd(0, k, &s->norm[k], &s->norm[DI + k]);
    s->x_lo[k] = init[k];
    s->x_hi[k] = init[kMaxCols + k];
  }
  for (int k = 0; k < DO; ++k) msd(2 * kMaxCols, k, &s->norm[2 * DI + k], &s->norm[2 * DI + DO + k]);
  s->det_lo = init[4 * kMaxCols];
  // error-gate bins span the training box
  double r2 = 0.0;
  for (int i = 0; i < s->dim; ++i)
    for (int j = 0; j < s->dim; ++j) {
      int k = i * s->dim + j;
      double dev = std::max(std::fabs(double(s->x_lo[k]) - (i == j)), std::fabs(double(s->x_hi[k]) - (i == j)));
      r2 += dev * dev;
    }
  s->r_max = std::sqrt(r2) + 1e-9;
  s->b_lo = s->x_lo[DI - 1];
  s->b_hi = s->x_hi[DI - 1] + 1e-9;
  s->bins_on = 0;

  TrainWs w;
  rs = train_ws(s, B, &w);
  if (rs) {
    (void)hipFree(T);
    return rs;
  }
  e = hipMemcpyAsync(s->norm_dev, s->norm, sizeof(s->norm), hipMemcpyHostToDevice, st);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  Rng rng{cfg->seed * 0x2545F4914F6CDD1Dull + 1};
  const int64_t steps_per_epoch = n_train / B;
  const int64_t total_steps = steps_per_epoch * cfg->epochs;
  // standardized gap at which a row counts as not laminating (hinge target)
  const float z_thr = (kZeroGap - ym(s)[0]) / ysd(s)[0];
  float last_loss = 0.0f;
  int64_t steps = 0;
  TrainArgs ta = batch_args(s, B, w, z_thr, cfg->energy_weight);
  ta.mode = 1;
  ta.X = X;
  ta.T = T;
  ta.n_train = n_train;
  if (e == hipSuccess) e = r1m_fill(s->n_params, s->grad, 0.0f, st);   // each Adam step clears it again
  for (int ep = 0; ep < cfg->epochs && e == hipSuccess; ++ep) {
    uint64_t a;
    do {
      a = 1 + rng.next() % uint64_t(n_train);
    } while (gcd64(a, uint64_t(n_train)) != 1);
    uint64_t c = rng.next() % uint64_t(n_train);
    e = r1m_fill(1, w.loss, 0.0f, st);
    ta.a = a;
    ta.c = c;
    for (int64_t sidx = 0; sidx < steps_per_epoch && e == hipSuccess; ++sidx) {
      ta.step = sidx;
      e = r1m_train_fwd(ta, st);
      if (e == hipSuccess) e = r1m_train_bwd(ta, st);
      if (e == hipSuccess) {
        ++s->t;
        // cosine decay of the step size to 2% over this call's steps
        const double frac = double(steps) / double(std::max<int64_t>(total_steps - 1, 1));
        const float lr = float(cfg->lr * (0.02 + 0.98 * 0.5 * (1.0 + std::cos(M_PI * frac))));
        e = adam_step(s, lr, cfg->beta1, cfg->beta2, cfg->eps, st);
      }
      ++steps;
    }
    if (e == hipSuccess && ep == cfg->epochs - 1) {
      e = hipMemcpyAsync(&last_loss, w.loss, sizeof(float), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      last_loss /= float(std::max<int64_t>(steps_per_epoch, 1));
    }
  }
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  float val = 0.0f;
  if (e == hipSuccess && n_val >= 32) {
    // held-out loss in chunks of B rows (last partial chunk dropped to a multiple of 32)
    e = r1m_fill(1, w.loss, 0.0f, st);
    int64_t chunks = 0;
    for (int64_t r0 = n_train; r0 + 32 <= n && e == hipSuccess; r0 += B) {
      TrainArgs va = ta;
      va.B = int(std::min<int64_t>(B, n - r0) / 32 * 32);
      va.mode = 2;
      va.r0 = r0;
      va.store = 0;
      e = r1m_train_fwd(va, st);
      ++chunks;
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&val, w.loss, sizeof(float), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    val /= float(std::max<int64_t>(chunks, 1));
  }
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  (void)hipFree(T);
  if (e != hipSuccess) return r1h::fail(h, e, "train");
  s->trained = true;
  if (report) {
    report->steps = steps;
    report->train_loss = last_loss;
    report->val_loss = val;
    report->ms = ms;
  }
  return R1_OK;
}

r1_status r1_surrogate_predict(r1_handle h, r1_surrogate s, const r1_material* mat, const float* X, int64_t n,
                               int32_t* cell, float* W_pred, float* gap_pred, void* stream) {
  if (!h || !s || !X || !cell || !W_pred || !gap_pred || n < 1 || n >= (int64_t(1) << 31)) return R1_EINVAL;
  r1_status rs = r1h::check_material(mat);
  if (rs) return rs;
  if (mat->dim != s->dim) return R1_EINVAL;
  if (!s->trained) return R1_ENOTTRAINED;
  if (hipSetDevice(h->device) != hipSuccess) return R1_EDEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int dd = s->dim * s->dim;
  rs = grow(s, al(sizeof(float) * size_t(n) * dd) + al(sizeof(float) * size_t(n)));
  if (rs) return rs;
  char* p = static_cast<char*>(s->ws);
  float* Fs = reinterpret_cast<float*>(p); p += al(sizeof(float) * size_t(n) * dd);
  float* bs = reinterpret_cast<float*>(p);
  InferParams ip = infer_params(s, mat, n);
  hipError_t e = r1m_unpack(s->dim, n, X, Fs, bs, st);
  if (e == hipSuccess) e = ensure_wfrag(s, st);
  if (e == hipSuccess) e = r1m_infer(R1_F32, s->dim, ip, 1, Fs, bs, nullptr, nullptr, nullptr, nullptr, nullptr,
                                     cell, W_pred, gap_pred, st);
  return e == hipSuccess ? R1_OK : r1h::fail(h, e, "surrogate predict");
}

r1_status r1_surrogate_calibrate(r1_handle h, r1_surrogate s, const r1_material* mat, const float* X,
                                 const float* Y, int64_t n, float tol, float quantile, int32_t* cells_allowed,
                                 void* stream) {
  if (!h || !s || !X || !Y || n < 1 || !(tol > 0.0f) || !(quantile > 0.0f && quantile <= 1.0f))
    return R1_EINVAL;
  r1_status rs = r1h::check_material(mat);
  if (rs) return rs;
  if (mat->dim != s->dim) return R1_EINVAL;
  if (!s->trained) return R1_ENOTTRAINED;
  if (hipSetDevice(h->device) != hipSuccess) return R1_EDEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int dd = s->dim * s->dim;
  size_t bytes = al(sizeof(float) * size_t(n) * dd) + al(sizeof(float) * size_t(n)) + al(sizeof(int) * size_t(n)) +
                 2 * al(sizeof(float) * size_t(n));
  rs = grow(s, bytes);
  if (rs) return rs;
  char* p = static_cast<char*>(s->ws);
  float* Fs = reinterpret_cast<float*>(p); p += al(sizeof(float) * size_t(n) * dd);
  float* bs = reinterpret_cast<float*>(p); p += al(sizeof(float) * size_t(n));
  int* cbin = reinterpret_cast<int*>(p); p += al(sizeof(int) * size_t(n));
  float* cw = reinterpret_cast<float*>(p); p += al(sizeof(float) * size_t(n));
  float* cg = reinterpret_cast<float*>(p);
  InferParams ip = infer_params(s, mat, n);
  hipError_t e = r1m_unpack(s->dim, n, X, Fs, bs, st);
  if (e == hipSuccess) e = ensure_wfrag(s, st);
  if (e == hipSuccess) e = r1m_infer(R1_F32, s->dim, ip, 1, Fs, bs, nullptr, nullptr, nullptr, nullptr, nullptr,
                                     cbin, cw, cg, st);
  std::vector<int> hbin(static_cast<size_t>(n));
  std::vector<float> hw(static_cast<size_t>(n)), hg(static_cast<size_t>(n)), hy(size_t(n) * s->d_out);
  if (e == hipSuccess) e = hipMemcpyAsync(hbin.data(), cbin, sizeof(int) * hbin.size(), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(hw.data(), cw, sizeof(float) * hw.size(), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(hg.data(), cg, sizeof(float) * hg.size(), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(hy.data(), Y, sizeof(float) * hy.size(), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return r1h::fail(h, e, "calibrate");
  // per cell: calibration points ordered by predicted gap; the threshold is
  // the largest predicted gap whose prefix (all points at or below it) has at
  // least 16 points and at least the requested quantile of them within tol
  // (relative energy error, |W| floored at 1e-2)
  std::vector<std::vector<std::pair<float, bool>>> cell(kGateCells);
  for (int64_t i = 0; i < n; ++i) {
    if (hbin[i] < 0 || hbin[i] >= kGateCells) continue;
    const float ref = hy[size_t(i) * s->d_out];
    const float err = std::fabs(hw[i] - ref) / std::max(std::fabs(ref), 1e-2f);
    cell[hbin[i]].push_back({hg[i], err <= tol});
  }
  int allowed = 0;
  for (int c = 0; c < kGateCells; ++c) {
    auto& v = cell[c];
    std::sort(v.begin(), v.end(), [](const std::pair<float, bool>& x, const std::pair<float, bool>& y) {
      return x.first < y.first;
    });
    float tau = -INFINITY;
    int64_t good = 0;
    for (size_t k = 0; k < v.size(); ++k) {
      good += v[k].second ? 1 : 0;
      const int64_t cnt = int64_t(k) + 1;
      const bool boundary = k + 1 == v.size() || v[k + 1].first > v[k].first;
      if (boundary && cnt >= 16 && double(good) >= double(quantile) * double(cnt)) tau = v[k].first;
    }
    s->gate_tau_h[c] = tau;
    allowed += tau > -INFINITY ? 1 : 0;
  }
  e = hipMemcpy(s->gate_tau, s->gate_tau_h, sizeof(float) * kGateCells, hipMemcpyHostToDevice);
  if (e != hipSuccess) return r1h::fail(h, e, "calibrate upload");
  s->bins_on = 1;
  if (cells_allowed) *cells_allowed = allowed;
  return R1_OK;
}

r1_status r1_surrogate_infer(r1_handle h, r1_surrogate s, const r1_material* mat, const r1_lamination* fallback,
                             int64_t n, r1_dtype dtype, const void* F, const void* beta_n, void* W, void* P,
                             int32_t* flags, int64_t* n_fallback, void* stream) {
  if (!h || !s) return R1_EINVAL;
  r1_status rs = r1h::check_material(mat);
  if (rs) return rs;
  if (mat->dim != s->dim) return R1_EINVAL;
  rs = r1h::check_lamination(fallback);
  if (rs) return rs;
  if (dtype != R1_F32 && dtype != R1_F64) return R1_EINVAL;
  if (n < 0 || n >= (int64_t(1) << 31)) return R1_EINVAL;
  if (n == 0) {
    if (n_fallback) *n_fallback = 0;
    return R1_OK;
  }
  if (!F || !beta_n || !W || !P) return R1_EINVAL;
  if (!s->trained) return R1_ENOTTRAINED;
  if (hipSetDevice(h->device) != hipSuccess) return R1_EDEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int dd = s->dim * s->dim;
  const size_t ts = dtype == R1_F32 ? 4 : 8;
  // workspace: fallback count and list, then (with the check) the candidates'
  // count and list, then the per-point status the lists are built from; the
  // fallback's compact arrays reuse all but the fallback list after the check
  const bool check = s->check_eps > 0.0f;
  size_t bytes = al(sizeof(int)) + al(sizeof(int32_t) * size_t(n));
  if (check) bytes += al(sizeof(int)) + al(sizeof(int32_t) * size_t(n));
  bytes += al(size_t(n));                   // per-point status (the lists are built from it)
  rs = grow(s, bytes);
  if (rs) return rs;
  char* p = static_cast<char*>(s->ws);
  int* cnt = reinterpret_cast<int*>(p); p += al(sizeof(int));
  int32_t* list = reinterpret_cast<int32_t*>(p); p += al(sizeof(int32_t) * size_t(n));
  InferParams ip = infer_params(s, mat, n);
  CheckArgs ca{};
  if (check) {
    ip.cand_count = reinterpret_cast<int*>(p); p += al(sizeof(int));
    ip.cand_list = reinterpret_cast<int32_t*>(p);
    const r1_level* lvs[1] = {&fallback->level[0]};
    rs = r1h::device_levels(h, lvs, 1, s->dim, &ca.lv);
    if (rs) return rs;
    ca.n = n;
    ca.F = F;
    ca.beta_n = beta_n;
    ca.W = W;
    ca.mat = ip.mat;
    ca.eps = s->check_eps;
    ca.n_off = r1_check_offsets(fallback->level[0].n_t, ca.off);
    ca.list = ip.cand_list;
    ca.count = ip.cand_count;
    ca.fb_count = cnt;
    ca.fb_list = list;
    p += al(sizeof(int32_t) * size_t(n));
  }
  ip.status = reinterpret_cast<uint8_t*>(p);
  hipError_t e = hipMemsetAsync(cnt, 0, sizeof(int), st);
  if (e == hipSuccess && check) e = hipMemsetAsync(ip.cand_count, 0, sizeof(int), st);
  if (e == hipSuccess) e = ensure_wfrag(s, st);
  if (e == hipSuccess)
    e = r1m_infer(dtype, s->dim, ip, 0, F, beta_n, W, P, flags, cnt, list, nullptr, nullptr, nullptr, st);
  if (e == hipSuccess && check) e = r1_launch_check(dtype, ca, st);
  int nfb = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&nfb, cnt, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return r1h::fail(h, e, "surrogate infer");
  if (n_fallback) *n_fallback = nfb;
  if (nfb == 0) return R1_OK;
  // compact the fallback points, laminate them, scatter back
  size_t need = al(sizeof(int)) + al(sizeof(int32_t) * size_t(n)) + 2 * al(ts * size_t(nfb) * dd) +
                3 * al(ts * size_t(nfb)) + al(sizeof(int32_t) * size_t(nfb));
  if (need > s->ws_bytes) {
    // keep the list: copy it out, grow, copy back
    std::vector<int32_t> hl(static_cast<size_t>(nfb));
    e = hipMemcpy(hl.data(), list, sizeof(int32_t) * size_t(nfb), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return r1h::fail(h, e, "fallback list");
    rs = grow(s, need);
    if (rs) return rs;
    p = static_cast<char*>(s->ws);
    p += al(sizeof(int));
    list = reinterpret_cast<int32_t*>(p);
    e = hipMemcpy(list, hl.data(), sizeof(int32_t) * size_t(nfb), hipMemcpyHostToDevice);
    if (e != hipSuccess) return r1h::fail(h, e, "fallback list");
  }
  p = static_cast<char*>(s->ws) + al(sizeof(int)) + al(sizeof(int32_t) * size_t(n));
  void* Fc = p; p += al(ts * size_t(nfb) * dd);
  void* Pc = p; p += al(ts * size_t(nfb) * dd);
  void* bc = p; p += al(ts * size_t(nfb));
  void* Wc = p; p += al(ts * size_t(nfb));
  p += al(ts * size_t(nfb));
  int32_t* fc = reinterpret_cast<int32_t*>(p);
  e = r1m_fb_gather(dtype, s->dim, n, nfb, list, F, beta_n, Fc, bc, st);
  if (e != hipSuccess) return r1h::fail(h, e, "fallback gather");
  rs = r1_envelope_stress(h, mat, fallback, nfb, dtype, Fc, bc, Wc, Pc, nullptr, fc, stream);
  if (rs) return rs;
  e = r1m_fb_scatter(dtype, s->dim, n, nfb, list, Wc, Pc, fc, W, P, flags, st);
  return e == hipSuccess ? R1_OK : r1h::fail(h, e, "fallback scatter");
}

r1_status r1_surrogate_check_offsets(int32_t n_t, int32_t* offsets, int32_t* count) {
  if (!offsets || !count || n_t < 3 || n_t > R1_MAX_NT || (n_t % 2) == 0) return R1_EINVAL;
  int off[kCheckMaxOffsets];
  const int k = r1_check_offsets(n_t, off);
  for (int i = 0; i < k; ++i) offsets[i] = off[i];
  *count = k;
  return R1_OK;
}

r1_status r1_surrogate_set_check(r1_surrogate s, float eps) {
  if (!s || !(eps >= 0.0f) || !std::isfinite(eps)) return R1_EINVAL;
  s->check_eps = eps;
  return R1_OK;
}

r1_status r1_surrogate_save(r1_surrogate s, const char* path) {
  if (!s || !path) return R1_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return R1_EDEVICE;
  std::vector<float> p(size_t(s->n_params)), m(size_t(s->n_params)), v(size_t(s->n_params));
  size_t pb = sizeof(float) * p.size();
  if (hipMemcpy(p.data(), s->params, pb, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(m.data(), s->m, pb, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(v.data(), s->v, pb, hipMemcpyDeviceToHost) != hipSuccess)
    return R1_EDEVICE;
  FILE* f = std::fopen(path, "wb");
  if (!f) return R1_EIO;
  const char magic[8] = {'R', '1', 'S', 'U', 'R', 'R', '0', '2'};
  int32_t hdr[6] = {s->dim, s->n_hidden, s->width, s->bins_on, int32_t(s->trained), 0};
  bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof(hdr), 1, f) == 1 &&
            std::fwrite(&s->t, sizeof(s->t), 1, f) == 1 && std::fwrite(s->norm, sizeof(s->norm), 1, f) == 1 &&
            std::fwrite(s->x_lo, sizeof(s->x_lo), 1, f) == 1 && std::fwrite(s->x_hi, sizeof(s->x_hi), 1, f) == 1 &&
            std::fwrite(&s->det_lo, sizeof(s->det_lo), 1, f) == 1 && std::fwrite(&s->r_max, sizeof(double), 1, f) == 1 &&
            std::fwrite(&s->b_lo, sizeof(double), 1, f) == 1 && std::fwrite(&s->b_hi, sizeof(double), 1, f) == 1 &&
            std::fwrite(s->gate_tau_h, sizeof(s->gate_tau_h), 1, f) == 1 &&
            std::fwrite(p.data(), pb, 1, f) == 1 && std::fwrite(m.data(), pb, 1, f) == 1 &&
            std::fwrite(v.data(), pb, 1, f) == 1;
  ok = (std::fclose(f) == 0) && ok;
  return ok ? R1_OK : R1_EIO;
}

r1_status r1_surrogate_load(r1_handle h, r1_surrogate* out, const char* path) {
  if (!h || !out || !path) return R1_EINVAL;
  *out = nullptr;
  FILE* f = std::fopen(path, "rb");
  if (!f) return R1_EIO;
  char magic[8];
  int32_t hdr[6];
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "R1SURR02", 8) == 0 &&
            std::fread(hdr, sizeof(hdr), 1, f) == 1;
  r1_surrogate s = nullptr;
  if (ok) {
    r1_status rs = r1_surrogate_create(h, &s, hdr[0], hdr[1], hdr[2], 0);
    ok = rs == R1_OK;
  }
  if (ok) {
    std::vector<float> p(size_t(s->n_params)), m(size_t(s->n_params)), v(size_t(s->n_params));
    size_t pb = sizeof(float) * p.size();
    ok = std::fread(&s->t, sizeof(s->t), 1, f) == 1 && std::fread(s->norm, sizeof(s->norm), 1, f) == 1 &&
         std::fread(s->x_lo, sizeof(s->x_lo), 1, f) == 1 && std::fread(s->x_hi, sizeof(s->x_hi), 1, f) == 1 &&
         std::fread(&s->det_lo, sizeof(s->det_lo), 1, f) == 1 && std::fread(&s->r_max, sizeof(double), 1, f) == 1 &&
         std::fread(&s->b_lo, sizeof(double), 1, f) == 1 && std::fread(&s->b_hi, sizeof(double), 1, f) == 1 &&
         std::fread(s->gate_tau_h, sizeof(s->gate_tau_h), 1, f) == 1 &&
         std::fread(p.data(), pb, 1, f) == 1 && std::fread(m.data(), pb, 1, f) == 1 &&
         std::fread(v.data(), pb, 1, f) == 1;
    if (ok) {
      s->bins_on = hdr[3];
      s->trained = hdr[4] != 0;
      ok = hipMemcpy(s->params, p.data(), pb, hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(s->m, m.data(), pb, hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(s->v, v.data(), pb, hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(s->gate_tau, s->gate_tau_h, sizeof(s->gate_tau_h), hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(s->norm_dev, s->norm, sizeof(s->norm), hipMemcpyHostToDevice) == hipSuccess &&
           refresh_bf16(s, nullptr) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
    }
  }
  std::fclose(f);
  if (!ok) {
    if (s) r1_surrogate_destroy(s);
    return R1_EIO;
  }
  *out = s;
  return R1_OK;
}

}  // extern "C"
