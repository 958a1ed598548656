// Host side of the uneven batch (r1_envelope_batched): the planner that turns
// the per-point table indices into an ordered work list, the captured HIP graph
// that replays the persistent launch, and the segment-width autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "r1_batched_kernels.hpp"
#include "r1_handle.hpp"

struct BatchedPlan {
  uint64_t key = 0;
  uint64_t serial = 0;
  void* dev = nullptr;          // table, items, order, pbase, counters, outer results
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t n_items = 0;
  int64_t n_outer = 0;
};

namespace {

uint64_t mix(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

template <typename V>
uint64_t mixv(uint64_t h, const V& v) { return mix(h, &v, sizeof(v)); }

void free_plan(BatchedPlan* pl) {
  if (!pl) return;
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  if (pl->dev) (void)hipFree(pl->dev);
  delete pl;
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Deterministic pseudo-random numbers for the tuning batch.
struct Lcg {
  uint64_t s;
  double next() {   // uniform in [-1, 1)
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return double(s >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
};

}  // namespace

// Samples per lane of the persistent kernel's layout for S lanes: the smallest K
// of a compiled variant with S*K/2 >= c (larger K only adds padding), or 0.
int r1h::batch_samples_per_lane(int S, int n_t) {
  int c = (n_t - 1) / 2;
  for (int K = 2; K <= 32; K *= 2)
    if (S * K / 2 >= c && r1_batch_variant(S, K) >= 0) return K;
  return 0;
}

void r1h::release_batched(r1_handle h) {
  for (auto& kv : h->plans) free_plan(kv.second);
  h->plans.clear();
  if (h->capture_stream) {
    (void)hipStreamDestroy(h->capture_stream);
    h->capture_stream = nullptr;
  }
}

// Times every admissible segment width for lines of n_t points and records
// the fastest for (n_t, dtype, dim, role).  Role kRoleLevel: a synthetic
// one-level batch (16384 points near the identity, 32 directions).  Role
// kRoleInner: the same 32 directions as the inner level of a depth-2 batch
// (1024 points, outer level of 8 directions x 129 points), timed through the
// depth-2 path, whose inner lines are sampled along outer lines.  Both batches
// launch several thousand blocks, many times what the chip holds at once, so
// the last partly filled round of blocks does not decide between layouts of
// different occupancy.
r1_status r1h::autotune(r1_handle h, const r1_material* mat, int n_t, int dtype, int dim, int role,
                        hipStream_t st, int* lanes) {
  const int key_dim = dim;
  std::vector<int> cands;
  for (int S = 8; S <= 64; S *= 2)
    if (batch_samples_per_lane(S, n_t) > 0) cands.push_back(S);
  if (cands.empty()) return R1_EINVAL;
  if (cands.size() == 1) {
    h->seg_tuned[tune_key(n_t, dtype, key_dim, role)] = cands[0];
    if (lanes) *lanes = cands[0];
    return R1_OK;
  }
  const bool inner = role == kRoleInner;
  const int n = inner ? 1024 : 16384, na = 8, nb = 4, dd = dim * dim;
  const int nao = 4, nbo = 2, nt_o = 129;
  const size_t ts = dtype == R1_F32 ? 4 : 8;
  std::vector<double> Fd(size_t(dd) * n), bnd(n), a(size_t(na * nb) * dim, 0.0), b(size_t(na * nb) * dim, 0.0);
  Lcg rng{0x9e3779b97f4a7c15ull ^ uint64_t(n_t)};
  for (int p = 0; p < n; ++p) {
    double G[9];
    for (;;) {
      for (int k = 0; k < dd; ++k) G[k] = ((k % (dim + 1)) == 0 ? 1.0 : 0.0) + 0.25 * rng.next();
      double det = dim == 2 ? G[0] * G[3] - G[1] * G[2]
                            : G[0] * (G[4] * G[8] - G[5] * G[7]) - G[1] * (G[3] * G[8] - G[5] * G[6]) +
                                  G[2] * (G[3] * G[7] - G[4] * G[6]);
      if (det > 0.2) break;
    }
    for (int k = 0; k < dd; ++k) Fd[size_t(k) * n + p] = G[k];
    bnd[p] = 0.25 * (rng.next() + 1.0);
  }
  for (int i = 0; i < na; ++i)
    for (int j = 0; j < nb; ++j) {
      int m = i * nb + j;
      a[m * dim + 0] = std::cos(M_PI * i / na);
      a[m * dim + 1] = std::sin(M_PI * i / na);
      b[m * dim + 0] = std::cos(M_PI * j / nb);
      b[m * dim + 1] = std::sin(M_PI * j / nb);
    }
  std::vector<double> ao(size_t(nao * nbo) * dim, 0.0), bo(size_t(nao * nbo) * dim, 0.0);
  for (int i = 0; i < nao; ++i)
    for (int j = 0; j < nbo; ++j) {
      int m = i * nbo + j;
      ao[m * dim + 0] = std::cos(M_PI * (i + 0.5) / nao);
      ao[m * dim + 1] = std::sin(M_PI * (i + 0.5) / nao);
      bo[m * dim + 0] = std::cos(M_PI * (j + 0.25) / nbo);
      bo[m * dim + 1] = std::sin(M_PI * (j + 0.25) / nbo);
    }
  std::vector<char> Fh(ts * Fd.size()), bnh(ts * n);
  for (size_t i = 0; i < Fd.size(); ++i) {
    if (ts == 4) { float v = float(Fd[i]); std::memcpy(&Fh[4 * i], &v, 4); }
    else std::memcpy(&Fh[8 * i], &Fd[i], 8);
  }
  for (int i = 0; i < n; ++i) {
    if (ts == 4) { float v = float(bnd[i]); std::memcpy(&bnh[4 * i], &v, 4); }
    else std::memcpy(&bnh[8 * i], &bnd[i], 8);
  }
  void* buf = nullptr;
  const size_t res_bytes = inner ? align_up(ts * n) + align_up(r1_outer_res_bytes(dtype) * n * nao * nbo) : 0;
  size_t bytes = align_up(Fh.size()) + align_up(bnh.size()) + align_up(ts * n) + res_bytes;
  if (hipMalloc(&buf, bytes) != hipSuccess) return R1_ENOMEM;
  char* base = static_cast<char*>(buf);
  void* dF = base;
  void* dB = base + align_up(Fh.size());
  void* dW = base + align_up(Fh.size()) + align_up(bnh.size());
  hipError_t e = hipMemcpy(dF, Fh.data(), Fh.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dB, bnh.data(), bnh.size(), hipMemcpyHostToDevice);
  r1_level lv{na * nb, a.data(), b.data(), n_t, 1.0};
  r1_level lvo{nao * nbo, ao.data(), bo.data(), nt_o, 1.0};
  KArgs ka{};
  ka.n = n;
  ka.F = dF;
  ka.beta_n = dB;
  ka.W = dW;
  ka.mat = r1d::Material{dim, mat->model, mat->mu, mat->lambda, mat->D_inf, mat->D0};
  r1_status s = e == hipSuccess ? R1_OK : fail(h, e, "hipMemcpy(tune)");
  if (!s && inner) {
    ka.scratch_w1f = static_cast<char*>(dW) + align_up(ts * n);
    ka.scratch_outer = static_cast<char*>(ka.scratch_w1f) + align_up(ts * n);
    s = device_level(h, lvo, dim, &ka.lv0);
    if (!s) s = device_level(h, lv, dim, &ka.lv1);
  } else if (!s) {
    s = device_level(h, lv, dim, &ka.lv0);
  }
  const int depth = inner ? 2 : 1;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!s && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) s = R1_EDEVICE;
  int best = cands[0];
  float best_ms = 1e30f;
  for (size_t ci = 0; !s && ci < cands.size(); ++ci) {
    int S = cands[ci], K = batch_samples_per_lane(S, n_t);
    e = r1_launch_envelope(ka, depth, dtype, S, K, st, nullptr);             // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int r = 0; r < 2 && e == hipSuccess; ++r) e = r1_launch_envelope(ka, depth, dtype, S, K, st, nullptr);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) { s = fail(h, e, "autotune"); break; }
    if (ms < best_ms) { best_ms = ms; best = S; }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  (void)hipFree(buf);
  if (s) return s;
  h->seg_tuned[tune_key(n_t, dtype, key_dim, role)] = best;
  if (lanes) *lanes = best;
  return R1_OK;
}

extern "C" r1_status r1_autotune(r1_handle h, const r1_material* mat, int32_t n_t, r1_dtype dtype,
                                 void* stream, int32_t* lanes) {
  if (!h) return R1_EINVAL;
  r1_status s = r1h::check_material(mat);
  if (s) return s;
  if (dtype != R1_F32 && dtype != R1_F64) return R1_EINVAL;
  if (n_t < 3 || n_t > R1_MAX_NT || (n_t % 2) == 0) return R1_EINVAL;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return r1h::fail(h, e, "hipSetDevice");
  int S = 0;
  s = r1h::autotune(h, mat, n_t, dtype, mat->dim, r1h::kRoleLevel, static_cast<hipStream_t>(stream), &S);
  if (!s && lanes) *lanes = S;
  return s;
}

extern "C" r1_status r1_autotune_inner(r1_handle h, const r1_material* mat, int32_t n_t, r1_dtype dtype,
                                       void* stream, int32_t* lanes) {
  if (!h) return R1_EINVAL;
  r1_status s = r1h::check_material(mat);
  if (s) return s;
  if (dtype != R1_F32 && dtype != R1_F64) return R1_EINVAL;
  if (n_t < 3 || n_t > R1_MAX_NT || (n_t % 2) == 0) return R1_EINVAL;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return r1h::fail(h, e, "hipSetDevice");
  int S = 0;
  s = r1h::autotune(h, mat, n_t, dtype, mat->dim, r1h::kRoleInner, static_cast<hipStream_t>(stream), &S);
  if (!s && lanes) *lanes = S;
  return s;
}

extern "C" r1_status r1_envelope_batched(r1_handle h, const r1_material* mat,
                                         const r1_lamination* table, int32_t n_table, int64_t n,
                                         const int32_t* lam_idx, r1_dtype dtype, const void* F,
                                         const void* beta_n, void* W, void* P, r1_laminate* tree,
                                         int32_t* flags, void* stream) {
  if (!h) return R1_EINVAL;
  r1_status s = r1h::check_material(mat);
  if (s) return s;
  if (!table || n_table < 1 || n_table > 4096) return R1_EINVAL;
  for (int k = 0; k < n_table; ++k) {
    s = r1h::check_lamination(&table[k]);
    if (s) return s;
  }
  if (dtype != R1_F32 && dtype != R1_F64) return R1_EINVAL;
  if (n < 0 || n >= (int64_t(1) << 31)) return R1_EINVAL;
  if (n == 0) return R1_OK;
  if (!lam_idx || !F || !beta_n || !W) return R1_EINVAL;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return r1h::fail(h, e, "hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int dim = mat->dim;

  // plan key: everything the captured launch bakes in
  uint64_t key = 1469598103934665603ull;
  key = mixv(key, *mat);
  key = mixv(key, n);
  key = mixv(key, dtype);
  const void* ptrs[8] = {F, beta_n, W, P, tree, flags, lam_idx, nullptr};
  key = mix(key, ptrs, sizeof(ptrs));
  for (int k = 0; k < n_table; ++k) {
    const r1_lamination& L = table[k];
    key = mixv(key, L.depth);
    for (int l = 0; l < L.depth; ++l) {
      const r1_level& lv = L.level[l];
      key = mixv(key, lv.n_dir);
      key = mixv(key, lv.n_t);
      key = mixv(key, lv.tau);
      key = mix(key, lv.a, sizeof(double) * size_t(lv.n_dir) * dim);
      key = mix(key, lv.b, sizeof(double) * size_t(lv.n_dir) * dim);
    }
  }
  auto found = h->plans.find(key);
  BatchedPlan* pl = found == h->plans.end() ? nullptr : found->second;

  if (!pl) {
    // ---- plan: read the table indices, order the work, upload
    std::vector<int32_t> idx(static_cast<size_t>(n));
    e = hipMemcpyAsync(idx.data(), lam_idx, sizeof(int32_t) * size_t(n), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return r1h::fail(h, e, "read lam_idx");
    for (int64_t p = 0; p < n; ++p)
      if (idx[p] < 0 || idx[p] >= n_table) return R1_EINVAL;
    std::vector<BEntry> ent(static_cast<size_t>(n_table));
    constexpr int NV = R1_N_BATCH_VARIANTS;
    size_t lds[NV] = {};
    const size_t ts = dtype == R1_F32 ? 4 : 8;
    for (int k = 0; k < n_table; ++k) {
      const r1_lamination& L = table[k];
      BEntry& b = ent[k];
      std::memset(&b, 0, sizeof(b));
      b.depth = L.depth;
      s = r1h::device_level(h, L.level[0], dim, &b.lv0);
      if (!s && L.depth == 2) s = r1h::device_level(h, L.level[1], dim, &b.lv1);
      if (s) return s;
      const int nti = L.level[L.depth - 1].n_t;
      const int role = L.depth == 2 ? r1h::kRoleInner : r1h::kRoleLevel;
      if (!h->seg_override.count(nti) && !h->seg_tuned.count(r1h::tune_key(nti, dtype, dim, role))) {
        s = r1h::autotune(h, mat, nti, dtype, dim, role, st, nullptr);
        if (s) return s;
      }
      int S = r1h::segment_width(h, nti, dtype, dim, role);
      int K = r1h::batch_samples_per_lane(S, nti);
      b.var = K > 0 ? r1_batch_variant(S, K) : -1;
      for (int S2 = 16; b.var < 0 && S2 <= 64; S2 *= 2) {   // width outside the variant set
        int K2 = r1h::batch_samples_per_lane(S2, nti);
        if (K2 > 0) b.var = r1_batch_variant(S2, K2);
      }
      if (b.var < 0) return R1_EUNSUPPORTED;
      if (L.depth == 2) {
        size_t need = r1k::outer_lds_bytes(ts, L.level[0].n_t, L.level[1].n_dir, mat->model);
        lds[b.var] = std::max(lds[b.var], need);
      }
    }
    // work lists per layout variant, each ordered largest first: point items
    // (groups of up to 4 depth-1 points; groups of up to 4 depth-2 points for
    // the centre values), outer lines of depth-2 points, depth-2 points to finalize
    std::vector<int64_t> d2[NV], d1[NV];
    for (int64_t p = 0; p < n; ++p) {
      const int c = ent[idx[p]].var;
      (table[idx[p]].depth == 2 ? d2[c] : d1[c]).push_back(p);
    }
    auto cost = [&](int64_t p) {
      const r1_lamination& L = table[idx[p]];
      if (L.depth == 1) return double(L.level[0].n_dir) * double(L.level[0].n_t - 1);
      return double(L.level[0].n_t - 1) *
             (double(L.level[1].n_dir) * double(L.level[1].n_t - 1) + 1.0);
    };
    std::vector<int64_t> pbase(static_cast<size_t>(n), 0);
    std::vector<int4> items;
    std::vector<int32_t> order;
    int64_t n_outer = 0;
    // per variant and kind: first item (or order entry for kBFinal) and count
    int64_t first[NV][3] = {}, count[NV][3] = {};
    for (int c = 0; c < NV; ++c) {
      std::stable_sort(d2[c].begin(), d2[c].end(), [&](int64_t x, int64_t y) { return cost(x) > cost(y); });
      std::stable_sort(d1[c].begin(), d1[c].end(), [&](int64_t x, int64_t y) { return cost(x) > cost(y); });
      first[c][kBPoint] = int64_t(items.size());
      for (int kind = 0; kind < 2; ++kind) {
        const std::vector<int64_t>& pts = kind == 0 ? d1[c] : d2[c];
        const int64_t o0 = int64_t(order.size());
        order.insert(order.end(), pts.begin(), pts.end());
        for (int64_t g = 0; 4 * g < int64_t(pts.size()); ++g) {
          int cnt = int(std::min<int64_t>(4, int64_t(pts.size()) - 4 * g));
          items.push_back(int4{kind == 0 ? 0 : 2, int(o0 + 4 * g), cnt, 0});
        }
      }
      count[c][kBPoint] = int64_t(items.size()) - first[c][kBPoint];
      first[c][kBOuter] = int64_t(items.size());
      for (int64_t p : d2[c]) {
        pbase[p] = n_outer;
        n_outer += table[idx[p]].level[0].n_dir;
        for (int mo = 0; mo < table[idx[p]].level[0].n_dir; ++mo) items.push_back(int4{1, int(p), mo, 0});
      }
      count[c][kBOuter] = int64_t(items.size()) - first[c][kBOuter];
      first[c][kBFinal] = int64_t(order.size());
      order.insert(order.end(), d2[c].begin(), d2[c].end());
      count[c][kBFinal] = int64_t(d2[c].size());
    }
    const int64_t n_items = int64_t(items.size());
    if (n_items >= (int64_t(1) << 31) || int64_t(order.size()) >= (int64_t(1) << 31)) return R1_EINVAL;
    const size_t res_sz = r1_outer_res_bytes(dtype);
    size_t off_tab = 0;
    size_t off_items = off_tab + align_up(sizeof(BEntry) * ent.size());
    size_t off_order = off_items + align_up(sizeof(int4) * std::max<size_t>(items.size(), 1));
    size_t off_pbase = off_order + align_up(sizeof(int32_t) * std::max<size_t>(order.size(), 1));
    size_t off_cnt = off_pbase + align_up(sizeof(int64_t) * size_t(n));
    size_t off_w1f = off_cnt + align_up(sizeof(int) * size_t(2 * NV));
    size_t off_outer = off_w1f + align_up(ts * size_t(n));
    size_t total = off_outer + align_up(res_sz * std::max<int64_t>(n_outer, 1));
    pl = new BatchedPlan();
    if (hipMalloc(&pl->dev, total) != hipSuccess) {
      free_plan(pl);
      return R1_ENOMEM;
    }
    char* base = static_cast<char*>(pl->dev);
    e = hipMemcpy(base + off_tab, ent.data(), sizeof(BEntry) * ent.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !items.empty())
      e = hipMemcpy(base + off_items, items.data(), sizeof(int4) * items.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !order.empty())
      e = hipMemcpy(base + off_order, order.data(), sizeof(int32_t) * order.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(base + off_pbase, pbase.data(), sizeof(int64_t) * size_t(n), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      free_plan(pl);
      return r1h::fail(h, e, "upload plan");
    }
    int n_cu = 0;
    e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, h->device);
    if (e != hipSuccess || n_cu < 1) {
      free_plan(pl);
      return e != hipSuccess ? r1h::fail(h, e, "device attribute") : R1_EUNSUPPORTED;
    }
    // launches: per variant k_bpoint, k_bouter, k_bfinal; counters [2c + kind]
    struct Launch { BArgs b; int var, kind, grid; size_t lds; };
    std::vector<Launch> launches;
    for (int c = 0; c < NV; ++c) {
      for (int kind = 0; kind < 3; ++kind) {
        if (count[c][kind] == 0) continue;
        Launch L{};
        BArgs& b = L.b;
        b.base.n = n;
        b.base.F = F;
        b.base.beta_n = beta_n;
        b.base.W = W;
        b.base.P = P;
        b.base.tree = tree;
        b.base.flags = flags;
        b.base.mat = r1d::Material{mat->dim, mat->model, mat->mu, mat->lambda, mat->D_inf, mat->D0};
        b.base.want_stress = P != nullptr;
        b.table = reinterpret_cast<const BEntry*>(base + off_tab);
        b.lam_idx = lam_idx;
        b.pbase = reinterpret_cast<const int64_t*>(base + off_pbase);
        b.outer = base + off_outer;
        b.w1f = base + off_w1f;
        b.n_items = int(count[c][kind]);
        if (kind == kBFinal) {
          b.order = reinterpret_cast<const int32_t*>(base + off_order) + first[c][kind];
          L.grid = int((count[c][kind] + 3) / 4);
        } else {
          b.order = reinterpret_cast<const int32_t*>(base + off_order);
          b.items = reinterpret_cast<const int4*>(base + off_items) + first[c][kind];
          b.counter = reinterpret_cast<int*>(base + off_cnt) + 2 * c + kind;
          L.lds = kind == kBOuter ? lds[c] : 0;
          int per_cu = 0;
          e = r1_occupancy_batched(dtype, dim, mat->model, c, kind, L.lds, &per_cu);
          if (e != hipSuccess || per_cu < 1) {
            free_plan(pl);
            return e != hipSuccess ? r1h::fail(h, e, "occupancy") : R1_EUNSUPPORTED;
          }
          L.grid = int(std::min<int64_t>(int64_t(per_cu) * n_cu, count[c][kind]));
        }
        L.var = c;
        L.kind = kind;
        launches.push_back(L);
      }
    }
    // capture the launch sequence once; replays run it unchanged
    if (!h->capture_stream) {
      e = hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking);
      if (e != hipSuccess) {
        h->capture_stream = nullptr;
        free_plan(pl);
        return r1h::fail(h, e, "hipStreamCreate");
      }
    }
    e = hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t le = hipSuccess;
      int zero_n = 2 * NV;                     // every queue head, once, by a fill kernel
      for (size_t k = 0; k < launches.size() && le == hipSuccess; ++k) {
        const Launch& L = launches[k];
        le = r1_launch_batched(L.b, dtype, dim, L.b.base.mat.model, L.var, L.kind, L.grid, L.lds, reinterpret_cast<int*>(base + off_cnt),
                               zero_n, h->capture_stream);
        zero_n = 0;
      }
      e = hipStreamEndCapture(h->capture_stream, &pl->graph);
      if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      free_plan(pl);
      return r1h::fail(h, e, "graph capture");
    }
    pl->key = key;
    pl->n_items = n_items;
    pl->n_outer = n_outer;
    pl->serial = ++h->plan_serial;
    if (h->plans.size() >= 8) {          // evict the oldest plan
      auto old = h->plans.begin();
      for (auto it = h->plans.begin(); it != h->plans.end(); ++it)
        if (it->second->serial < old->second->serial) old = it;
      (void)hipDeviceSynchronize();
      free_plan(old->second);
      h->plans.erase(old);
    }
    h->plans[key] = pl;
  }
  if (h->timer.on) h->timer.begin("batched", st);
  e = hipGraphLaunch(pl->exec, st);
  if (h->timer.on) h->timer.end(st);
  if (e != hipSuccess) return r1h::fail(h, e, "hipGraphLaunch");
  return R1_OK;
}
