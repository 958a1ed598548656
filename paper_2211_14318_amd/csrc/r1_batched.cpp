// Host side of the uneven batch (r1_batched_plan_*, r1_envelope_batched): the
// plan that owns the ordered work lists, the table's directions and a copy of
// the per-point table indices, the captured HIP graphs that replay its
// persistent launches, and the segment-width autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "r1_batched_kernels.hpp"
#include "r1_batched_plan.hpp"
#include "r1_handle.hpp"

struct r1_batched_plan_s {
  r1_handle h = nullptr;
  uint64_t key = 0;             // content key (r1_envelope_batched's cache)
  uint64_t serial = 0;
  int dtype = 0;
  int64_t n = 0;
  void* dev = nullptr;          // table, directions, table indices, items, order, pbase, counters, results
  int* counters = nullptr;      // queue heads, cleared at the start of every replay
  int n_counters = 0;
  struct Launch {
    BArgs b;                    // plan-owned pointers; the caller's buffers are set at capture
    int var, kind, grid;
    size_t lds;
  };
  std::vector<Launch> launches;
  struct Graph {                // one captured sequence per set of caller buffers
    const void* ptrs[6];
    hipGraph_t graph;
    hipGraphExec_t exec;
    uint64_t used;
  };
  std::vector<Graph> graphs;
  uint64_t clock = 0;
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

void free_graph(r1_batched_plan_s::Graph& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g.exec = nullptr;
  g.graph = nullptr;
}

// Frees a plan; the caller has made sure no replay of it is still running.
void free_plan(r1_batched_plan_s* pl) {
  if (!pl) return;
  for (auto& g : pl->graphs) free_graph(g);
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
  for (r1_batched_plan_s* pl : h->user_plans) free_plan(pl);
  h->user_plans.clear();
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
    const r1_level* lvs[2] = {&lvo, &lv};
    r1d::Level out[2];
    s = device_levels(h, lvs, 2, dim, out);
    ka.lv0 = out[0];
    ka.lv1 = out[1];
  } else if (!s) {
    const r1_level* lvs[1] = {&lv};
    s = device_levels(h, lvs, 1, dim, &ka.lv0);
  }
  const int depth = inner ? 2 : 1;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!s && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) s = R1_EDEVICE;
  // each candidate warmed up once, then timed in three interleaved rounds of two
  // launches; the fastest round counts (layouts within a few percent of each other
  // are otherwise picked by noise)
  std::vector<float> cand_ms(cands.size(), 1e30f);
  for (size_t ci = 0; !s && ci < cands.size(); ++ci) {
    e = r1_launch_envelope(ka, depth, dtype, cands[ci], batch_samples_per_lane(cands[ci], n_t), st, nullptr);
    if (e != hipSuccess) s = fail(h, e, "autotune");
  }
  for (int round = 0; !s && round < 3; ++round)
    for (size_t ci = 0; !s && ci < cands.size(); ++ci) {
      const int S = cands[ci], K = batch_samples_per_lane(S, n_t);
      e = hipEventRecord(e0, st);
      for (int r = 0; r < 2 && e == hipSuccess; ++r) e = r1_launch_envelope(ka, depth, dtype, S, K, st, nullptr);
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) { s = fail(h, e, "autotune"); break; }
      cand_ms[ci] = std::min(cand_ms[ci], ms);
    }
  int best = cands[0];
  float best_ms = 1e30f;
  for (size_t ci = 0; ci < cands.size(); ++ci)
    if (cand_ms[ci] < best_ms) { best_ms = cand_ms[ci]; best = cands[ci]; }
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


namespace {

r1_status check_table(const r1_material* mat, const r1_lamination* table, int32_t n_table) {
  r1_status s = r1h::check_material(mat);
  if (s) return s;
  if (!table || n_table < 1 || n_table > 4096) return R1_EINVAL;
  for (int k = 0; k < n_table; ++k) {
    s = r1h::check_lamination(&table[k]);
    if (s) return s;
  }
  return R1_OK;
}

// Reads the caller's per-point table indices (device) into idx and checks them.
r1_status read_indices(r1_handle h, const int32_t* lam_idx, int64_t n, int32_t n_table, hipStream_t st,
                       std::vector<int32_t>* idx) {
  idx->resize(static_cast<size_t>(n));
  hipError_t e = hipMemcpyAsync(idx->data(), lam_idx, sizeof(int32_t) * size_t(n), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return r1h::fail(h, e, "read lam_idx");
  for (int64_t p = 0; p < n; ++p)
    if ((*idx)[size_t(p)] < 0 || (*idx)[size_t(p)] >= n_table) return R1_EINVAL;
  return R1_OK;
}

// Builds a plan for table indices idx (host copy, checked): tunes the segment
// widths it needs, orders the work, and uploads the table (with its own copy of
// every level's directions), the indices and the work lists into one device
// buffer owned by the plan.  No graph is captured yet.
r1_status make_plan(r1_handle h, const r1_material* mat, const r1_lamination* table, int32_t n_table,
                    const std::vector<int32_t>& idx, r1_dtype dtype, hipStream_t st, r1_batched_plan_s** out) {
  const int dim = mat->dim;
  const int64_t n = int64_t(idx.size());
  constexpr int NV = R1_N_BATCH_VARIANTS;
  const size_t ts = dtype == R1_F32 ? 4 : 8;
  std::vector<BEntry> ent(static_cast<size_t>(n_table));
  std::vector<r1plan::Entry> pent(static_cast<size_t>(n_table));
  std::vector<size_t> dir_off(static_cast<size_t>(2 * n_table), 0);   // doubles into the direction block
  std::vector<double> dirs;
  size_t lds[NV] = {};
  r1_status s = R1_OK;
  for (int k = 0; k < n_table; ++k) {
    const r1_lamination& L = table[k];
    BEntry& b = ent[size_t(k)];
    std::memset(&b, 0, sizeof(b));
    b.depth = L.depth;
    for (int l = 0; l < L.depth; ++l) {
      const r1_level& lv = L.level[l];
      r1h::level_meta(lv, dim, l == 0 ? &b.lv0 : &b.lv1);
      dir_off[size_t(2 * k + l)] = dirs.size();
      dirs.insert(dirs.end(), lv.a, lv.a + size_t(lv.n_dir) * dim);
      dirs.insert(dirs.end(), lv.b, lv.b + size_t(lv.n_dir) * dim);
    }
    const int nti = L.level[L.depth - 1].n_t;
    const int role = L.depth == 2 ? r1h::kRoleInner : r1h::kRoleLevel;
    if (!h->seg_override.count(nti) && !h->seg_tuned.count(r1h::tune_key(nti, dtype, dim, role))) {
      s = r1h::autotune(h, mat, nti, dtype, dim, role, st, nullptr);
      if (s) return s;
    }
    const int S = r1h::segment_width(h, nti, dtype, dim, role);
    const int K = r1h::batch_samples_per_lane(S, nti);
    b.var = K > 0 ? r1_batch_variant(S, K) : -1;
    for (int S2 = 16; b.var < 0 && S2 <= 64; S2 *= 2) {   // width outside the variant set
      const int K2 = r1h::batch_samples_per_lane(S2, nti);
      if (K2 > 0) b.var = r1_batch_variant(S2, K2);
    }
    if (b.var < 0) return R1_EUNSUPPORTED;
    if (L.depth == 2) {
      const size_t need = r1k::outer_lds_bytes(ts, L.level[0].n_t, L.level[1].n_dir, mat->model);
      lds[b.var] = std::max(lds[b.var], need);
    }
    pent[size_t(k)] = r1plan::Entry{L.depth, L.level[0].n_dir, L.level[0].n_t,
                                    L.depth == 2 ? L.level[1].n_dir : 0, L.depth == 2 ? L.level[1].n_t : 0, b.var};
  }
  const r1plan::Plan wk = r1plan::plan_work(pent, idx, NV);
  if (int64_t(wk.items.size()) >= (int64_t(1) << 31) || int64_t(wk.order.size()) >= (int64_t(1) << 31) ||
      wk.n_outer >= (int64_t(1) << 31))
    return R1_EINVAL;
  const size_t res_sz = r1_outer_res_bytes(dtype);
  const size_t off_tab = 0;
  const size_t off_dirs = off_tab + align_up(sizeof(BEntry) * ent.size());
  const size_t off_idx = off_dirs + align_up(sizeof(double) * std::max<size_t>(dirs.size(), 1));
  const size_t off_items = off_idx + align_up(sizeof(int32_t) * size_t(n));
  const size_t off_order = off_items + align_up(sizeof(int4) * std::max<size_t>(wk.items.size(), 1));
  const size_t off_pbase = off_order + align_up(sizeof(int32_t) * std::max<size_t>(wk.order.size(), 1));
  const size_t off_cnt = off_pbase + align_up(sizeof(int64_t) * size_t(n));
  const size_t off_w1f = off_cnt + align_up(sizeof(int) * size_t(2 * NV));
  const size_t off_outer = off_w1f + align_up(ts * size_t(n));
  const size_t total = off_outer + align_up(res_sz * size_t(std::max<int64_t>(wk.n_outer, 1)));
  r1_batched_plan_s* pl = new (std::nothrow) r1_batched_plan_s();
  if (!pl) return R1_ENOMEM;
  if (hipMalloc(&pl->dev, total) != hipSuccess) {
    pl->dev = nullptr;
    free_plan(pl);
    return R1_ENOMEM;
  }
  char* base = static_cast<char*>(pl->dev);
  const double* ddirs = reinterpret_cast<const double*>(base + off_dirs);
  for (int k = 0; k < n_table; ++k) {
    BEntry& b = ent[size_t(k)];
    for (int l = 0; l < b.depth; ++l) {
      r1d::Level& lv = l == 0 ? b.lv0 : b.lv1;
      lv.a = ddirs + dir_off[size_t(2 * k + l)];
      lv.b = lv.a + size_t(lv.n_dir) * dim;
    }
  }
  static_assert(sizeof(r1plan::Item) == sizeof(int4), "work item layout");
  hipError_t e = hipMemcpy(base + off_tab, ent.data(), sizeof(BEntry) * ent.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !dirs.empty())
    e = hipMemcpy(base + off_dirs, dirs.data(), sizeof(double) * dirs.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(base + off_idx, idx.data(), sizeof(int32_t) * size_t(n), hipMemcpyHostToDevice);
  if (e == hipSuccess && !wk.items.empty())
    e = hipMemcpy(base + off_items, wk.items.data(), sizeof(int4) * wk.items.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !wk.order.empty())
    e = hipMemcpy(base + off_order, wk.order.data(), sizeof(int32_t) * wk.order.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(base + off_pbase, wk.pbase.data(), sizeof(int64_t) * size_t(n), hipMemcpyHostToDevice);
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
  for (int c = 0; c < NV; ++c) {
    for (int kind = 0; kind < 3; ++kind) {
      const int64_t first = wk.first[size_t(c) * 3 + kind], count = wk.count[size_t(c) * 3 + kind];
      if (count == 0) continue;
      r1_batched_plan_s::Launch L{};
      BArgs& b = L.b;
      b.base.n = n;
      b.base.mat = r1d::Material{mat->dim, mat->model, mat->mu, mat->lambda, mat->D_inf, mat->D0};
      b.table = reinterpret_cast<const BEntry*>(base + off_tab);
      b.lam_idx = reinterpret_cast<const int32_t*>(base + off_idx);
      b.pbase = reinterpret_cast<const int64_t*>(base + off_pbase);
      b.outer = base + off_outer;
      b.w1f = base + off_w1f;
      b.n_items = int(count);
      if (kind == kBFinal) {
        b.order = reinterpret_cast<const int32_t*>(base + off_order) + first;
        L.grid = int((count + 3) / 4);
      } else {
        b.order = reinterpret_cast<const int32_t*>(base + off_order);
        b.items = reinterpret_cast<const int4*>(base + off_items) + first;
        b.counter = reinterpret_cast<int*>(base + off_cnt) + 2 * c + kind;
        L.lds = kind == kBOuter ? lds[c] : 0;
        int per_cu = 0;
        e = r1_occupancy_batched(dtype, dim, mat->model, c, kind, L.lds, &per_cu);
        if (e != hipSuccess || per_cu < 1) {
          free_plan(pl);
          return e != hipSuccess ? r1h::fail(h, e, "occupancy") : R1_EUNSUPPORTED;
        }
        L.grid = int(std::min<int64_t>(int64_t(per_cu) * n_cu, count));
      }
      L.var = c;
      L.kind = kind;
      pl->launches.push_back(L);
    }
  }
  pl->h = h;
  pl->dtype = dtype;
  pl->n = n;
  pl->counters = reinterpret_cast<int*>(base + off_cnt);
  pl->n_counters = 2 * NV;
  *out = pl;
  return R1_OK;
}

// Captures the plan's launch sequence for the given caller buffers into a graph
// (the queue heads are cleared by a fill kernel at its start, no memset node).
r1_status capture(r1_batched_plan_s* pl, const void* const ptrs[6], r1_batched_plan_s::Graph* g) {
  r1_handle h = pl->h;
  hipError_t e = hipSuccess;
  if (!h->capture_stream) {
    e = hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      h->capture_stream = nullptr;
      return r1h::fail(h, e, "hipStreamCreate");
    }
  }
  *g = r1_batched_plan_s::Graph{};
  for (int k = 0; k < 6; ++k) g->ptrs[k] = ptrs[k];
  e = hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t le = hipSuccess;
    int zero_n = pl->n_counters;             // every queue head, once
    for (size_t k = 0; k < pl->launches.size() && le == hipSuccess; ++k) {
      const r1_batched_plan_s::Launch& L = pl->launches[k];
      BArgs b = L.b;
      b.base.F = ptrs[0];
      b.base.beta_n = ptrs[1];
      b.base.W = const_cast<void*>(ptrs[2]);
      b.base.P = const_cast<void*>(ptrs[3]);
      b.base.tree = static_cast<r1_laminate*>(const_cast<void*>(ptrs[4]));
      b.base.flags = static_cast<int32_t*>(const_cast<void*>(ptrs[5]));
      b.base.want_stress = ptrs[3] != nullptr;
      le = r1_launch_batched(b, pl->dtype, b.base.mat.dim, b.base.mat.model, L.var, L.kind, L.grid, L.lds,
                             pl->counters, zero_n, h->capture_stream);
      zero_n = 0;
    }
    e = hipStreamEndCapture(h->capture_stream, &g->graph);
    if (le != hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    free_graph(*g);
    return r1h::fail(h, e, "graph capture");
  }
  return R1_OK;
}

// Replays the plan for the given buffers on st; up to 4 captured graphs (one per
// set of buffers) are kept, the least recently used one is replaced.
r1_status execute(r1_batched_plan_s* pl, const void* F, const void* beta_n, void* W, void* P, r1_laminate* tree,
                  int32_t* flags, hipStream_t st) {
  r1_handle h = pl->h;
  if (!F || !beta_n || !W) return R1_EINVAL;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return r1h::fail(h, e, "hipSetDevice");
  const void* ptrs[6] = {F, beta_n, W, P, tree, flags};
  r1_batched_plan_s::Graph* g = nullptr;
  for (auto& x : pl->graphs)
    if (std::equal(ptrs, ptrs + 6, x.ptrs)) g = &x;
  if (!g) {
    r1_batched_plan_s::Graph ng;
    r1_status s = capture(pl, ptrs, &ng);
    if (s) return s;
    if (pl->graphs.size() >= 4) {
      auto old = std::min_element(pl->graphs.begin(), pl->graphs.end(),
                                  [](const r1_batched_plan_s::Graph& a, const r1_batched_plan_s::Graph& b) {
                                    return a.used < b.used;
                                  });
      e = hipDeviceSynchronize();             // a replay of it may still run
      if (e != hipSuccess) {
        free_graph(ng);
        return r1h::fail(h, e, "hipDeviceSynchronize");
      }
      free_graph(*old);
      *old = ng;
      g = &*old;
    } else {
      pl->graphs.push_back(ng);
      g = &pl->graphs.back();
    }
  }
  g->used = ++pl->clock;
  if (h->timer.on) h->timer.begin("batched", st);
  e = hipGraphLaunch(g->exec, st);
  if (h->timer.on) h->timer.end(st);
  if (e != hipSuccess) return r1h::fail(h, e, "hipGraphLaunch");
  return R1_OK;
}

}  // namespace

extern "C" r1_status r1_batched_plan_create(r1_handle h, const r1_material* mat, const r1_lamination* table,
                                            int32_t n_table, int64_t n, const int32_t* lam_idx, r1_dtype dtype,
                                            void* stream, r1_batched_plan* plan) {
  if (!h || !plan) return R1_EINVAL;
  *plan = nullptr;
  r1_status s = check_table(mat, table, n_table);
  if (s) return s;
  if (dtype != R1_F32 && dtype != R1_F64) return R1_EINVAL;
  if (n < 1 || n >= (int64_t(1) << 31) || !lam_idx) return R1_EINVAL;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return r1h::fail(h, e, "hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<int32_t> idx;
  s = read_indices(h, lam_idx, n, n_table, st, &idx);
  if (s) return s;
  r1_batched_plan_s* pl = nullptr;
  s = make_plan(h, mat, table, n_table, idx, dtype, st, &pl);
  if (s) return s;
  h->user_plans.insert(pl);
  *plan = pl;
  return R1_OK;
}

extern "C" r1_status r1_batched_plan_execute(r1_batched_plan plan, const void* F, const void* beta_n, void* W,
                                             void* P, r1_laminate* tree, int32_t* flags, void* stream) {
  if (!plan) return R1_EINVAL;
  return execute(plan, F, beta_n, W, P, tree, flags, static_cast<hipStream_t>(stream));
}

extern "C" r1_status r1_batched_plan_destroy(r1_batched_plan plan) {
  if (!plan) return R1_EINVAL;
  r1_handle h = plan->h;
  if (!h->user_plans.erase(plan)) return R1_EINVAL;
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();           // replays of it may still run
  free_plan(plan);
  return R1_OK;
}

extern "C" r1_status r1_envelope_batched(r1_handle h, const r1_material* mat,
                                         const r1_lamination* table, int32_t n_table, int64_t n,
                                         const int32_t* lam_idx, r1_dtype dtype, const void* F,
                                         const void* beta_n, void* W, void* P, r1_laminate* tree,
                                         int32_t* flags, void* stream) {
  if (!h) return R1_EINVAL;
  r1_status s = check_table(mat, table, n_table);
  if (s) return s;
  if (dtype != R1_F32 && dtype != R1_F64) return R1_EINVAL;
  if (n < 0 || n >= (int64_t(1) << 31)) return R1_EINVAL;
  if (n == 0) return R1_OK;
  if (!lam_idx || !F || !beta_n || !W) return R1_EINVAL;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return r1h::fail(h, e, "hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int dim = mat->dim;
  std::vector<int32_t> idx;
  s = read_indices(h, lam_idx, n, n_table, st, &idx);
  if (s) return s;

  // plan key: the contents that decide the plan (material, sizes, table, indices)
  uint64_t key = 1469598103934665603ull;
  key = mixv(key, *mat);
  key = mixv(key, n);
  key = mixv(key, dtype);
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
  key = mix(key, idx.data(), sizeof(int32_t) * idx.size());
  auto found = h->plans.find(key);
  r1_batched_plan_s* pl = found == h->plans.end() ? nullptr : found->second;
  if (!pl) {
    s = make_plan(h, mat, table, n_table, idx, dtype, st, &pl);
    if (s) return s;
    pl->key = key;
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
  return execute(pl, F, beta_n, W, P, tree, flags, st);
}
