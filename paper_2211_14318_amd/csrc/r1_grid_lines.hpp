// Mesh and direction bookkeeping of the grid variant (Section 4.1 of arXiv
// 2211.14318): the mesh of Section 5.2 as node counts and strides, and for a
// direction (an integer step s) the starts of its lines.  The lines of a step
// partition the mesh; a line starts at every node whose predecessor (the node
// one step back) lies outside the box.  Those nodes are the box minus the box of
// nodes whose predecessor is inside, which splits into at most d*d disjoint
// slabs by the first component that leaves it: slab c holds components c' < c
// in their "predecessor inside" range, component c outside it and components
// c' > c free.  Lines of at least m nodes start where, besides, the node m - 1
// steps ahead lies inside: each range intersected with one more interval, so
// the slabs stay boxes.  Line start t is decoded from t in mixed radix with the
// last component fastest, so consecutive t are consecutive nodes within a slab.
// Host and device share these functions.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>

#include "r1.h"

namespace r1g {

constexpr int kGridMaxLen = 512;  // nodes per component (bounds a line's length)

struct GridArgs {
  int dd;                  // d*d components
  int n[9];                // nodes per component (1 beyond dd)
  int64_t stride[9];       // node index step of each component (component 0 slowest)
  double lo[9];            // first node value per component
  double delta;            // mesh width
  int64_t size;            // nodes
};

struct Step {
  int s[9];              // the step (0 beyond dd)
  int lo[9], hi[9];      // per component: predecessor inside (components before the slab's), [lo, hi)
  int slo[9], shi[9];    // per component: predecessor outside (the slab's component), [slo, shi)
  int flo[9], fhi[9];    // per component: free (components after the slab's), [flo, fhi)
  int64_t slab_end[9];   // starts in slabs 0..c (INT64_MAX beyond dd)
  int64_t count;         // lines (of at least min_len nodes) of the direction
  int64_t ds;            // node index step along a line
  int len;               // longest line
};

// Mesh arguments of a caller's grid; R1_EINVAL for a bad grid (dim not 2 or 3,
// delta not finite and positive, a count outside 1..512, a non-finite lo, more
// than 2^31 nodes).
inline r1_status grid_args(const r1_grid* grid, GridArgs* g) {
  if (!grid || (grid->dim != 2 && grid->dim != 3)) return R1_EINVAL;
  if (!(grid->delta > 0.0) || !std::isfinite(grid->delta)) return R1_EINVAL;
  g->dd = grid->dim * grid->dim;
  g->delta = grid->delta;
  int64_t size = 1;
  for (int c = 0; c < g->dd; ++c) {
    if (grid->n[c] < 1 || grid->n[c] > kGridMaxLen || !std::isfinite(grid->lo[c])) return R1_EINVAL;
    g->n[c] = grid->n[c];
    g->lo[c] = grid->lo[c];
    size *= grid->n[c];
    if (size > (int64_t(1) << 31)) return R1_EINVAL;
  }
  for (int c = g->dd; c < 9; ++c) {
    g->n[c] = 1;
    g->lo[c] = 0.0;
  }
  int64_t st = 1;
  for (int c = g->dd - 1; c >= 0; --c) {
    g->stride[c] = st;
    st *= g->n[c];
  }
  for (int c = g->dd; c < 9; ++c) g->stride[c] = 0;
  g->size = size;
  return R1_OK;
}

// Fills the slabs, line count, index step and longest line of step s->s
// (|s_c| <= 512, not all zero) on mesh g, for the lines of at least min_len >= 1
// nodes.
inline void step_slabs(const GridArgs& g, Step* s, int min_len = 1) {
  s->len = kGridMaxLen;
  s->ds = 0;
  const int64_t m = min_len - 1;
  for (int c = 0; c < 9; ++c) {
    const int n = g.n[c];
    const int v = c < g.dd ? s->s[c] : 0;
    s->s[c] = v;
    // the node min_len - 1 steps ahead lies inside: [rlo, rhi)
    const int rlo = int(std::min<int64_t>(v < 0 ? -m * v : 0, n));
    const int rhi = int(std::max<int64_t>(v > 0 ? n - m * v : n, rlo));
    auto clip = [&](int a, int b, int* lo, int* hi) {
      *lo = std::max(a, rlo);
      *hi = std::max(std::min(b, rhi), *lo);
    };
    clip(v >= 0 ? std::min(v, n) : 0, v >= 0 ? n : std::max(n + v, 0), &s->lo[c], &s->hi[c]);
    clip(v > 0 ? 0 : (v < 0 ? std::max(n + v, 0) : 0), v > 0 ? std::min(v, n) : (v < 0 ? n : 0), &s->slo[c],
         &s->shi[c]);
    clip(0, n, &s->flo[c], &s->fhi[c]);
    if (v != 0) s->len = std::min(s->len, (n - 1) / std::abs(v) + 1);
    s->ds += int64_t(v) * g.stride[c];
  }
  int64_t end = 0;
  for (int c = 0; c < 9; ++c) {
    int64_t cnt = 0;
    if (c < g.dd) {
      cnt = s->shi[c] - s->slo[c];
      for (int k = 0; k < g.dd; ++k)
        if (k != c) cnt *= k < c ? int64_t(s->hi[k] - s->lo[k]) : int64_t(s->fhi[k] - s->flo[k]);
    }
    end += cnt;
    s->slab_end[c] = c < g.dd ? end : INT64_MAX;
  }
  s->count = end;
}

// Node index (and multi-index I, first dd entries) of line start t, 0 <= t < s.count
// (< 2^31, so the mixed-radix decoding runs in 32-bit arithmetic); *slab receives
// the slab of t.
__host__ __device__ inline int64_t line_start(const GridArgs& g, const Step& s, int64_t t, int* I,
                                              int* slab = nullptr) {
  int c = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) c += t >= s.slab_end[k] ? 1 : 0;
  int64_t r64 = t;
#pragma unroll
  for (int k = 1; k < 9; ++k)
    if (k == c) r64 -= s.slab_end[k - 1];
  uint32_t r = uint32_t(r64);
  int64_t p = 0;
#pragma unroll
  for (int k = 8; k >= 0; --k) {
    if (k < g.dd) {
      const int lo = k < c ? s.lo[k] : (k == c ? s.slo[k] : s.flo[k]);
      const uint32_t w = uint32_t(k < c ? s.hi[k] - s.lo[k] : (k == c ? s.shi[k] - s.slo[k] : s.fhi[k] - s.flo[k]));
      const uint32_t qt = r / w;
      I[k] = lo + int(r - qt * w);
      r = qt;
      p += int64_t(I[k]) * g.stride[k];
    }
  }
  if (slab) *slab = c;
  return p;
}

// Advances (I, *p) from line start t to start t + delta (delta >= 0) within slab c:
// the mixed-radix counter adds delta to its last component and carries (a division
// only for the components the carry reaches).  False when that leaves slab c (the
// start, if any, lies in a later slab; decode it with line_start).
__host__ __device__ inline bool line_advance(const GridArgs& g, const Step& s, int c, int* I, int64_t* p,
                                             uint32_t delta) {
  for (int k = g.dd - 1; k >= 0 && delta; --k) {
    const int lo = k < c ? s.lo[k] : (k == c ? s.slo[k] : s.flo[k]);
    const int hi = k < c ? s.hi[k] : (k == c ? s.shi[k] : s.fhi[k]);
    const uint32_t w = uint32_t(hi - lo);
    const uint32_t v = uint32_t(I[k] - lo) + delta;
    const uint32_t qt = v < w ? 0u : v / w;
    const int nv = lo + int(v - qt * w);
    *p += int64_t(nv - I[k]) * g.stride[k];
    I[k] = nv;
    delta = qt;
  }
  return delta == 0;
}

// Nodes of the line that starts at multi-index I.
__host__ __device__ inline int line_length(const GridArgs& g, const Step& s, const int* I) {
  int L = kGridMaxLen;
  for (int c = 0; c < g.dd; ++c) {
    const int v = s.s[c];
    if (v == 0) continue;
    const int room = v > 0 ? g.n[c] - 1 - I[c] : I[c];     // steps left inside the box
    const int a = v > 0 ? v : -v;
    L = std::min(L, (a == 1 ? room : room / a) + 1);
  }
  return L;
}

}  // namespace r1g
