// Global rank-one lamination on a deformation-gradient mesh (Section 4.1 of
// arXiv 2211.14318): node values W^0 = W on the mesh of Section 5.2 (one mesh
// width for every component), then iterations of eq. 4.3 -- every node takes
// the minimum over the directions of the lower hull (Algorithm 1) of the line
// of eq. 4.4 through it, clipped to the mesh's box -- until the maximal decrease
// of an iteration is at most the tolerance or k_max iterations are done
// (Section 6); off-mesh values by multilinear interpolation.  Node stresses and
// tangent moduli, when requested, follow the laminates that lower the nodes
// (eq. 5.2, first case; Algorithm 3's moduli with the same weights);
// interpolating them gives the off-mesh values (eq. 5.2, second case).
//
// A direction is an integer step s in Z^{d x d}; its lines advance the node
// index by a constant stride and partition the mesh.  The directions of an
// iteration all read the previous iterate, so their hulls are independent; only
// the choice among them is ordered (a later direction replaces a node's value
// only when lower by more than a rounding margin).  An iteration therefore runs,
// per group of up to 16 directions, a hull launch -- one thread per line of every
// direction of the group; the line starts (nodes whose predecessor lies outside
// the box) form at most d*d disjoint boxes and are decoded from the thread index;
// the thread stages its line in its own LDS column, builds the lower hull with a
// monotone chain and writes every node's candidate value (and, when stresses or
// moduli are carried, its laminate's offsets) -- then a pick launch, one thread
// per node, that takes the group's candidates in direction order.  The last
// pick of an iteration also takes the maximal decrease and writes the carried
// stresses and moduli, so nothing is copied between iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "r1.h"
#include "r1_device.hpp"
#include "r1_grid_lines.hpp"
#include "r1_handle.hpp"

namespace {

using namespace r1g;

constexpr int kLineThreads = 64;        // threads per block of the line kernel
constexpr int kStageBytes = 56 * 1024;  // LDS of a block that stages its lines

__device__ __forceinline__ void node_multi(const GridArgs& g, int64_t p, int* I) {
  for (int c = g.dd - 1; c >= 0; --c) {
    I[c] = int(p % g.n[c]);
    p /= g.n[c];
  }
}

template <typename T>
__device__ __forceinline__ T inf_t() { return T(__builtin_inf()); }

// Unit roundoff of T: a hull value lowers a node only by more than 4 of these
// relative to max(|W|, 1e-3) -- a node on a straight hull run reads its own value
// back up to rounding, which is no lamination, and of directions that tie to
// rounding the first keeps the node.
template <typename T>
__device__ __forceinline__ T eps_t() { return sizeof(T) == 4 ? T(1.1920928955078125e-07) : T(2.220446049250313e-16); }

// W^0 at every node: the library's W (neo-Hooke: +inf where det F <= 0); with P,
// also P^0 = dW/dF, with A the moduli d^2W/dFdF (component-major, NaN where W is
// +inf).
template <typename T, int D>
__global__ __launch_bounds__(256) void k_grid_energy(GridArgs g, r1d::Material mat, double bn, T* W, T* P, T* A) {
  const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (p >= g.size) return;
  int I[9];
  node_multi(g, p, I);
  double F[D * D];
#pragma unroll
  for (int c = 0; c < D * D; ++c) F[c] = g.lo[c] + I[c] * g.delta;
  const r1d::Point<T> q = r1d::make_point_any<T>(mat, bn);
  double cof[D * D];
  r1d::cofactor<D>(F, cof);
  const T w = r1d::w_point_any<T, D>(q, F, cof);
  W[p] = w < inf_t<T>() ? w : inf_t<T>();
  if (P) {
    double S[D * D];
    r1d::stress0_any<D>(mat, bn, F, S);
#pragma unroll
    for (int c = 0; c < D * D; ++c) P[int64_t(c) * g.size + p] = T(S[c]);
  }
  if (A) r1d::tangent0_store<D>(mat, bn, F, A + p, g.size);
}

// Hulls of some directions of a group of up to kGroupMax directions of one
// iteration.  A block takes R * 64 consecutive line starts of one direction, its
// lanes R of them 64 apart (lanes on consecutive starts, so accesses coalesce;
// the first decoded, the next ones stepped to by a mixed-radix add).  The blocks
// of the launch's i-th direction, group slot slot[i], are block_end[i-1] ..
// block_end[i]-1, so a block's direction (and its Step, read through scalar
// loads) is uniform.
// A node's candidate is the hull value ((b - q) w_a + (q - a) w_b) / (b - a)
// where it lies strictly inside a hull segment [a, b] and its own value is
// finite, +inf otherwise; with offs, also the offsets (q - a) | (b - q) << 16 of
// its laminate.  Dense (mask null): the launch covers every line and writes
// every slot (the lines of a direction partition the mesh, so each once).
// Sparse: it covers only the lines of at least 3 nodes (shorter ones hold no
// node strictly inside a segment), writes the finite candidates only and marks
// them in the node's mask (bit = group slot); unmarked slots are never read.
// Non-finite values are absent from a hull.  STAGED: the line's values sit in
// the thread's LDS column (entry q at [q * kLineThreads]); otherwise they are
// read in place.
constexpr int kGroupMax = 16;
constexpr int kShortLine = 8;  // lines of at most this many nodes go to their own hull launch
constexpr int kShortRun = 8;   // line starts per thread there
constexpr int kLenClasses = 6; // hull launches per group: lines of <= 8, 16, 32, 64, 128 nodes, longer

inline int len_class(int len) {
  return len <= kShortLine ? 0 : len <= 16 ? 1 : len <= 32 ? 2 : len <= 64 ? 3 : len <= 128 ? 4 : 5;
}

struct Group {
  int d0;                      // first direction of the group
  int n;                       // directions of this launch ...
  int slot[kGroupMax];         // ... their slots in the group (direction d0 + slot)
  int block_end[kGroupMax];    // prefix sums of their blocks
};

// One line of L nodes from node p, index step ds: hull, then the candidates.
template <typename T, bool STAGED, int CHUNK>
__device__ __forceinline__ void hull_line(const T* __restrict__ Win, T* __restrict__ cd, uint32_t* __restrict__ od,
                                          uint32_t* __restrict__ mask, uint32_t bit, int64_t p, int64_t ds, int L,
                                          T* vin, uint16_t* st) {
  if (L == 3) {
    // three nodes (most lines of the 9-D meshes): the chain pops the middle one
    // exactly when it lies on or above the chord, and its candidate is the chord's
    // midpoint -- the general path's arithmetic, without its loops
    const T w0 = Win[p], w1 = Win[p + ds], w2 = Win[p + 2 * ds];
    const bool fin = w0 < inf_t<T>() && w1 < inf_t<T>() && w2 < inf_t<T>();
    const bool cand1 = fin && (w1 - w0) * T(1) >= (w2 - w1) * T(1);
    const T val = cand1 ? (T(1) * w0 + T(1) * w2) / T(2) : inf_t<T>();
    if (!mask) {
      cd[p] = inf_t<T>();
      cd[p + 2 * ds] = inf_t<T>();
      if (od) od[p] = od[p + 2 * ds] = 0u;
    }
    if (!mask || cand1) {
      cd[p + ds] = val;
      if (od) od[p + ds] = cand1 ? (1u | (1u << 16)) : 0u;
      if (mask) atomicOr(mask + p + ds, bit);
    }
    return;
  }
  auto win = [&](int q) -> T { return STAGED ? vin[q * kLineThreads] : Win[p + q * ds]; };
  if constexpr (STAGED) {
    // chunks of independent loads: a line costs one or two memory round trips, not L
    for (int q0 = 0; q0 < L; q0 += CHUNK) {
      T a[CHUNK];
#pragma unroll
      for (int i = 0; i < CHUNK; ++i) a[i] = q0 + i < L ? Win[p + (q0 + i) * ds] : T(0);
#pragma unroll
      for (int i = 0; i < CHUNK; ++i)
        if (q0 + i < L) vin[(q0 + i) * kLineThreads] = a[i];
    }
  }
  // monotone chain: the top vertex is popped while the slope into it is at least
  // the slope from it to the new point (collinear points are not kept).  One flat
  // loop of pops and pushes (at most 2L trips), so the lanes of a wave, whose hulls
  // differ, stay within the longest line's trip count.
  int h = 0, i1 = 0, i2 = 0;
  T v1 = T(0), v2 = T(0);
  {
    int q = 0;
    T w = L > 0 ? win(0) : T(0);
    while (q < L) {
      const bool fin = w < inf_t<T>();
      if (fin && h >= 2 && (v2 - v1) * T(q - i2) >= (w - v2) * T(i2 - i1)) {
        --h;
        i2 = i1;
        v2 = v1;
        if (h >= 2) {
          i1 = st[(h - 2) * kLineThreads];
          v1 = win(i1);
        }
        continue;
      }
      if (fin) {
        st[h * kLineThreads] = uint16_t(q);
        ++h;
        i1 = i2;
        v1 = v2;
        i2 = q;
        v2 = w;
      }
      ++q;
      if (q < L) w = win(q);
    }
  }
  // candidates along the line, one flat loop; (a, b) is the segment holding q
  int k = 1, a = 0, b = 0, last = -1;
  T wa = T(0), wb = T(0);
  if (h >= 2) {
    a = st[0];
    b = st[kLineThreads];
    wa = win(a);
    wb = win(b);
    last = st[(h - 1) * kLineThreads];
  }
  for (int q = 0; q < L; ++q) {
    T val = inf_t<T>();
    uint32_t off = 0;
    if (q > a && q < last) {
      if (q == b) {
        a = b;
        wa = wb;
        ++k;
        b = st[k * kLineThreads];
        wb = win(b);
      } else if (win(q) < inf_t<T>()) {
        val = (T(b - q) * wa + T(q - a) * wb) / T(b - a);
        off = uint32_t(q - a) | (uint32_t(b - q) << 16);
      }
    }
    if (!mask || val < inf_t<T>()) {
      cd[p + q * ds] = val;
      if (od) od[p + q * ds] = off;
      if (mask) atomicOr(mask + p + q * ds, bit);
    }
  }
}

template <typename T, bool STAGED, int R>
__global__ __launch_bounds__(kLineThreads) void k_grid_hulls(GridArgs g, const Step* __restrict__ steps, Group grp,
                                                            const T* __restrict__ Win, T* __restrict__ cand,
                                                            uint32_t* __restrict__ offs, uint32_t* __restrict__ mask,
                                                            int len) {
  extern __shared__ __align__(8) unsigned char line_mem[];
  const int tid = threadIdx.x;
  const int blk = blockIdx.x;
  int i = 0;
#pragma unroll
  for (int k = 0; k < kGroupMax; ++k) i += (k < grp.n && blk >= grp.block_end[k]) ? 1 : 0;
  const int j = grp.slot[i];
  const Step& s = steps[grp.d0 + j];
  const int64_t t0 = int64_t(blk - (i ? grp.block_end[i - 1] : 0)) * kLineThreads * R + tid;
  T* const cd = cand + int64_t(j) * g.size;
  uint32_t* const od = offs ? offs + int64_t(j) * g.size : nullptr;
  T* const vin = reinterpret_cast<T*>(line_mem) + tid;  // STAGED only
  uint16_t* const st = reinterpret_cast<uint16_t*>(reinterpret_cast<T*>(line_mem) +
                                                   (STAGED ? len * kLineThreads : 0)) + tid;
  constexpr int kChunk = R > 1 ? kShortLine : 32;
  int I[9];
  int slab = 0;
  int64_t p = 0;
  for (int r = 0; r < R; ++r) {
    const int64_t t = t0 + int64_t(r) * kLineThreads;
    if (t >= s.count) break;
    if (r == 0 || !line_advance(g, s, slab, I, &p, kLineThreads)) p = line_start(g, s, t, I, &slab);
    hull_line<T, STAGED, kChunk>(Win, cd, od, mask, 1u << j, p, s.ds, line_length(g, s, I), vin, st);
  }
}

// The group's candidates in direction order, per node: a candidate replaces the
// running value only when lower by more than 4 units of rounding relative to
// max(|W|, 1e-3), so directions that tie to rounding leave the node to the first.
// kFirst: the running value starts from Win (else Wout, and with sel the running
// laminate) and every node is written.  Sparse (mask): only the marked slots of
// the nodes with a mark are read, and the mask goes back to 0.
// The maximal decrease Win - W over nodes with finite Win goes to *dec (atomic
// maximum of the non-negative doubles' bit patterns; W only decreases over the
// groups, so the maximum over the nodes the groups lower is the iteration's).
// kLast: the node stresses / moduli of the laminate that lowered a node, with the
// weights of its value (eq. 5.2, first case), or the node's own, go to Pout / Aout.
enum : int { kFirst = 1, kLast = 2 };
constexpr unsigned kPickBlocks = 2048;  // grid-stride pick launches: 8 blocks per CU

template <typename T>
struct Carry {
  const T* Pin;
  T* Pout;
  const T* Ain;
  T* Aout;
  int32_t* sel;            // running laminate: direction (-1: none) ...
  uint32_t* soff;          // ... and its offsets, kept between groups
};

template <typename T>
__global__ __launch_bounds__(256) void k_grid_pick(GridArgs g, const Step* __restrict__ steps, int d0, int nd,
                                                   const T* __restrict__ Win, T* __restrict__ Wout,
                                                   const T* __restrict__ cand, const uint32_t* __restrict__ offs,
                                                   uint32_t* __restrict__ mask, Carry<T> cy, int flags,
                                                   unsigned long long* dec) {
  const int64_t n = g.size;
  const bool first = flags & kFirst;
  const bool carry = cy.Pout || cy.Aout;
  double m = 0.0;
  for (int64_t node = int64_t(blockIdx.x) * 256 + threadIdx.x; node < n; node += int64_t(gridDim.x) * 256) {
    const uint32_t mk = mask ? mask[node] : (1u << nd) - 1u;
    if (mk || first || (carry && (flags & kLast))) {
      const T w0 = Win[node];
      T cur = first || !mk ? w0 : Wout[node];
      int32_t sl = -1;
      uint32_t so = 0;
      if (carry && !first) {
        sl = cy.sel[node];
        so = cy.soff[node];
      }
      bool changed = false;
      if (mk) {
        T v[kGroupMax];                            // all loads first, then the ordered choice
#pragma unroll
        for (int j = 0; j < kGroupMax; ++j) v[j] = (mk >> j) & 1u ? cand[int64_t(j) * n + node] : inf_t<T>();
        if (mask) mask[node] = 0u;
#pragma unroll
        for (int j = 0; j < kGroupMax; ++j) {
          if (v[j] < cur - T(4) * eps_t<T>() * fmax(fabs(cur), T(1e-3))) {
            cur = v[j];
            sl = d0 + j;
            if (offs) so = offs[int64_t(j) * n + node];
            changed = true;
          }
        }
      }
      if (first || changed) Wout[node] = cur;
      if (changed && w0 < inf_t<T>()) m = double(w0) - double(cur);
      if (carry && !(flags & kLast) && (first || changed)) {
        cy.sel[node] = sl;
        cy.soff[node] = so;
      }
      if (carry && (flags & kLast)) {
        int64_t ia = node, ib = node;
        int qa = 0, bq = 0;
        if (sl >= 0) {
          qa = int(so & 0xffffu);
          bq = int(so >> 16);
          ia = node - qa * steps[sl].ds;
          ib = node + bq * steps[sl].ds;
        }
        if (cy.Pout)
          for (int c = 0; c < g.dd; ++c)
            cy.Pout[c * n + node] = sl < 0 ? cy.Pin[c * n + node]
                                           : (T(bq) * cy.Pin[c * n + ia] + T(qa) * cy.Pin[c * n + ib]) / T(qa + bq);
        if (cy.Aout)
          for (int c = 0; c < g.dd * g.dd; ++c)
            cy.Aout[c * n + node] = sl < 0 ? cy.Ain[c * n + node]
                                           : (T(bq) * cy.Ain[c * n + ia] + T(qa) * cy.Ain[c * n + ib]) / T(qa + bq);
      }
    }
  }
  // one atomic per block (the launch has a bounded number of blocks)
  __shared__ double red[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    if (m > 0.0) atomicMax(dec, static_cast<unsigned long long>(__double_as_longlong(m)));
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_grid_fill(int64_t n, T* a, T v) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ __launch_bounds__(256) void k_grid_zero(unsigned long long* dec, int n) {
  const int i = int(blockIdx.x) * 256 + int(threadIdx.x);
  if (i < n) dec[i] = 0ull;
}

// Multilinear interpolation of the node values at n points F (SoA, d*d x n):
// corners of zero weight do not take part; NaN outside the box (beyond a
// rounding margin of 1e-9 mesh widths).
template <typename T, int D>
__global__ __launch_bounds__(256) void k_grid_interp(GridArgs g, const T* W, int64_t n, const T* F, T* out) {
  const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (p >= n) return;
  constexpr int DD = D * D;
  int base[DD];
  double frac[DD];
  bool inside = true;
#pragma unroll
  for (int c = 0; c < DD; ++c) {
    double u = (double(F[int64_t(c) * n + p]) - g.lo[c]) / g.delta;
    const double top = double(g.n[c] - 1);
    inside = inside && u >= -1e-9 && u <= top + 1e-9;
    u = u < 0.0 ? 0.0 : (u > top ? top : u);
    int i = int(floor(u));
    i = i > g.n[c] - 2 ? g.n[c] - 2 : i;
    i = i < 0 ? 0 : i;
    base[c] = i;
    frac[c] = g.n[c] > 1 ? u - i : 0.0;
  }
  if (!inside) {
    out[p] = T(__builtin_nan(""));
    return;
  }
  double sum = 0.0;
  for (int corner = 0; corner < (1 << DD); ++corner) {
    double wgt = 1.0;
    int64_t idx = 0;
#pragma unroll
    for (int c = 0; c < DD; ++c) {
      const int up = (corner >> (DD - 1 - c)) & 1;
      if (up && g.n[c] == 1) wgt = 0.0;
      wgt *= up ? frac[c] : 1.0 - frac[c];
      idx += int64_t(base[c] + up) * g.stride[c];
    }
    if (wgt != 0.0) sum += wgt * double(W[idx]);
  }
  out[p] = T(sum);
}

inline unsigned blocks_of(int64_t n, int b) { return unsigned((n + b - 1) / b); }

// Device scratch of one laminate call: the other iterate (and stress / moduli
// iterates), the per-iteration decreases, the steps, and one group's candidates.
template <typename T>
struct GridWork {
  T* W2 = nullptr;
  T* P2 = nullptr;
  T* A2 = nullptr;
  unsigned long long* dec = nullptr;
  Step* steps = nullptr;
  T* cand = nullptr;
  uint32_t* offs = nullptr;
  uint32_t* mask = nullptr;    // sparse mode only
  int32_t* sel = nullptr;
  uint32_t* soff = nullptr;
};

inline size_t round256(size_t b) { return (b + 255) & ~size_t(255); }


// One iteration: for each group of directions, the hull launch then the pick launch.
template <typename T>
hipError_t grid_sweep(const GridArgs& g, const std::vector<Step>& steps, const GridWork<T>& wk, const T* Win,
                      T* Wout, Carry<T> cy, unsigned long long* dec, hipStream_t st, KTimer* tm) {
  const int n_dir = int(steps.size());
  const bool carry = cy.Pout || cy.Aout;
  for (int d0 = 0; d0 < n_dir; d0 += kGroupMax) {
    const int nd = std::min(kGroupMax, n_dir - d0);
    // one hull launch per length class of the group's lines, each with the LDS of
    // its own longest line (short lines would otherwise run at the occupancy of the
    // longest); the candidates keep their group slots, so the order is unchanged
    for (int part = 0; part < kLenClasses; ++part) {
      const int R = part == 0 ? kShortRun : 1;
      Group grp{};
      grp.d0 = d0;
      int blocks = 0, len = 1;
      for (int j = 0; j < nd; ++j) {
        const Step& s = steps[d0 + j];
        if (len_class(s.len) != part) continue;
        blocks += int(blocks_of(s.count, kLineThreads * R));
        grp.slot[grp.n] = j;
        grp.block_end[grp.n] = blocks;
        ++grp.n;
        len = std::max(len, s.len);
      }
      if (grp.n == 0) continue;
      const size_t staged = (sizeof(T) + sizeof(uint16_t)) * size_t(kLineThreads) * size_t(len);
      uint32_t* offs = carry ? wk.offs : nullptr;
      if (blocks == 0) continue;
      if (tm) tm->begin("grid_lines", st);
      if (part == 0)
        hipLaunchKernelGGL((k_grid_hulls<T, true, kShortRun>), dim3(blocks), dim3(kLineThreads), staged, st, g,
                           wk.steps, grp, Win, wk.cand, offs, wk.mask, len);
      else if (staged <= size_t(kStageBytes))
        hipLaunchKernelGGL((k_grid_hulls<T, true, 1>), dim3(blocks), dim3(kLineThreads), staged, st, g, wk.steps,
                           grp, Win, wk.cand, offs, wk.mask, len);
      else
        hipLaunchKernelGGL((k_grid_hulls<T, false, 1>), dim3(blocks), dim3(kLineThreads),
                           sizeof(uint16_t) * size_t(kLineThreads) * size_t(len), st, g, wk.steps, grp, Win,
                           wk.cand, offs, wk.mask, len);
      if (tm) tm->end(st);
    }
    const int flags = (d0 == 0 ? kFirst : 0) | (d0 + nd == n_dir ? kLast : 0);
    Carry<T> c = cy;
    c.sel = carry ? wk.sel : nullptr;
    c.soff = carry ? wk.soff : nullptr;
    if (tm) tm->begin("grid_pick", st);
    hipLaunchKernelGGL((k_grid_pick<T>), dim3(std::min<unsigned>(blocks_of(g.size, 256), kPickBlocks)), dim3(256), 0,
                       st, g, wk.steps, d0, nd,
                       Win, Wout, wk.cand, carry ? wk.offs : nullptr, wk.mask, c, flags, dec);
    if (tm) tm->end(st);
  }
  return hipGetLastError();
}

// steps enumerate every line (dense) or the lines of at least 3 nodes (sparse).
template <typename T>
r1_status grid_laminate_T(r1_handle h, const GridArgs& g, const std::vector<Step>& steps, bool sparse, T* W, T* P,
                          T* A, int k_max, double tol, int32_t* iterations, double* decrease, hipStream_t st) {
  const size_t n = size_t(g.size);
  const bool carry = P || A;
  const int G = std::min<int>(kGroupMax, int(steps.size()));
  const size_t sizes[10] = {round256(sizeof(T) * n),
                           P ? round256(sizeof(T) * n * size_t(g.dd)) : 0,
                           A ? round256(sizeof(T) * n * size_t(g.dd * g.dd)) : 0,
                           round256(sizeof(unsigned long long) * size_t(k_max)),
                           round256(sizeof(Step) * steps.size()),
                           round256(sizeof(T) * n * size_t(G)),
                           carry ? round256(sizeof(uint32_t) * n * size_t(G)) : 0,
                           carry ? round256(sizeof(int32_t) * n) : 0,
                           carry ? round256(sizeof(uint32_t) * n) : 0,
                           sparse ? round256(sizeof(uint32_t) * n) : 0};
  size_t total = 0;
  for (size_t b : sizes) total += b;
  void* base = nullptr;
  r1_status s = r1h::scratch(h, total, &base);
  if (s) return s;
  char* at = static_cast<char*>(base);
  auto take = [&](int i) -> void* {
    void* q = sizes[i] ? at : nullptr;
    at += sizes[i];
    return q;
  };
  GridWork<T> wk;
  wk.W2 = static_cast<T*>(take(0));
  wk.P2 = static_cast<T*>(take(1));
  wk.A2 = static_cast<T*>(take(2));
  wk.dec = static_cast<unsigned long long*>(take(3));
  wk.steps = static_cast<Step*>(take(4));
  wk.cand = static_cast<T*>(take(5));
  wk.offs = static_cast<uint32_t*>(take(6));
  wk.sel = static_cast<int32_t*>(take(7));
  wk.soff = static_cast<uint32_t*>(take(8));
  wk.mask = static_cast<uint32_t*>(take(9));
  hipError_t e = hipMemcpyAsync(wk.steps, steps.data(), sizeof(Step) * steps.size(), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return r1h::fail(h, e, "grid steps");
  if (sparse)  // the invariant the sparse launches keep: no marks between groups
    hipLaunchKernelGGL((k_grid_fill<uint32_t>), dim3(blocks_of(int64_t(n), 256)), dim3(256), 0, st, int64_t(n),
                       wk.mask, 0u);
  hipLaunchKernelGGL(k_grid_zero, dim3(blocks_of(k_max, 256)), dim3(256), 0, st, wk.dec, k_max);
  KTimer* tm = h->timer.on ? &h->timer : nullptr;
  T* cur = W;
  T* nxt = wk.W2;
  T* pcur = P;
  T* pnxt = wk.P2;
  T* acur = A;
  T* anxt = wk.A2;
  int k = 0;
  while (k < k_max) {
    Carry<T> cy{pcur, pnxt, acur, anxt, nullptr, nullptr};
    e = grid_sweep<T>(g, steps, wk, cur, nxt, cy, wk.dec + k, st, tm);
    unsigned long long bits = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&bits, wk.dec + k, sizeof(bits), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return r1h::fail(h, e, "grid iteration");
    double md;
    std::memcpy(&md, &bits, sizeof(md));
    if (decrease) decrease[k] = md;
    ++k;
    std::swap(cur, nxt);
    std::swap(pcur, pnxt);
    std::swap(acur, anxt);
    if (md <= tol) break;
  }
  if (cur != W) {
    e = hipMemcpyAsync(W, cur, sizeof(T) * n, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && P) e = hipMemcpyAsync(P, pcur, sizeof(T) * n * size_t(g.dd), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && A)
      e = hipMemcpyAsync(A, acur, sizeof(T) * n * size_t(g.dd * g.dd), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return r1h::fail(h, e, "grid copy");
  }
  if (iterations) *iterations = k;
  return R1_OK;
}

template <typename T>
void launch_energy(int dim, dim3 grd, hipStream_t st, const GridArgs& g, const r1d::Material& m, double beta_n,
                   void* W, void* P, void* A) {
  T* w = static_cast<T*>(W);
  T* p = static_cast<T*>(P);
  T* a = static_cast<T*>(A);
  if (dim == 2)
    hipLaunchKernelGGL((k_grid_energy<T, 2>), grd, dim3(256), 0, st, g, m, beta_n, w, p, a);
  else
    hipLaunchKernelGGL((k_grid_energy<T, 3>), grd, dim3(256), 0, st, g, m, beta_n, w, p, a);
}

}  // namespace

extern "C" {

r1_status r1_grid_r11(int32_t dim, int32_t* steps, int32_t* n_dir) {
  if ((dim != 2 && dim != 3) || !steps || !n_dir) return R1_EINVAL;
  const int dd = dim * dim;
  int count = 0;
  // a (x) b for a, b in {-1, 0, 1}^dim \ {0}; s ~ -s, kept with a positive first non-zero entry
  const int na = dim == 2 ? 9 : 27;
  for (int ia = 0; ia < na; ++ia)
    for (int ib = 0; ib < na; ++ib) {
      int a[3], b[3];
      bool az = true, bz = true;
      for (int i = 0, ra = ia, rb = ib; i < dim; ++i, ra /= 3, rb /= 3) {
        a[dim - 1 - i] = ra % 3 - 1;
        b[dim - 1 - i] = rb % 3 - 1;
      }
      for (int i = 0; i < dim; ++i) {
        az = az && a[i] == 0;
        bz = bz && b[i] == 0;
      }
      if (az || bz) continue;
      int s[9];
      int sign = 0;
      for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) {
          s[i * dim + j] = a[i] * b[j];
          if (!sign && s[i * dim + j]) sign = s[i * dim + j];
        }
      for (int c = 0; c < dd; ++c) s[c] *= sign;
      bool dup = false;
      for (int m = 0; m < count && !dup; ++m) dup = std::memcmp(steps + m * dd, s, sizeof(int) * dd) == 0;
      if (!dup) {
        std::memcpy(steps + count * dd, s, sizeof(int) * dd);
        ++count;
      }
    }
  *n_dir = count;
  return R1_OK;
}

r1_status r1_grid_energy(r1_handle h, const r1_material* mat, const r1_grid* grid, double beta_n, r1_dtype dtype,
                         void* W, void* P, void* A, void* stream) {
  if (!h || !W) return R1_EINVAL;
  r1_status s = r1h::check_material(mat);
  if (s) return s;
  GridArgs g;
  s = grid_args(grid, &g);
  if (s) return s;
  if (mat->dim != grid->dim || !std::isfinite(beta_n) || (dtype != R1_F32 && dtype != R1_F64)) return R1_EINVAL;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return r1h::fail(h, e, "hipSetDevice");
  const r1d::Material m{mat->dim, mat->model, mat->mu, mat->lambda, mat->D_inf, mat->D0};
  hipStream_t st = static_cast<hipStream_t>(stream);
  const dim3 grd(blocks_of(g.size, 256));
  if (dtype == R1_F32)
    launch_energy<float>(grid->dim, grd, st, g, m, beta_n, W, P, A);
  else
    launch_energy<double>(grid->dim, grd, st, g, m, beta_n, W, P, A);
  e = hipGetLastError();
  return e == hipSuccess ? R1_OK : r1h::fail(h, e, "kernel launch");
}

r1_status r1_grid_laminate(r1_handle h, const r1_grid* grid, int32_t n_dir, const int32_t* steps, r1_dtype dtype,
                           void* W, void* P, void* A, int32_t k_max, double tol, int32_t* iterations,
                           double* decrease, void* stream) {
  if (!h || !W || !steps || n_dir < 1 || n_dir > R1_MAX_DIRS || k_max < 1 || !(tol >= 0.0)) return R1_EINVAL;
  if (dtype != R1_F32 && dtype != R1_F64) return R1_EINVAL;
  GridArgs g;
  r1_status s = grid_args(grid, &g);
  if (s) return s;
  std::vector<Step> st_list(static_cast<size_t>(n_dir));
  for (int m = 0; m < n_dir; ++m) {
    bool zero = true;
    for (int c = 0; c < 9; ++c) st_list[m].s[c] = c < g.dd ? steps[m * g.dd + c] : 0;
    for (int c = 0; c < g.dd; ++c) {
      if (st_list[m].s[c] < -kGridMaxLen || st_list[m].s[c] > kGridMaxLen) return R1_EINVAL;
      zero = zero && st_list[m].s[c] == 0;
    }
    if (zero) return R1_EINVAL;
  }
  // sparse when the lines of at least 3 nodes -- the only ones that can lower a
  // node -- cover under half of the direction-node pairs (the 9-D meshes: under a
  // third; the 4-D ones: nearly all)
  double covered = 0.0;
  for (int m = 0; m < n_dir; ++m) {
    Step t = st_list[m];
    for (int len = 3; len <= kGridMaxLen; ++len) {
      step_slabs(g, &t, len);
      if (t.count == 0) break;
      covered += double(t.count) * (len == 3 ? 3.0 : 1.0);
    }
  }
  const bool sparse = covered < 0.5 * double(n_dir) * double(g.size);
  for (int m = 0; m < n_dir; ++m) step_slabs(g, &st_list[m], sparse ? 3 : 1);
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return r1h::fail(h, e, "hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == R1_F32)
    return grid_laminate_T<float>(h, g, st_list, sparse, static_cast<float*>(W), static_cast<float*>(P),
                                  static_cast<float*>(A), k_max, tol, iterations, decrease, st);
  return grid_laminate_T<double>(h, g, st_list, sparse, static_cast<double*>(W), static_cast<double*>(P),
                                 static_cast<double*>(A), k_max, tol, iterations, decrease, st);
}

r1_status r1_grid_interpolate(r1_handle h, const r1_grid* grid, r1_dtype dtype, const void* W, int64_t n,
                              const void* F, void* out, void* stream) {
  if (!h) return R1_EINVAL;
  GridArgs g;
  r1_status s = grid_args(grid, &g);
  if (s) return s;
  if (n < 0 || n > (int64_t(1) << 31) || (dtype != R1_F32 && dtype != R1_F64)) return R1_EINVAL;
  if (n == 0) return R1_OK;
  if (!W || !F || !out) return R1_EINVAL;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return r1h::fail(h, e, "hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const dim3 grd(blocks_of(n, 256));
  if (dtype == R1_F32) {
    if (grid->dim == 2)
      hipLaunchKernelGGL((k_grid_interp<float, 2>), grd, dim3(256), 0, st, g, static_cast<const float*>(W), n,
                         static_cast<const float*>(F), static_cast<float*>(out));
    else
      hipLaunchKernelGGL((k_grid_interp<float, 3>), grd, dim3(256), 0, st, g, static_cast<const float*>(W), n,
                         static_cast<const float*>(F), static_cast<float*>(out));
  } else {
    if (grid->dim == 2)
      hipLaunchKernelGGL((k_grid_interp<double, 2>), grd, dim3(256), 0, st, g, static_cast<const double*>(W), n,
                         static_cast<const double*>(F), static_cast<double*>(out));
    else
      hipLaunchKernelGGL((k_grid_interp<double, 3>), grd, dim3(256), 0, st, g, static_cast<const double*>(W), n,
                         static_cast<const double*>(F), static_cast<double*>(out));
  }
  e = hipGetLastError();
  return e == hipSuccess ? R1_OK : r1h::fail(h, e, "kernel launch");
}

}  // extern "C"
