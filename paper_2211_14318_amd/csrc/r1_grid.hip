// Global rank-one lamination on a deformation-gradient mesh (Section 4.1 of
// arXiv 2211.14318): node values W^0 = W on the mesh of Section 5.2 (one mesh
// width for every component), then iterations of eq. 4.3 -- every node takes
// the minimum over the directions of the lower hull (Algorithm 1) of the line
// of eq. 4.4 through it, clipped to the mesh's box -- until the maximal decrease
// of an iteration is at most the tolerance or k_max iterations are done
// (Section 6); off-mesh values by multilinear interpolation.  Node stresses, when
// requested, follow the laminates that lower the nodes (eq. 5.2, first case);
// interpolating them gives the off-mesh stress (eq. 5.2, second case).
//
// A direction is an integer step s in Z^{d x d}; its lines advance the node
// index by a constant stride.  One launch per direction and iteration: the
// thread of each line's first node walks the line from the previous iterate,
// builds the lower hull with a monotone chain (vertex indices on an LDS stack,
// the two top values in registers) and lowers every node inside a hull segment
// in the next iterate, which starts as a copy of the previous one.  Lines of one
// direction share no node, so the updates do not race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "r1.h"
#include "r1_device.hpp"
#include "r1_handle.hpp"

namespace {

constexpr int kGridMaxLen = 512;     // nodes per component (bounds a line's length)
constexpr int kLineThreads = 64;     // threads per block of the line kernel
constexpr int kDecBlocks = 256;      // blocks of the maximal-decrease reduction

struct GridArgs {
  int dd;                  // d*d components
  int n[9];                // nodes per component
  int64_t stride[9];       // node index step of each component (component 0 slowest)
  double lo[9];            // first node value per component
  double delta;            // mesh width
  int64_t size;            // nodes
  int maxlen;              // longest component
};

struct Step {
  int s[9];
};

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
// also P^0 = dW/dF (component-major, NaN where W is +inf).
template <typename T, int D>
__global__ __launch_bounds__(256) void k_grid_energy(GridArgs g, r1d::Material mat, double bn, T* W, T* P) {
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
}

// One direction of one iteration: the lines of step s, one per thread of their
// first node.  Non-finite values are absent from a hull and stay as they are.
// With Pin/Pout (node stresses), a lowered node takes the stress of its laminate
// with the weights of its value (eq. 5.2, first case).
template <typename T>
__global__ __launch_bounds__(kLineThreads) void k_grid_lines(GridArgs g, Step s, const T* __restrict__ Win,
                                                            T* __restrict__ Wout, const T* __restrict__ Pin,
                                                            T* __restrict__ Pout) {
  extern __shared__ uint16_t stack_mem[];
  const int64_t p = int64_t(blockIdx.x) * kLineThreads + threadIdx.x;
  if (p >= g.size) return;
  int I[9];
  node_multi(g, p, I);
  bool start = false;
  int L = kGridMaxLen;
  int64_t ds = 0;
  for (int c = 0; c < g.dd; ++c) {
    const int y = I[c] - s.s[c];
    start = start || y < 0 || y >= g.n[c];
    if (s.s[c] > 0) L = min(L, (g.n[c] - 1 - I[c]) / s.s[c] + 1);
    if (s.s[c] < 0) L = min(L, I[c] / -s.s[c] + 1);
    ds += int64_t(s.s[c]) * g.stride[c];
  }
  if (!start) return;
  uint16_t* st = stack_mem + threadIdx.x;                  // entry h at st[h * kLineThreads]
  // monotone chain: the top vertex is popped while the slope into it is at least
  // the slope from it to the new point (collinear points are not kept)
  int h = 0, i1 = 0, i2 = 0;
  T v1 = T(0), v2 = T(0);
  for (int q = 0; q < L; ++q) {
    const T w = Win[p + q * ds];
    if (!(w < inf_t<T>())) continue;
    while (h >= 2 && (v2 - v1) * T(q - i2) >= (w - v2) * T(i2 - i1)) {
      --h;
      i2 = i1;
      v2 = v1;
      if (h >= 2) {
        i1 = st[(h - 2) * kLineThreads];
        v1 = Win[p + i1 * ds];
      }
    }
    st[h * kLineThreads] = uint16_t(q);
    ++h;
    i1 = i2;
    v1 = v2;
    i2 = q;
    v2 = w;
  }
  if (h < 2) return;
  // nodes strictly inside a hull segment [a, b] read ((b - q) w_a + (q - a) w_b) / (b - a)
  int a = st[0];
  T wa = Win[p + a * ds];
  for (int k = 1; k < h; ++k) {
    const int b = st[k * kLineThreads];
    const T wb = Win[p + b * ds];
    for (int q = a + 1; q < b; ++q) {
      const int64_t idx = p + q * ds;
      if (!(Win[idx] < inf_t<T>())) continue;
      const T val = (T(b - q) * wa + T(q - a) * wb) / T(b - a);
      const T cur = Wout[idx];
      if (val < cur - T(4) * eps_t<T>() * fmax(fabs(cur), T(1e-3))) {
        Wout[idx] = val;
        if (Pout) {
          const int64_t ia = p + a * ds, ib = p + b * ds;
          for (int c = 0; c < g.dd; ++c)
            Pout[c * g.size + idx] = (T(b - q) * Pin[c * g.size + ia] + T(q - a) * Pin[c * g.size + ib]) / T(b - a);
        }
      }
    }
    a = b;
    wa = wb;
  }
}

// Per-block maxima of Win - Wout over nodes with finite Win (in double).
template <typename T>
__global__ __launch_bounds__(256) void k_grid_maxdec(int64_t n, const T* Win, const T* Wout, double* partial) {
  __shared__ double red[256];
  double m = 0.0;
  for (int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x; p < n; p += int64_t(gridDim.x) * 256) {
    const T a = Win[p];
    if (a < inf_t<T>()) m = fmax(m, double(a) - double(Wout[p]));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
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

r1_status grid_args(const r1_grid* grid, GridArgs* g) {
  if (!grid || (grid->dim != 2 && grid->dim != 3)) return R1_EINVAL;
  if (!(grid->delta > 0.0) || !std::isfinite(grid->delta)) return R1_EINVAL;
  g->dd = grid->dim * grid->dim;
  g->delta = grid->delta;
  g->maxlen = 1;
  int64_t size = 1;
  for (int c = 0; c < g->dd; ++c) {
    if (grid->n[c] < 1 || grid->n[c] > kGridMaxLen || !std::isfinite(grid->lo[c])) return R1_EINVAL;
    g->n[c] = grid->n[c];
    g->lo[c] = grid->lo[c];
    g->maxlen = std::max(g->maxlen, int(grid->n[c]));
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

inline unsigned blocks_of(int64_t n, int b) { return unsigned((n + b - 1) / b); }

template <typename T>
hipError_t grid_sweep(const GridArgs& g, const std::vector<Step>& steps, const T* Win, T* Wout, const T* Pin,
                      T* Pout, double* partial, hipStream_t st, KTimer* tm) {
  hipError_t e = hipMemcpyAsync(Wout, Win, sizeof(T) * size_t(g.size), hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && Pout)
    e = hipMemcpyAsync(Pout, Pin, sizeof(T) * size_t(g.size) * size_t(g.dd), hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  const size_t lds = sizeof(uint16_t) * size_t(kLineThreads) * size_t(g.maxlen);
  for (const Step& s : steps) {
    if (tm) tm->begin("grid_lines", st);
    hipLaunchKernelGGL((k_grid_lines<T>), dim3(blocks_of(g.size, kLineThreads)), dim3(kLineThreads), lds, st, g, s,
                       Win, Wout, Pin, Pout);
    if (tm) tm->end(st);
  }
  const int nb = int(std::min<int64_t>(kDecBlocks, (g.size + 255) / 256));
  hipLaunchKernelGGL((k_grid_maxdec<T>), dim3(nb), dim3(256), 0, st, g.size, Win, Wout, partial);
  return hipGetLastError();
}

template <typename T>
r1_status grid_laminate_T(r1_handle h, const GridArgs& g, const std::vector<Step>& steps, T* W, T* P, int k_max,
                          double tol, int32_t* iterations, double* decrease, hipStream_t st) {
  const size_t wbytes = (sizeof(T) * size_t(g.size) + 255) & ~size_t(255);
  const size_t pbytes = P ? (sizeof(T) * size_t(g.size) * size_t(g.dd) + 255) & ~size_t(255) : 0;
  void* base = nullptr;
  r1_status s = r1h::scratch(h, wbytes + pbytes + sizeof(double) * kDecBlocks, &base);
  if (s) return s;
  T* other = static_cast<T*>(base);
  T* pother = P ? reinterpret_cast<T*>(static_cast<char*>(base) + wbytes) : nullptr;
  double* partial = reinterpret_cast<double*>(static_cast<char*>(base) + wbytes + pbytes);
  const int nb = int(std::min<int64_t>(kDecBlocks, (g.size + 255) / 256));
  std::vector<double> host(nb);
  KTimer* tm = h->timer.on ? &h->timer : nullptr;
  T* cur = W;
  T* nxt = other;
  T* pcur = P;
  T* pnxt = pother;
  int k = 0;
  while (k < k_max) {
    hipError_t e = grid_sweep<T>(g, steps, cur, nxt, pcur, pnxt, partial, st, tm);
    if (e == hipSuccess) e = hipMemcpyAsync(host.data(), partial, sizeof(double) * nb, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return r1h::fail(h, e, "grid iteration");
    double md = 0.0;
    for (double v : host) md = std::max(md, v);
    if (decrease) decrease[k] = md;
    ++k;
    std::swap(cur, nxt);
    std::swap(pcur, pnxt);
    if (md <= tol) break;
  }
  if (cur != W) {
    hipError_t e = hipMemcpyAsync(W, cur, sizeof(T) * size_t(g.size), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && P)
      e = hipMemcpyAsync(P, pcur, sizeof(T) * size_t(g.size) * size_t(g.dd), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return r1h::fail(h, e, "grid copy");
  }
  if (iterations) *iterations = k;
  return R1_OK;
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
                         void* W, void* P, void* stream) {
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
  if (dtype == R1_F32) {
    if (grid->dim == 2) hipLaunchKernelGGL((k_grid_energy<float, 2>), grd, dim3(256), 0, st, g, m, beta_n, static_cast<float*>(W), static_cast<float*>(P));
    else hipLaunchKernelGGL((k_grid_energy<float, 3>), grd, dim3(256), 0, st, g, m, beta_n, static_cast<float*>(W), static_cast<float*>(P));
  } else {
    if (grid->dim == 2) hipLaunchKernelGGL((k_grid_energy<double, 2>), grd, dim3(256), 0, st, g, m, beta_n, static_cast<double*>(W), static_cast<double*>(P));
    else hipLaunchKernelGGL((k_grid_energy<double, 3>), grd, dim3(256), 0, st, g, m, beta_n, static_cast<double*>(W), static_cast<double*>(P));
  }
  e = hipGetLastError();
  return e == hipSuccess ? R1_OK : r1h::fail(h, e, "kernel launch");
}

r1_status r1_grid_laminate(r1_handle h, const r1_grid* grid, int32_t n_dir, const int32_t* steps, r1_dtype dtype,
                           void* W, void* P, int32_t k_max, double tol, int32_t* iterations, double* decrease,
                           void* stream) {
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
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return r1h::fail(h, e, "hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == R1_F32)
    return grid_laminate_T<float>(h, g, st_list, static_cast<float*>(W), static_cast<float*>(P), k_max, tol,
                                  iterations, decrease, st);
  return grid_laminate_T<double>(h, g, st_list, static_cast<double*>(W), static_cast<double*>(P), k_max, tol,
                                 iterations, decrease, st);
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
