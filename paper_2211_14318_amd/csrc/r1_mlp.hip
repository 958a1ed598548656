// Kernels of the learned surrogate (gfx950) outside the training step (which is
// in r1_train.hip): data packing and statistics, and the fused inference kernel
// with the routing gates -- BF16 MFMA (v_mfma_f32_32x32x16_bf16, FP32
// accumulation) for the width x width layers, FP32 for the small first and last
// layers.
//
// MFMA 32x32x16 lane layout (64 lanes): A fragment = row (lane % 32), k =
// 8*(lane/32) .. +7; B fragment = column (lane % 32), same k; accumulator j of
// lane l holds row 8*(j/4) + 4*(l/32) + (j%4), column l % 32.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "r1_device.hpp"
#include "r1_mlp.hpp"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kWaveM = 64;

namespace r1m {

// Logistic function with the hardware reciprocal (about 1 ulp): the activations
// are rounded to BF16 next (or feed an FP32 dot product of ~1e-4 accuracy), so
// the exactly rounded divide bought nothing and cost 9 instructions per unit.
__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }

// Packed rows -> SoA F (float) and beta_n.
__global__ void k_unpack(int dd, int64_t n, const float* X, float* F, float* bn) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  for (int k = 0; k < dd; ++k) F[int64_t(k) * n + p] = X[p * (dd + 1) + k];
  bn[p] = X[p * (dd + 1) + dd];
}

__global__ void k_fill(int64_t n, float* p, float v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Gap-form targets from packed rows: T = (W(F) - W^k, P0(F) - P^k), W and P0 of
// the unrelaxed potential (eq. 2.9, 2.12) in double.
template <int D>
__global__ void k_targets(int64_t n, r1d::Material mat, const float* X, const float* Y, float* T) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  constexpr int DI = D * D + 1;
  double G[D * D], cof[D * D], P0[D * D];
  for (int k = 0; k < D * D; ++k) G[k] = X[p * DI + k];
  const double bn = X[p * DI + D * D];
  r1d::Point<double> q = r1d::make_point_any<double>(mat, bn);
  r1d::cofactor<D>(G, cof);
  const double w = r1d::w_point_any<double, D>(q, G, cof);
  r1d::stress0_any<D>(mat, bn, G, P0);
  T[p * DI] = float(w - double(Y[p * DI]));
  for (int k = 0; k < D * D; ++k) T[p * DI + 1 + k] = float(P0[k] - double(Y[p * DI + 1 + k]));
}

__device__ __forceinline__ void atomic_min_f(float* a, float v) {
  int* ai = reinterpret_cast<int*>(a);
  int old = *ai;
  while (v < __int_as_float(old)) {
    int assumed = old;
    old = atomicCAS(ai, assumed, __float_as_int(v));
    if (old == assumed) break;
  }
}
__device__ __forceinline__ void atomic_max_f(float* a, float v) {
  int* ai = reinterpret_cast<int*>(a);
  int old = *ai;
  while (v > __int_as_float(old)) {
    int assumed = old;
    old = atomicCAS(ai, assumed, __float_as_int(v));
    if (old == assumed) break;
  }
}

// Per-column sum, sum of squares, minimum and maximum over rows [0, n) of a
// row-major n x ncol matrix (ncol <= kMaxCols), and (when dF > 0) the smallest
// det of the dF x dF matrices in the first dF*dF columns.  Block-reduced, one
// atomic per block and column.  stats layout: sum[c], sum2[c] (double);
// mn[c], mx[c], det_min (float).
__global__ __launch_bounds__(256) void k_colstats(int64_t n, int ncol, int dF, const float* A,
                                                  double* sum, double* sum2, float* mn, float* mx,
                                                  float* det_min) {
  double s[kMaxCols], s2[kMaxCols];
  float lo[kMaxCols], hi[kMaxCols];
  float dmin = __builtin_inff();
  for (int c = 0; c < kMaxCols; ++c) { s[c] = 0; s2[c] = 0; lo[c] = __builtin_inff(); hi[c] = -__builtin_inff(); }
  for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n; p += int64_t(gridDim.x) * blockDim.x) {
    const float* row = A + p * ncol;
    for (int c = 0; c < kMaxCols; ++c) {
      if (c >= ncol) break;
      float v = row[c];
      s[c] += v; s2[c] += double(v) * v;
      lo[c] = fminf(lo[c], v); hi[c] = fmaxf(hi[c], v);
    }
    if (dF == 2) dmin = fminf(dmin, row[0] * row[3] - row[1] * row[2]);
    if (dF == 3)
      dmin = fminf(dmin, row[0] * (row[4] * row[8] - row[5] * row[7]) - row[1] * (row[3] * row[8] - row[5] * row[6]) +
                             row[2] * (row[3] * row[7] - row[4] * row[6]));
  }
  __shared__ double rs[256];
  __shared__ float rf[256];
  for (int c = 0; c < ncol; ++c) {
    rs[threadIdx.x] = s[c];
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) { if (threadIdx.x < k) rs[threadIdx.x] += rs[threadIdx.x + k]; __syncthreads(); }
    if (threadIdx.x == 0) atomicAdd(&sum[c], rs[0]);
    __syncthreads();
    rs[threadIdx.x] = s2[c];
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) { if (threadIdx.x < k) rs[threadIdx.x] += rs[threadIdx.x + k]; __syncthreads(); }
    if (threadIdx.x == 0) atomicAdd(&sum2[c], rs[0]);
    __syncthreads();
    rf[threadIdx.x] = lo[c];
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) { if (threadIdx.x < k) rf[threadIdx.x] = fminf(rf[threadIdx.x], rf[threadIdx.x + k]); __syncthreads(); }
    if (threadIdx.x == 0) atomic_min_f(&mn[c], rf[0]);
    __syncthreads();
    rf[threadIdx.x] = hi[c];
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) { if (threadIdx.x < k) rf[threadIdx.x] = fmaxf(rf[threadIdx.x], rf[threadIdx.x + k]); __syncthreads(); }
    if (threadIdx.x == 0) atomic_max_f(&mx[c], rf[0]);
    __syncthreads();
  }
  if (dF > 0) {
    rf[threadIdx.x] = dmin;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) { if (threadIdx.x < k) rf[threadIdx.x] = fminf(rf[threadIdx.x], rf[threadIdx.x + k]); __syncthreads(); }
    if (threadIdx.x == 0) atomic_min_f(det_min, rf[0]);
  }
}

// Packs SoA lamination data into rows: X = (F, beta_n), Y = (W, P).
template <typename T, int D>
__global__ void k_pack(int64_t n, const T* F, const T* bn, const T* W, const T* P, float* X, float* Y) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  constexpr int DI = D * D + 1;
  for (int k = 0; k < D * D; ++k) X[p * DI + k] = float(F[int64_t(k) * n + p]);
  X[p * DI + D * D] = float(bn[p]);
  Y[p * DI] = float(W[p]);
  for (int k = 0; k < D * D; ++k) Y[p * DI + 1 + k] = float(P[int64_t(k) * n + p]);
}

// Bin of a point for the error gate: radius |F - I|_F over [0, r_max) and beta_n
// over [b_lo, b_hi), clamped.
template <int D>
__device__ __forceinline__ int gate_bin(const InferParams& ip, const double* F, double bn) {
  double r2 = 0.0;
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) {
      double e = F[i * D + j] - (i == j ? 1.0 : 0.0);
      r2 += e * e;
    }
  int br = int(sqrt(r2) / ip.r_max * kBinsR);
  int bb = int((bn - ip.b_lo) / (ip.b_hi - ip.b_lo) * kBinsB);
  br = br < 0 ? 0 : (br >= kBinsR ? kBinsR - 1 : br);
  bb = bb < 0 ? 0 : (bb >= kBinsB ? kBinsB - 1 : bb);
  return br * kBinsB + bb;
}

// Fused inference for widths whose weights do not fit in LDS (see
// k_infer_lds): 4 waves x 32 points per block.  Per point: load F, beta_n;
// gates; first layer (FP32) into the wave's LDS activations (BF16); each hidden
// width x width layer as 32 x 16-deep MFMA tiles with B fragments read from the
// BF16 weights in global memory (L2-resident), bias + SiLU, back to LDS; output
// layer in FP32; exact W(F), P0(F); W = W(F) - max(g, 0), P = P0 - dP.
// MODE 0: gates on, each point's status (fallback / served) to ip.status.
// MODE 1 (calibration): box gate only; the gate cell, predicted W and
// predicted gap go to cal_bin / cal_w / cal_gap, rejected points get cell -1.
template <typename T, int D, int WID, int MODE, int FAM>
__global__ __launch_bounds__(256, 2) void k_infer(InferParams ip, const T* F, const T* bn, T* W,
                                               T* P, int32_t* flags, int* cal_bin, float* cal_w,
                                               float* cal_gap) {
  constexpr int DI = D * D + 1, DO = D * D + 1;
  constexpr int LD = WID + 8;                      // padded BF16 row stride (bank spread)
  extern __shared__ char smem[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __bf16* act = reinterpret_cast<__bf16*>(smem) + wave * 32 * LD;
  const int r = lane & 31, half = lane >> 5;
  const int64_t pt = int64_t(blockIdx.x) * 128 + wave * 32 + r;
  const bool valid = pt < ip.n;
  const int64_t pc = valid ? pt : ip.n - 1;        // clamp for loads
  double G[D * D];
  for (int k = 0; k < D * D; ++k) G[k] = double(F[int64_t(k) * ip.n + pc]);
  const double b = double(bn[pc]);
  float x[DI];
  bool ok = true;
  for (int k = 0; k < DI; ++k) {
    float raw = k < D * D ? float(G[k]) : float(b);
    ok = ok && raw >= ip.x_lo[k] && raw <= ip.x_hi[k];
    x[k] = (raw - ip.x_mean[k]) / ip.x_std[k];
  }
  double cof[D * D];
  r1d::cofactor<D>(G, cof);
  const double det = r1d::det_of<D>(G, cof);
  ok = ok && det >= double(ip.det_lo);
  const int bin = gate_bin<D>(ip, G, b);
  // first layer: this lane computes features [half*WID/2, (half+1)*WID/2)
  for (int f = half * (WID / 2); f < (half + 1) * (WID / 2); ++f) {
    float z = ip.b[0][f];
    for (int k = 0; k < DI; ++k) z = fmaf(ip.w0[f * DI + k], x[k], z);
    act[r * LD + f] = __bf16(silu(z));
  }
  __syncthreads();
  // hidden width x width layers on the matrix cores; a k step's B fragments
  // (one per 32-column tile) are loaded together, and the next step's while
  // this step's products run, so their L2 latency overlaps the matrix cores
  constexpr int NT = WID / 32;
  for (int l = 1; l < ip.n_hidden; ++l) {
    // fragment (k step ks, tile t) of this lane: wf[(ks NT + t) 64] (r1m_wfrag)
    const bf16x8* wf = static_cast<const bf16x8*>(ip.wfrag) + int64_t(l - 1) * (WID * WID / 8) + lane;
    f32x16 acc[NT];
    bf16x8 bw[NT], bn[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      acc[t] = f32x16{};
      bw[t] = wf[t * 64];
    }
    for (int k0 = 0; k0 < WID; k0 += 16) {
      const int kn = k0 + 16 < WID ? k0 / 16 + 1 : k0 / 16;   // the last step reloads its own fragments
#pragma unroll
      for (int t = 0; t < NT; ++t) bn[t] = wf[(kn * NT + t) * 64];
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(act + r * LD + k0 + 8 * half);
      // keep the next step's loads ahead of this step's products (the scheduler
      // would otherwise sink each load to its use to save registers)
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int t = 0; t < WID / 32; ++t) acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bw[t], acc[t], 0, 0, 0);
#pragma unroll
      for (int t = 0; t < WID / 32; ++t) bw[t] = bn[t];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < WID / 32; ++t)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int row = 8 * (j >> 2) + 4 * half + (j & 3);
        const int col = t * 32 + r;
        act[row * LD + col] = __bf16(silu(acc[t][j] + ip.b[l][col]));
      }
    __syncthreads();
  }
  // output layer: each lane sums half the features of its point, partner completes
  float out[DO];
  for (int j = 0; j < DO; ++j) {
    float s = 0.0f;
    for (int k = half * (WID / 2); k < (half + 1) * (WID / 2); ++k)
      s = fmaf(ip.wout[j * WID + k], float(act[r * LD + k]), s);
    s += __shfl_xor(s, 32);
    out[j] = s + ip.bout[j];
  }
  if (half != 0 || !valid) return;
  // de-standardize; a non-positive gap means no lamination: W(F), P0(F) exactly
  const float rawf = out[0] * ip.y_std[0] + ip.y_mean[0];
  const double raw = double(rawf);
  const bool convex = raw <= 0.0;
  r1d::Point<double> q = r1d::make_point<double, FAM>(ip.mat, b);
  const double w_un = r1d::w_point<double, D, FAM>(q, G, cof);
  const double wpred = convex ? w_un : w_un - raw;
  if (MODE == 1) {
    cal_bin[pt] = ok ? bin : -1;
    cal_w[pt] = float(wpred);
    cal_gap[pt] = rawf;
    return;
  }
  if (ip.bins_on) ok = ok && rawf <= ip.gate_tau[bin];
  ok = ok && det > 0.0;
  ip.status[pt] = ok ? 2 : 1;
  if (!ok) return;
  double P0[D * D];
  r1d::stress0<D, FAM>(ip.mat, b, G, P0);
  W[pt] = T(wpred);
  for (int k = 0; k < D * D; ++k)
    P[int64_t(k) * ip.n + pt] =
        T(convex ? P0[k] : P0[k] - double(out[1 + k] * ip.y_std[1 + k] + ip.y_mean[1 + k]));
  if (flags) flags[pt] = 0;
}

// Bytes of LDS k_infer_lds needs: the BF16 hidden layers (rows padded by 8)
// and the FP32 first layer, biases, last layer.
__host__ __device__ inline size_t infer_lds_bytes(int width, int n_hidden, int d_in, int d_out) {
  return size_t(n_hidden - 1) * width * (width + 8) * 2 +
         sizeof(float) * (size_t(width) * d_in + size_t(n_hidden) * width + size_t(d_out) * width + d_out);
}

// Fused inference with LDS-resident weights and register-resident activations.
// A persistent block of 8 waves stages the hidden layers (BF16), the first and
// last layers and the biases in LDS once; each wave then takes tiles of 32
// points.  Lane (p = lane % 32, half = lane / 32) of a tile:
//  * first layer in FP32 for the 8 features per 16-deep k step that its B
//    fragments hold (features 16 s + 8 half + i);
//  * each width x width layer as (width/32) x (width/16) MFMA 32x32x16 steps with
//    the weights as A (rows = output features) and the activations as B
//    (columns = points); bias + SiLU on the accumulators (lane holds features
//    8 (j/4) + 4 half + j%4 of each 32-feature tile), and one exchange of four
//    packed values with the lane 32 away forms the next layer's B fragments;
//  * last layer: FP32 dot products over each lane's half of the features,
//    completed by the same exchange;
//  * gates, then W(F) (lower half) and P0(F) (upper half) in FP64.
// MODE as in k_infer.
template <typename T, int D, int WID, int MODE, int FAM>
__global__ __launch_bounds__(512) void k_infer_lds(InferParams ip, const T* F, const T* bn, T* W, T* P,
                                                   int32_t* flags, int* cal_bin, float* cal_w, float* cal_gap) {
  constexpr int DI = D * D + 1, DO = D * D + 1;
  constexpr int LDW = WID + 8;
  constexpr int NS = WID / 16, NT = WID / 32;
  extern __shared__ char smem[];
  const int L = ip.n_hidden;
  __bf16* wl = reinterpret_cast<__bf16*>(smem);                       // (L-1) x WID x LDW
  float* w0 = reinterpret_cast<float*>(wl + size_t(L - 1) * WID * LDW);  // WID x DI
  float* bb = w0 + WID * DI;                                          // L x WID
  float* wo = bb + L * WID;                                           // DO x WID
  float* bo = wo + DO * WID;                                          // DO
  for (int i = threadIdx.x; i < (L - 1) * WID * (WID / 8); i += blockDim.x) {
    const int l = i / (WID * (WID / 8)), rem = i % (WID * (WID / 8));
    const int row = rem / (WID / 8), c8 = rem % (WID / 8);
    *reinterpret_cast<bf16x8*>(wl + (size_t(l) * WID + row) * LDW + c8 * 8) =
        *reinterpret_cast<const bf16x8*>(static_cast<const __bf16*>(ip.wbf[l + 1]) + row * WID + c8 * 8);
  }
  for (int i = threadIdx.x; i < WID * DI; i += blockDim.x) w0[i] = ip.w0[i];
  for (int i = threadIdx.x; i < L * WID; i += blockDim.x) bb[i] = ip.b[i / WID][i % WID];
  for (int i = threadIdx.x; i < DO * WID; i += blockDim.x) wo[i] = ip.wout[i];
  if (threadIdx.x < DO) bo[threadIdx.x] = ip.bout[threadIdx.x];
  __syncthreads();

  const int lane = threadIdx.x & 63, r = lane & 31, half = lane >> 5;
  const int64_t waves = int64_t(gridDim.x) * (blockDim.x >> 6);
  for (int64_t tile = int64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6); tile * 32 < ip.n;
       tile += waves) {
    const int64_t pt = tile * 32 + r;
    const bool valid = pt < ip.n;
    const int64_t pc = valid ? pt : ip.n - 1;        // clamp for loads
    double G[D * D];
    for (int k = 0; k < D * D; ++k) G[k] = double(F[int64_t(k) * ip.n + pc]);
    const double b = double(bn[pc]);
    float x[DI];
    bool ok = true;
    for (int k = 0; k < DI; ++k) {
      const float raw = k < D * D ? float(G[k]) : float(b);
      ok = ok && raw >= ip.x_lo[k] && raw <= ip.x_hi[k];
      x[k] = (raw - ip.x_mean[k]) / ip.x_std[k];
    }
    // first layer: the features of this lane's B fragments
    bf16x8 bf[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int f = s * 16 + 8 * half + i;
        float z = bb[f];
#pragma unroll
        for (int k = 0; k < DI; ++k) z = fmaf(w0[f * DI + k], x[k], z);
        bf[s][i] = __bf16(silu(z));
      }
    // hidden layers on the matrix cores
    f32x16 acc[NT];
    for (int l = 1; l < L; ++l) {
      const __bf16* wlay = wl + size_t(l - 1) * WID * LDW;
      // the accumulators start at the bias (the MFMA sums onto it)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[t][j] = bb[l * WID + t * 32 + 8 * (j >> 2) + 4 * half + (j & 3)];
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const bf16x8 a = *reinterpret_cast<const bf16x8*>(wlay + (t * 32 + r) * LDW + s * 16 + 8 * half);
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bf[s], acc[t], 0, 0, 0);
        }
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int j = 0; j < 16; ++j)
          acc[t][j] = silu(acc[t][j]);
      if (l + 1 < L) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int t = s >> 1, j0 = 8 * (s & 1);
          __bf16 keep[4], send[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            keep[i] = __bf16(half ? acc[t][j0 + 4 + i] : acc[t][j0 + i]);
            send[i] = __bf16(half ? acc[t][j0 + i] : acc[t][j0 + 4 + i]);
          }
          const uint32_t s01 = uint32_t(__builtin_bit_cast(uint16_t, send[0])) |
                               (uint32_t(__builtin_bit_cast(uint16_t, send[1])) << 16);
          const uint32_t s23 = uint32_t(__builtin_bit_cast(uint16_t, send[2])) |
                               (uint32_t(__builtin_bit_cast(uint16_t, send[3])) << 16);
          const uint32_t r01 = uint32_t(__shfl_xor(int(s01), 32, kWaveM));
          const uint32_t r23 = uint32_t(__shfl_xor(int(s23), 32, kWaveM));
          __bf16 recv[4] = {__builtin_bit_cast(__bf16, uint16_t(r01 & 0xffffu)),
                            __builtin_bit_cast(__bf16, uint16_t(r01 >> 16)),
                            __builtin_bit_cast(__bf16, uint16_t(r23 & 0xffffu)),
                            __builtin_bit_cast(__bf16, uint16_t(r23 >> 16))};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            bf[s][i] = half ? recv[i] : keep[i];
            bf[s][4 + i] = half ? keep[i] : recv[i];
          }
        }
      }
    }
    // last layer: this lane's features, completed by the lane 32 away
    float out[DO];
#pragma unroll
    for (int o = 0; o < DO; ++o) {
      float sacc = 0.0f;
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int j = 0; j < 16; ++j)
          sacc = fmaf(wo[o * WID + t * 32 + 8 * (j >> 2) + 4 * half + (j & 3)], acc[t][j], sacc);
      sacc += __shfl_xor(sacc, 32, kWaveM);
      out[o] = sacc + bo[o];
    }
    double cof[D * D];
    r1d::cofactor<D>(G, cof);
    const double det = r1d::det_of<D>(G, cof);
    ok = ok && det >= double(ip.det_lo);
    const int bin = gate_bin<D>(ip, G, b);
    const float rawf = out[0] * ip.y_std[0] + ip.y_mean[0];
    const double raw = double(rawf);
    const bool convex = raw <= 0.0;
    if (MODE == 1) {
      if (valid && half == 0) {
        r1d::Point<double> q = r1d::make_point<double, FAM>(ip.mat, b);
        const double w_un = r1d::w_point<double, D, FAM>(q, G, cof);
        cal_bin[pt] = ok ? bin : -1;
        cal_w[pt] = float(convex ? w_un : w_un - raw);
        cal_gap[pt] = rawf;
      }
      continue;
    }
    if (ip.bins_on) ok = ok && rawf <= ip.gate_tau[bin];
    ok = ok && det > 0.0;
    if (valid && half == 0) ip.status[pt] = ok ? 2 : 1;
    if (!valid || !ok) continue;
    if (half == 0) {
      r1d::Point<double> q = r1d::make_point<double, FAM>(ip.mat, b);
      const double w_un = r1d::w_point<double, D, FAM>(q, G, cof);
      W[pt] = T(convex ? w_un : w_un - raw);
      if (flags) flags[pt] = 0;
    } else {
      double P0[D * D];
      r1d::stress0<D, FAM>(ip.mat, b, G, P0);
      for (int k = 0; k < D * D; ++k)
        P[int64_t(k) * ip.n + pt] =
            T(convex ? P0[k] : P0[k] - double(out[1 + k] * ip.y_std[1 + k] + ip.y_mean[1 + k]));
    }
  }
}

// The fallback and candidate lists from the inference kernels' per-point status
// (1 = fallback, 2 = served): each block takes 2048 consecutive points, counts
// them by wave ballots and reserves its slots with one atomic per list.  Building
// the lists here rather than in the inference kernels keeps those free of
// atomics whose returned slot a wave had to wait for on every tile.
constexpr int kListPer = 8;
__global__ __launch_bounds__(256) void k_lists(int64_t n, const uint8_t* status, int* fb_count, int32_t* fb_list,
                                               int* cand_count, int32_t* cand_list) {
  __shared__ int wsum[2][4], wbase[2][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t b0 = int64_t(blockIdx.x) * 256 * kListPer;
  const unsigned long long lt = (1ull << lane) - 1ull;
  int v[kListPer];
  int cf = 0, cc = 0;
#pragma unroll
  for (int j = 0; j < kListPer; ++j) {
    const int64_t p = b0 + j * 256 + threadIdx.x;
    v[j] = p < n ? status[p] : 0;
  }
#pragma unroll
  for (int j = 0; j < kListPer; ++j) {
    cf += __popcll(__ballot(v[j] == 1));
    cc += __popcll(__ballot(v[j] == 2));
  }
  if (lane == 0) { wsum[0][wave] = cf; wsum[1][wave] = cc; }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int li = threadIdx.x;
    int tot = 0;
    for (int w = 0; w < 4; ++w) tot += wsum[li][w];
    int base = 0;
    if (tot > 0) base = li == 0 ? atomicAdd(fb_count, tot) : (cand_list ? atomicAdd(cand_count, tot) : 0);
    for (int w = 0; w < 4; ++w) { wbase[li][w] = base; base += wsum[li][w]; }
  }
  __syncthreads();
  int of = wbase[0][wave], oc = wbase[1][wave];
#pragma unroll
  for (int j = 0; j < kListPer; ++j) {
    const int64_t p = b0 + j * 256 + threadIdx.x;
    const unsigned long long mf = __ballot(v[j] == 1), mc = __ballot(v[j] == 2);
    if (v[j] == 1) fb_list[of + __popcll(mf & lt)] = int32_t(p);
    if (v[j] == 2 && cand_list) cand_list[oc + __popcll(mc & lt)] = int32_t(p);
    of += __popcll(mf);
    oc += __popcll(mc);
  }
}

// Gather fallback points into compact SoA arrays, and scatter their results back.
template <typename T, int D>
__global__ void k_fb_gather(int64_t n, int nfb, const int32_t* list, const T* F, const T* bn, T* Fc,
                            T* bc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nfb) return;
  const int64_t p = list[i];
  for (int k = 0; k < D * D; ++k) Fc[int64_t(k) * nfb + i] = F[int64_t(k) * n + p];
  bc[i] = bn[p];
}

template <typename T, int D>
__global__ void k_fb_scatter(int64_t n, int nfb, const int32_t* list, const T* Wc, const T* Pc,
                             const int32_t* fc, T* W, T* P, int32_t* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nfb) return;
  const int64_t p = list[i];
  W[p] = Wc[i];
  for (int k = 0; k < D * D; ++k) P[int64_t(k) * n + p] = Pc[int64_t(k) * nfb + i];
  if (flags) flags[p] = fc[i] | R1_PT_FALLBACK;
}

}  // namespace r1m

// ---- launchers -----------------------------------------------------------------

using namespace r1m;

static inline unsigned nblk(int64_t n, int b = 256) { return unsigned((n + b - 1) / b); }

hipError_t r1m_unpack(int dim, int64_t n, const float* X, float* F, float* bn, hipStream_t st) {
  hipLaunchKernelGGL(k_unpack, dim3(nblk(n)), dim3(256), 0, st, dim * dim, n, X, F, bn);
  return hipGetLastError();
}

// one thread per destination element, in destination order (see r1m_wfrag)
__global__ void k_wfrag(int64_t total, int width, const __bf16* wbf, __bf16* wfrag) {
  const int64_t d = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (d >= total) return;
  const int nt = width / 32, ks_n = width / 16;
  const int e = int(d % 8), lane = int((d / 8) % 64);
  const int t = int((d / 512) % nt), ks = int((d / (512 * int64_t(nt))) % ks_n);
  const int64_t l1 = d / (int64_t(width) * width);
  const int r = lane & 31, half = lane >> 5;
  wfrag[d] = wbf[l1 * width * width + int64_t(t * 32 + r) * width + ks * 16 + 8 * half + e];
}

hipError_t r1m_wfrag(int width, int n_hidden, const void* wbf, void* wfrag, hipStream_t st) {
  const int64_t total = int64_t(n_hidden - 1) * width * width;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_wfrag, dim3(nblk(total)), dim3(256), 0, st, total, width, static_cast<const __bf16*>(wbf),
                     static_cast<__bf16*>(wfrag));
  return hipGetLastError();
}

hipError_t r1m_fill(int64_t n, float* p, float v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3(nblk(n)), dim3(256), 0, st, n, p, v);
  return hipGetLastError();
}

hipError_t r1m_targets(int dim, int64_t n, const r1d::Material& mat, const float* X, const float* Y,
                       float* T, hipStream_t st) {
  if (dim == 2) hipLaunchKernelGGL(k_targets<2>, dim3(nblk(n)), dim3(256), 0, st, n, mat, X, Y, T);
  else hipLaunchKernelGGL(k_targets<3>, dim3(nblk(n)), dim3(256), 0, st, n, mat, X, Y, T);
  return hipGetLastError();
}

hipError_t r1m_colstats(int64_t n, int ncol, int dF, const float* A, double* sum, double* sum2, float* mn,
                        float* mx, float* det_min, hipStream_t st) {
  unsigned g = nblk(n);
  if (g > 1024) g = 1024;
  hipLaunchKernelGGL(k_colstats, dim3(g), dim3(256), 0, st, n, ncol, dF, A, sum, sum2, mn, mx, det_min);
  return hipGetLastError();
}

hipError_t r1m_pack(int dtype, int dim, int64_t n, const void* F, const void* bn, const void* W,
                    const void* P, float* X, float* Y, hipStream_t st) {
#define R1P(T, D) hipLaunchKernelGGL((k_pack<T, D>), dim3(nblk(n)), dim3(256), 0, st, n, static_cast<const T*>(F), \
                                     static_cast<const T*>(bn), static_cast<const T*>(W), static_cast<const T*>(P), X, Y)
  if (dtype == R1_F32) { if (dim == 2) R1P(float, 2); else R1P(float, 3); }
  else { if (dim == 2) R1P(double, 2); else R1P(double, 3); }
#undef R1P
  return hipGetLastError();
}

size_t r1m_infer_lds(int width) { return size_t(4) * 32 * (width + 8) * 2; }

template <typename T, int D, int FAM>
static hipError_t infer_TD(const InferParams& ip, int mode, const void* F, const void* bn, void* W, void* P,
                           int32_t* flags, int* fb_count, int32_t* fb_list, int* cal_bin, float* cal_w,
                           float* cal_gap, hipStream_t st) {
  const size_t lds2 = infer_lds_bytes(ip.width, ip.n_hidden, D * D + 1, D * D + 1);
  if (ip.width <= 128 && lds2 <= size_t(160) * 1024) {
    // weights resident in LDS: one persistent block of 8 waves per CU
    int dev = 0, n_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const int64_t blocks = (ip.n + 255) / 256;
    dim3 grid(unsigned(blocks < n_cu ? blocks : n_cu));
#define R1L(WID, MODE) (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_infer_lds<T, D, WID, MODE, FAM>), \
      hipFuncAttributeMaxDynamicSharedMemorySize, int(lds2)); \
  hipLaunchKernelGGL((k_infer_lds<T, D, WID, MODE, FAM>), grid, dim3(512), lds2, st, ip, \
      static_cast<const T*>(F), static_cast<const T*>(bn), static_cast<T*>(W), static_cast<T*>(P), flags, \
      cal_bin, cal_w, cal_gap)
#define R1V(WID) if (ip.width == WID) { if (mode == 0) { R1L(WID, 0); } else { R1L(WID, 1); } return hipGetLastError(); }
    R1V(32) R1V(64) R1V(128)
#undef R1V
#undef R1L
    return hipErrorInvalidValue;
  }
  dim3 grid(unsigned((ip.n + 127) / 128));
  size_t lds = r1m_infer_lds(ip.width);
#define R1I(WID, MODE) (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_infer<T, D, WID, MODE, FAM>), \
      hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)); \
  hipLaunchKernelGGL((k_infer<T, D, WID, MODE, FAM>), grid, dim3(256), lds, st, ip, \
      static_cast<const T*>(F), static_cast<const T*>(bn), static_cast<T*>(W), static_cast<T*>(P), flags, \
      cal_bin, cal_w, cal_gap)
#define R1W(WID) if (ip.width == WID) { if (mode == 0) { R1I(WID, 0); } else { R1I(WID, 1); } return hipGetLastError(); }
  R1W(256)
#undef R1W
#undef R1I
  return hipErrorInvalidValue;
}

hipError_t r1m_infer(int dtype, int dim, const InferParams& ip, int mode, const void* F, const void* bn,
                     void* W, void* P, int32_t* flags, int* fb_count, int32_t* fb_list, int* cal_bin,
                     float* cal_w, float* cal_gap, hipStream_t st) {
  // one set of kernels per model family (exact W and P0 of the material in the epilogue)
#define R1F(T, D) (ip.mat.model == R1_STVK_DAMAGE                                                                   \
                       ? infer_TD<T, D, r1d::kFamSTVK>(ip, mode, F, bn, W, P, flags, fb_count, fb_list, cal_bin, \
                                                       cal_w, cal_gap, st)                                       \
                       : infer_TD<T, D, r1d::kFamNH>(ip, mode, F, bn, W, P, flags, fb_count, fb_list, cal_bin,   \
                                                     cal_w, cal_gap, st))
  hipError_t e = dtype == R1_F32 ? (dim == 2 ? R1F(float, 2) : R1F(float, 3))
                                 : (dim == 2 ? R1F(double, 2) : R1F(double, 3));
#undef R1F
  if (e != hipSuccess || mode != 0) return e;
  const int64_t blocks = (ip.n + 256 * kListPer - 1) / (256 * kListPer);
  hipLaunchKernelGGL(k_lists, dim3(unsigned(blocks)), dim3(256), 0, st, ip.n, ip.status, fb_count, fb_list,
                     ip.cand_count, ip.cand_list);
  return hipGetLastError();
}

hipError_t r1m_fb_gather(int dtype, int dim, int64_t n, int nfb, const int32_t* list, const void* F,
                         const void* bn, void* Fc, void* bc, hipStream_t st) {
#define R1FG(T, D) hipLaunchKernelGGL((k_fb_gather<T, D>), dim3(nblk(nfb)), dim3(256), 0, st, n, nfb, list, \
    static_cast<const T*>(F), static_cast<const T*>(bn), static_cast<T*>(Fc), static_cast<T*>(bc))
  if (dtype == R1_F32) { if (dim == 2) R1FG(float, 2); else R1FG(float, 3); }
  else { if (dim == 2) R1FG(double, 2); else R1FG(double, 3); }
#undef R1FG
  return hipGetLastError();
}

hipError_t r1m_fb_scatter(int dtype, int dim, int64_t n, int nfb, const int32_t* list, const void* Wc,
                          const void* Pc, const int32_t* fc, void* W, void* P, int32_t* flags,
                          hipStream_t st) {
#define R1FS(T, D) hipLaunchKernelGGL((k_fb_scatter<T, D>), dim3(nblk(nfb)), dim3(256), 0, st, n, nfb, list, \
    static_cast<const T*>(Wc), static_cast<const T*>(Pc), fc, static_cast<T*>(W), static_cast<T*>(P), flags)
  if (dtype == R1_F32) { if (dim == 2) R1FS(float, 2); else R1FS(float, 3); }
  else { if (dim == 2) R1FS(double, 2); else R1FS(double, 3); }
#undef R1FS
  return hipGetLastError();
}
