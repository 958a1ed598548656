// Training step of the learned surrogate (gfx950) in four launches:
//
//   k_train_fwd    per block of 32 batch rows: the rows (gathered and
//                  standardized), the FP32 first layer, every width x width
//                  layer on BF16 MFMA with the activations kept in LDS, the
//                  FP32 output layer, the loss and dL/dout.  Stores what the
//                  backward pass needs: Z of every layer (FP32) and the BF16
//                  activations transposed (width x B, K-contiguous for the
//                  weight gradients).
//   k_train_bwd    per block of 32 rows: the delta chain through the width x
//                  width layers (BF16 MFMA against the transposed weights) with
//                  SiLU' from Z, and the block's share of the output- and
//                  first-layer weight gradients and of every bias gradient
//                  (stored as per-block partials); stores the BF16 deltas
//                  transposed.
//   k_train_wgrad  dW_l += Delta_l^T H_{l-1} for every width x width layer in
//                  one launch (both operands K-contiguous), split over the batch
//                  in chunks whose partial sums meet in atomics; and the sum of
//                  k_train_bwd's partials into the small layers' gradients.
//   k_train_adam   Adam on every parameter, clearing its gradient for the next
//                  step and refreshing the BF16 copies of W_l and W_l^T.
//
// The arithmetic is that of a plain layer-by-layer pass: BF16 operands
// (activations and deltas rounded to nearest even) with FP32 accumulation for
// the width x width products, FP32 elsewhere; only the order of the batch sums
// differs.  MFMA 32x32x16 lane layout as in r1_mlp.hip.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "r1_mlp.hpp"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {

constexpr int kR = 32;           // batch rows per block of the fused passes

// Batch rows per partial sum of the weight gradients: the largest of 512 .. 32
// dividing B (B is a multiple of kR).
__host__ __device__ inline int wgrad_chunk(int B) {
  int c = 512;
  while (B % c != 0) c /= 2;
  return c;
}

__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float silu_d(float z) {
  const float s = sigm(z);
  return s * (1.0f + z * (1.0f - s));
}

// Index i of the small layers' partial gradients (train_n_small) and the
// parameter it belongs to.
__device__ __forceinline__ int small_b(const TrainArgs& a) { return a.width * a.d_in; }
__device__ __forceinline__ int small_wo(const TrainArgs& a) { return small_b(a) + a.n_hidden * a.width; }
__device__ __forceinline__ int small_bo(const TrainArgs& a) { return small_wo(a) + a.d_out * a.width; }
__device__ __forceinline__ int64_t small_param(const TrainArgs& a, int i) {
  if (i < small_b(a)) return a.off_w[0] + i;
  if (i < small_wo(a)) {
    const int j = i - small_b(a);
    return a.off_b[j / a.width] + j % a.width;
  }
  if (i < small_bo(a)) return a.off_w[a.n_hidden] + (i - small_wo(a));
  return a.off_b[a.n_hidden] + (i - small_bo(a));
}

// Source row of batch row b (modes 1 and 2; see TrainArgs).
__device__ __forceinline__ int64_t source_row(const TrainArgs& a, int64_t b) {
  if (a.mode == 2) return a.r0 + b;
  const uint64_t n = uint64_t(a.n_train);
  const uint64_t q = (uint64_t(a.step) * uint64_t(a.B) + uint64_t(b)) % n;
  return int64_t(((a.a % n) * q % n + a.c % n) % n);
}

// The block's rows into LDS (sx: inputs, sy: targets, kMaxCols apart),
// standardized; srow (kR entries of LDS) holds their source rows.
__device__ __forceinline__ void load_rows(const TrainArgs& a, int64_t row0, float* sx, float* sy, int64_t* srow) {
  if (a.mode != 0 && threadIdx.x < kR) srow[threadIdx.x] = source_row(a, row0 + threadIdx.x);
  __syncthreads();
  const int per = a.d_in + a.d_out;
  for (int e = threadIdx.x; e < kR * per; e += blockDim.x) {
    const int r = e / per, k = e % per;
    const int64_t b = row0 + r;
    float v;
    if (a.mode == 0) {
      v = k < a.d_in ? a.Xn[b * a.d_in + k] : a.Yn[b * a.d_out + (k - a.d_in)];
    } else {
      // norm = x_mean (d_in), x_std (d_in), y_mean (d_out), y_std (d_out)
      const int64_t src = srow[r];
      if (k < a.d_in) {
        v = (a.X[src * a.d_in + k] - a.norm[k]) / a.norm[a.d_in + k];
      } else {
        const int j = k - a.d_in;
        v = (a.T[src * a.d_out + j] - a.norm[2 * a.d_in + j]) / a.norm[2 * a.d_in + a.d_out + j];
      }
    }
    if (k < a.d_in) {
      sx[r * kMaxCols + k] = v;
      if (a.store) a.Xb[b * a.d_in + k] = v;
    } else {
      sy[r * kMaxCols + (k - a.d_in)] = v;
    }
  }
}

// 32 x 32 tile n0.. of the block's rows times a BF16 weight block: acc(m, n) =
// sum_k A[m][k] B[n][k], A in LDS (row stride lda), B row-major (width x width).
template <int W>
__device__ __forceinline__ f32x16 tile_mfma(const __bf16* A, int lda, const __bf16* B, int n0) {
  const int lane = threadIdx.x & 63, r = lane & 31, kq = 8 * (lane >> 5);
  f32x16 acc = {};
#pragma unroll
  for (int k0 = 0; k0 < W; k0 += 16) {
    const bf16x8 av = *reinterpret_cast<const bf16x8*>(A + r * lda + k0 + kq);
    const bf16x8 bv = *reinterpret_cast<const bf16x8*>(B + int64_t(n0 + r) * W + k0 + kq);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
  }
  return acc;
}

// Transposed store of a kR x W BF16 block (LDS, row stride ld) into dst[c * B + row0 + r].
template <int W>
__device__ __forceinline__ void store_transposed(const __bf16* s, int ld, __bf16* dst, int64_t B, int64_t row0) {
  for (int e = threadIdx.x; e < W * (kR / 2); e += blockDim.x) {
    const int c = e / (kR / 2), r = 2 * (e % (kR / 2));
    __bf16 two[2] = {s[r * ld + c], s[(r + 1) * ld + c]};
    *reinterpret_cast<uint32_t*>(dst + int64_t(c) * B + row0 + r) = *reinterpret_cast<const uint32_t*>(two);
  }
}

template <int W>
__global__ __launch_bounds__(256) void k_train_fwd(TrainArgs a) {
  constexpr int LD = W + 8;                      // LDS row stride (BF16), 16-byte aligned rows
  __shared__ __attribute__((aligned(16))) __bf16 sh[2][kR * LD];
  __shared__ float sx[kR * kMaxCols], sy[kR * kMaxCols];
  __shared__ float swo[kMaxCols * W];            // output-layer weights
  __shared__ float red[256];
  __shared__ int64_t srow[kR];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t B = a.B, row0 = int64_t(blockIdx.x) * kR;
  const int L = a.n_hidden;
  for (int e = tid; e < a.d_out * W; e += blockDim.x) swo[e] = a.params[a.off_w[L] + e];
  load_rows(a, row0, sx, sy, srow);
  __syncthreads();
  // first layer (FP32): Z0 = X W0^T + b0, H0 = SiLU(Z0).  A thread keeps one
  // unit c (its weights and bias in registers) over rows r = tid / W, + 256 / W ...
  static_assert(256 % W == 0, "width divides the block");
  {
    const int c = tid % W;
    const float* W0 = a.params + a.off_w[0];
    float w0c[kMaxCols];
#pragma unroll
    for (int k = 0; k < kMaxCols; ++k) w0c[k] = k < a.d_in ? W0[c * a.d_in + k] : 0.0f;
    const float b0c = a.params[a.off_b[0] + c];
    for (int r = tid / W; r < kR; r += 256 / W) {
      float z = b0c;
#pragma unroll
      for (int k = 0; k < kMaxCols; ++k)
        if (k < a.d_in) z = fmaf(w0c[k], sx[r * kMaxCols + k], z);
      if (a.store) a.Z[(row0 + r) * W + c] = z;
      sh[0][r * LD + c] = __bf16(silu(z));
    }
  }
  __syncthreads();
  if (a.store) store_transposed<W>(sh[0], LD, static_cast<__bf16*>(a.Ht), B, row0);
  // width x width layers: Z_l = H_{l-1} W_l^T + b_l on BF16 MFMA
  for (int l = 1; l < L; ++l) {
    const __bf16* src = sh[(l - 1) & 1];
    __bf16* dst = sh[l & 1];
    const __bf16* Wl = static_cast<const __bf16*>(a.wbf) + int64_t(l - 1) * W * W;
    const float* bl = a.params + a.off_b[l];
    for (int t = wave; t < W / 32; t += 4) {
      const int col = 32 * t + (lane & 31);
      const float bias = bl[col];
      const f32x16 acc = tile_mfma<W>(src, LD, Wl, 32 * t);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int row = 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
        const float z = acc[j] + bias;
        if (a.store) a.Z[(int64_t(l) * B + row0 + row) * W + col] = z;
        dst[row * LD + col] = __bf16(silu(z));
      }
    }
    __syncthreads();
    if (a.store) store_transposed<W>(dst, LD, static_cast<__bf16*>(a.Ht) + int64_t(l) * W * B, B, row0);
  }
  // output layer (FP32 weights, BF16 activations), loss and dL/dout.  Rows whose
  // standardized gap target is <= z_thr did not laminate: their gap output only
  // has to stay below z_thr - margin (one-sided squared hinge) and their stress
  // outputs are not trained.  The energy output's squared error is weighted by ew.
  // Row r = tid / 8: its 8 threads (consecutive lanes) each sum a W/8 slice of
  // k, then meet in three exchanges.
  const __bf16* hl = sh[(L - 1) & 1];
  const float* bo = a.params + a.off_b[L];
  const float inv_n = 1.0f / float(B * a.d_out);
  const int r = tid >> 3, k0 = (tid & 7) * (W / 8);
  float part[kMaxCols];
#pragma unroll
  for (int j = 0; j < kMaxCols; ++j) {
    part[j] = 0.0f;
    if (j < a.d_out)
      for (int k = k0; k < k0 + W / 8; ++k) part[j] = fmaf(swo[j * W + k], float(hl[r * LD + k]), part[j]);
  }
#pragma unroll
  for (int off = 1; off < 8; off <<= 1)
#pragma unroll
    for (int j = 0; j < kMaxCols; ++j) part[j] += __shfl_xor(part[j], off);
  float e2 = 0.0f;
  if ((tid & 7) == 0) {
    const bool convex = sy[r * kMaxCols] <= a.z_thr;
#pragma unroll
    for (int j = 0; j < kMaxCols; ++j) {
      if (j >= a.d_out) break;
      const float o = bo[j] + part[j];
      float err;
      if (!convex) err = o - sy[r * kMaxCols + j];
      else if (j == 0) err = fmaxf(0.0f, o - (a.z_thr - a.margin));
      else err = 0.0f;
      const float wj = j == 0 ? a.ew : 1.0f;
      e2 += wj * err * err;
      if (a.store) a.G[(row0 + r) * a.d_out + j] = 2.0f * wj * err * inv_n;
    }
  }
  red[tid] = e2;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) atomicAdd(a.loss, red[0] * inv_n);
}

template <int W>
__global__ __launch_bounds__(256) void k_train_bwd(TrainArgs a) {
  constexpr int LD = W + 8;
  __shared__ float sd[kR * W];                   // FP32 delta of the current layer
  __shared__ __attribute__((aligned(16))) __bf16 sb[kR * LD];   // BF16 delta (MFMA operand) / H_{L-1}
  __shared__ float sg[kR * kMaxCols], sxb[kR * kMaxCols];
  __shared__ float swo[kMaxCols * W];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t B = a.B, row0 = int64_t(blockIdx.x) * kR;
  const int L = a.n_hidden;
  float* part = a.part + int64_t(blockIdx.x) * train_n_small(a.d_in, a.d_out, W, L);
  const __bf16* Ht = static_cast<const __bf16*>(a.Ht);
  for (int e = tid; e < kR * a.d_out; e += blockDim.x) {
    const int r = e / a.d_out, j = e % a.d_out;
    sg[r * kMaxCols + j] = a.G[(row0 + r) * a.d_out + j];
  }
  for (int e = tid; e < kR * a.d_in; e += blockDim.x) {
    const int r = e / a.d_in, i = e % a.d_in;
    sxb[r * kMaxCols + i] = a.Xb[(row0 + r) * a.d_in + i];
  }
  for (int e = tid; e < a.d_out * W; e += blockDim.x) swo[e] = a.params[a.off_w[L] + e];
  for (int e = tid; e < kR * W; e += blockDim.x) {
    const int c = e / kR, r = e % kR;
    sb[r * LD + c] = Ht[(int64_t(L - 1) * W + c) * B + row0 + r];
  }
  __syncthreads();
  // output layer: dWout += G^T H_{L-1}, dbout += colsum G
  for (int e = tid; e < a.d_out * W; e += blockDim.x) {
    const int j = e / W, k = e % W;
    float s = 0.0f;
    for (int r = 0; r < kR; ++r) s = fmaf(sg[r * kMaxCols + j], float(sb[r * LD + k]), s);
    part[small_wo(a) + e] = s;
  }
  if (tid < a.d_out) {
    float s = 0.0f;
    for (int r = 0; r < kR; ++r) s += sg[r * kMaxCols + tid];
    part[small_bo(a) + tid] = s;
  }
  // delta of the last hidden layer: (G Wout) * SiLU'(Z)
  for (int e = tid; e < kR * W; e += blockDim.x) {
    const int r = e / W, c = e % W;
    float s = 0.0f;
    for (int j = 0; j < a.d_out; ++j) s = fmaf(sg[r * kMaxCols + j], swo[j * W + c], s);
    sd[r * W + c] = s * silu_d(a.Z[(int64_t(L - 1) * B + row0 + r) * W + c]);
  }
  __syncthreads();
  for (int l = L - 1; l >= 1; --l) {
    // db_l += colsum delta_l; the BF16 delta, in LDS and transposed in memory
    for (int c = tid; c < W; c += blockDim.x) {
      float s = 0.0f;
      for (int r = 0; r < kR; ++r) s += sd[r * W + c];
      part[small_b(a) + l * W + c] = s;
    }
    for (int e = tid; e < kR * W; e += blockDim.x) {
      const int r = e / W, c = e % W;
      sb[r * LD + c] = __bf16(sd[r * W + c]);
    }
    __syncthreads();
    store_transposed<W>(sb, LD, static_cast<__bf16*>(a.Dt) + int64_t(l) * W * B, B, row0);
    // delta_{l-1} = (delta_l W_l) * SiLU'(Z_{l-1}): B operand W_l^T (row n = input unit)
    const __bf16* Wt = static_cast<const __bf16*>(a.wbf_t) + int64_t(l - 1) * W * W;
    for (int t = wave; t < W / 32; t += 4) {
      const int col = 32 * t + (lane & 31);
      float zv[16];                              // issued before the products, used after
#pragma unroll
      for (int j = 0; j < 16; ++j)
        zv[j] = a.Z[(int64_t(l - 1) * B + row0 + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3)) * W + col];
      const f32x16 acc = tile_mfma<W>(sb, LD, Wt, 32 * t);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int row = 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
        sd[row * W + col] = acc[j] * silu_d(zv[j]);
      }
    }
    __syncthreads();
  }
  // first layer: db0 += colsum delta_0, dW0 += delta_0^T X
  for (int c = tid; c < W; c += blockDim.x) {
    float s = 0.0f;
    for (int r = 0; r < kR; ++r) s += sd[r * W + c];
    part[small_b(a) + c] = s;
  }
  for (int e = tid; e < W * a.d_in; e += blockDim.x) {
    const int c = e / a.d_in, i = e % a.d_in;
    float s = 0.0f;
    for (int r = 0; r < kR; ++r) s = fmaf(sd[r * W + c], sxb[r * kMaxCols + i], s);
    part[e] = s;
  }
}

// Two kinds of block of 4 waves.  The first (n_hidden - 1) TILES chunks / 4:
// one wave per (layer, 32 x 32 tile, batch chunk), dW_l[m][n] += sum over the
// chunk's rows k of Dt_l[m][k] Ht_{l-1}[n][k], the chunks' partial sums meeting
// in atomics.  The rest sum k_train_bwd's per-block partials into the small
// layers' gradients: 64 elements per block, wave w adding the partials of batch
// blocks w, w + 4, ... (a wave's loads are 64 consecutive elements), the four
// waves' sums meeting in LDS.
template <int W>
__device__ __forceinline__ int wgrad_tasks(const TrainArgs& a) {
  return (a.n_hidden - 1) * (W / 32) * (W / 32) * (a.B / wgrad_chunk(a.B));
}

template <int W>
__global__ __launch_bounds__(256) void k_train_wgrad(TrainArgs a) {
  constexpr int TILES = (W / 32) * (W / 32);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r = lane & 31, kq = 8 * (lane >> 5);
  const int task_blocks = (wgrad_tasks<W>(a) + 3) / 4;
  if (int(blockIdx.x) >= task_blocks) {        // block-uniform
    __shared__ float red[4 * 64];
    const int ns = train_n_small(a.d_in, a.d_out, W, a.n_hidden), nb = a.B / kR;
    const int i = (int(blockIdx.x) - task_blocks) * 64 + lane;
    float s = 0.0f;
    if (i < ns) {
#pragma unroll 8
      for (int b = wave; b < nb; b += 4) s += a.part[int64_t(b) * ns + i];
    }
    red[wave * 64 + lane] = s;
    __syncthreads();
    if (wave == 0 && i < ns) a.grad[small_param(a, i)] += red[lane] + red[64 + lane] + red[128 + lane] + red[192 + lane];
    return;
  }
  const int64_t B = a.B;
  const int chunk_rows = wgrad_chunk(a.B), chunks = int(B / chunk_rows);
  const int task = int(blockIdx.x) * 4 + wave;
  if (task >= wgrad_tasks<W>(a)) return;       // wave-uniform
  const int chunk = task % chunks;
  const int tile = (task / chunks) % TILES;
  const int l = 1 + task / (chunks * TILES);
  const int m0 = 32 * (tile / (W / 32)), n0 = 32 * (tile % (W / 32));
  const __bf16* A = static_cast<const __bf16*>(a.Dt) + (int64_t(l) * W + m0 + r) * B;
  const __bf16* Bm = static_cast<const __bf16*>(a.Ht) + (int64_t(l - 1) * W + n0 + r) * B;
  f32x16 acc = {};
  const int64_t k1 = int64_t(chunk + 1) * chunk_rows;
  for (int64_t k0 = int64_t(chunk) * chunk_rows; k0 < k1; k0 += 16) {
    const bf16x8 av = *reinterpret_cast<const bf16x8*>(A + k0 + kq);
    const bf16x8 bv = *reinterpret_cast<const bf16x8*>(Bm + k0 + kq);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
  }
  float* g = a.grad + a.off_w[l];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int row = m0 + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
    atomicAdd(&g[row * W + n0 + r], acc[j]);
  }
}

// Adam on every parameter; the gradient is cleared for the next step and the BF16
// copies of the width x width layers (W_l and W_l^T) are refreshed.
__global__ void k_train_adam(AdamArgs a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  float p = a.p[i];
  if (a.lr != 0.0f) {
    const float gi = a.g[i];
    a.g[i] = 0.0f;
    const float mi = a.b1 * a.m[i] + (1.0f - a.b1) * gi;
    const float vi = a.b2 * a.v[i] + (1.0f - a.b2) * gi * gi;
    a.m[i] = mi;
    a.v[i] = vi;
    p -= a.lr * (mi / a.c1) / (sqrtf(vi / a.c2) + a.eps);
    a.p[i] = p;
  }
  for (int l = 1; l < a.n_hidden; ++l) {
    const int64_t o = i - a.off_w[l];
    if (o >= 0 && o < int64_t(a.width) * a.width) {
      const int64_t blk = int64_t(l - 1) * a.width * a.width;
      const int out = int(o / a.width), in = int(o % a.width);
      static_cast<__bf16*>(a.wbf)[blk + o] = __bf16(p);
      static_cast<__bf16*>(a.wbf_t)[blk + int64_t(in) * a.width + out] = __bf16(p);
    }
  }
}

template <int W>
hipError_t launch_step(const TrainArgs& a, int pass, hipStream_t st) {
  const unsigned rows = unsigned(a.B / kR);
  if (pass == 0) {
    hipLaunchKernelGGL(k_train_fwd<W>, dim3(rows), dim3(256), 0, st, a);
  } else if (pass == 1) {
    hipLaunchKernelGGL(k_train_bwd<W>, dim3(rows), dim3(256), 0, st, a);
  } else {
    const int ns = train_n_small(a.d_in, a.d_out, W, a.n_hidden);
    const int tasks = (a.n_hidden - 1) * (W / 32) * (W / 32) * (a.B / wgrad_chunk(a.B));
    hipLaunchKernelGGL(k_train_wgrad<W>, dim3(unsigned((tasks + 3) / 4 + (ns + 63) / 64)), dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_pass(const TrainArgs& args, int pass, hipStream_t st) {
  if (args.B < kR || args.B % kR != 0 || args.n_hidden < 2 || args.n_hidden > kMaxHidden)
    return hipErrorInvalidValue;
  const TrainArgs& a = args;
  switch (a.width) {
    case 32: return launch_step<32>(a, pass, st);
    case 64: return launch_step<64>(a, pass, st);
    case 128: return launch_step<128>(a, pass, st);
    case 256: return launch_step<256>(a, pass, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t r1m_train_fwd(const TrainArgs& a, hipStream_t st) { return launch_pass(a, 0, st); }

hipError_t r1m_train_bwd(const TrainArgs& a, hipStream_t st) {
  hipError_t e = launch_pass(a, 1, st);
  return e == hipSuccess ? launch_pass(a, 2, st) : e;
}

hipError_t r1m_train_adam(const AdamArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_train_adam, dim3(unsigned((a.n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}
