// Interface between the surrogate host code (r1_surrogate.cpp) and its kernels
// (r1_mlp.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "r1.h"
#include "r1_device.hpp"

constexpr int kEpiBiasSilu = 0;   // C = acc + bias, H = SiLU(C)
constexpr int kEpiDsilu = 1;      // C = acc * SiLU'(zaux)
constexpr int kEpiAtomic = 2;     // C += acc (split-K weight gradients)
constexpr int kMaxCols = 10;      // d_in, d_out <= 10
constexpr int kMaxHidden = 8;
constexpr int kBinsR = 16;        // error-gate bins over |F - I|_F
constexpr int kBinsB = 8;         // ... and over beta_n
constexpr int kGateCells = kBinsR * kBinsB;   // each with a threshold on the predicted gap
constexpr float kZeroGap = 1e-6f;  // gap targets at or below this did not laminate
constexpr float kHingeMargin = 0.25f;  // standardized margin below the no-lamination threshold

struct InferParams {
  int64_t n;
  int width, n_hidden;
  r1d::Material mat;
  const float* w0;                  // first layer, width x d_in
  const float* b[kMaxHidden];       // biases of the hidden layers
  const void* wbf[kMaxHidden];      // BF16 width x width weights of hidden layers 1.. (index 0 unused)
  const float* wout;                // d_out x width
  const float* bout;
  float x_mean[kMaxCols], x_std[kMaxCols], x_lo[kMaxCols], x_hi[kMaxCols];
  float y_mean[kMaxCols], y_std[kMaxCols];
  float det_lo;
  double r_max, b_lo, b_hi;
  int bins_on;
  const float* gate_tau;            // kGateCells: accept when the predicted gap is <= the cell's value
  int* cand_count;                  // nullable: points served by the network are also listed here
  int32_t* cand_list;               // (the candidates of the a-posteriori check)
};

hipError_t r1m_gemm(int epi, bool b_bf16, int M, int N, int K, const float* A, int64_t sam,
                    int64_t sak, const void* B, int64_t sbn, int64_t sbk, float* C, int64_t ldc,
                    const float* bias, const float* zaux, float* H, int ksplit, hipStream_t st);
hipError_t r1m_first_fwd(int B, int d_in, int w, const float* X, const float* W, const float* b,
                         float* Z, float* H, hipStream_t st);
hipError_t r1m_out_fwd_loss(int B, int w, int d_out, const float* H, const float* Wo, const float* bo,
                            const float* Y, float z_thr, float margin, float ew, float* G, float* loss,
                            hipStream_t st);
hipError_t r1m_out_bwd_dh(int B, int w, int d_out, const float* G, const float* Wo, const float* Z,
                          float* Dl, hipStream_t st);
hipError_t r1m_colsum(int B, int ncol, int ld, const float* A, float* out, hipStream_t st);
hipError_t r1m_outer_small(int B, int no, int ni, const float* D, int ldd, const float* X, int ldx,
                           int round_x, float* out, hipStream_t st);
hipError_t r1m_adam(int64_t n, float* p, const float* g, float* m, float* v, float lr, float b1,
                    float b2, float eps, int64_t t, hipStream_t st);
hipError_t r1m_to_bf16(int64_t n, const float* src, void* dst, hipStream_t st);
hipError_t r1m_fill(int64_t n, float* p, float v, hipStream_t st);
hipError_t r1m_gather(int B, int64_t n_train, uint64_t a, uint64_t c, int64_t step, int d_in, int d_out,
                      const float* X, const float* T, const float* norm, float* Xb, float* Yb,
                      hipStream_t st);
hipError_t r1m_standardize(int64_t r0, int64_t r1, int d_in, int d_out, const float* X, const float* T,
                           const float* norm, float* Xb, float* Yb, hipStream_t st);
hipError_t r1m_targets(int dim, int64_t n, const r1d::Material& mat, const float* X, const float* Y,
                       float* T, hipStream_t st);
hipError_t r1m_colstats(int64_t n, int ncol, int dF, const float* A, double* sum, double* sum2, float* mn,
                        float* mx, float* det_min, hipStream_t st);
hipError_t r1m_pack(int dtype, int dim, int64_t n, const void* F, const void* bn, const void* W,
                    const void* P, float* X, float* Y, hipStream_t st);
hipError_t r1m_unpack(int dim, int64_t n, const float* X, float* F, float* bn, hipStream_t st);
size_t r1m_infer_lds(int width);
hipError_t r1m_infer(int dtype, int dim, const InferParams& ip, int mode, const void* F, const void* bn,
                     void* W, void* P, int32_t* flags, int* fb_count, int32_t* fb_list, int* cal_bin,
                     float* cal_w, float* cal_gap, hipStream_t st);
hipError_t r1m_fb_gather(int dtype, int dim, int64_t n, int nfb, const int32_t* list, const void* F,
                         const void* bn, void* Fc, void* bc, hipStream_t st);
hipError_t r1m_fb_scatter(int dtype, int dim, int64_t n, int nfb, const int32_t* list, const void* Wc,
                          const void* Pc, const int32_t* fc, void* W, void* P, int32_t* flags,
                          hipStream_t st);
