// Interface between the surrogate host code (r1_surrogate.cpp) and its kernels
// (r1_mlp.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "r1.h"
#include "r1_device.hpp"

constexpr int kMaxCols = 10;      // d_in, d_out <= 10
constexpr int kMaxHidden = 8;

// Gradients of the small layers per block of 32 batch rows in a training step:
// W_0 (width x d_in), the biases b_0 .. b_{n_hidden-1} (width each), W_out
// (d_out x width) and b_out (d_out), in that order.
__host__ __device__ constexpr int train_n_small(int d_in, int d_out, int width, int n_hidden) {
  return width * d_in + n_hidden * width + d_out * width + d_out;
}
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
  const void* wfrag;                // the same weights in MFMA fragment order (r1m_wfrag), for k_infer
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
  uint8_t* status;                  // MODE 0: n bytes, per point 1 = fallback, 2 = served, from which
                                    // r1m_infer then builds the fallback and candidate lists
};

// One batch of the training step (r1_train.hip).  Rows (mode): 0 = Xn / Yn given,
// already standardized; 1 = training row (a (step B + b) + c) mod n_train of X / T
// for batch row b (a permutation when gcd(a, n_train) = 1); 2 = rows r0 .. r0 + B
// of X / T; modes 1 and 2 standardize with norm = x_mean, x_std (d_in each),
// y_mean, y_std (d_out each).  B is a multiple of 32.
struct TrainArgs {
  int B, d_in, d_out, width, n_hidden;
  const float* params;                // FP32 master weights (off_w / off_b layout)
  int64_t off_w[kMaxHidden + 1], off_b[kMaxHidden + 1];
  const void* wbf;                    // BF16 W_l, l = 1 .. n_hidden - 1 (out x in, width^2 each)
  const void* wbf_t;                  // BF16 W_l^T (in x out)
  float* grad;                        // accumulated into (+=)
  int mode;
  const float* Xn;
  const float* Yn;
  const float* X;
  const float* T;
  const float* norm;
  int64_t n_train, r0, step;
  uint64_t a, c;
  float z_thr, margin, ew;            // loss (see k_train_fwd)
  float* loss;                        // += mean loss of the batch
  int store;                          // 0: loss only (the workspace below is not touched)
  float* Xb;                          // B x d_in: standardized inputs
  float* G;                           // B x d_out: dL/dout
  float* Z;                           // n_hidden x B x width: pre-activations
  void* Ht;                           // n_hidden x width x B BF16: activations, transposed
  void* Dt;                           // n_hidden x width x B BF16: deltas, transposed (layers >= 1)
  float* part;                        // (B / 32) x train_n_small: per-block partial gradients of the
                                      // small layers (k_train_bwd), summed by the weight-gradient launch
};

// Adam step on n parameters (lr = 0: only the BF16 copies are refreshed), then
// W_l and W_l^T of the width x width layers rounded to BF16.
struct AdamArgs {
  int64_t n;
  float* p;
  float* g;                           // cleared after use
  float* m;
  float* v;
  float lr, b1, b2, eps, c1, c2;
  int n_hidden, width;
  int64_t off_w[kMaxHidden + 1];
  void* wbf;
  void* wbf_t;
};

hipError_t r1m_train_fwd(const TrainArgs& a, hipStream_t st);        // forward, loss, dL/dout
hipError_t r1m_train_bwd(const TrainArgs& a, hipStream_t st);        // every gradient (after fwd)
hipError_t r1m_train_adam(const AdamArgs& a, hipStream_t st);

hipError_t r1m_fill(int64_t n, float* p, float v, hipStream_t st);
hipError_t r1m_targets(int dim, int64_t n, const r1d::Material& mat, const float* X, const float* Y,
                       float* T, hipStream_t st);
hipError_t r1m_colstats(int64_t n, int ncol, int dF, const float* A, double* sum, double* sum2, float* mn,
                        float* mx, float* det_min, hipStream_t st);
hipError_t r1m_pack(int dtype, int dim, int64_t n, const void* F, const void* bn, const void* W,
                    const void* P, float* X, float* Y, hipStream_t st);
hipError_t r1m_unpack(int dim, int64_t n, const float* X, float* F, float* bn, hipStream_t st);
// The BF16 hidden weights wbf (n_hidden - 1 layers of width x width, out x in)
// rewritten in the order k_infer reads its B fragments: per layer, k step ks
// (16 inputs), 32-output tile t and lane (r = lane % 32, half = lane / 32), the
// 8 inputs ks 16 + 8 half .. + 7 of output t 32 + r, so that each fragment load
// of a wave is 1 KB contiguous.
hipError_t r1m_wfrag(int width, int n_hidden, const void* wbf, void* wfrag, hipStream_t st);
size_t r1m_infer_lds(int width);
hipError_t r1m_infer(int dtype, int dim, const InferParams& ip, int mode, const void* F, const void* bn,
                     void* W, void* P, int32_t* flags, int* fb_count, int32_t* fb_list, int* cal_bin,
                     float* cal_w, float* cal_gap, hipStream_t st);
hipError_t r1m_fb_gather(int dtype, int dim, int64_t n, int nfb, const int32_t* list, const void* F,
                         const void* bn, void* Fc, void* bc, hipStream_t st);
hipError_t r1m_fb_scatter(int dtype, int dim, int64_t n, int nfb, const int32_t* list, const void* Wc,
                          const void* Pc, const int32_t* fc, void* W, void* P, int32_t* flags,
                          hipStream_t st);
