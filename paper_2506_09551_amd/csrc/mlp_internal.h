// Internal declarations of the surrogate network (k_mlp.hip, mlp_api.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace msb {

constexpr int kMlpIn = 6;       // (U, t', U_c, Gamma, w_in, w)
constexpr int kMlpH = 512;      // hidden width
// flat float32 parameter vector of one network: W1[6][512] b1 W2[512][512] b2
// W3[512][512] b3 W4[512] b4 (weights stored [in][out])
constexpr int64_t kOffW1 = 0;
constexpr int64_t kOffB1 = kOffW1 + kMlpIn * kMlpH;
constexpr int64_t kOffW2 = kOffB1 + kMlpH;
constexpr int64_t kOffB2 = kOffW2 + (int64_t)kMlpH * kMlpH;
constexpr int64_t kOffW3 = kOffB2 + kMlpH;
constexpr int64_t kOffB3 = kOffW3 + (int64_t)kMlpH * kMlpH;
constexpr int64_t kOffW4 = kOffB3 + kMlpH;
constexpr int64_t kOffB4 = kOffW4 + kMlpH;
constexpr int64_t kMlpParams = kOffB4 + 1;

enum { kEpiFwd = 0, kEpiDh = 1, kEpiStore = 2 };
constexpr int kRowsPerPart = 256;    // batch rows per partial sum of the column reductions
constexpr int kMaxSplitK = 8;        // K slices of the weight-gradient product
constexpr int kMaxRows = 131072;     // largest batch

// C[M][N] = sum_k A[m][k] B[n][k] (both operands k-contiguous, bfloat16)
struct GemmArgs {
  const __bf16* A; int64_t lda, sA;     // s*: stride between ensemble members (elements)
  const __bf16* B; int64_t ldb, sB;
  int M, N, K;                          // multiples of 128, 128, 64 * splitk
  int splitk;                           // K slices (weight gradient only; 0 or 1 = none)
  float* C; int64_t ldc, sC, sCk;       // float32 output (z or dW); sCk: stride between K slices
  const float* bias; int64_t sBias;     // forward epilogue
  __bf16* H; int64_t ldh, sH;           // bfloat16 output (h or dz)
  __bf16* HT; int64_t ldht, sHT;        // optional transposed bfloat16 output [n][m]
  const float* Zp; int64_t ldz, sZ;     // pre-activations for gelu' (input-gradient epilogue)
};
hipError_t launch_gemm(int epi, const GemmArgs& g, int members, hipStream_t st);

struct MlpFwdArgs {
  const float* X;          // [points][6] raw inputs
  const float* T;          // [points] raw targets (nullptr: no loss)
  const int* perm;         // [members][steps * batch] point indices (nullptr: rows base + b)
  int64_t perm_stride;
  const int* step;         // device step counter (offset into perm)
  int64_t base;            // first point of this batch (when perm == nullptr)
  int batch;               // rows (multiple of 128)
  int valid;               // rows that hold points (the rest are zero padding)
  const float* in_shift; const float* in_scale;  // device [6]
  float out_scale;         // model output = out_scale * I
  const float* params; int64_t pstride;
  float *z1, *z2, *z3;     // [members][batch][512] gelu'(z) of layers 1-3 for the backward pass (nullptr: not kept)
  __bf16 *h1, *h2, *h3;
  __bf16 *dz1, *dz2, *dz3;
  int64_t act_stride;
  __bf16 *h1T, *h2T, *dz2T, *dz3T;  // transposed copies [members][512][ldT] (weight-gradient operands; h1T, h2T nullptr: not written)
  int64_t actT_stride, ldT;
  float* y; float* g; int64_t y_stride;          // [members][batch]
  double* loss_part;       // [members][batch / 4]
};
hipError_t launch_layer1_fwd(const MlpFwdArgs& a, int members, hipStream_t st);
hipError_t launch_layer4_fwd(const MlpFwdArgs& a, int members, hipStream_t st);
hipError_t launch_layer4_bwd(const MlpFwdArgs& a, int members, hipStream_t st);
hipError_t launch_layer1_bwd(const MlpFwdArgs& a, float* part, int max_parts, float* grads, int64_t gstride,
                             int members, hipStream_t st);
// loss_hist[m][*step] = sum of the loss partials / valid rows
hipError_t launch_loss_record(const MlpFwdArgs& a, double* loss_hist, int64_t hist_stride, int members,
                              hipStream_t st);

struct ColSumArgs {
  const __bf16* src_bf16; const float* src_f32;  // one of them
  int64_t src_stride, ld;
  const float* wgt; int64_t wgt_stride;          // optional row weights
  int nrows, ncols, rows_per_part, max_parts;
  float* part;                                    // [members][max_parts][ncols]
  float* out; int64_t out_stride;
};
hipError_t launch_colsum(const ColSumArgs& a, int members, hipStream_t st);
// out[m][i] = sum_k part[k][m][i] for i < n (part stride split_stride per slice)
hipError_t launch_splitk_sum(const float* part, int64_t split_stride, int splits, float* out, int64_t out_stride,
                             int64_t n, int members, hipStream_t st);

struct AdamArgs {
  float* params; float* grads; float* m; float* v; int64_t pstride;
  __bf16* w2b; __bf16* w3b;   // bfloat16 copies [in][out]
  __bf16* w2t; __bf16* w3t;   // and [out][in]
  int* step;                // Adam step (advanced after the update)
  int* call_step;           // step within the training call (advanced too)
  float lr, b1, b2, eps;
};
hipError_t launch_adam(const AdamArgs& a, int members, hipStream_t st);
hipError_t launch_weights_bf16(const float* params, int64_t pstride, __bf16* w2b, __bf16* w3b, __bf16* w2t,
                               __bf16* w3t, int members, hipStream_t st);
hipError_t launch_ensemble_stats(const float* y, int64_t y_stride, int members, int n, float inv_scale,
                                 float* mean, float* sd, hipStream_t st);

}  // namespace msb
