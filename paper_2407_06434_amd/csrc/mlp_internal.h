// Internal declarations of the learned support proposal (network kernels and
// their host driver). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "omp_internal.h"

namespace bomp {

// Epilogues of the BF16 "NT" product C[m][n] = sum_k P[m][k] Q[n][k].
enum {
  EPI_FEATURES = 0,  // out bf16 = |c| * colscale[n] * rowscale[m] * scale
  EPI_BIAS_RELU = 1, // out bf16 = relu(c + bias[n])
  EPI_BIAS = 2,      // out f32  = c + bias[n]
  EPI_BCE = 3,       // out bf16 = (sigmoid(c + bias[n]) - t[m][n]) * scale; loss terms per block
  EPI_RELU_MASK = 4, // out bf16 = c where mask[m][n] > 0, else 0
  EPI_PARTIAL = 5,   // out f32 [split][m][n] = this split's partial sum
};

struct GemmEpi {
  void *out;
  int64_t ldo;               // output row stride (elements)
  const float *bias;         // [n]
  const float *colscale;     // [n]
  const float *rowscale;     // [m]
  const uint16_t *mask;      // [m][ldo] BF16 activations (EPI_RELU_MASK)
  const uint32_t *labels;    // [m][ldl] multi-hot bits (EPI_BCE)
  int64_t ldl;
  int64_t mvalid;            // rows below this are real signals (EPI_BCE)
  float scale;               // EPI_BCE: 1 / batch; EPI_FEATURES: sqrt(M)
  float *loss_part;          // EPI_BCE: one partial per block
};

// One layer's parameters and optimiser state (device pointers).
struct LayerView {
  int64_t n_in, n_out;
  float *W32;      // [out][in] FP32 master weights
  uint16_t *W16;   // [out][in] BF16 copy (forward operand)
  uint16_t *W16T;  // [in][out] BF16 transposed copy (backward operand)
  float *b32;      // [out]
  float *mW, *vW;  // Adam moments of W
  float *mb, *vb;  // Adam moments of b
};

int64_t gemm_blocks(int64_t M, int64_t N, int splits);
hipError_t launch_gemm_bf16(int epi, const uint16_t *P, int64_t ldp, const uint16_t *Q, int64_t ldq, int64_t M,
                            int64_t N, int64_t K, int splits, const GemmEpi &e, hipStream_t st);
hipError_t launch_prep_signals(const float *Y, int64_t ldy, int64_t B, int64_t M, int64_t Mp, int64_t Bp,
                               uint16_t *Y16, float *yinv, hipStream_t st);
hipError_t launch_pad_rows16(const uint16_t *src, int64_t ld, const int32_t *rows, int64_t B, int64_t cols,
                             int64_t Bp, uint16_t *dst, hipStream_t st);
hipError_t launch_labels(const int32_t *sup, const int32_t *rows, int64_t B, int S, int64_t n_out, int64_t Bp,
                         uint32_t *bits, hipStream_t st);
hipError_t launch_transpose16(const uint16_t *src, int64_t R, int64_t C, uint16_t *dst, hipStream_t st);
hipError_t launch_colsum16(const uint16_t *src, int64_t R, int64_t C, int chunks, float *part, hipStream_t st);
hipError_t launch_loss_sum(const float *part, int64_t n, float scale, float *out, hipStream_t st);
hipError_t launch_adam_w(const LayerView &L, const float *gpart, int splits, float lr, float b1, float b2, float eps,
                         float c1, float c2, int update, hipStream_t st);
hipError_t launch_adam_b(const LayerView &L, const float *gpart, int chunks, float lr, float b1, float b2, float eps,
                         float c1, float c2, hipStream_t st);
hipError_t launch_sum_parts(const float *part, int parts, int64_t n, float *out, hipStream_t st);
hipError_t launch_copy32(const float *src, int64_t n, float *dst, hipStream_t st);
hipError_t launch_topk(const float *Z, int64_t ldz, int64_t N, int64_t B, int S, int32_t *P, hipStream_t st);
hipError_t launch_ls_check(const DictView &d, const float *Y, int64_t ldy, int64_t B, const int32_t *P, int S,
                           const float *eps_per, float eps, int32_t *support_out, float *coef_out, int32_t *status_out,
                           float *rnorm_out, int32_t *accept, hipStream_t st);
hipError_t launch_compact(const int32_t *accept, int64_t B, int32_t *idx, int32_t *count, hipStream_t st);
hipError_t launch_gather_rejects(const float *Y, int64_t ldy, int64_t M, const float *eps_per, float eps,
                                 const int32_t *idx, int64_t n, float *Yr, float *eps_r, hipStream_t st);
hipError_t launch_scatter_fallback(const int32_t *idx, int64_t n, int S, const int32_t *sup_r, const float *coef_r,
                                   const int32_t *st_r, const float *rn_r, int32_t *support_out, float *coef_out,
                                   int32_t *status_out, float *rnorm_out, hipStream_t st);

}  // namespace bomp
