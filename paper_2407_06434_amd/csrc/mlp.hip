// Kernels of the learned support proposal (an extension of the paper's
// method): a multilayer perceptron maps the magnitude of the normalised first
// correlation of a signal, f_n = sqrt(M) |a_n^T y| / (||a_n|| ||y||) (Algorithm
// 1's first selection statistic, scaled to unit size),
// to one score per atom; the S best-scored atoms are checked by one
// least-squares solve (Eq. 2, by the Cholesky factorisation of the Gram
// block, Section 2.2), and plain OMP handles the signals whose residual misses
// the tolerance.
//
// Network: h1 = relu(W1 f + b1), h2 = relu(W2 h1 + b2), z = W3 h2 + b3, with
// BF16 operands and FP32 accumulation; W_l is stored [out][in]. Training
// minimises binary cross-entropy with logits against the multi-hot OMP
// support, averaged over the batch, with Adam (Kingma and Ba, 2015).
//
// All matrix products are the "NT" BF16 MFMA product of mfma_tile.h with a
// fused epilogue; every layout below keeps the reduction index contiguous:
//   forward   H1[b][o]  = F[b][:]   . W1[o][:]          (+ b1, relu)
//   backward  dH2[b][i] = dZ[b][:]  . W3T[i][:]         (x (H2 > 0))
//   weights   dW3[o][i] = dZT[o][:] . H2T[i][:]         (split over the batch)
// with W_lT the transposed BF16 copy kept by the optimiser and the activation
// transposes made per step.

#include <cmath>

#include "../../include/batched_omp.h"
#include "mfma_tile.h"
#include "mlp_internal.h"
#include "omp_internal.h"

namespace bomp {
namespace {

using GT = Tile<128, 128, 2, 2>;  // 128 x 128 tiles, 4 wavefronts of 64 x 64

__device__ inline uint16_t bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline float sigmoidf(float z) {
  const float e = expf(-fabsf(z));
  return z >= 0.f ? 1.f / (1.f + e) : e / (1.f + e);
}
__device__ inline float softplusf(float z) { return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))); }

// ---------------------------------------------------------------------------
// BF16 "NT" product C[m][n] = sum_k P[m][k] Q[n][k] with a fused epilogue.
// P: [rows][ldp] BF16, Q: [cols][ldq] BF16, K a multiple of 64. The grid is
// (M/128) x (N/128) tiles times `splits` slices of K (EPI_PARTIAL only).
// ---------------------------------------------------------------------------
template <int EPI>
__global__ __launch_bounds__(GT::NTHR) void k_gemm_nt(const uint16_t *__restrict__ P, int64_t ldp,
                                                     const uint16_t *__restrict__ Q, int64_t ldq, int64_t Mrows,
                                                     int64_t Ncols, int64_t K, int splits, GemmEpi e) {
  using T = GT;
  extern __shared__ u32x4 lds[];
  const int64_t ntm = Mrows / T::TN, ntn = Ncols / T::TB;
  const int64_t tile = blockIdx.x % (ntm * ntn);
  const int split = (int)(blockIdx.x / (ntm * ntn));
  const int64_t tm = tile % ntm, tn = tile / ntm;
  const int64_t kc = K / splits;  // elements of K per split (a multiple of 64)
  const int64_t prs = ldp / 8, qrs = ldq / 8;
  const u32x4 *Pp = reinterpret_cast<const u32x4 *>(P) + tm * T::TN * prs + (split * kc) / 8;
  const u32x4 *Qp = reinterpret_cast<const u32x4 *>(Q) + tn * T::TB * qrs + (split * kc) / 8;
  f32x16 acc[T::FN][T::FB];
  mainloop<OpBF16, T>(Pp, prs, Qp, qrs, (int)(kc / 64), lds, acc);

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wn = wave % T::WN, wb = wave / T::WN;
  float lsum = 0.f;
#pragma unroll
  for (int i = 0; i < T::FN; ++i)
#pragma unroll
    for (int j = 0; j < T::FB; ++j) {
      const int64_t n = tn * T::TB + wb * T::FB * 32 + j * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t m = tm * T::TN + wn * T::FN * 32 + i * 32 + frag_row(lane, r);
        const float c = acc[i][j][r];
        const int64_t o = m * e.ldo + n;
        if (EPI == EPI_FEATURES) {
          reinterpret_cast<uint16_t *>(e.out)[o] = bf16_rne(fabsf(c) * e.colscale[n] * e.rowscale[m] * e.scale);
        } else if (EPI == EPI_BIAS_RELU) {
          reinterpret_cast<uint16_t *>(e.out)[o] = bf16_rne(fmaxf(c + e.bias[n], 0.f));
        } else if (EPI == EPI_BIAS) {
          reinterpret_cast<float *>(e.out)[o] = c + e.bias[n];
        } else if (EPI == EPI_BCE) {
          // rows at or beyond the batch are padding: no gradient, no loss
          float dz = 0.f;
          if (m < e.mvalid) {
            const float z = c + e.bias[n];
            const float t = (float)((e.labels[m * e.ldl + (n >> 5)] >> (n & 31)) & 1u);
            dz = (sigmoidf(z) - t) * e.scale;
            lsum += softplusf(z) - t * z;
          }
          reinterpret_cast<uint16_t *>(e.out)[o] = bf16_rne(dz);
        } else if (EPI == EPI_RELU_MASK) {
          const bool on = bf16_to_f32(e.mask[o]) > 0.f;
          reinterpret_cast<uint16_t *>(e.out)[o] = bf16_rne(on ? c : 0.f);
        } else {  // EPI_PARTIAL: split-K partial sums, summed by the optimiser
          reinterpret_cast<float *>(e.out)[(int64_t)split * Mrows * e.ldo + o] = c;
        }
      }
    }
  if (EPI == EPI_BCE) {
    // block sum of the loss terms, one partial per block (summed in block order)
    __shared__ float red[GT::NTHR / 64];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) lsum += __shfl_xor(lsum, off);
    if (lane == 0) red[wave] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) {
      float s = 0.f;
      for (int i = 0; i < GT::NTHR / 64; ++i) s += red[i];
      e.loss_part[blockIdx.x] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// Signals to BF16 (padded) and 1/||y|| (0 for a zero or non-finite signal).
// One wavefront per padded signal.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_prep_signals(const float *__restrict__ Y, int64_t ldy, int64_t B, int64_t M,
                                                     int64_t Mp, uint16_t *__restrict__ Y16,
                                                     float *__restrict__ yinv) {
  const int64_t b = blockIdx.x;
  const int lane = threadIdx.x;
  double s = 0.0;
  int finite = 1;
  for (int64_t m = lane; m < Mp; m += 64) {
    const float v = (b < B && m < M) ? Y[b * ldy + m] : 0.f;
    finite &= isfinite(v) ? 1 : 0;
    const float vz = isfinite(v) ? v : 0.f;
    Y16[b * Mp + m] = bf16_rne(vz);
    s += (double)vz * (double)vz;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  const bool ok = __all(finite) && s > 0.0;
  if (lane == 0) yinv[b] = ok ? (float)(1.0 / sqrt(s)) : 0.f;
}

// Zero-padded copy of B rows of a BF16 matrix into [Bp][cols]; row b is source
// row rows[b] when `rows` is given.
__global__ __launch_bounds__(256) void k_pad_rows16(const uint16_t *__restrict__ src, int64_t lds_,
                                                    const int32_t *__restrict__ rows, int64_t B, int64_t cols,
                                                    uint16_t *__restrict__ dst) {
  const int64_t b = blockIdx.x;
  const int64_t sb = b < B ? (rows ? (int64_t)rows[b] : b) : 0;
  for (int64_t c = threadIdx.x; c < cols; c += blockDim.x) dst[b * cols + c] = b < B ? src[sb * lds_ + c] : 0;
}

// Multi-hot labels from supports [.][S] (-1 padded; row rows[b] when given):
// bits [Bp][n/32]. One wavefront per row; the atomics order nothing (OR).
__global__ __launch_bounds__(64) void k_labels(const int32_t *__restrict__ sup, const int32_t *__restrict__ rows,
                                               int64_t B, int S, int64_t words, uint32_t *__restrict__ bits) {
  const int64_t b = blockIdx.x;
  for (int64_t t = threadIdx.x; t < words; t += 64) bits[b * words + t] = 0u;
  __syncthreads();
  if (b >= B) return;
  const int64_t sb = rows ? (int64_t)rows[b] : b;
  for (int j = threadIdx.x; j < S; j += 64) {
    const int n = sup[sb * S + j];
    if (n >= 0 && n < words * 32) atomicOr(&bits[b * words + (n >> 5)], 1u << (n & 31));
  }
}

// BF16 transpose dst[c][r] = src[r][c]; R and C multiples of 64.
__global__ __launch_bounds__(256) void k_transpose16(const uint16_t *__restrict__ src, int64_t R, int64_t C,
                                                     uint16_t *__restrict__ dst) {
  __shared__ uint16_t t[64][66];
  const int64_t tc = blockIdx.x % (C / 64), tr = blockIdx.x / (C / 64);
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < 64; i += 4) t[i][tx] = src[(tr * 64 + i) * C + tc * 64 + tx];
  __syncthreads();
  for (int i = ty; i < 64; i += 4) dst[(tc * 64 + i) * R + tr * 64 + tx] = t[tx][i];
}

// Column sums of a BF16 [R][C] matrix in row chunks: part[chunk][c].
__global__ __launch_bounds__(256) void k_colsum16(const uint16_t *__restrict__ src, int64_t R, int64_t C,
                                                  int64_t rows_per_chunk, float *__restrict__ part) {
  const int64_t c = (int64_t)(blockIdx.x % (C / 256)) * 256 + threadIdx.x;
  const int64_t chunk = blockIdx.x / (C / 256);
  const int64_t r0 = chunk * rows_per_chunk, r1 = min(R, r0 + rows_per_chunk);
  float s = 0.f;
  for (int64_t r = r0; r < r1; ++r) s += bf16_to_f32(src[r * C + c]);
  part[chunk * C + c] = s;
}

// Sum of the loss partials, in block order.
__global__ __launch_bounds__(64) void k_loss_sum(const float *__restrict__ part, int64_t n, float scale,
                                                 float *__restrict__ out) {
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 64) s += part[i];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if (threadIdx.x == 0) out[0] = (float)(s * scale);
}

// ---------------------------------------------------------------------------
// Adam on one weight matrix W [out][in] (64 x 64 tiles): gradient = sum of the
// split-K partials; moments, master weights, the BF16 copy and its transpose.
// c1 = 1/(1 - beta1^t), c2 = 1/(1 - beta2^t). lr = 0 only copies (no update).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_adam_w(LayerView L, const float *__restrict__ gpart, int splits,
                                                float lr, float b1, float b2, float eps, float c1, float c2,
                                                int update) {
  __shared__ uint16_t t[64][66];
  const int64_t nin = L.n_in, nout = L.n_out;
  const int64_t ti = blockIdx.x % (nin / 64), to = blockIdx.x / (nin / 64);
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < 64; i += 4) {
    const int64_t o = to * 64 + i, in = ti * 64 + tx, idx = o * nin + in;
    float w = L.W32[idx];
    if (update) {
      float g = 0.f;
      for (int s = 0; s < splits; ++s) g += gpart[(int64_t)s * nout * nin + idx];
      const float m = b1 * L.mW[idx] + (1.f - b1) * g;
      const float v = b2 * L.vW[idx] + (1.f - b2) * g * g;
      L.mW[idx] = m;
      L.vW[idx] = v;
      w -= lr * (m * c1) / (sqrtf(v * c2) + eps);
      L.W32[idx] = w;
    }
    const uint16_t h = bf16_rne(w);
    L.W16[idx] = h;
    t[i][tx] = h;
  }
  __syncthreads();
  for (int i = ty; i < 64; i += 4) L.W16T[(ti * 64 + i) * nout + to * 64 + tx] = t[tx][i];
}

__global__ __launch_bounds__(256) void k_adam_b(LayerView L, const float *__restrict__ gpart, int chunks, float lr,
                                                float b1, float b2, float eps, float c1, float c2) {
  const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (o >= L.n_out) return;
  float g = 0.f;
  for (int s = 0; s < chunks; ++s) g += gpart[(int64_t)s * L.n_out + o];
  const float m = b1 * L.mb[o] + (1.f - b1) * g;
  const float v = b2 * L.vb[o] + (1.f - b2) * g * g;
  L.mb[o] = m;
  L.vb[o] = v;
  L.b32[o] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
}

// Gradient export: sum the partials into a dense FP32 array.
__global__ __launch_bounds__(256) void k_sum_parts(const float *__restrict__ part, int parts, int64_t n,
                                                   float *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float g = 0.f;
  for (int s = 0; s < parts; ++s) g += part[(int64_t)s * n + i];
  out[i] = g;
}

// Plain FP32 copies and zero fills (kernels, so that captured graphs hold no memset).
__global__ __launch_bounds__(256) void k_copy32(const float *__restrict__ src, int64_t n, float *__restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src ? src[i] : 0.f;
}

// ---------------------------------------------------------------------------
// Top-S of N scores per signal (one wavefront; NPL = N / 64 scores per lane):
// S rounds of a wavefront max over packed keys (orderable score bits, then
// the complement of the index so that ties go to the lowest index).
// ---------------------------------------------------------------------------
__device__ inline uint32_t orderable(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

template <int NPL>
__global__ __launch_bounds__(64) void k_topk(const float *__restrict__ Z, int64_t ldz, int S,
                                             int32_t *__restrict__ P) {
  const int64_t b = blockIdx.x;
  const int lane = threadIdx.x;
  uint64_t key[NPL];
#pragma unroll
  for (int q = 0; q < NPL; ++q) {
    const int n = q * 64 + lane;
    key[q] = ((uint64_t)orderable(Z[b * ldz + n]) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)n);
  }
  for (int s = 0; s < S; ++s) {
    uint64_t best = 0;
#pragma unroll
    for (int q = 0; q < NPL; ++q) best = key[q] > best ? key[q] : best;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const uint64_t o = __shfl_xor(best, off);
      best = o > best ? o : best;
    }
#pragma unroll
    for (int q = 0; q < NPL; ++q) key[q] = key[q] == best ? 0ull : key[q];  // keys are distinct
    if (lane == 0) P[b * S + s] = (int32_t)(0xFFFFFFFFu - (uint32_t)(best & 0xFFFFFFFFull));
  }
}

// ---------------------------------------------------------------------------
// Least-squares check of a proposed support (one wavefront per signal, S <= 64):
// Cholesky of the Gram block G[P, P] (pivots in FP64; a pivot below the
// dependency threshold rejects the proposal), beta = A_P^T y with exact
// products and FP64 sums, forward and back solves, the residual
// r = y - A_P x in FP32 and ||r|| in FP64; accepted when ||r|| <= eps_b.
// LDS: L (S x (S+1) floats) per wavefront.
// ---------------------------------------------------------------------------
constexpr int LS_WAVES = 4;

__global__ __launch_bounds__(64 * LS_WAVES) void k_ls_check(DictView d, const float *__restrict__ Y, int64_t ldy,
                                                            int64_t B, const int32_t *__restrict__ P, int S,
                                                            const float *__restrict__ eps_per, float eps,
                                                            int32_t *__restrict__ support_out,
                                                            float *__restrict__ coef_out,
                                                            int32_t *__restrict__ status_out,
                                                            float *__restrict__ rnorm_out,
                                                            int32_t *__restrict__ accept) {
  extern __shared__ float lsm[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t b = (int64_t)blockIdx.x * LS_WAVES + wv;
  if (b >= B) return;
  const int LD = S + 1;
  float *Ls = lsm + (size_t)wv * S * LD;
  const int pi = lane < S ? P[b * S + lane] : 0;
  // Gram block rows: lane i holds row i of G[P, P] in LDS.
  for (int j = 0; j < S; ++j) {
    const int pj = __shfl(pi, j);
    if (lane < S) Ls[lane * LD + j] = d.G[(int64_t)pj * d.Np + pi];
  }
  // beta_j = a_{P_j}^T y and the signal's own finiteness.
  const float *y = Y + b * ldy;
  double bj = 0.0;
  int finite = 1;
  for (int j = 0; j < S; ++j) {
    const int pj = __shfl(pi, j);
    double s = 0.0;
    for (int64_t m = lane; m < d.M; m += 64) {
      const float v = y[m];
      finite &= isfinite(v) ? 1 : 0;
      s += (double)d.A32[(int64_t)pj * d.Mp + m] * (double)v;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if (lane == j) bj = s;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  // Cholesky, column by column: L[j][j] = sqrt(G[j][j] - sum_k L[j][k]^2) (FP64),
  // L[i][j] = (G[i][j] - sum_k L[i][k] L[j][k]) / L[j][j] for i > j.
  bool dependent = !__all(finite);
  float rdj = 0.f;  // lane j keeps 1 / L[j][j]
  for (int j = 0; j < S && !dependent; ++j) {
    double dd = 0.0;
    float off = 0.f;
    for (int k = 0; k < j; ++k) {
      const float ljk = Ls[j * LD + k];
      dd += (double)ljk * (double)ljk;
      if (lane > j && lane < S) off = fmaf(Ls[lane * LD + k], ljk, off);
    }
    const double nu2 = d.nu2[__shfl(pi, j)];
    const double d2 = (double)Ls[j * LD + j] - dd;
    if (!(d2 > DEP_TOL2 * nu2)) {
      dependent = true;
      break;
    }
    const float dj = (float)sqrt(d2);
    if (lane == j) {
      Ls[j * LD + j] = dj;
      rdj = 1.f / dj;
    }
    if (lane > j && lane < S) Ls[lane * LD + j] = (Ls[lane * LD + j] - off) / dj;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  float x = 0.f;
  double rn = 0.0;
  if (!dependent) {
    // forward solve L u = beta (row by row: u_j = (beta_j - sum_k L[j][k] u_k) / L[j][j])
    float u = 0.f;
    for (int j = 0; j < S; ++j) {
      float acc = (float)__shfl(bj, j);
      for (int k = 0; k < j; ++k) acc = fmaf(-Ls[j * LD + k], __shfl(u, k), acc);
      const float uj = acc * __shfl(rdj, j);
      if (lane == j) u = uj;
    }
    // back solve L^T x = u, last unknown first: x_j = (u_j - sum_{i>j} L[i][j] x_i) / L[j][j]
    for (int j = S - 1; j >= 0; --j) {
      float acc = __shfl(u, j);
      for (int i = j + 1; i < S; ++i) acc = fmaf(-Ls[i * LD + j], __shfl(x, i), acc);
      const float xj = acc * __shfl(rdj, j);
      if (lane == j) x = xj;
    }
    // residual and its norm
    for (int64_t m = lane; m < d.M; m += 64) {
      float r = y[m];
      for (int j = 0; j < S; ++j) r = fmaf(-__shfl(x, j), d.A32[(int64_t)__shfl(pi, j) * d.Mp + m], r);
      rn += (double)r * (double)r;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) rn += __shfl_xor(rn, off);
    rn = sqrt(rn);
  }
  float eb = eps_per ? eps_per[b] : eps;
  eb = fmaxf(eb, 0.f);
  const bool ok = !dependent && rn <= (double)eb;
  if (lane < S) {
    support_out[b * S + lane] = ok ? pi : -1;
    coef_out[b * S + lane] = ok ? x : 0.f;
  }
  if (lane == 0) {
    accept[b] = ok ? 1 : 0;
    if (ok) {
      status_out[b] = (S << 8) | OMP_SIG_EPS | OMP_SIG_LEARNED;
      rnorm_out[b] = (float)rn;
    }
  }
}

// Rejected signals: compacted index list (order irrelevant: each signal's
// fallback result does not depend on the others) and their signals and
// tolerances gathered for the fallback solve.
__global__ __launch_bounds__(256) void k_compact(const int32_t *__restrict__ accept, int64_t B,
                                                 int32_t *__restrict__ idx, int32_t *__restrict__ count) {
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b < B && !accept[b]) idx[atomicAdd(count, 1)] = (int32_t)b;
}

__global__ __launch_bounds__(64) void k_gather_rejects(const float *__restrict__ Y, int64_t ldy, int64_t M,
                                                       const float *__restrict__ eps_per, float eps,
                                                       const int32_t *__restrict__ idx, float *__restrict__ Yr,
                                                       float *__restrict__ eps_r) {
  const int64_t i = blockIdx.x;
  const int64_t b = idx[i];
  for (int64_t m = threadIdx.x; m < M; m += 64) Yr[i * M + m] = Y[b * ldy + m];
  if (threadIdx.x == 0) eps_r[i] = eps_per ? eps_per[b] : eps;
}

__global__ __launch_bounds__(64) void k_scatter_fallback(const int32_t *__restrict__ idx, int S,
                                                         const int32_t *__restrict__ sup_r,
                                                         const float *__restrict__ coef_r,
                                                         const int32_t *__restrict__ st_r,
                                                         const float *__restrict__ rn_r, int32_t *__restrict__ support_out,
                                                         float *__restrict__ coef_out, int32_t *__restrict__ status_out,
                                                         float *__restrict__ rnorm_out) {
  const int64_t i = blockIdx.x;
  const int64_t b = idx[i];
  for (int j = threadIdx.x; j < S; j += 64) {
    support_out[b * S + j] = sup_r[i * S + j];
    coef_out[b * S + j] = coef_r[i * S + j];
  }
  if (threadIdx.x == 0) {
    status_out[b] = st_r[i];
    rnorm_out[b] = rn_r[i];
  }
}

template <class K>
hipError_t lds_limit(K kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

template <int EPI>
hipError_t gemm_t(const uint16_t *P, int64_t ldp, const uint16_t *Q, int64_t ldq, int64_t M, int64_t N, int64_t K,
                  int splits, const GemmEpi &e, hipStream_t st) {
  hipError_t err = lds_limit(k_gemm_nt<EPI>, GT::LDS_BYTES);
  if (err != hipSuccess) return err;
  const unsigned grid = (unsigned)((M / GT::TN) * (N / GT::TB) * splits);
  hipLaunchKernelGGL(k_gemm_nt<EPI>, dim3(grid), dim3(GT::NTHR), GT::LDS_BYTES, st, P, ldp, Q, ldq, M, N, K, splits,
                     e);
  return hipGetLastError();
}

}  // namespace

int64_t gemm_blocks(int64_t M, int64_t N, int splits) { return (M / GT::TN) * (N / GT::TB) * splits; }

hipError_t launch_gemm_bf16(int epi, const uint16_t *P, int64_t ldp, const uint16_t *Q, int64_t ldq, int64_t M,
                            int64_t N, int64_t K, int splits, const GemmEpi &e, hipStream_t st) {
  if (M % GT::TN || N % GT::TB || K % (64 * splits) || ldp % 8 || ldq % 8) return hipErrorInvalidValue;
  switch (epi) {
    case EPI_FEATURES: return gemm_t<EPI_FEATURES>(P, ldp, Q, ldq, M, N, K, splits, e, st);
    case EPI_BIAS_RELU: return gemm_t<EPI_BIAS_RELU>(P, ldp, Q, ldq, M, N, K, splits, e, st);
    case EPI_BIAS: return gemm_t<EPI_BIAS>(P, ldp, Q, ldq, M, N, K, splits, e, st);
    case EPI_BCE: return gemm_t<EPI_BCE>(P, ldp, Q, ldq, M, N, K, splits, e, st);
    case EPI_RELU_MASK: return gemm_t<EPI_RELU_MASK>(P, ldp, Q, ldq, M, N, K, splits, e, st);
    default: return gemm_t<EPI_PARTIAL>(P, ldp, Q, ldq, M, N, K, splits, e, st);
  }
}

hipError_t launch_prep_signals(const float *Y, int64_t ldy, int64_t B, int64_t M, int64_t Mp, int64_t Bp,
                               uint16_t *Y16, float *yinv, hipStream_t st) {
  hipLaunchKernelGGL(k_prep_signals, dim3((unsigned)Bp), dim3(64), 0, st, Y, ldy, B, M, Mp, Y16, yinv);
  return hipGetLastError();
}

hipError_t launch_pad_rows16(const uint16_t *src, int64_t ld, const int32_t *rows, int64_t B, int64_t cols,
                             int64_t Bp, uint16_t *dst, hipStream_t st) {
  hipLaunchKernelGGL(k_pad_rows16, dim3((unsigned)Bp), dim3(256), 0, st, src, ld, rows, B, cols, dst);
  return hipGetLastError();
}

hipError_t launch_labels(const int32_t *sup, const int32_t *rows, int64_t B, int S, int64_t n_out, int64_t Bp,
                         uint32_t *bits, hipStream_t st) {
  hipLaunchKernelGGL(k_labels, dim3((unsigned)Bp), dim3(64), 0, st, sup, rows, B, S, n_out / 32, bits);
  return hipGetLastError();
}

hipError_t launch_transpose16(const uint16_t *src, int64_t R, int64_t C, uint16_t *dst, hipStream_t st) {
  hipLaunchKernelGGL(k_transpose16, dim3((unsigned)((R / 64) * (C / 64))), dim3(256), 0, st, src, R, C, dst);
  return hipGetLastError();
}

hipError_t launch_colsum16(const uint16_t *src, int64_t R, int64_t C, int chunks, float *part, hipStream_t st) {
  const int64_t rpc = (R + chunks - 1) / chunks;
  hipLaunchKernelGGL(k_colsum16, dim3((unsigned)((C / 256) * chunks)), dim3(256), 0, st, src, R, C, rpc, part);
  return hipGetLastError();
}

hipError_t launch_loss_sum(const float *part, int64_t n, float scale, float *out, hipStream_t st) {
  hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(64), 0, st, part, n, scale, out);
  return hipGetLastError();
}

hipError_t launch_adam_w(const LayerView &L, const float *gpart, int splits, float lr, float b1, float b2, float eps,
                         float c1, float c2, int update, hipStream_t st) {
  hipLaunchKernelGGL(k_adam_w, dim3((unsigned)((L.n_out / 64) * (L.n_in / 64))), dim3(256), 0, st, L, gpart, splits,
                     lr, b1, b2, eps, c1, c2, update);
  return hipGetLastError();
}

hipError_t launch_adam_b(const LayerView &L, const float *gpart, int chunks, float lr, float b1, float b2, float eps,
                         float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(k_adam_b, dim3((unsigned)((L.n_out + 255) / 256)), dim3(256), 0, st, L, gpart, chunks, lr, b1,
                     b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_sum_parts(const float *part, int parts, int64_t n, float *out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part, parts, n, out);
  return hipGetLastError();
}

hipError_t launch_copy32(const float *src, int64_t n, float *dst, hipStream_t st) {
  hipLaunchKernelGGL(k_copy32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, n, dst);
  return hipGetLastError();
}

hipError_t launch_topk(const float *Z, int64_t ldz, int64_t N, int64_t B, int S, int32_t *P, hipStream_t st) {
  switch (N / 64) {
    case 4: hipLaunchKernelGGL(k_topk<4>, dim3((unsigned)B), dim3(64), 0, st, Z, ldz, S, P); break;
    case 8: hipLaunchKernelGGL(k_topk<8>, dim3((unsigned)B), dim3(64), 0, st, Z, ldz, S, P); break;
    case 16: hipLaunchKernelGGL(k_topk<16>, dim3((unsigned)B), dim3(64), 0, st, Z, ldz, S, P); break;
    case 32: hipLaunchKernelGGL(k_topk<32>, dim3((unsigned)B), dim3(64), 0, st, Z, ldz, S, P); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ls_check(const DictView &d, const float *Y, int64_t ldy, int64_t B, const int32_t *P, int S,
                           const float *eps_per, float eps, int32_t *support_out, float *coef_out, int32_t *status_out,
                           float *rnorm_out, int32_t *accept, hipStream_t st) {
  if (S < 1 || S > 64) return hipErrorInvalidValue;
  const size_t lds = (size_t)LS_WAVES * S * (S + 1) * sizeof(float);
  const unsigned blocks = (unsigned)((B + LS_WAVES - 1) / LS_WAVES);
  hipLaunchKernelGGL(k_ls_check, dim3(blocks), dim3(64 * LS_WAVES), lds, st, d, Y, ldy, B, P, S, eps_per, eps,
                     support_out, coef_out, status_out, rnorm_out, accept);
  return hipGetLastError();
}

hipError_t launch_compact(const int32_t *accept, int64_t B, int32_t *idx, int32_t *count, hipStream_t st) {
  hipLaunchKernelGGL(k_copy32, dim3(1), dim3(256), 0, st, nullptr, 1, reinterpret_cast<float *>(count));
  hipLaunchKernelGGL(k_compact, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, accept, B, idx, count);
  return hipGetLastError();
}

hipError_t launch_gather_rejects(const float *Y, int64_t ldy, int64_t M, const float *eps_per, float eps,
                                 const int32_t *idx, int64_t n, float *Yr, float *eps_r, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rejects, dim3((unsigned)n), dim3(64), 0, st, Y, ldy, M, eps_per, eps, idx, Yr, eps_r);
  return hipGetLastError();
}

hipError_t launch_scatter_fallback(const int32_t *idx, int64_t n, int S, const int32_t *sup_r, const float *coef_r,
                                   const int32_t *st_r, const float *rn_r, int32_t *support_out, float *coef_out,
                                   int32_t *status_out, float *rnorm_out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_fallback, dim3((unsigned)n), dim3(64), 0, st, idx, S, sup_r, coef_r, st_r, rn_r,
                     support_out, coef_out, status_out, rnorm_out);
  return hipGetLastError();
}

}  // namespace bomp
