// Per-signal kernels of the OMP iteration for gfx950: dictionary preparation,
// solve set-up, the update step after each correlation product, and the output
// scatter. One 64-lane wavefront owns one signal in the update step.
//
// The update step is the least-squares half of Algorithm 1 done by the
// progressive Cholesky factorisation of Section 2.2 (Eqs. 4-5), with the Gram
// row taken from the precomputed A^T A:
//
//   g   = G[n*, support]                  (A_{k-1}^T a_n*, Eq. 3 via the Gram)
//   z   = V_{k-1}^{-1} g                  (forward solve, Eq. 5)
//   d   = sqrt(||a_n*||^2 - ||z||^2)      (new pivot, Eq. 5; FP64 subtraction)
//   V_k = [[V_{k-1}, 0], [z^T, d]]        (append one row)
//   beta = a_n*^T y                       (append to A_k^T y, Eq. 2)
//   u_k = (beta - z^T u_{k-1}) / d        (forward solve V_k u = A_k^T y, one new entry)
//   x   = V_k^{-T} u                      (back solve)
//   r   = y - A_k x                       (recomputed from y, no drift)
//
// The paper's code re-factorised A_k^T A_k at every step and names the
// Cholesky update as its next step (Section 3.6); this file implements that
// update. V is kept packed (row i at offset i(i+1)/2), the packed storage of
// Section 3.3, and is staged through LDS for the two triangular solves.

#include <cmath>

#include "../../include/batched_omp.h"
#include "omp_internal.h"

namespace bomp {
namespace {

__device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ inline uint64_t wave_max(uint64_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint64_t w = __shfl_xor(v, o);
    v = w > v ? w : v;
  }
  return v;
}

// Select element p (wave-uniform) of a small per-lane register array without
// dynamic register indexing.
template <int R>
__device__ inline float pick(const float (&a)[R], int p) {
  float v = a[0];
#pragma unroll
  for (int i = 1; i < R; ++i) v = (p == i) ? a[i] : v;
  return v;
}
template <int R>
__device__ inline void put(float (&a)[R], int p, float v) {
#pragma unroll
  for (int i = 0; i < R; ++i) a[i] = (p == i) ? v : a[i];
}

__device__ inline float readlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Rigorous bound on |s_bf16 - s| for one atom, where s = |a^T r| / ||a|| is the
// score of the FP32 residual r and s_bf16 the score computed from BF16-rounded
// a and r with FP32 accumulation over K terms:
//   |c_bf16 - c| <= ((2 u_b + u_b^2) + gamma_K (1 + u_b)^2) sum_m |a_m r_m|
//                <= (...) ||a|| ||r||                      (Cauchy-Schwarz),
// u_b = 2^-8 (BF16 unit roundoff), gamma_K = K u / (1 - K u), u = 2^-24, plus
// one FP32 rounding for the scaling by 1/||a||; a 1% margin covers the
// rounding of ||r|| itself.
__device__ inline double bf16_tau(double rn, int64_t K) {
  const double ub = 1.0 / 256.0;
  const double u = 1.0 / 16777216.0;
  const double gk = (double)K * u / (1.0 - (double)K * u);
  return 1.01 * ((2.0 * ub + ub * ub) + gk * (1.0 + ub) * (1.0 + ub) + 2.0 * u) * rn;
}

// Score of atom n against the FP32 residual r, |a_n^T r| / ||a_n||, with exact
// products and FP64 accumulation (the whole wavefront cooperates).
__device__ inline double rescore(const DictView &d, const float4 *__restrict__ r4, int n, int lane) {
  const int64_t nc4 = d.Mp / 4;
  const float4 *a4 = reinterpret_cast<const float4 *>(d.A32) + (int64_t)n * nc4;
  double acc = 0.0;
  for (int64_t c = lane; c < nc4; c += 64) {
    const float4 a = a4[c], r = r4[c];
    acc += (double)a.x * r.x + (double)a.y * r.y + (double)a.z * r.z + (double)a.w * r.w;
  }
  acc = wave_sum(acc);
  return fabs(acc) / sqrt(d.nu2[n]);
}

__device__ inline bool better(double s, int n, double bs, int bn) { return s > bs || (s == bs && n < bn); }

// BF16 form of the pick. The epilogue left, per subgroup of atoms, the keys of
// its best and second-best BF16 score. With tau the bound above:
//   1. s_max = largest BF16 score; every listed atom with s_bf16 >= s_max - 2 tau
//      is re-scored exactly; the best re-scored atom w is the provisional pick.
//      (The atom holding s_max has s >= s_max - tau, so a listed atom below the
//      window, s <= s_bf16 + tau < s_max - tau, cannot beat w.)
//   2. an unlisted atom of a subgroup has s <= theta + tau, theta the
//      subgroup's second BF16 score; when theta + tau >= s_w the whole
//      subgroup is re-scored (and the signal is flagged OMP_SIG_WIDENED).
// The result is the exact argmax of s over the selectable atoms, ties to the
// lowest index. Returns -1 when no atom is selectable.
__device__ int select_bf16(const DictView &d, const WorkView &w, int64_t b, int lane, int *widened) {
  const int nkeys = w.ntile * w.ncand;
  const uint64_t *keys = w.part + b * nkeys;
  const float4 *r4 = reinterpret_cast<const float4 *>(w.R32) + b * (d.Mp / 4);
  float smax = -1.f;
  for (int t = lane; t < nkeys; t += 64) {
    const uint64_t k = keys[t];
    if (k) smax = fmaxf(smax, __uint_as_float((uint32_t)(k >> 32)));
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) smax = fmaxf(smax, __shfl_xor(smax, o));
  if (smax < 0.f) return -1;
  const double tau = bf16_tau((double)w.rn[b], d.Mp);
  const double thr = (double)smax - 2.0 * tau;
  double bs = -1.0;
  int bn = 0x7fffffff;
  for (int t0 = 0; t0 < nkeys; t0 += 64) {
    const int t = t0 + lane;
    const uint64_t k = t < nkeys ? keys[t] : 0ull;
    const bool cand = k && (double)__uint_as_float((uint32_t)(k >> 32)) >= thr;
    uint64_t m = __ballot(cand);
    const int n_l = (int)(0xFFFFFFFFu - (uint32_t)(k & 0xFFFFFFFFull));
    while (m) {
      const int l = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      const int n = __builtin_amdgcn_readlane(n_l, l);
      const double sc = rescore(d, r4, n, lane);
      if (better(sc, n, bs, bn)) { bs = sc; bn = n; }
    }
  }
  const int64_t mwords = d.Np / 32;
  const uint32_t *mk = w.mask + b * mwords;
  for (int t0 = 0; t0 < nkeys; t0 += 64) {
    const int t = t0 + lane;
    const uint64_t k = (t < nkeys && (t & 1)) ? keys[t] : 0ull;
    const bool open = k && (double)__uint_as_float((uint32_t)(k >> 32)) + tau >= bs;
    uint64_t m = __ballot(open);
    while (m) {
      const int l = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      const int slot = t0 + l;
      const int tile = slot / w.ncand;
      const int sg = (slot % w.ncand) >> 1;
      const int wn = sg >> 1, hh = sg & 1;
      *widened = 1;
      for (int i = 0; i < w.sub_fn; ++i)
        for (int g = 0; g < 4; ++g)
          for (int e = 0; e < 4; ++e) {
            const int n = tile * w.tile_atoms + wn * w.sub_atoms + 32 * i + 8 * g + 4 * hh + e;
            if (d.inv_nu[n] <= 0.f || ((mk[n >> 5] >> (n & 31)) & 1u)) continue;
            const double sc = rescore(d, r4, n, lane);
            if (better(sc, n, bs, bn)) { bs = sc; bn = n; }
          }
    }
  }
  return bn;
}

// ---------------------------------------------------------------------------
// Dictionary preparation: one wavefront per (padded) atom.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_dict_prep(const float *__restrict__ A, int64_t lda, int64_t M,
                                                  int64_t N, int64_t Mp, double *__restrict__ nu2,
                                                  float *__restrict__ inv_nu, float *__restrict__ A32,
                                                  uint16_t *__restrict__ A16) {
  const int64_t n = blockIdx.x;
  const int lane = threadIdx.x;
  double s = 0.0;
  for (int64_t m = lane; m < Mp; m += 64) {
    const float v = (n < N && m < M) ? A[n * lda + m] : 0.f;
    A32[n * Mp + m] = v;
    if (A16) A16[n * Mp + m] = f32_to_bf16_rne(v);
    s += (double)v * (double)v;
  }
  s = wave_sum(s);
  if (lane == 0) {
    nu2[n] = s;
    inv_nu[n] = s > 0.0 ? (float)(1.0 / sqrt(s)) : 0.f;
  }
}

// ---------------------------------------------------------------------------
// Solve set-up: one wavefront per (padded) signal.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_init(const float *__restrict__ Y, int64_t ldy,
                                             const int32_t *__restrict__ S_per,
                                             const float *__restrict__ eps_per, float eps, int64_t M,
                                             WorkView w) {
  const int64_t b = blockIdx.x;
  const int lane = threadIdx.x;
  const bool real = b < w.B;
  double s = 0.0;
  int finite = 1;
  for (int64_t m = lane; m < w.Mp; m += 64) {
    const float v = (real && m < M) ? Y[b * ldy + m] : 0.f;
    finite &= isfinite(v) ? 1 : 0;
    const float vz = isfinite(v) ? v : 0.f;
    w.Yp[b * w.Mp + m] = vz;
    w.R32[b * w.Mp + m] = vz;
    if (w.R16) w.R16[b * w.Mp + m] = f32_to_bf16_rne(vz);
    s += (double)vz * (double)vz;
  }
  const int64_t mwords = w.Np / 32;
  for (int64_t t = lane; t < mwords; t += 64) w.mask[b * mwords + t] = 0u;
  s = wave_sum(s);
  const bool all_finite = __all(finite);
  if (lane == 0) {
    int Sb = w.S;
    if (S_per && real) Sb = min(max(S_per[b], 0), w.S);
    float eb = (eps_per && real) ? eps_per[b] : eps;
    eb = fmaxf(eb, 0.f);  // also maps NaN to 0
    const double rn = sqrt(s);
    int fl = 0;
    if (!real) fl = FLAG_DONE;
    else if (!all_finite) fl = FLAG_DONE | OMP_SIG_NONFINITE;
    else if (rn <= (double)eb) fl = FLAG_DONE | OMP_SIG_EPS | (Sb == 0 ? OMP_SIG_SMAX : 0);
    else if (Sb == 0) fl = FLAG_DONE | OMP_SIG_SMAX;
    w.flags[b] = fl;
    w.k[b] = 0;
    w.rn[b] = real && all_finite ? (float)rn : 0.f;
    w.Sb[b] = Sb;
    w.epsb[b] = eb;
  }
}

// ---------------------------------------------------------------------------
// Update step. One 64-lane block per signal; RPL = rows of V per lane
// (S <= 64 RPL; RPL in {1, 2, 4}).
// LDS: V (S(S+1)/2 floats), coefficients (S floats), support (S ints).
// ---------------------------------------------------------------------------
template <int RPL, bool BF16>
__global__ __launch_bounds__(64) void k_update(DictView d, WorkView w) {
  extern __shared__ float smem[];
  const int64_t b = blockIdx.x;
  const int lane = threadIdx.x;
  const int fl0 = w.flags[b];
  if (fl0 & FLAG_DONE) return;  // whole block exits together
  const int S = w.S;
  const int64_t VS = (int64_t)S * (S + 1) / 2;
  float *Vs = smem;
  float *xs = Vs + VS;
  int *ss = reinterpret_cast<int *>(xs + S);
  const int k = w.k[b];

  // 1. The pick: the winner over all atom tiles (largest score, then lowest
  //    index); in the BF16 form, the certified exact re-score of the candidates.
  int nstar = -1;
  int widened = 0;
  if (BF16) {
    nstar = select_bf16(d, w, b, lane, &widened);
  } else {
    uint64_t best = 0;
    const int nkeys = w.ntile * w.ncand;
    for (int t = lane; t < nkeys; t += 64) {
      const uint64_t v = w.part[b * nkeys + t];
      best = v > best ? v : best;
    }
    best = wave_max(best);
    if (best != 0ull) nstar = (int)(0xFFFFFFFFu - (uint32_t)(best & 0xFFFFFFFFull));
  }
  if (nstar < 0) {  // nothing selectable is left
    if (lane == 0) w.flags[b] = fl0 | FLAG_DONE | OMP_SIG_EXHAUSTED;
    return;
  }
  const int fl1 = fl0 | (widened ? OMP_SIG_WIDENED : 0);

  // 2. Support and packed factor into LDS.
  for (int t = lane; t < k; t += 64) ss[t] = w.sup[b * S + t];
  const int64_t vlen = (int64_t)k * (k + 1) / 2;
  for (int64_t t = lane; t < vlen; t += 64) Vs[t] = w.V[b * VS + t];
  __syncthreads();

  // 3. Gram row g_i = G[n*, support_i]; lane holds rows i = lane + 64 p.
  float g[RPL], z[RPL];
#pragma unroll
  for (int p = 0; p < RPL; ++p) {
    const int i = lane + 64 * p;
    g[p] = i < k ? d.G[(int64_t)nstar * d.Np + ss[i]] : 0.f;
    z[p] = 0.f;
  }

  // 4. Forward solve V_{k-1} z = g, column by column.
  for (int j = 0; j < k; ++j) {
    const int pj = j >> 6, jl = j & 63;
    const int64_t rj = (int64_t)j * (j + 1) / 2;
    const float zj = readlane(pick(g, pj), jl) / Vs[rj + j];
    if (lane == jl) put(z, pj, zj);
#pragma unroll
    for (int p = 0; p < RPL; ++p) {
      const int i = lane + 64 * p;
      if (i > j && i < k) g[p] = fmaf(-Vs[(int64_t)i * (i + 1) / 2 + j], zj, g[p]);
    }
  }

  // 5. Pivot d^2 = ||a_n*||^2 - ||z||^2 in FP64.
  double zz = 0.0;
#pragma unroll
  for (int p = 0; p < RPL; ++p) zz += (double)z[p] * (double)z[p];
  zz = wave_sum(zz);
  const double nu2 = d.nu2[nstar];
  const double d2 = nu2 - zz;
  if (!(d2 > DEP_TOL2 * nu2)) {  // dependent atom: stop without appending
    if (lane == 0) w.flags[b] = fl1 | FLAG_DONE | OMP_SIG_DEPENDENT;
    return;
  }
  const float dk = (float)sqrt(d2);

  // 6. beta = a_n*^T y; u_k = (beta - z^T u_{k-1}) / d.
  const int64_t nc4 = d.Mp / 4;
  const float4 *A4 = reinterpret_cast<const float4 *>(d.A32);
  const float4 *Y4 = reinterpret_cast<const float4 *>(w.Yp) + b * nc4;
  const float4 *an = A4 + (int64_t)nstar * nc4;
  float bp = 0.f;
  for (int64_t c = lane; c < nc4; c += 64) {
    const float4 a = an[c], y = Y4[c];
    bp = fmaf(a.x, y.x, bp);
    bp = fmaf(a.y, y.y, bp);
    bp = fmaf(a.z, y.z, bp);
    bp = fmaf(a.w, y.w, bp);
  }
  const double beta = wave_sum((double)bp);
  float uo[RPL];
  double zu = 0.0;
#pragma unroll
  for (int p = 0; p < RPL; ++p) {
    const int i = lane + 64 * p;
    uo[p] = i < k ? w.u[b * S + i] : 0.f;
    zu += (double)z[p] * (double)uo[p];
  }
  zu = wave_sum(zu);
  const float uk = (float)((beta - zu) / (double)dk);

  // 7. Append row k of V, u_k and n* (LDS and memory).
  const int64_t rk = (int64_t)k * (k + 1) / 2;
#pragma unroll
  for (int p = 0; p < RPL; ++p) {
    const int i = lane + 64 * p;
    if (i < k) {
      Vs[rk + i] = z[p];
      w.V[b * VS + rk + i] = z[p];
    }
  }
  if (lane == 0) {
    Vs[rk + k] = dk;
    w.V[b * VS + rk + k] = dk;
    ss[k] = nstar;
    w.sup[b * S + k] = nstar;
    w.u[b * S + k] = uk;
    const int64_t mwords = d.Np / 32;
    w.mask[b * mwords + nstar / 32] |= 1u << (nstar & 31);
  }
  __syncthreads();
  const int K = k + 1;

  // 8. Back solve V_K^T x = u, last unknown first.
  float t[RPL], x[RPL];
#pragma unroll
  for (int p = 0; p < RPL; ++p) {
    const int i = lane + 64 * p;
    t[p] = i < k ? uo[p] : (i == k ? uk : 0.f);
    x[p] = 0.f;
  }
  for (int j = K - 1; j >= 0; --j) {
    const int pj = j >> 6, jl = j & 63;
    const int64_t rj = (int64_t)j * (j + 1) / 2;
    const float xj = readlane(pick(t, pj), jl) / Vs[rj + j];
    if (lane == jl) put(x, pj, xj);
#pragma unroll
    for (int p = 0; p < RPL; ++p) {
      const int i = lane + 64 * p;
      if (i < j) t[p] = fmaf(-Vs[rj + i], xj, t[p]);
    }
  }
#pragma unroll
  for (int p = 0; p < RPL; ++p) {
    const int i = lane + 64 * p;
    if (i < K) {
      xs[i] = x[p];
      w.xh[b * S + i] = x[p];
    }
  }
  __syncthreads();

  // 9. Residual r = y - sum_j x_j a_{s_j}, recomputed from y; ||r||^2 in FP64.
  float4 *R4 = reinterpret_cast<float4 *>(w.R32) + b * nc4;
  double nrm = 0.0;
  for (int64_t base = 0; base < nc4; base += 256) {
    float4 r[4];
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
      const int64_t c = base + lane + 64 * cc;
      r[cc] = c < nc4 ? Y4[c] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll 4
    for (int j = 0; j < K; ++j) {
      const float xj = -xs[j];
      const float4 *a = A4 + (int64_t)ss[j] * nc4 + base + lane;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        if (base + lane + 64 * cc < nc4) {
          const float4 av = a[64 * cc];
          r[cc].x = fmaf(xj, av.x, r[cc].x);
          r[cc].y = fmaf(xj, av.y, r[cc].y);
          r[cc].z = fmaf(xj, av.z, r[cc].z);
          r[cc].w = fmaf(xj, av.w, r[cc].w);
        }
      }
    }
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
      const int64_t c = base + lane + 64 * cc;
      if (c < nc4) {
        R4[c] = r[cc];
        if (BF16) {
          ushort4 h;
          h.x = f32_to_bf16_rne(r[cc].x);
          h.y = f32_to_bf16_rne(r[cc].y);
          h.z = f32_to_bf16_rne(r[cc].z);
          h.w = f32_to_bf16_rne(r[cc].w);
          reinterpret_cast<ushort4 *>(w.R16)[b * nc4 + c] = h;
        }
        nrm += (double)r[cc].x * r[cc].x + (double)r[cc].y * r[cc].y + (double)r[cc].z * r[cc].z +
               (double)r[cc].w * r[cc].w;
      }
    }
  }
  nrm = wave_sum(nrm);

  // 10. Stop test.
  if (lane == 0) {
    const double rn = sqrt(nrm);
    int fl = fl1;
    if (rn <= (double)w.epsb[b]) fl |= FLAG_DONE | OMP_SIG_EPS;
    if (K >= w.Sb[b]) fl |= FLAG_DONE | OMP_SIG_SMAX;
    w.k[b] = K;
    w.rn[b] = (float)rn;
    w.flags[b] = fl;
  }
}

// ---------------------------------------------------------------------------
// Outputs: one 256-thread block per signal.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_finalize(WorkView w, int64_t N, float *__restrict__ X_out,
                                                  int32_t *__restrict__ support_out,
                                                  float *__restrict__ coef_out,
                                                  int32_t *__restrict__ status_out,
                                                  float *__restrict__ rnorm_out) {
  __shared__ int ss[OMP_MAX_S];
  __shared__ float xs[OMP_MAX_S];
  const int64_t b = blockIdx.x;
  const int S = w.S;
  const int k = w.k[b];
  for (int j = threadIdx.x; j < S; j += blockDim.x) {
    const int sj = j < k ? w.sup[b * S + j] : -1;
    const float xj = j < k ? w.xh[b * S + j] : 0.f;
    ss[j] = sj;
    xs[j] = xj;
    support_out[b * S + j] = sj;
    if (coef_out) coef_out[b * S + j] = xj;
  }
  __syncthreads();
  if (X_out) {
    const int64_t mwords = w.Np / 32;
    for (int64_t n = threadIdx.x; n < N; n += blockDim.x) {
      float v = 0.f;
      if ((w.mask[b * mwords + n / 32] >> (n & 31)) & 1u) {
        for (int j = 0; j < k; ++j)
          if (ss[j] == n) v = xs[j];
      }
      X_out[b * N + n] = v;
    }
  }
  if (threadIdx.x == 0) {
    if (status_out) status_out[b] = (k << 8) | (w.flags[b] & 0xff);
    if (rnorm_out) rnorm_out[b] = w.rn[b];
  }
}

}  // namespace

hipError_t launch_dict_prep(const float *A, int64_t lda, const DictView &d, hipStream_t st) {
  hipLaunchKernelGGL(k_dict_prep, dim3((unsigned)d.Np), dim3(64), 0, st, A, lda, d.M, d.N, d.Mp, d.nu2,
                     d.inv_nu, d.A32, d.A16);
  return hipGetLastError();
}

hipError_t launch_init(const float *Y, int64_t ldy, const int32_t *S_per, const float *eps_per, float eps,
                       const DictView &d, const WorkView &w, int precision, hipStream_t st) {
  (void)precision;
  hipLaunchKernelGGL(k_init, dim3((unsigned)w.Bp), dim3(64), 0, st, Y, ldy, S_per, eps_per, eps, d.M, w);
  return hipGetLastError();
}

hipError_t launch_update(const DictView &d, const WorkView &w, int precision, hipStream_t st) {
  const size_t lds = ((size_t)w.S * (w.S + 1) / 2 + 2 * (size_t)w.S) * 4;
  const dim3 grid((unsigned)w.B), block(64);
  if (w.B == 0) return hipSuccess;
  const bool bf = precision == OMP_PREC_BF16;
  if (w.S <= 64) {
    if (bf) hipLaunchKernelGGL((k_update<1, true>), grid, block, lds, st, d, w);
    else hipLaunchKernelGGL((k_update<1, false>), grid, block, lds, st, d, w);
  } else if (w.S <= 128) {
    if (bf) hipLaunchKernelGGL((k_update<2, true>), grid, block, lds, st, d, w);
    else hipLaunchKernelGGL((k_update<2, false>), grid, block, lds, st, d, w);
  } else {
    static bool attr[2] = {false, false};
    const void *fn = bf ? reinterpret_cast<const void *>(k_update<4, true>)
                        : reinterpret_cast<const void *>(k_update<4, false>);
    if (!attr[bf]) {
      hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      if (e != hipSuccess) return e;
      attr[bf] = true;
    }
    if (bf) hipLaunchKernelGGL((k_update<4, true>), grid, block, lds, st, d, w);
    else hipLaunchKernelGGL((k_update<4, false>), grid, block, lds, st, d, w);
  }
  return hipGetLastError();
}

hipError_t launch_finalize(const DictView &d, const WorkView &w, float *X_out, int32_t *support_out,
                           float *coef_out, int32_t *status_out, float *rnorm_out, hipStream_t st) {
  if (w.B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)w.B), dim3(256), 0, st, w, d.N, X_out, support_out, coef_out,
                     status_out, rnorm_out);
  return hipGetLastError();
}

}  // namespace bomp
