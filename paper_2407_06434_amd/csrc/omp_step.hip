// Per-signal kernels of the OMP iteration for gfx950: dictionary preparation,
// solve set-up, the two kernels that follow each correlation product, and the
// output scatter.
//
// After the correlation product has scored every atom, one iteration of
// Algorithm 1 finishes in two kernels:
//
// k_solve (one 64-lane wavefront per signal): the pick and the least-squares
// update by the progressive Cholesky factorisation of Section 2.2 (Eqs. 4-5),
// with the Gram row taken from the precomputed A^T A:
//
//   g    = G[n*, support]                 (A_{k-1}^T a_n*, Eq. 3 via the Gram)
//   z    = V_{k-1}^{-1} g                 (forward solve, Eq. 5)
//   d    = sqrt(||a_n*||^2 - ||z||^2)     (new pivot, Eq. 5; FP64 subtraction)
//   V_k  = [[V_{k-1}, 0], [z^T, d]]       (append one row)
//   beta = a_n*^T y                       (append to A_k^T y, Eq. 2), evaluated
//        = a_n*^T r + g^T x_{k-1}         as the exact score of the pick plus the
//                                         Gram row times the current coefficients
//                                         (r = y - A_{k-1} x_{k-1}), so that only
//                                         a_n* and r are read
//   u_k  = (beta - z^T u_{k-1}) / d       (forward solve V_k u = A_k^T y, one new entry)
//   x    = V_k^{-T} u                     (back solve)
//
// k_residual: r = y - A_k x, recomputed from y at every step (no drift), with
// ||r||^2 accumulated in FP64 per slice of the signal. The signal is cut into
// up to 8 slices of M and workgroup i works on slice i mod 8: workgroups are
// dispatched round-robin over the 8 XCDs, so every XCD only ever gathers its
// own eighth of every atom (one slice of M), which then stays in its L2. For a
// dictionary of at most 4 MiB in FP32 (one XCD's L2) the solve's wavefront
// forms r itself after its back solve, in the same order per element, and
// k_residual is not launched (except for
// signals shorter than 256 samples in batches larger than the solve's resident
// wavefronts, where the residual kernel's packing of several signals per
// wavefront wins, and for S > 64 where the solve holds the residual in
// registers).
//
// The paper's code re-factorised A_k^T A_k at every step and names the
// Cholesky update as its next step (Section 3.6); this file implements that
// update. V is kept packed (row i at offset i(i+1)/2), the packed storage of
// Section 3.3, and is staged through LDS for the two triangular solves.

#include <cmath>
#include <cstring>

#include "../../include/batched_omp.h"
#include "omp_internal.h"

namespace bomp {

// The solve reads the residual into registers in its first memory round when
// a lane's share fills most of its four 16-byte register chunks (512 < M <=
// 1024) and the form keeps residual vectors. Shorter signals keep the memory path: with one or two
// chunks per lane the register path's fixed four loads per operand cost more
// than the round they save (2.3% slower at M = 64 and 256). Not in the slot
// scheduler's solve either, whose retire-and-admit code would then leave three
// wavefronts per SIMD instead of four.
bool solve_rr(const DictView &d, const WorkView &w) { return !w.gram_dom && d.Mp > 512 && d.Mp <= 1024; }

// Whether the solve forms the residual itself instead of a residual launch, for
// the residual-vector forms on a batch of B signals: dictionaries of at most
// 4 MiB in FP32 (one XCD's L2; beyond that gathering whole atoms leaves the L2s
// and the XCD-sliced residual kernel wins), except signals shorter than 256
// samples in batches of more than 4096 (the solve's resident wavefronts): one
// wavefront per signal then leaves lanes idle, and each later generation of
// solve wavefronts waits for its gathers again, where the residual kernel packs
// several signals per wavefront and holds every one of them at once.
bool residual_in_solve(const DictView &d, int64_t B) {
  return d.Mp * d.Np * 4 <= ((int64_t)4 << 20) && (d.Mp >= 256 || B <= 4096);
}

namespace {

__device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// FP16 (IEEE binary16) round to nearest even, and back.
__device__ inline uint16_t f32_to_f16_rne(float f) { return __builtin_bit_cast(uint16_t, (_Float16)f); }
__device__ inline float f16_to_f32(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }

// The value the product may take for a stored 16-bit code: the code's own value, or 0
// where the code is subnormal (an MFMA that flushes subnormal inputs uses 0). The
// rounding errors of the copies are measured against it, so the certificate's bound
// holds whether or not subnormals are flushed (|v - sub| <= |v - 0| for a subnormal sub
// that v rounds to).
__device__ inline double bf16_used(uint16_t h) {
  return (h & 0x7F80u) == 0 ? 0.0 : (double)__uint_as_float((uint32_t)h << 16);
}
__device__ inline double f16_used(uint16_t h) { return (h & 0x7C00u) == 0 ? 0.0 : (double)f16_to_f32(h); }

// The power of two 2^-e with x 2^-e in [1/2, 1) (1 for x = 0 or non-finite x): the
// FP16 form stores sigma v so that every stored value lies in [-1, 1].
__device__ inline float pow2_scale(double x) {
  if (!(x > 0.0) || !isfinite(x)) return 1.f;
  int e;
  (void)frexp(x, &e);
  return ldexpf(1.f, -e);
}

// Cross-lane moves within 16-lane rows by DPP (no LDS round trip): the two
// 32-bit halves of a 64-bit value move together.
template <int CTRL>
__device__ inline uint64_t dpp64(uint64_t v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, 0xF, 0xF, false);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
template <int CTRL>
__device__ inline double dppd(double v) {
  return __longlong_as_double((long long)dpp64<CTRL>((uint64_t)__double_as_longlong(v)));
}
__device__ inline uint64_t readlane64(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}
// DPP controls: swap neighbours (quad_perm 1,0,3,2), swap pairs (quad_perm
// 2,3,0,1), reverse 8 lanes (row_half_mirror), reverse 16 lanes (row_mirror).
constexpr int DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140;

// Sum over the 64 lanes, returned to every lane: each 16-lane row is reduced
// by four DPP steps (after them every lane of a row holds the row's sum), then
// the four row sums are read out and added in a fixed order. Must be called
// with every lane active.
__device__ inline double wave_sum(double v) {
  v += dppd<DPP_XOR1>(v);
  v += dppd<DPP_XOR2>(v);
  v += dppd<DPP_HALF_MIRROR>(v);
  v += dppd<DPP_MIRROR>(v);
  const double r0 = __longlong_as_double((long long)readlane64((uint64_t)__double_as_longlong(v), 0));
  const double r1 = __longlong_as_double((long long)readlane64((uint64_t)__double_as_longlong(v), 16));
  const double r2 = __longlong_as_double((long long)readlane64((uint64_t)__double_as_longlong(v), 32));
  const double r3 = __longlong_as_double((long long)readlane64((uint64_t)__double_as_longlong(v), 48));
  return (r0 + r1) + (r2 + r3);
}

__device__ inline uint64_t wave_max(uint64_t v) {
  uint64_t w = dpp64<DPP_XOR1>(v);
  v = w > v ? w : v;
  w = dpp64<DPP_XOR2>(v);
  v = w > v ? w : v;
  w = dpp64<DPP_HALF_MIRROR>(v);
  v = w > v ? w : v;
  w = dpp64<DPP_MIRROR>(v);
  v = w > v ? w : v;
  uint64_t m = readlane64(v, 0);
#pragma unroll
  for (int r = 16; r < 64; r += 16) {
    const uint64_t x = readlane64(v, r);
    m = x > m ? x : m;
  }
  return m;
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
__device__ inline int pick_i(const int (&a)[R], int p) {
  int v = a[0];
#pragma unroll
  for (int i = 1; i < R; ++i) v = (p == i) ? a[i] : v;
  return v;
}

__device__ inline float readlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Element j (wave-uniform) of an array held one element per lane, rows
// j = lane + 64 p: lane j mod 64 of every register is read first and the
// register chosen by j / 64 afterwards, among the read (uniform) values. Unlike
// readlane(pick(a, j >> 6), j & 63) this is exact where some lanes are inactive:
// pick's per-lane select is not executed by inactive lanes, whose stale values
// readlane would then return.
template <int R>
__device__ inline int lane_elem(const int (&a)[R], int j) {
  int v = __builtin_amdgcn_readlane(a[0], j & 63);
#pragma unroll
  for (int i = 1; i < R; ++i) {
    const int u = __builtin_amdgcn_readlane(a[i], j & 63);
    v = (j >> 6) == i ? u : v;
  }
  return v;
}
template <int R>
__device__ inline float lane_elem(const float (&a)[R], int j) {
  float v = readlane(a[0], j & 63);
#pragma unroll
  for (int i = 1; i < R; ++i) {
    const float u = readlane(a[i], j & 63);
    v = (j >> 6) == i ? u : v;
  }
  return v;
}

// Current ||r|| of signal b from its per-slice partial sums of squares.
__device__ inline double residual_norm(const WorkView &w, int64_t b) {
  double s = 0.0;
  for (int i = 0; i < NSLICE_MAX; ++i) s += w.pnorm[b * NSLICE_MAX + i];
  return sqrt(s);
}

// Rigorous bound on |s_bf16 - s| for every atom, where s = |a^T r| / ||a|| is
// the exact score of the FP32 residual r and s_bf16 the score the BF16 product
// computed from a~ = bf16(a), r~ = bf16(r). With e = a - a~, delta = r - r~:
//   a^T r - a~^T r~ = a~^T delta + e^T r~ + e^T delta
//   |a^T r - a~^T r~| <= ||a|| ((1 + 2 E) D + E R~)       (Cauchy-Schwarz)
// where E = max_n ||e_n|| / ||a_n|| (measured once per dictionary), D = ||delta||
// (measured with each residual) and R~ = ||r~|| <= ||r|| + D. The BF16 products
// are exact in FP32; their FP32 accumulation over K terms adds at most
// gamma_K ||a~|| ||r~|| <= gamma_K (1 + E) ||a|| R~, gamma_K = K u / (1 - K u),
// u = 2^-24; scaling by the FP32 1/||a|| adds 2 u (s + T) <= 2 u (||r|| + T).
// This is far tighter than the worst case u_bf16 ||a|| ||r||: rounding errors
// have norm ~ 2^-8 / sqrt(3) relative, not 2^-8.
__device__ inline double bf16_tau(double rn, double dn, double E, int64_t K) {
  const double u = 1.0 / 16777216.0;
  const double gk = (double)K * u / (1.0 - (double)K * u);
  const double Rt = rn + dn;
  const double T = (1.0 + 2.0 * E) * dn + E * Rt + gk * (1.0 + E) * Rt;
  return (T * (1.0 + 4.0 * u) + 2.0 * u * (rn + T)) * (1.0 + 1e-9) + 1e-30;
}

__device__ inline bool better(double s, int n, double bs, int bn) { return s > bs || (s == bs && n < bn); }

__device__ inline double dot4d(const float4 &a, const float4 &v) {
  return (double)a.x * v.x + (double)a.y * v.y + (double)a.z * v.z + (double)a.w * v.w;
}

// FP64 dot products of up to NA atoms (n[i] < 0: unused) with the vector v:
// exact products, FP64 accumulation. The whole wavefront cooperates; each lane
// keeps CP 16-byte chunks of every operand in flight per pass, and the
// reductions run interleaved.
template <int NA, int CP>
__device__ __attribute__((always_inline)) inline void atom_dots(const DictView &d, const int (&n)[NA],
                                                                const float4 *__restrict__ v4, int lane,
                                                                double (&av)[NA]) {
  const int64_t nc4 = d.Mp / 4;
  const float4 *A4 = reinterpret_cast<const float4 *>(d.A32);
  // Every load reads a valid address (unused atoms read row 0, chunks past the
  // end read chunk 0) and the value is then masked: a conditional choice between
  // a load and a constant would be compiled as a choice of pointers.
  int64_t row[NA];
  bool use[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    use[i] = n[i] >= 0;
    row[i] = (int64_t)(use[i] ? n[i] : 0) * nc4;
  }
#pragma unroll
  for (int i = 0; i < NA; ++i) av[i] = 0.0;
  for (int64_t c0 = 0; c0 < nc4; c0 += 64 * CP) {
    float4 vv[CP], aa[NA][CP];
    bool ok[CP];
#pragma unroll
    for (int q = 0; q < CP; ++q) {
      const int64_t c = c0 + lane + 64 * q;
      ok[q] = c < nc4;
      const int64_t cs = ok[q] ? c : 0;
      vv[q] = v4[cs];
#pragma unroll
      for (int i = 0; i < NA; ++i) aa[i][q] = A4[row[i] + cs];
    }
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
      for (int q = 0; q < CP; ++q) {
        const double pa = dot4d(aa[i][q], vv[q]);
        av[i] += (use[i] && ok[q]) ? pa : 0.0;
      }
  }
#pragma unroll
  for (int i = 0; i < NA; ++i) av[i] = wave_sum(av[i]);
}

// The residual's chunks a lane holds in registers when the solve reads r in
// its first memory round (512 < M <= 64 * 4 * RREG).
constexpr int RREG = 4;
static_assert(64 * 4 * RREG == 1024, "solve_rr selects the register path for M <= 1024");

// atom_dots with the vector already in registers: lane l holds chunks
// l + 64 q (q < RREG) of v, zero past the end (requires M <= 64 * 4 * RREG).
// The atoms' chunks are loaded CP at a time.
template <int NA, int CP>
__device__ __attribute__((always_inline)) inline void atom_dots_reg(const DictView &d, const int (&n)[NA],
                                                                    const float4 (&vr)[RREG], int lane,
                                                                    double (&av)[NA]) {
  static_assert(RREG % CP == 0, "whole passes");
  const int64_t nc4 = d.Mp / 4;
  const float4 *A4 = reinterpret_cast<const float4 *>(d.A32);
  int64_t row[NA];
  bool use[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    use[i] = n[i] >= 0;
    row[i] = (int64_t)(use[i] ? n[i] : 0) * nc4;
    av[i] = 0.0;
  }
#pragma unroll
  for (int q0 = 0; q0 < RREG; q0 += CP) {
    float4 aa[NA][CP];
    bool ok[CP];
#pragma unroll
    for (int q = 0; q < CP; ++q) {
      const int64_t c = lane + 64 * (q0 + q);
      ok[q] = c < nc4;
      const int64_t cs = ok[q] ? c : 0;
#pragma unroll
      for (int i = 0; i < NA; ++i) aa[i][q] = A4[row[i] + cs];
    }
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
      for (int q = 0; q < CP; ++q) {
        const double pa = dot4d(aa[i][q], vr[q0 + q]);
        av[i] += (use[i] && ok[q]) ? pa : 0.0;
      }
  }
#pragma unroll
  for (int i = 0; i < NA; ++i) av[i] = wave_sum(av[i]);
}

typedef __attribute__((address_space(3))) void lds_void_t;

// Asynchronous global-to-LDS loads (gfx950 global_load_lds): lane l's element
// lands at dst + l (lane order), dst being wave-uniform. Completion is awaited
// with s_waitcnt before the LDS data is read.
__device__ inline void lds_load16(const float4 *src, float4 *dst_wave) {
  __builtin_amdgcn_global_load_lds(reinterpret_cast<const void *>(src), (lds_void_t *)(dst_wave), 16, 0,
                                   0);
}

// Intra-wavefront LDS ordering: one wavefront's LDS instructions execute in
// order, so it suffices that the compiler keeps them in program order.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Queue of atoms to re-score against r, flushed two at a time (all values
// wave-uniform; a pick has about two candidates on the benchmark workload).
// A flush fetches, in one round with the dot products, each candidate's
// ||a_n||^2. Keeps the best exact score, its atom, its signed a^T r and
// ||a||^2. The winner's Gram row is read after the pick: fetching every
// candidate's row in the re-score round instead saves that round but reads
// about twice the Gram lines, and measured 2.3% slower on the benchmark step.
template <bool RR>
struct RescoreQueue {
  const float4 *r4;          // the residual in memory ...
  const float4 (&rr)[RREG];  // ... and in registers (RR)
  __device__ RescoreQueue(const float4 *r, const float4 (&regs)[RREG]) : r4(r), rr(regs) {}
  int n0 = -1, n1 = -1;
  double bs = -1.0;
  double bs2 = -1.0;  // best exact score of any other atom (near-tie flagging)
  double bar = 0.0, bnu2 = 0.0;
  int bn = 0x7fffffff;
  template <int NA>
  __device__ __attribute__((always_inline)) void rescore(const DictView &d, const int (&n)[NA], int lane) {
    double nu2[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) nu2[i] = n[i] >= 0 ? d.nu2[n[i]] : 1.0;
    double ar[NA];
    if constexpr (RR)
      atom_dots_reg<NA, 2>(d, n, rr, lane, ar);
    else
      atom_dots<NA, 2>(d, n, r4, lane, ar);
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      if (n[i] < 0) continue;
      const double sc = fabs(ar[i]) / sqrt(nu2[i]);
      if (better(sc, n[i], bs, bn)) {
        if (n[i] != bn) bs2 = bs;  // (an atom may be re-scored twice: it is not its own runner-up)
        bs = sc;
        bn = n[i];
        bar = ar[i];
        bnu2 = nu2[i];
      } else if (n[i] != bn && sc > bs2) {
        bs2 = sc;
      }
    }
  }
  __device__ __attribute__((always_inline)) void flush(const DictView &d, int lane) {
    if (n0 < 0) return;
    if (n1 < 0) {  // a single atom: half the loads and dot products
      const int n[1] = {n0};
      rescore<1>(d, n, lane);
    } else {
      const int n[2] = {n0, n1};
      rescore<2>(d, n, lane);
    }
    n0 = n1 = -1;
  }
  __device__ __attribute__((always_inline)) void push(int atom, const DictView &d, int lane) {
    if (n0 < 0) {
      n0 = atom;
    } else {
      n1 = atom;
      flush(d, lane);
    }
  }
};

// Keys kept in registers per lane by the solve's first memory round (BF16 form):
// up to 64 * KREG keys per signal, otherwise they are read again in batches.
constexpr int KREG = 8;

// BF16 keys (32 bits): the BF16 score's bits with the low five replaced by
// 31 - loc (loc = the atom's place in its 32-atom subgroup), bit 31 set when
// the atom is selected, zero-norm or padding. Key slot t of a signal belongs
// to subgroup (t / NKEEP) of the correlation tile's layout.
__device__ inline bool key_valid(uint32_t key) { return !(key >> 31); }
__device__ inline double key_score(uint32_t key) { return (double)__uint_as_float(key & 0x7FFFFFE0u); }
__device__ inline int key_loc(uint32_t key) { return 31 - (int)(key & 31u); }

// Atom of subgroup slot `t` (tile t / ncand, subgroup ((wn * subs_per_half +
// ig) * 2 + h) within it) at place loc = ii * 16 + r: the epilogue's row
// 8 (r / 4) + 4 h + r % 4 of fragment ig * sub_frags + ii of wavefront row wn.
__device__ inline int key_atom(const WorkView &w, int t, int loc) {
  const int tile = t / w.ncand;
  const int sgl = (t % w.ncand) / NKEEP;
  const int hh = sgl & 1;
  const int ig = (sgl >> 1) % w.subs_per_half;
  const int wn = (sgl >> 1) / w.subs_per_half;
  const int ii = loc >> 4, r = loc & 15;
  return tile * w.tile_atoms + wn * w.wave_atoms + 32 * (ig * w.sub_frags + ii) + 8 * (r >> 2) + 4 * hh + (r & 3);
}

// One batch of keys (KB per lane, key t0 + 64 j + lane in kb[j]): candidates
// (valid, score >= thr) are appended to clist, subgroups whose bounding key
// could reach the exact winner (theta (1 + et) >= mthr) to mlist.
// Bits of the largest float <= x, for x >= 0 (0 for x <= 0): a score s (a
// non-negative float, compared through its bits, which order like the values)
// satisfies s >= x exactly when bits(s) >= this, up to the floats in
// [result, x), which are taken as well.
__device__ inline uint32_t float_bits_floor(double x) {
  if (!(x > 0.0)) return 0u;
  float f = (float)x;
  if ((double)f > x) f = __uint_as_float(__float_as_uint(f) - 1u);
  return __float_as_uint(f);
}

template <int KB>
__device__ __attribute__((always_inline)) inline void scan_keys(const uint32_t (&kb)[KB], int t0, int nkeys,
                                                                uint32_t thr_bits, uint32_t mthr_bits, int *clist,
                                                                int *mlist, int &ncand, int &nmaybe) {
#pragma unroll
  for (int j = 0; j < KB; ++j) {
    const int t = t0 + 64 * j + (int)(threadIdx.x & 63);
    const uint32_t sb = kb[j] & 0x7FFFFFE0u;  // score bits
    const bool cand = key_valid(kb[j]) && sb >= thr_bits;
    const uint64_t m = __ballot(cand);
    if (m) {
      const int pos = ncand + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
      if (cand) clist[pos] = t * 32 + key_loc(kb[j]);
      ncand += __popcll(m);
    }
    const bool maybe = t < nkeys && (t % NKEEP) == NKEEP - 1 && sb >= mthr_bits;
    const uint64_t mm = __ballot(maybe);
    if (mm) {
      const int mpos = nmaybe + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mm >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)mm, 0u));
      if (maybe && mpos < MAYBE_CAP) mlist[mpos] = t;
      nmaybe += __popcll(mm);
    }
  }
}

// Ablation A3 (re-factorisation instead of the progressive update): the packed
// lower triangle of G[S, S] in LDS is replaced by its Cholesky factor, column
// by column (left-looking: lane i forms row i's dot product with row j in
// FP64, the pivot comes from lane j).
template <int RPL>
__device__ void cholesky_lds(float *Vs, int k, int lane) {
  for (int j = 0; j < k; ++j) {
    const int tj = j * (j + 1) / 2;
    double sp[RPL];
#pragma unroll
    for (int p = 0; p < RPL; ++p) {
      const int i = lane + 64 * p;
      const int ti = i * (i + 1) / 2;
      double acc = 0.0;
      if (i >= j && i < k)
        for (int q = 0; q < j; ++q) acc += (double)Vs[ti + q] * (double)Vs[tj + q];
      sp[p] = acc;
    }
    double sj = sp[0];
#pragma unroll
    for (int p = 1; p < RPL; ++p) sj = ((j >> 6) == p) ? sp[p] : sj;
    sj = __longlong_as_double((long long)readlane64((uint64_t)__double_as_longlong(sj), j & 63));
    const double piv = fmax((double)Vs[tj + j] - sj, 1e-300);
    const double djj = sqrt(piv);
#pragma unroll
    for (int p = 0; p < RPL; ++p) {
      const int i = lane + 64 * p;
      const int ti = i * (i + 1) / 2;
      if (i > j && i < k) Vs[ti + j] = (float)(((double)Vs[ti + j] - sp[p]) / djj);
      if (i == j) Vs[tj + j] = (float)djj;
    }
    wave_lds_sync();
  }
}

// Ablation of the Gram precomputation: g_i = a_{s_i}^T a_n* for the rows i < k
// this lane holds, from the FP32 atoms (exact products, FP64 sum, rounded to
// FP32 like the stored Gram).
template <int RPL>
__device__ void gram_row_from_atoms(const DictView &d, int nstar, const int (&si)[RPL], int k, int lane,
                                    float (&g)[RPL]) {
  const int64_t nc4 = d.Mp / 4;
  const float4 *A4 = reinterpret_cast<const float4 *>(d.A32);
  const float4 *an = A4 + (int64_t)nstar * nc4;
#pragma unroll
  for (int p = 0; p < RPL; ++p) {
    const int i = lane + 64 * p;
    const bool use = i < k;
    const float4 *as = A4 + (int64_t)(use ? si[p] : 0) * nc4;
    double acc = 0.0;
    for (int64_t c = 0; c < nc4; ++c) acc += dot4d(as[c], an[c]);
    g[p] = use ? (float)acc : 0.f;
  }
}

// BF16 form of the pick. The epilogue left, per subgroup of atoms, keys for
// its NKEEP best BF16 scores, each score rounded down by less than 2^-18
// relative (et below); keys of selected, zero or padding atoms carry their
// score but no index. With tau the bound above and s_max the largest score of
// a valid listed key:
//   1. every valid listed atom with s >= s_max - 2 tau - et s_max is re-scored
//      exactly; the best re-scored atom w is the provisional pick. (The atom
//      holding s_max has exact score >= s_max - tau, and a listed atom below
//      the window has exact score <= s (1 + et) + tau < s_max - tau.)
//   2. an unlisted atom of a subgroup has exact score <= theta (1 + et) + tau,
//      theta the subgroup's last kept score; when that reaches s_w the whole
//      subgroup is re-scored (and the signal is flagged OMP_SIG_WIDENED). Since
//      s_w >= s_max - tau, only subgroups with theta (1 + et) >= s_max - 2 tau
//      can open: they are listed while the keys are scanned for step 1 and
//      tested against s_w afterwards.
// The result is the exact argmax of s over the selectable atoms, ties to the
// lowest index; *cdot and *nu2 receive a_n*^T r and ||a_n*||^2 of the pick
// (fetched in the same round as its score). kv holds the signal's keys when
// kreg (read in the first memory round).
template <bool RR>
__device__ int select_bf16(const DictView &d, const WorkView &w, int64_t b, float smax_key, double ks, double tau,
                           int lane, int *widened, double *cdot, double *nu2, int *clist,
                           const uint32_t (&kv)[KREG], bool kreg, const float4 (&rr)[RREG], int *neartie) {
  // Key scores carry the scale ks of the 16-bit residual copy (1 in the BF16 form, a
  // power of two in the FP16 form): a score s is stored as ks s, exactly.
  const double smax = (double)smax_key / ks;
  const int nkeys = w.ntile * w.ncand;
  const uint32_t *keys = reinterpret_cast<const uint32_t *>(w.part) + b * nkeys;
  const float4 *r4 = reinterpret_cast<const float4 *>(w.R32) + b * (d.Mp / 4);
  const double et = 1.0 / 262144.0;  // 2^-18: the epilogue's rounding of listed scores
  // Near-tie flagging widens both windows by TIE_REL s_max, so that every atom
  // whose exact score can reach (1 - TIE_REL) s_w is re-scored too.
  const double tw = w.flag_ties ? TIE_REL * smax : 0.0;
  const double thr = smax - 2.0 * tau - et * smax - tw;
  const double mthr = smax - 2.0 * tau - tw;
  // the same tests on score bits: s >= thr, and s (1 + et) >= mthr taken as
  // s >= mthr / (1 + et) lowered by 1e-12 relative (a superset of the list), both
  // in the keys' scale
  const uint32_t thr_bits = float_bits_floor(thr * ks);
  const uint32_t mthr_bits = float_bits_floor(mthr / (1.0 + et) * (1.0 - 1e-12) * ks);
  int *mlist = clist + solve_cand_len(nkeys);
  RescoreQueue<RR> q(r4, rr);
  // Candidates and possibly open subgroups, from the keys in registers or, for
  // more keys than that, read again KREG per lane at a time.
  int ncand = 0, nmaybe = 0;
  if (kreg) {
    scan_keys<KREG>(kv, 0, nkeys, thr_bits, mthr_bits, clist, mlist, ncand, nmaybe);
  } else {
    for (int t0 = 0; t0 < nkeys; t0 += 64 * KREG) {
      uint32_t kb[KREG];
#pragma unroll
      for (int j = 0; j < KREG; ++j) {
        const int t = t0 + 64 * j + lane;
        const uint32_t v = keys[t < nkeys ? t : 0];
        kb[j] = t < nkeys ? v : 0x80000000u;
      }
      scan_keys<KREG>(kb, t0, nkeys, thr_bits, mthr_bits, clist, mlist, ncand, nmaybe);
    }
  }
  wave_lds_sync();
  for (int i = 0; i < ncand; ++i) {
    const int e = __builtin_amdgcn_readfirstlane(clist[i]);
    q.push(key_atom(w, e >> 5, e & 31), d, lane);
  }
  q.flush(d, lane);

  // The listed subgroups (all bounding keys if the list overflowed) against
  // the exact winner; an open subgroup is re-scored whole.
  const int64_t mwords = d.Np / 32;
  const uint32_t *mk = w.mask + b * mwords;
  const bool movf = nmaybe > MAYBE_CAP;
  const int npass = movf ? nkeys / NKEEP : nmaybe;
  for (int i = 0; i < npass; ++i) {
    const int slot = movf ? i * NKEEP + NKEEP - 1 : __builtin_amdgcn_readfirstlane(mlist[i]);
    const double theta = key_score(keys[slot]) / ks;
    if (!(theta * (1.0 + et) + tau >= (w.flag_ties ? (1.0 - TIE_REL) * q.bs : q.bs))) continue;
    const int tile = slot / w.ncand;
    const int sgl = (slot % w.ncand) / NKEEP;  // ((wn * subs_per_half + ig) * 2 + h)
    const int hh = sgl & 1;
    const int ig = (sgl >> 1) % w.subs_per_half;
    const int wn = (sgl >> 1) / w.subs_per_half;
    *widened = 1;
    for (int ii = 0; ii < w.sub_frags; ++ii)
      for (int g4 = 0; g4 < 4; ++g4)
        for (int e = 0; e < 4; ++e) {
          const int n = tile * w.tile_atoms + wn * w.wave_atoms + 32 * (ig * w.sub_frags + ii) + 8 * g4 + 4 * hh + e;
          if (d.inv_nu[n] <= 0.f || ((mk[n >> 5] >> (n & 31)) & 1u)) continue;
          q.push(n, d, lane);
        }
    q.flush(d, lane);
  }
  *cdot = q.bar;
  *nu2 = q.bnu2;
  *neartie = (w.flag_ties && q.bs2 >= (1.0 - TIE_REL) * q.bs) ? 1 : 0;
  return q.bn == 0x7fffffff ? -1 : q.bn;
}


// ---------------------------------------------------------------------------
// Dictionary preparation: one wavefront per (padded) atom.
// ---------------------------------------------------------------------------
// The FP16 form (inv_nu_h set) stores fp16(sigma_n a_n) with sigma_n = pow2_scale(max_m
// |a_n,m|) and scores by inv_nu_h[n] = 1/(sigma_n ||a_n||); the rounding error ratio is
// measured in the atom's own scale.
__global__ __launch_bounds__(64) void k_dict_prep(const float *__restrict__ A, int64_t lda, int64_t M,
                                                  int64_t N, int64_t Mp, double *__restrict__ nu2,
                                                  float *__restrict__ inv_nu, float *__restrict__ A32,
                                                  uint16_t *__restrict__ A16, float *__restrict__ aerr,
                                                  float *__restrict__ inv_nu_h) {
  const int64_t n = blockIdx.x;
  const int lane = threadIdx.x;
  float sig = 1.f;
  if (inv_nu_h) {
    float mx = 0.f;
    for (int64_t m = lane; m < M; m += 64) mx = fmaxf(mx, n < N ? fabsf(A[n * lda + m]) : 0.f);
    for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    sig = pow2_scale((double)mx);
  }
  double s = 0.0, e = 0.0;
  for (int64_t m = lane; m < Mp; m += 64) {
    const float v = (n < N && m < M) ? A[n * lda + m] : 0.f;
    A32[n * Mp + m] = v;
    if (A16) {
      uint16_t h;
      double dv;
      if (inv_nu_h) {
        h = f32_to_f16_rne(v * sig);
        dv = (double)v - f16_used(h) / (double)sig;
      } else {
        h = f32_to_bf16_rne(v);
        dv = (double)v - bf16_used(h);
      }
      A16[n * Mp + m] = h;
      e += dv * dv;
    }
    s += (double)v * (double)v;
  }
  s = wave_sum(s);
  e = wave_sum(e);
  if (lane == 0) {
    nu2[n] = s;
    inv_nu[n] = s > 0.0 ? (float)(1.0 / sqrt(s)) : 0.f;
    if (inv_nu_h) inv_nu_h[n] = s > 0.0 ? (float)(1.0 / (sqrt(s) * (double)sig)) : 0.f;
    // rounded up so that the float is an upper bound of the ratio
    aerr[n] = s > 0.0 ? __double2float_ru(sqrt(e / s) * (1.0 + 1e-12)) : 0.f;
  }
}

// 1/||a_n|| in FP64 from the FP64 squared norms (0 for zero and padding atoms).
__global__ __launch_bounds__(256) void k_inv_nu64(const double *__restrict__ nu2, int64_t Np,
                                                  double *__restrict__ inv) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n < Np) inv[n] = nu2[n] > 0.0 ? 1.0 / sqrt(nu2[n]) : 0.0;
}

// max_n aerr[n] over the dictionary (one block).
__global__ __launch_bounds__(1024) void k_dict_aerr_max(const float *__restrict__ aerr, int64_t Np,
                                                        float *__restrict__ out) {
  __shared__ float red[1024];
  float m = 0.f;
  for (int64_t n = threadIdx.x; n < Np; n += 1024) m = fmaxf(m, aerr[n]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 512; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// ---------------------------------------------------------------------------
// Solve set-up.
// ---------------------------------------------------------------------------
__device__ inline int signal_S(const int32_t *S_per, int64_t i, int S) {
  return S_per ? min(max(S_per[i], 0), S) : S;
}
__device__ inline float signal_eps(const float *eps_per, int64_t i, float eps) {
  return eps_per ? eps_per[i] : eps;
}

// Puts signal y (length M; null = no signal) into column b of the workspace: the
// padded copy, r = y in FP32 (and BF16), ||y||^2 and ||y - bf16(y)||^2, a clear
// atom mask, k = 0, and the stops that need no pick (non-finite y, ||y|| <= eps,
// S_b = 0). A column without a signal gets `idle` as its flags. One wavefront.
__device__ void init_column(const WorkView &w, int64_t b, const float *__restrict__ y, int64_t M, int Sb,
                            float eb, int idle, int lane) {
  double s = 0.0, dl = 0.0;
  int finite = 1;
  if ((M & 3) == 0 && (reinterpret_cast<uintptr_t>(y) & 15) == 0) {
    // 16-byte chunks (a chunk lies wholly inside or wholly past the signal)
    const float4 *y4 = reinterpret_cast<const float4 *>(y);
    float4 *Y4 = reinterpret_cast<float4 *>(w.Yp + b * w.Mp);
    float4 *R4 = reinterpret_cast<float4 *>(w.R32 + b * w.Mp);
    for (int64_t c = lane; c < w.Mp / 4; c += 64) {
      float4 v = (y && 4 * c < M) ? y4[c] : make_float4(0.f, 0.f, 0.f, 0.f);
      finite &= (isfinite(v.x) && isfinite(v.y) && isfinite(v.z) && isfinite(v.w)) ? 1 : 0;
      v.x = isfinite(v.x) ? v.x : 0.f;
      v.y = isfinite(v.y) ? v.y : 0.f;
      v.z = isfinite(v.z) ? v.z : 0.f;
      v.w = isfinite(v.w) ? v.w : 0.f;
      Y4[c] = v;
      R4[c] = v;
      if (w.R16 && !w.fp16) {
        ushort4 h;
        h.x = f32_to_bf16_rne(v.x);
        h.y = f32_to_bf16_rne(v.y);
        h.z = f32_to_bf16_rne(v.z);
        h.w = f32_to_bf16_rne(v.w);
        reinterpret_cast<ushort4 *>(w.R16 + b * w.Mp)[c] = h;
        const double d0 = (double)v.x - bf16_used(h.x);
        const double d1 = (double)v.y - bf16_used(h.y);
        const double d2 = (double)v.z - bf16_used(h.z);
        const double d3 = (double)v.w - bf16_used(h.w);
        dl += d0 * d0 + d1 * d1 + d2 * d2 + d3 * d3;
      }
      s += (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w;
    }
  } else {
    for (int64_t m = lane; m < w.Mp; m += 64) {
      const float v = (y && m < M) ? y[m] : 0.f;
      finite &= isfinite(v) ? 1 : 0;
      const float vz = isfinite(v) ? v : 0.f;
      w.Yp[b * w.Mp + m] = vz;
      w.R32[b * w.Mp + m] = vz;
      if (w.R16 && !w.fp16) {
        const uint16_t h = f32_to_bf16_rne(vz);
        w.R16[b * w.Mp + m] = h;
        const double dv = (double)vz - bf16_used(h);
        dl += dv * dv;
      }
      s += (double)vz * (double)vz;
    }
  }
  const int64_t mwords = w.Np / 32;
  for (int64_t t = lane; t < mwords; t += 64) w.mask[b * mwords + t] = 0u;
  s = wave_sum(s);
  dl = wave_sum(dl);
  const bool all_finite = __all(finite);
  if (w.fp16) {
    // FP16 form: the 16-bit copy is fp16(sigma y), sigma = pow2_scale(||y||), so every
    // stored value lies in [-1, 1]; ||y - fp16(sigma y) / sigma||^2 replaces dl
    const float sig = all_finite ? pow2_scale(sqrt(s)) : 1.f;
    double d16 = 0.0;
    for (int64_t m = lane; m < w.Mp; m += 64) {
      float v = (y && m < M) ? y[m] : 0.f;
      v = isfinite(v) ? v : 0.f;
      const uint16_t h = f32_to_f16_rne(v * sig);
      w.R16[b * w.Mp + m] = h;
      const double dv = (double)v - f16_used(h) / (double)sig;
      d16 += dv * dv;
    }
    dl = wave_sum(d16);
    if (lane == 0) w.rscale[b] = sig;
  }
  if (lane < NSLICE_MAX) {
    w.pnorm[b * NSLICE_MAX + lane] = (lane == 0 && all_finite) ? s : 0.0;
    // (the Gram-domain and v0 forms keep ||y||^2 there: the rounding scale of their running ||r||^2)
    w.pdelta[b * NSLICE_MAX + lane] = (lane == 0 && all_finite) ? ((w.gram_dom || w.v0) ? s : dl) : 0.0;
  }
  if (lane == 0) {
    eb = fmaxf(eb, 0.f);  // also maps NaN to 0
    const double rn = sqrt(s);
    int fl = 0;
    if (!y) fl = idle;
    else if (!all_finite) fl = FLAG_DONE | OMP_SIG_NONFINITE;
    else if (rn <= (double)eb || Sb == 0) fl = FLAG_DONE;
    w.flags[b] = fl;
    w.k[b] = 0;
    w.Sb[b] = Sb;
    w.epsb[b] = eb;
  }
}

// One wavefront per (padded) signal.
__global__ __launch_bounds__(64) void k_init(const float *__restrict__ Y, int64_t ldy,
                                             const int32_t *__restrict__ S_per,
                                             const float *__restrict__ eps_per, float eps, int64_t M,
                                             WorkView w) {
  const int64_t b = blockIdx.x;
  const bool real = b < w.B;
  init_column(w, b, real ? Y + b * ldy : nullptr, M, real ? signal_S(S_per, b, w.S) : w.S,
              real ? signal_eps(eps_per, b, eps) : eps, FLAG_DONE, threadIdx.x);
}

// Slot scheduler set-up: slot i takes signal i while signals last; block 0
// also resets the queue (next signal to admit, signals finished).
__global__ __launch_bounds__(64) void k_init_slots(WorkView w, SlotView sv) {
  const int64_t b = blockIdx.x;
  const int lane = threadIdx.x;
  const bool real = b < sv.nsig;
  if (lane == 0) sv.sig[b] = real ? (int32_t)b : -1;
  if (b == 0 && lane == 0) {
    sv.ctrl[0] = (int32_t)min<int64_t>(sv.nsig, w.B);
    sv.ctrl[1] = 0;
  }
  init_column(w, b, real ? sv.Y + b * sv.ldy : nullptr, sv.M, real ? signal_S(sv.S_per, b, w.S) : w.S,
              real ? signal_eps(sv.eps_per, b, sv.eps) : sv.eps, FLAG_DONE | FLAG_EMPTY, lane);
}

// Slot scheduler: the signal in slot b has stopped (flags fl, k atoms, residual
// norm rn). Writes its support, coefficients, status and ||r|| (same stop
// reasons and order as the output kernel), then admits the next waiting
// signal into the slot, or marks the slot empty. One wavefront.
__device__ void retire_and_admit(const WorkView &w, const SlotView &sv, int64_t b, int fl, int k, double rn,
                                 int lane) {
  const int S = w.S;
  const int64_t sg = sv.sig[b];
  for (int j = lane; j < S; j += 64) {
    const bool in = j < k;
    sv.support_out[sg * S + j] = in ? w.sup[b * S + j] : -1;
    sv.coef_out[sg * S + j] = in ? w.xh[b * S + j] : 0.f;
  }
  int nxt = 0;
  if (lane == 0) {
    int st = fl & (OMP_SIG_NONFINITE | OMP_SIG_DEPENDENT | OMP_SIG_EXHAUSTED);
    if (st == 0) {
      if (rn <= (double)w.epsb[b]) st |= OMP_SIG_EPS;
      if (k >= w.Sb[b]) st |= OMP_SIG_SMAX;
    }
    st |= fl & (OMP_SIG_WIDENED | OMP_SIG_NEARTIE);
    if (sv.status_out) sv.status_out[sg] = (k << 8) | st;
    if (sv.rnorm_out) sv.rnorm_out[sg] = (float)rn;
    nxt = atomicAdd(sv.ctrl, 1);
    atomicAdd(sv.ctrl + 1, 1);
  }
  nxt = __shfl(nxt, 0);
  if (nxt < sv.nsig) {
    if (lane == 0) sv.sig[b] = nxt;
    init_column(w, b, sv.Y + (int64_t)nxt * sv.ldy, sv.M, signal_S(sv.S_per, nxt, S),
                signal_eps(sv.eps_per, nxt, sv.eps), FLAG_DONE | FLAG_EMPTY, lane);
  } else if (lane == 0) {
    sv.sig[b] = -1;
    w.flags[b] = FLAG_DONE | FLAG_EMPTY;
  }
}

// ---------------------------------------------------------------------------
// Solve step. One 64-lane wavefront per signal, up to SOLVE_WAVES signals per
// block, fewer when their LDS would not fit (the wavefronts share nothing;
// each has its own LDS region). RPL = rows of V per lane (S <= 64 RPL; RPL in
// {1, 2, 4}).
// LDS per wavefront: V (vstride floats), then in the BF16 form the candidate
// and possibly-open lists (a multiple of 4 ints, so every wavefront's region
// stays 16-byte aligned).
// Memory is read in two dependent rounds: first everything whose address
// depends on the signal only (state, norms, the epilogue's keys, support, u,
// x), then the packed factor together with what depends on the pick (Gram row,
// ||a_n*||^2, a_n*^T r; in the BF16 form fetched for every re-scored
// candidate alongside its exact score).
// The triangular solves run column by column; the reciprocal diagonal is
// computed up front in parallel and the next columns are read from LDS while
// the current ones are applied, so the sequential chain holds no division and
// no LDS latency.
// ---------------------------------------------------------------------------

// A stop found by the solve step: record the flags, or (slot scheduler) write
// the signal out and admit the next one.
template <bool SLOTS>
__device__ inline void stop_signal(const WorkView &w, const SlotView &sv, int64_t b, int fl, int k, double rn,
                                   int lane) {
  if (SLOTS) retire_and_admit(w, sv, b, fl, k, rn, lane);
  else if (lane == 0) w.flags[b] = fl;
}

// RPL: support rows per lane (S <= 64 RPL); BF16: the 16-bit forms' certified
// pick; SLOTS: the slot scheduler's retire and admit; RR: the residual is held
// in registers (512 < M <= 1024); RRF: that variant also forms the next residual
// (a variant of its own, so that the one that does not keeps its registers).
template <int RPL, bool BF16, bool SLOTS, bool RR, bool RRF = false>
__global__ __launch_bounds__(64 * SOLVE_WAVES) void k_solve(DictView d, WorkView w, SlotView sv) {
  extern __shared__ float smem[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t b = (int64_t)blockIdx.x * (blockDim.x >> 6) + wv;  // blocks of solve_waves(w) wavefronts
  if (b >= w.B) return;
  const int S = w.S;
  const int64_t VS = w.vstride;
  float *Vs = smem + (size_t)wv * (VS + solve_list_len(w));
  int *clist = reinterpret_cast<int *>(Vs + VS);  // BF16 pick: candidate list (one entry per key at most)

  // ---- memory round 1: state, residual norms, keys, support, u and (RR) the
  // residual (none of these addresses depends on another load)
  int fl = w.flags[b];
  const int k = __builtin_amdgcn_readfirstlane(w.k[b]);  // wave-uniform: scalar loop bounds
  const float eps_b = w.epsb[b];  // read here, with the rest of memory round 1
  const int S_b = w.Sb[b];
  const double pn = lane < NSLICE_MAX ? w.pnorm[b * NSLICE_MAX + lane] : 0.0;
  const double pd = (BF16 && lane < NSLICE_MAX) ? w.pdelta[b * NSLICE_MAX + lane] : 0.0;
  const double y2 = w.gram_dom ? w.pdelta[b * NSLICE_MAX] : 0.0;  // Gram-domain form: ||y||^2
  const double ks = (BF16 && w.fp16) ? (double)w.rscale[b] : 1.0;    // FP16 form: scale of the keys
  // Every stop found below leaves through the `stop` label with these set, so
  // that the stop's code (slot scheduler: the retire and admit) exists once.
  int stopfl = 0;
  double rn = 0.0;
  {
  int si[RPL];
  float uo[RPL], xo[RPL];
#pragma unroll
  for (int p = 0; p < RPL; ++p) {
    const int i = lane + 64 * p;
    si[p] = i < S ? w.sup[b * S + i] : 0;  // only entries below k are meaningful
    uo[p] = i < S ? w.u[b * S + i] : 0.f;
    xo[p] = i < S ? w.xh[b * S + i] : 0.f;
  }
  const int nkeys = w.ntile * w.ncand;
  // FP32 form: the largest valid 64-bit key (a valid key has a non-zero index
  // word). BF16 form: (score bits << 32) | 1 of the best valid 32-bit key.
  uint64_t kmax = 0;
  // RR (512 < M <= 1024, residual-vector forms): the residual is read in this
  // round too, so the pick's exact scores need only the atoms.
  const float4 *r4 = reinterpret_cast<const float4 *>(w.R32) + b * (d.Mp / 4);
  float4 rr[RREG];
#pragma unroll
  for (int q = 0; q < RREG; ++q) {
    if constexpr (RR) {
      const int64_t c = lane + 64 * q;
      const float4 v = r4[c < d.Mp / 4 ? c : 0];
      rr[q] = c < d.Mp / 4 ? v : make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
      rr[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  // BF16 form: up to 64 KREG keys stay in registers for the pick
  uint32_t kv[KREG];
  const bool kreg = BF16 && nkeys <= 64 * KREG;
  if (BF16) {
    const uint32_t *keys = reinterpret_cast<const uint32_t *>(w.part) + b * nkeys;
    if (kreg) {
#pragma unroll
      for (int j = 0; j < KREG; ++j) {
        const int t = 64 * j + lane;
        const uint32_t v = keys[t < nkeys ? t : 0];
        kv[j] = t < nkeys ? v : 0x80000000u;
        const uint64_t m = ((uint64_t)(kv[j] & ~31u) << 32) | 1ull;
        kmax = (key_valid(kv[j]) && m > kmax) ? m : kmax;
      }
    } else {
#pragma unroll
      for (int j = 0; j < KREG; ++j) kv[j] = 0x80000000u;
#pragma unroll 4
      for (int t = lane; t < nkeys; t += 64) {
        const uint32_t v = keys[t];
        const uint64_t m = ((uint64_t)(v & ~31u) << 32) | 1ull;
        kmax = (key_valid(v) && m > kmax) ? m : kmax;
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < KREG; ++j) kv[j] = 0x80000000u;
    const uint64_t *keys = w.part + b * nkeys;
#pragma unroll 4
    for (int t = lane; t < nkeys; t += 64) {
      const uint64_t v = keys[t];
      kmax = ((v & 0xFFFFFFFFull) && v > kmax) ? v : kmax;
    }
  }
  if (fl & FLAG_NEWX) {
    fl &= ~FLAG_NEWX;
    if (lane == 0) w.flags[b] = fl;
  }
  if (fl & FLAG_DONE) {  // the wavefront exits as a whole
    // slot scheduler: a signal that stopped at its last pick leaves now that
    // its final residual is known
    if (SLOTS && !(fl & FLAG_EMPTY)) {
      rn = sqrt(wave_sum(pn));
      stopfl = fl;
      goto stop;
    }
    return;
  }

  // 0. Stop test on the current residual (Algorithm 1 stops once ||r|| <= eps).
  rn = sqrt(wave_sum(pn));
  if (rn <= (double)eps_b) {
    stopfl = fl | FLAG_DONE;
    goto stop;
  }
  kmax = wave_max(kmax);
  if (kmax == 0ull) {  // nothing selectable is left
    stopfl = fl | FLAG_DONE | OMP_SIG_EXHAUSTED;
    goto stop;
  }
  if (!BF16 && w.flag_ties) {
    // Near-tie flagging (FP32 and Gram-domain forms): the keys hold every tile's
    // best and second best atom, so the largest key below kmax is the second
    // best atom overall; flag the step when its score is within 1e-5 of the best.
    const uint64_t *keys = w.part + b * nkeys;
    uint64_t k2 = 0;
    for (int t = lane; t < nkeys; t += 64) {
      const uint64_t v = keys[t];
      k2 = ((v & 0xFFFFFFFFull) && v < kmax && v > k2) ? v : k2;
    }
    k2 = wave_max(k2);
    const double s1 = (double)__uint_as_float((uint32_t)(kmax >> 32));
    const double s2 = (double)__uint_as_float((uint32_t)(k2 >> 32));
    if (k2 != 0ull && s2 >= (1.0 - TIE_REL) * s1) fl |= OMP_SIG_NEARTIE;
  }
#pragma unroll
  for (int p = 0; p < RPL; ++p)
    if (lane + 64 * p >= k) uo[p] = xo[p] = 0.f;

  // ---- memory round 2: the packed factor straight into LDS (asynchronous
  // global-to-LDS loads: no registers, no wait until it is read) ...
  if (w.refactor) {
    // ablation A3: the Gram block G[S, S] (packed lower triangle) instead of the
    // stored factor; it is factorised below
    const int nv = k * (k + 1) / 2;
    for (int t = lane; t < nv; t += 64) {
      int i = (int)((sqrtf(8.f * (float)t + 1.f) - 1.f) * 0.5f);
      while ((i + 1) * (i + 2) / 2 <= t) ++i;
      while (i * (i + 1) / 2 > t) --i;
      const int j = t - i * (i + 1) / 2;
      Vs[t] = d.G[(int64_t)w.sup[b * S + i] * d.Np + w.sup[b * S + j]];
    }
  } else {
    const int nv4 = (k * (k + 1) / 2 + 3) / 4;
    const float4 *V4 = reinterpret_cast<const float4 *>(w.V + b * VS);
    float4 *Vs4 = reinterpret_cast<float4 *>(Vs);
    for (int t0 = 0; t0 < nv4; t0 += 64)
      if (t0 + lane < nv4) lds_load16(V4 + t0 + lane, Vs4 + t0);
  }

  // ... and the pick: the best key over all atom tiles (largest score, then
  // lowest index), or in the BF16 form the certified exact re-score of the
  // candidates; cdot = a_n*^T r (exact products, FP64 sum). The Gram row of the
  // pick, g_i = G[n*, support_i] (lane holds rows i = lane + 64 p), and
  // ||a_n*||^2 are fetched in this same round in the FP32 form; in the BF16
  // form the row is read once the re-score has decided the pick.
  int nstar;
  int widened = 0;
  double cdot = 0.0, nu2 = 0.0;
  float g[RPL];
  if (BF16) {
    const double tau = bf16_tau(rn, sqrt(wave_sum(pd)), (double)d.aerr_max[0], d.Mp);
    int neartie = 0;
    nstar = select_bf16<RR>(d, w, b, __uint_as_float((uint32_t)(kmax >> 32)), ks, tau, lane, &widened, &cdot,
                            &nu2, clist, kv, kreg, rr, &neartie);
    // FP16 form: the next residual copy is scaled by ||r_k||, which bounds ||r_k+1||
    if (w.fp16 && lane == 0) w.rscale_next[b] = pow2_scale(rn);
    if (nstar < 0) {
      stopfl = fl | FLAG_DONE | OMP_SIG_EXHAUSTED;
      goto stop;
    }
    if (neartie) fl |= OMP_SIG_NEARTIE;
  } else {
    nstar = (int)(0xFFFFFFFFu - (uint32_t)(kmax & 0xFFFFFFFFull));
    nu2 = d.nu2[nstar];
#pragma unroll
    for (int p = 0; p < RPL; ++p) {
      const int i = lane + 64 * p;
      g[p] = (i < k && !w.gram_fly) ? d.G[(int64_t)nstar * d.Np + si[p]] : 0.f;
    }
    if (!w.gram_dom) {  // the Gram-domain form keeps no residual vectors
      const int na[1] = {nstar};
      double ar[1];
      if constexpr (RR)
        atom_dots_reg<1, 4>(d, na, rr, lane, ar);
      else
        atom_dots<1, 4>(d, na, r4, lane, ar);
      cdot = ar[0];
    }
  }
  if (w.gram_fly) {
    gram_row_from_atoms<RPL>(d, nstar, si, k, lane, g);
  } else if (BF16) {  // the pick's Gram row, now that the pick is known
#pragma unroll
    for (int p = 0; p < RPL; ++p) {
      const int i = lane + 64 * p;
      g[p] = i < k ? d.G[(int64_t)nstar * d.Np + si[p]] : 0.f;
    }
  }
  // beta = a_n*^T y = a_n*^T r + sum_j G[n*, s_j] x_j (r = y - A_{k-1} x_{k-1})
  double gx = 0.0;
#pragma unroll
  for (int p = 0; p < RPL; ++p) gx += (double)g[p] * (double)xo[p];
  double beta = cdot + wave_sum(gx);
  if (w.gram_dom) beta = (double)w.P[b * w.Np + nstar];  // the stored a_n*^T y
  if (widened) fl |= OMP_SIG_WIDENED;
  __builtin_amdgcn_s_waitcnt(0);  // the global-to-LDS loads have landed
  wave_lds_sync();
  if (w.refactor) cholesky_lds<RPL>(Vs, k, lane);

  float z[RPL], rd[RPL];
  int tri[RPL];  // i (i + 1) / 2: start of row i in the packed factor
#pragma unroll
  for (int p = 0; p < RPL; ++p) {
    const int i = lane + 64 * p;
    tri[p] = i * (i + 1) / 2;
    rd[p] = i < k ? 1.0f / Vs[tri[p] + i] : 0.f;  // reciprocal diagonal, all rows at once
    z[p] = 0.f;
  }

  // 4. Forward solve V_{k-1} z = g, column by column. Column j is applied as
  //    g_i -= (V_ij / V_jj) g_j on every lane: the column is read masked to the
  //    rows j < i < k (other lanes add zero) and scaled by the reciprocal
  //    diagonal while the previous block is applied, so a column costs one
  //    broadcast and one FMA on the critical path. Finally z_i = g_i / V_ii.
  //    Columns are handled four at a time, the loop rounded up to a whole
  //    block (columns j >= k are all zero).
  {
    constexpr int QB = 4;
    float va[QB][RPL], vx[QB][RPL];
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const float rj = readlane(pick(rd, q >> 6), q & 63);
#pragma unroll
      for (int p = 0; p < RPL; ++p) {
        const int i = lane + 64 * p;
        const bool in = i > q && i < k;
        const float v = Vs[in ? tri[p] + q : 0];
        va[q][p] = in ? v * rj : 0.f;
      }
    }
    for (int j0 = 0; j0 < k; j0 += QB) {
#pragma unroll
      for (int q = 0; q < QB; ++q)
#pragma unroll
        for (int p = 0; p < RPL; ++p) {
          const int i = lane + 64 * p, j = j0 + QB + q;
          const bool in = i > j && i < k;
          vx[q][p] = Vs[in ? tri[p] + j : 0];
        }
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        const int j = j0 + q;
        const float gj = readlane(pick(g, j >> 6), j & 63);
#pragma unroll
        for (int p = 0; p < RPL; ++p) g[p] = fmaf(-va[q][p], gj, g[p]);
      }
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        const int j = j0 + QB + q;
        const int jc = j < 64 * RPL ? j : 0;
        const float rj = readlane(pick(rd, jc >> 6), jc & 63);
#pragma unroll
        for (int p = 0; p < RPL; ++p) {
          const int i = lane + 64 * p;
          va[q][p] = (i > j && i < k) ? vx[q][p] * rj : 0.f;
        }
      }
    }
#pragma unroll
    for (int p = 0; p < RPL; ++p) z[p] = g[p] * rd[p];  // rd is 0 on rows >= k
  }

  // 5. Pivot d^2 = ||a_n*||^2 - ||z||^2 in FP64.
  double zz = 0.0;
#pragma unroll
  for (int p = 0; p < RPL; ++p) zz += (double)z[p] * (double)z[p];
  zz = wave_sum(zz);
  const double d2 = nu2 - zz;
  if (!(d2 > DEP_TOL2 * nu2)) {  // dependent atom: stop without appending
    stopfl = fl | FLAG_DONE | OMP_SIG_DEPENDENT;
    goto stop;
  }
  const float dk = (float)sqrt(d2);

  // 6. u_k = (beta - z^T u_{k-1}) / d, beta = a_n*^T y (Eq. 2).
  double zu = 0.0;
#pragma unroll
  for (int p = 0; p < RPL; ++p) zu += (double)z[p] * (double)uo[p];
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
    if (i == k) rd[p] = 1.0f / dk;
  }
  if (lane == 0) {
    Vs[rk + k] = dk;
    w.V[b * VS + rk + k] = dk;
    w.sup[b * S + k] = nstar;
    w.u[b * S + k] = uk;
    const int64_t mwords = d.Np / 32;
    // no returned value: the wavefront does not wait for this update
    __hip_atomic_fetch_or(&w.mask[b * mwords + nstar / 32], 1u << (nstar & 31), __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_AGENT);
  }
  wave_lds_sync();
  const int K = k + 1;

  // 8. Back solve V_K^T x = u, last unknown first. Row j is applied as
  //    t_i -= (V_ji / V_jj) t_j on every lane (the row is read masked to
  //    i < j and scaled while the previous block is applied); finally
  //    x_i = t_i / V_ii. Rows are handled four at a time from the top of the
  //    block holding row K-1 (rows j >= K are all zero).
  float t[RPL], x[RPL];
#pragma unroll
  for (int p = 0; p < RPL; ++p) {
    const int i = lane + 64 * p;
    t[p] = i < k ? uo[p] : (i == k ? uk : 0.f);
  }
  {
    constexpr int QB = 4;
    const int jt = ((K + QB - 1) / QB) * QB - 1;  // top row of the first block
    float va[QB][RPL], vx[QB][RPL];
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int j = jt - q;
      const bool row = j < K;
      const float rj = readlane(pick(rd, j >> 6), j & 63);
#pragma unroll
      for (int p = 0; p < RPL; ++p) {
        const int i = lane + 64 * p;
        const bool in = row && i < j;
        const float v = Vs[in ? j * (j + 1) / 2 + i : 0];
        va[q][p] = in ? v * rj : 0.f;
      }
    }
    for (int j0 = jt; j0 >= 0; j0 -= QB) {
#pragma unroll
      for (int q = 0; q < QB; ++q)
#pragma unroll
        for (int p = 0; p < RPL; ++p) {
          const int i = lane + 64 * p, j = j0 - QB - q;
          const bool in = j >= 0 && i < j;
          vx[q][p] = Vs[in ? j * (j + 1) / 2 + i : 0];
        }
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        const int j = j0 - q;
        const float tj = readlane(pick(t, j >> 6), j & 63);
#pragma unroll
        for (int p = 0; p < RPL; ++p) t[p] = fmaf(-va[q][p], tj, t[p]);
      }
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        const int j = j0 - QB - q;
        const int jc = j >= 0 ? j : 0;
        const float rj = readlane(pick(rd, jc >> 6), jc & 63);
#pragma unroll
        for (int p = 0; p < RPL; ++p) {
          const int i = lane + 64 * p;
          va[q][p] = (j >= 0 && i < j) ? vx[q][p] * rj : 0.f;
        }
      }
    }
  }
#pragma unroll
  for (int p = 0; p < RPL; ++p) {
    x[p] = t[p] * rd[p];  // rd is 0 on rows >= K
    const int i = lane + 64 * p;
    if (i < K) w.xh[b * S + i] = x[p];
  }

  if ((!RR || RRF) && w.fuse_res) {
    // Residual fused into the solve (dictionaries of at most 4 MiB in FP32): this
    // wavefront forms r = y - A_K x for its own signal as the residual kernel
    // does (the same FMA order per element), its 16-bit copy, ||r||^2 and, in
    // the 16-bit forms, the copy's error norm, and stores the norms in slice 0
    // (the other slices' entries stay at the zero the set-up wrote).
    const int64_t nc4 = d.Mp / 4;
    const float4 *A4 = reinterpret_cast<const float4 *>(d.A32);
    const float4 *Y4 = reinterpret_cast<const float4 *>(w.Yp) + b * nc4;
    float4 *R4 = reinterpret_cast<float4 *>(w.R32) + b * nc4;
    // FP16 form: the copy is fp16(sigma r) with the scale chosen from ||r_k|| above
    const float sig = (BF16 && w.fp16) ? pow2_scale(rn) : 1.f;
    double nrm = 0.0, dlt = 0.0;
    for (int64_t c = lane; c < nc4; c += 64) {
      float4 r = Y4[c];
      // rounds of four atoms, their loads issued together; the sums run in
      // support order (lanes past nc4 are inactive in the last pass: lane_elem,
      // not pick)
      for (int j0 = 0; j0 < K; j0 += 4) {
        float4 a[4];
        float xj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = j0 + u < K ? j0 + u : K - 1;  // past K: a repeated load, not summed
          const int sj = j < k ? lane_elem(si, j) : nstar;
          xj[u] = -lane_elem(x, j);
          a[u] = A4[(int64_t)sj * nc4 + c];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (j0 + u < K) {
            r.x = fmaf(xj[u], a[u].x, r.x); r.y = fmaf(xj[u], a[u].y, r.y);
            r.z = fmaf(xj[u], a[u].z, r.z); r.w = fmaf(xj[u], a[u].w, r.w);
          }
      }
      R4[c] = r;
      if (BF16 && w.fp16) {
        ushort4 h;
        h.x = f32_to_f16_rne(r.x * sig);
        h.y = f32_to_f16_rne(r.y * sig);
        h.z = f32_to_f16_rne(r.z * sig);
        h.w = f32_to_f16_rne(r.w * sig);
        reinterpret_cast<ushort4 *>(w.R16)[b * nc4 + c] = h;
        const double e0 = (double)r.x - f16_used(h.x) / (double)sig;
        const double e1 = (double)r.y - f16_used(h.y) / (double)sig;
        const double e2 = (double)r.z - f16_used(h.z) / (double)sig;
        const double e3 = (double)r.w - f16_used(h.w) / (double)sig;
        dlt += e0 * e0 + e1 * e1 + e2 * e2 + e3 * e3;
      } else if (BF16) {
        ushort4 h;
        h.x = f32_to_bf16_rne(r.x);
        h.y = f32_to_bf16_rne(r.y);
        h.z = f32_to_bf16_rne(r.z);
        h.w = f32_to_bf16_rne(r.w);
        reinterpret_cast<ushort4 *>(w.R16)[b * nc4 + c] = h;
        const double e0 = (double)r.x - bf16_used(h.x);
        const double e1 = (double)r.y - bf16_used(h.y);
        const double e2 = (double)r.z - bf16_used(h.z);
        const double e3 = (double)r.w - bf16_used(h.w);
        dlt += e0 * e0 + e1 * e1 + e2 * e2 + e3 * e3;
      }
      nrm += (double)r.x * r.x + (double)r.y * r.y + (double)r.z * r.z + (double)r.w * r.w;
    }
    nrm = wave_sum(nrm);
    if (BF16) dlt = wave_sum(dlt);
    if (lane == 0) {
      w.pnorm[b * NSLICE_MAX] = nrm;  // entries 1 .. NSLICE_MAX-1 stay 0
      if (BF16) w.pdelta[b * NSLICE_MAX] = dlt;
      if (BF16 && w.fp16) w.rscale[b] = sig;
    }
  }

  if (w.gram_dom) {
    // Gram-domain form (no residual vectors): ||r_K||^2 = ||r_k||^2 - u_K^2, u_K
    // being y's component along the new orthonormal direction, kept in FP64
    // where the residual kernel would have left the slice norms. That running
    // value carries the rounding of the FP32 quantities it is built from, about
    // K u ||y||^2; once it falls to that level, or to within it of eps_b^2 (where
    // it would decide the stop), ||y - A_S x||^2 is formed explicitly instead:
    // exact FP64 products of the FP32 atoms and coefficients, FP64 sums.
    const double ud = (beta - zu) / (double)dk;
    double r2 = rn * rn - ud * ud;
    const double floor2 = 64.0 * (double)(K + 1) * (1.0 / 16777216.0) * y2;
    const double e2 = (double)eps_b * (double)eps_b;
    if (!(r2 > floor2) || fabs(r2 - e2) <= floor2) {
      const float *yb = w.Yp + b * w.Mp;
      double acc = 0.0;
      for (int64_t m = lane; m < d.M; m += 64) {
        double rm = (double)yb[m];
        for (int j = 0; j < K; ++j) {
          // (lanes past M are inactive in the last pass: lane_elem, not pick)
          const int sj = j < k ? lane_elem(si, j) : nstar;
          const float xj = lane_elem(x, j);
          rm -= (double)xj * (double)d.A32[(int64_t)sj * d.Mp + m];
        }
        acc += rm * rm;
      }
      r2 = wave_sum(acc);
    }
    if (lane == 0) w.pnorm[b * NSLICE_MAX] = r2;
  }

  // 9. New state; the residual kernel picks the signal up through FLAG_NEWX
  //    (it is not launched when the residual is fused above).
  if (lane == 0) {
    fl |= FLAG_NEWX;
    if (K >= S_b) fl |= FLAG_DONE;
    w.k[b] = K;
    w.flags[b] = fl;
  }
  }
  return;
stop:
  // A stop after the factor's global-to-LDS loads were issued (no selectable
  // atom left) must not leave them writing this block's LDS after it ends.
  __builtin_amdgcn_s_waitcnt(0);
  stop_signal<SLOTS>(w, sv, b, stopfl, k, rn, lane);
}

// ---------------------------------------------------------------------------
// Gram-domain select (tall dictionaries; the Gram solver of Section 2.1): the
// correlations of the current residual are c_n = P[b][n] - sum_j G[s_j][n] x_j
// (P = A^T y once per signal; G is symmetric, so row s_j of G is its column),
// scored |c_n| / ||a_n|| over the atoms not yet selected, each slice's best
// atom carried by its key (the FP32 correlation epilogue's key format) in
// w.part[b][slice]. One wavefront per (signal, atom slice); workgroup i runs
// on XCD i mod 8 and takes slice i mod GSLICE, so an XCD reads only its
// 1/GSLICE of the columns of G (L2-resident), in runs of 64 consecutive atoms.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_gram_select(DictView d, WorkView w) {
  __shared__ int ss[OMP_MAX_S];
  __shared__ float xs[OMP_MAX_S];
  const int64_t b = blockIdx.x / GSLICE;
  const int x = blockIdx.x % GSLICE;
  const int lane = threadIdx.x;
  if (w.flags[b] & FLAG_DONE) return;  // the whole wavefront leaves
  const int k = __builtin_amdgcn_readfirstlane(w.k[b]);
  const int S = w.S;
  for (int j = lane; j < k; j += 64) {
    ss[j] = w.sup[b * S + j];
    xs[j] = w.xh[b * S + j];
  }
  __syncthreads();
  const int64_t Np = d.Np, len = Np / GSLICE;
  const float *Pb = w.P + b * Np;
  const uint32_t *mk = w.mask + b * (Np / 32);
  // NA atoms per lane at a time and JR support rows per round, so that JR NA
  // independent loads are in flight before their FMAs (c_n accumulates in
  // support order). Addresses past the slice are clamped to its last atom and
  // their results dropped.
  constexpr int NA = 4, JR = 8;
  const int64_t end = (x + 1) * len;
  const bool ties = w.ncand == 2;  // near-tie flagging: the slice's second best key too
  uint64_t kbest = 0, ksec = 0;
  for (int64_t n0 = x * len + lane; n0 < end; n0 += 64 * NA) {
    int64_t nn[NA];
    float c[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      const int64_t n = n0 + 64 * a;
      nn[a] = n < end ? n : end - 1;
      c[a] = Pb[nn[a]];
    }
    int j = 0;
    for (; j + JR <= k; j += JR) {
      float v[JR][NA];
#pragma unroll
      for (int q = 0; q < JR; ++q) {
        const float *g = d.G + (int64_t)ss[j + q] * Np;
#pragma unroll
        for (int a = 0; a < NA; ++a) v[q][a] = g[nn[a]];
      }
#pragma unroll
      for (int q = 0; q < JR; ++q)
#pragma unroll
        for (int a = 0; a < NA; ++a) c[a] = fmaf(-v[q][a], xs[j + q], c[a]);
    }
    for (; j < k; ++j) {
      const float *g0 = d.G + (int64_t)ss[j] * Np;
#pragma unroll
      for (int a = 0; a < NA; ++a) c[a] = fmaf(-g0[nn[a]], xs[j], c[a]);
    }
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      const int64_t n = n0 + 64 * a;
      if (n >= end) continue;
      const float iv = d.inv_nu[n];
      const bool taken = (mk[n >> 5] >> (n & 31)) & 1u;
      if (iv > 0.f && !taken) {
        const uint64_t key = ((uint64_t)__float_as_uint(fabsf(c[a]) * iv) << 32) | (0xFFFFFFFFull - (uint64_t)n);
        ksec = max(ksec, min(kbest, key));
        kbest = key > kbest ? key : kbest;
      }
    }
  }
  if (ties) {
    // the slice's second best: the best key below the slice's best (keys are distinct)
    const uint64_t top = wave_max(kbest);
    ksec = wave_max(kbest == top ? ksec : kbest);
    if (lane == 0) {
      w.part[(b * GSLICE + x) * 2] = top;
      w.part[(b * GSLICE + x) * 2 + 1] = ksec;
    }
    return;
  }
  kbest = wave_max(kbest);
  if (lane == 0) w.part[b * GSLICE + x] = kbest;  // ntile = GSLICE keys per signal in this form
}

// ---------------------------------------------------------------------------
// Algorithm v0 of the paper (Section 2.3): the inverse Cholesky factor
// F_k = V_k^{-T} (upper triangular) and D_k = A^T A_k F_k = A^T Q_k, Q_k = A_k F_k
// having orthonormal columns. No correlation product and no residual vectors:
// every step works on N-long rows of one signal.
//   c_0 = A^T y (the projection product, stored in w.P), n* = argmax |c| / ||a||
//   z   = D_{k-1}[n*, :]                 (a_n*^T q_j, j < k)
//   g   = 1 / sqrt(||a_n*||^2 - ||z||^2)   (FP64 pivot)
//   d_k = g (G[:, n*] - D_{k-1} z)        (new column of D: A^T q_k)
//   u_k = g c_{k-1}[n*]                   (q_k^T y)
//   c_k = c_{k-1} - u_k d_k               (A^T r_k)
//   F_k = [[F_{k-1}, -g F_{k-1} z], [0, g]]
//   ||r_k||^2 = ||r_{k-1}||^2 - u_k^2, and at the end x = F_S u.
// The signal's next pick is found while c_k is written (one key per signal in
// w.part), so a step reads c once. One workgroup of V0_THREADS per signal;
// D is [Bp][S][Np] (column j of D_k contiguous), F packed by columns in w.V.
// ---------------------------------------------------------------------------
constexpr int V0_THREADS = 256;

// Block-wide maximum of a 64-bit key (every thread gets it). red: LDS [V0_THREADS / 64].
__device__ inline uint64_t block_max(uint64_t v, uint64_t *red) {
  v = wave_max(v);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[wv] = v;
  __syncthreads();
  uint64_t m = red[0];
#pragma unroll
  for (int i = 1; i < V0_THREADS / 64; ++i) m = red[i] > m ? red[i] : m;
  __syncthreads();
  return m;
}

// Key of atom n with correlation c (0: not a candidate), as the FP32 select writes it.
__device__ inline uint64_t v0_key(float c, float iv, bool taken, int64_t n) {
  return (iv > 0.f && !taken) ? ((uint64_t)__float_as_uint(fabsf(c) * iv) << 32) | (0xFFFFFFFFull - (uint64_t)n)
                              : 0ull;
}

// The block's best and second best keys (threads hold their own best and second),
// stored as the signal's two keys for the next step.
__device__ inline void v0_store_pick(const WorkView &w, int64_t b, uint64_t best, uint64_t sec, uint64_t *red) {
  const uint64_t top = block_max(best, red);
  const uint64_t second = block_max(best == top ? sec : best, red);
  if (threadIdx.x == 0) {
    w.part[2 * b] = top;
    w.part[2 * b + 1] = second;
  }
}

// First pick of every signal from c_0 = P (one workgroup per signal).
__global__ __launch_bounds__(V0_THREADS) void k_v0_first(DictView d, WorkView w) {
  __shared__ uint64_t red[V0_THREADS / 64];
  const int64_t b = blockIdx.x;
  const float *c = w.P + b * d.Np;
  uint64_t best = 0, sec = 0;
  for (int64_t n = threadIdx.x; n < d.Np; n += V0_THREADS) {
    const uint64_t key = v0_key(c[n], d.inv_nu[n], false, n);
    sec = max(sec, min(best, key));
    best = key > best ? key : best;
  }
  v0_store_pick(w, b, best, sec, red);
}

// One v0 step for every live signal.
__global__ __launch_bounds__(V0_THREADS) void k_v0_step(DictView d, WorkView w) {
  extern __shared__ uint32_t v0s[];
  __shared__ uint64_t red[V0_THREADS / 64];
  __shared__ double zzs;
  const int64_t b = blockIdx.x;
  const int tid = threadIdx.x;
  int fl = w.flags[b];
  if (fl & FLAG_DONE) return;  // the whole block leaves
  const int k = w.k[b];
  const int S = w.S;
  const int64_t Np = d.Np, mwords = Np / 32;
  float *zs = reinterpret_cast<float *>(v0s);                 // [S]
  uint32_t *mk = v0s + S;                                     // [Np / 32] selected-atom mask
  const double rn = sqrt(w.pnorm[b * NSLICE_MAX]);
  const float eps_b = w.epsb[b];
  const uint64_t key = w.part[2 * b], key2 = w.part[2 * b + 1];
  // stop test on the current residual, then the pick found by the previous step
  if (rn <= (double)eps_b || key == 0ull) {
    if (tid == 0) w.flags[b] = fl | FLAG_DONE | (rn <= (double)eps_b ? 0 : OMP_SIG_EXHAUSTED);
    return;
  }
  const int nstar = (int)(0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull));
  if (w.flag_ties && key2 != 0ull &&
      (double)__uint_as_float((uint32_t)(key2 >> 32)) >= (1.0 - TIE_REL) * (double)__uint_as_float((uint32_t)(key >> 32)))
    fl |= OMP_SIG_NEARTIE;
  float *Db = w.D + b * (int64_t)S * Np;
  float *c = w.P + b * Np;
  for (int j = tid; j < k; j += V0_THREADS) zs[j] = Db[(int64_t)j * Np + nstar];
  for (int64_t t = tid; t < mwords; t += V0_THREADS) mk[t] = w.mask[b * mwords + t];
  if (tid < 64) {
    double zz = 0.0;
    for (int j = tid; j < k; j += 64) {
      const double z = (double)Db[(int64_t)j * Np + nstar];
      zz += z * z;
    }
    zz = wave_sum(zz);
    if (tid == 0) zzs = zz;
  }
  __syncthreads();
  const double nu2 = d.nu2[nstar];
  const double d2 = nu2 - zzs;
  if (!(d2 > DEP_TOL2 * nu2)) {  // dependent atom: stop without appending
    if (tid == 0) w.flags[b] = fl | FLAG_DONE | OMP_SIG_DEPENDENT;
    return;
  }
  const double gd = 1.0 / sqrt(d2);
  const float g = (float)gd;
  const float uk = (float)(gd * (double)c[nstar]);
  // new column of F: f_i = -g sum_{j=i}^{k-1} F[i][j] z_j (i < k), f_k = g
  const float *Fb = w.V + b * w.vstride;
  float *Fk = w.V + b * w.vstride + (int64_t)k * (k + 1) / 2;
  for (int i = tid; i <= k; i += V0_THREADS) {
    if (i == k) {
      Fk[k] = g;
    } else {
      double acc = 0.0;
      for (int j = i; j < k; ++j) acc += (double)Fb[(int64_t)j * (j + 1) / 2 + i] * (double)zs[j];
      Fk[i] = (float)(-gd * acc);
    }
  }
  // d_k = g (G[n*, :] - D_{k-1} z), c_k = c_{k-1} - u_k d_k, and the next pick
  const float4 *G4 = reinterpret_cast<const float4 *>(d.G + (int64_t)nstar * Np);
  const float4 *D4 = reinterpret_cast<const float4 *>(Db);
  float4 *Dk4 = reinterpret_cast<float4 *>(Db + (int64_t)k * Np);
  float4 *c4 = reinterpret_cast<float4 *>(c);
  const int64_t n4 = Np / 4;
  uint64_t best = 0, sec = 0;
  for (int64_t t = tid; t < n4; t += V0_THREADS) {
    float4 a = G4[t];
    int j = 0;
    for (; j + 4 <= k; j += 4) {
      const float4 e0 = D4[(int64_t)j * n4 + t], e1 = D4[(int64_t)(j + 1) * n4 + t];
      const float4 e2 = D4[(int64_t)(j + 2) * n4 + t], e3 = D4[(int64_t)(j + 3) * n4 + t];
      const float z0 = zs[j], z1 = zs[j + 1], z2 = zs[j + 2], z3 = zs[j + 3];
      a.x = fmaf(-z0, e0.x, a.x); a.y = fmaf(-z0, e0.y, a.y); a.z = fmaf(-z0, e0.z, a.z); a.w = fmaf(-z0, e0.w, a.w);
      a.x = fmaf(-z1, e1.x, a.x); a.y = fmaf(-z1, e1.y, a.y); a.z = fmaf(-z1, e1.z, a.z); a.w = fmaf(-z1, e1.w, a.w);
      a.x = fmaf(-z2, e2.x, a.x); a.y = fmaf(-z2, e2.y, a.y); a.z = fmaf(-z2, e2.z, a.z); a.w = fmaf(-z2, e2.w, a.w);
      a.x = fmaf(-z3, e3.x, a.x); a.y = fmaf(-z3, e3.y, a.y); a.z = fmaf(-z3, e3.z, a.z); a.w = fmaf(-z3, e3.w, a.w);
    }
    for (; j < k; ++j) {
      const float4 e = D4[(int64_t)j * n4 + t];
      const float z = zs[j];
      a.x = fmaf(-z, e.x, a.x); a.y = fmaf(-z, e.y, a.y); a.z = fmaf(-z, e.z, a.z); a.w = fmaf(-z, e.w, a.w);
    }
    a.x *= g; a.y *= g; a.z *= g; a.w *= g;
    Dk4[t] = a;
    float4 cv = c4[t];
    const float dv[4] = {a.x, a.y, a.z, a.w};
    float cc[4] = {cv.x, cv.y, cv.z, cv.w};
    const float4 iv4 = reinterpret_cast<const float4 *>(d.inv_nu)[t];
    const float iv[4] = {iv4.x, iv4.y, iv4.z, iv4.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t n = 4 * t + e;
      const bool taken = n == nstar || ((mk[n >> 5] >> (n & 31)) & 1u);
      cc[e] = taken ? 0.f : fmaf(-uk, dv[e], cc[e]);
      const uint64_t kk = v0_key(cc[e], iv[e], taken, n);
      sec = max(sec, min(best, kk));
      best = kk > best ? kk : best;
    }
    c4[t] = make_float4(cc[0], cc[1], cc[2], cc[3]);
  }
  v0_store_pick(w, b, best, sec, red);
  const int K = k + 1;
  // ||r_K||^2 = ||r_k||^2 - u_K^2 (FP64 running value); at its own rounding level,
  // or within it of eps_b^2, formed explicitly from y - A_S x, x = F_K u.
  double r2 = rn * rn - (double)uk * (double)uk;
  const double y2 = w.pdelta[b * NSLICE_MAX];
  const double floor2 = 64.0 * (double)(K + 1) * (1.0 / 16777216.0) * y2;
  const double e2 = (double)eps_b * (double)eps_b;
  if (!(r2 > floor2) || fabs(r2 - e2) <= floor2) {
    // x_i = sum_{j=i}^{K-1} F[i][j] u_j into LDS (zs reused), then r over m
    __syncthreads();
    const float *Fu = w.V + b * w.vstride;
    for (int i = tid; i < K; i += V0_THREADS) {
      double acc = 0.0;
      for (int j = i; j < K; ++j)
        acc += (double)Fu[(int64_t)j * (j + 1) / 2 + i] * (double)(j == k ? uk : w.u[b * S + j]);
      zs[i] = (float)acc;
    }
    __syncthreads();
    const float *yb = w.Yp + b * w.Mp;
    double acc = 0.0;
    for (int64_t m = tid; m < d.M; m += V0_THREADS) {
      double rm = (double)yb[m];
      for (int j = 0; j < K; ++j) {
        const int sj = j == k ? nstar : w.sup[b * S + j];
        rm -= (double)zs[j] * (double)d.A32[(int64_t)sj * d.Mp + m];
      }
      acc += rm * rm;
    }
    acc = wave_sum(acc);
    __shared__ double part4[V0_THREADS / 64];
    if ((tid & 63) == 0) part4[tid >> 6] = acc;
    __syncthreads();
    r2 = 0.0;
#pragma unroll
    for (int i = 0; i < V0_THREADS / 64; ++i) r2 += part4[i];
  }
  if (tid == 0) {
    w.pnorm[b * NSLICE_MAX] = r2;
    w.sup[b * S + k] = nstar;
    w.u[b * S + k] = uk;
    w.mask[b * mwords + nstar / 32] = mk[nstar / 32] | (1u << (nstar & 31));
    w.k[b] = K;
    w.flags[b] = fl | (K >= w.Sb[b] ? FLAG_DONE : 0);
  }
}

// Coefficients x = F_k u of every signal (one wavefront per signal), into w.xh.
__global__ __launch_bounds__(64) void k_v0_coef(WorkView w) {
  const int64_t b = blockIdx.x;
  const int k = w.k[b];
  const int S = w.S;
  const float *F = w.V + b * w.vstride;
  for (int i = threadIdx.x; i < k; i += 64) {
    double acc = 0.0;
    for (int j = i; j < k; ++j) acc += (double)F[(int64_t)j * (j + 1) / 2 + i] * (double)w.u[b * S + j];
    w.xh[b * S + i] = (float)acc;
  }
}

// ---------------------------------------------------------------------------
// FP64 form (OMP_PREC_FP64): Algorithm v0 of Section 2.3 with every quantity in
// FP64 -- the projection P = A^T y and the Gram matrix (exact products of the FP32
// inputs, FP64 sums), the correlations c, the columns of D, the inverse factor F,
// u and x. The paper notes that double precision halves the speed of its v0 code;
// this form is the library's accurate mode (picks decided by FP64 scores, no FP32
// cancellation in the solves).
// ---------------------------------------------------------------------------

// C[r][c] = sum_m X[r][m] Z[c][m] in FP64 from FP32 operands (rows of X and Z are Mp
// floats, Mp a multiple of 32); 64 x 64 tiles, 256 threads, 4 x 4 outputs each.
constexpr int G64_T = 64, G64_K = 32;
__global__ __launch_bounds__(256) void k_gemm64(const float *__restrict__ X, const float *__restrict__ Z, int64_t Mp,
                                                int ntc, double *__restrict__ C, int64_t ldc) {
  __shared__ double Xs[G64_K][G64_T + 1];
  __shared__ double Zs[G64_K][G64_T + 1];
  const int tr = blockIdx.x / ntc, tc = blockIdx.x % ntc;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const float *Xb = X + (int64_t)tr * G64_T * Mp;
  const float *Zb = Z + (int64_t)tc * G64_T * Mp;
  double acc[4][4] = {};
  for (int64_t k0 = 0; k0 < Mp; k0 += G64_K) {
    // 64 rows x 32 floats per operand: 512 float4, two per thread
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int f = tid + 256 * q;
      const int r = f >> 3, c4 = f & 7;
      const float4 xv = *reinterpret_cast<const float4 *>(Xb + (int64_t)r * Mp + k0 + 4 * c4);
      const float4 zv = *reinterpret_cast<const float4 *>(Zb + (int64_t)r * Mp + k0 + 4 * c4);
      Xs[4 * c4 + 0][r] = xv.x; Xs[4 * c4 + 1][r] = xv.y; Xs[4 * c4 + 2][r] = xv.z; Xs[4 * c4 + 3][r] = xv.w;
      Zs[4 * c4 + 0][r] = zv.x; Zs[4 * c4 + 1][r] = zv.y; Zs[4 * c4 + 2][r] = zv.z; Zs[4 * c4 + 3][r] = zv.w;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < G64_K; ++k) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = Xs[k][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Zs[k][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      C[((int64_t)tr * G64_T + ty * 4 + i) * ldc + (int64_t)tc * G64_T + tx * 4 + j] = acc[i][j];
}

// A candidate atom in FP64: score |c_n| / ||a_n|| (negative: none) and its index;
// the larger score wins, ties to the lower index.
struct Pick64 {
  double s;
  int n;
};
__device__ inline bool pick_better(double s, int n, double bs, int bn) { return s > bs || (s == bs && n < bn); }

// Merge the top two (b1 > b2) of another set of distinct atoms into (a1 > a2).
__device__ inline void pick_merge(Pick64 &a1, Pick64 &a2, const Pick64 &b1, const Pick64 &b2) {
  if (pick_better(b1.s, b1.n, a1.s, a1.n)) {
    a2 = pick_better(a1.s, a1.n, b2.s, b2.n) ? a1 : b2;
    a1 = b1;
  } else if (pick_better(b1.s, b1.n, a2.s, a2.n)) {
    a2 = b1;
  }
}

// Block-wide best and second best of the threads' (best, second) pairs, stored as the
// signal's two (score, index) pairs of doubles in w.part. red: LDS [2 V0_THREADS / 64].
__device__ inline void v0_store_pick64(const WorkView &w, int64_t b, Pick64 p1, Pick64 p2, Pick64 *red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const Pick64 q1{__shfl_xor(p1.s, off), __shfl_xor(p1.n, off)};
    const Pick64 q2{__shfl_xor(p2.s, off), __shfl_xor(p2.n, off)};
    pick_merge(p1, p2, q1, q2);
  }
  const int tid = threadIdx.x;
  if ((tid & 63) == 0) {
    red[2 * (tid >> 6)] = p1;
    red[2 * (tid >> 6) + 1] = p2;
  }
  __syncthreads();
  if (tid == 0) {
    Pick64 b1 = red[0], b2 = red[1];
    for (int i = 1; i < V0_THREADS / 64; ++i) pick_merge(b1, b2, red[2 * i], red[2 * i + 1]);
    double *pk = reinterpret_cast<double *>(w.part) + 4 * b;
    pk[0] = b1.s;
    pk[1] = (double)b1.n;
    pk[2] = b2.s;
    pk[3] = (double)b2.n;
  }
  __syncthreads();
}

__device__ inline void pick_insert(double s, int n, Pick64 &p1, Pick64 &p2) {
  if (pick_better(s, n, p1.s, p1.n)) {
    p2 = p1;
    p1 = Pick64{s, n};
  } else if (pick_better(s, n, p2.s, p2.n)) {
    p2 = Pick64{s, n};
  }
}

__global__ __launch_bounds__(V0_THREADS) void k_v0_first64(DictView d, WorkView w) {
  __shared__ Pick64 red[2 * V0_THREADS / 64];
  const int64_t b = blockIdx.x;
  const double *c = w.P64 + b * d.Np;
  Pick64 p1{-1.0, 0x7fffffff}, p2{-1.0, 0x7fffffff};
  for (int64_t n = threadIdx.x; n < d.Np; n += V0_THREADS) {
    const double iv = d.inv_nu64[n];
    if (iv > 0.0) pick_insert(fabs(c[n]) * iv, (int)n, p1, p2);
  }
  v0_store_pick64(w, b, p1, p2, red);
}

// One FP64 v0 step per live signal (the FP32 step's arithmetic in FP64).
__global__ __launch_bounds__(V0_THREADS) void k_v0_step64(DictView d, WorkView w) {
  extern __shared__ uint32_t v0s[];
  __shared__ Pick64 red[2 * V0_THREADS / 64];
  __shared__ double part4[V0_THREADS / 64];
  const int64_t b = blockIdx.x;
  const int tid = threadIdx.x;
  int fl = w.flags[b];
  if (fl & FLAG_DONE) return;
  const int k = w.k[b];
  const int S = w.S;
  const int64_t Np = d.Np, mwords = Np / 32;
  double *zs = reinterpret_cast<double *>(v0s);              // [S]
  uint32_t *mk = v0s + 2 * S;                                 // [Np / 32]
  const double rn = sqrt(w.pnorm[b * NSLICE_MAX]);
  const float eps_b = w.epsb[b];
  const double *pk = reinterpret_cast<const double *>(w.part) + 4 * b;
  const double s1 = pk[0], s2 = pk[2];
  if (rn <= (double)eps_b || !(s1 >= 0.0)) {
    if (tid == 0) w.flags[b] = fl | FLAG_DONE | (rn <= (double)eps_b ? 0 : OMP_SIG_EXHAUSTED);
    return;
  }
  const int nstar = (int)pk[1];
  if (w.flag_ties && s2 >= 0.0 && s2 >= (1.0 - TIE_REL) * s1) fl |= OMP_SIG_NEARTIE;
  double *Db = w.D64 + b * (int64_t)S * Np;
  double *c = w.P64 + b * Np;
  for (int j = tid; j < k; j += V0_THREADS) zs[j] = Db[(int64_t)j * Np + nstar];
  for (int64_t t = tid; t < mwords; t += V0_THREADS) mk[t] = w.mask[b * mwords + t];
  __syncthreads();
  if (tid < 64) {
    double zz = 0.0;
    for (int j = tid; j < k; j += 64) zz += zs[j] * zs[j];
    zz = wave_sum(zz);
    if (tid == 0) part4[0] = zz;
  }
  __syncthreads();
  const double nu2 = d.nu2[nstar];
  const double d2 = nu2 - part4[0];
  if (!(d2 > DEP_TOL2 * nu2)) {
    if (tid == 0) w.flags[b] = fl | FLAG_DONE | OMP_SIG_DEPENDENT;
    return;
  }
  const double g = 1.0 / sqrt(d2);
  const double uk = g * c[nstar];
  const double *Fb = w.V64 + b * w.vstride;
  double *Fk = w.V64 + b * w.vstride + (int64_t)k * (k + 1) / 2;
  for (int i = tid; i <= k; i += V0_THREADS) {
    if (i == k) {
      Fk[k] = g;
    } else {
      double acc = 0.0;
      for (int j = i; j < k; ++j) acc += Fb[(int64_t)j * (j + 1) / 2 + i] * zs[j];
      Fk[i] = -g * acc;
    }
  }
  const double *Gr = d.G64 + (int64_t)nstar * Np;
  double *Dk = Db + (int64_t)k * Np;
  Pick64 p1{-1.0, 0x7fffffff}, p2{-1.0, 0x7fffffff};
  for (int64_t n = tid; n < Np; n += V0_THREADS) {
    double a = Gr[n];
    int j = 0;
    for (; j + 4 <= k; j += 4) {
      const double e0 = Db[(int64_t)j * Np + n], e1 = Db[(int64_t)(j + 1) * Np + n];
      const double e2 = Db[(int64_t)(j + 2) * Np + n], e3 = Db[(int64_t)(j + 3) * Np + n];
      a = fma(-zs[j], e0, a);
      a = fma(-zs[j + 1], e1, a);
      a = fma(-zs[j + 2], e2, a);
      a = fma(-zs[j + 3], e3, a);
    }
    for (; j < k; ++j) a = fma(-zs[j], Db[(int64_t)j * Np + n], a);
    a *= g;
    Dk[n] = a;
    const bool taken = n == nstar || ((mk[n >> 5] >> (n & 31)) & 1u);
    const double cn = taken ? 0.0 : fma(-uk, a, c[n]);
    c[n] = cn;
    const double iv = d.inv_nu64[n];
    if (!taken && iv > 0.0) pick_insert(fabs(cn) * iv, (int)n, p1, p2);
  }
  v0_store_pick64(w, b, p1, p2, red);
  const int K = k + 1;
  double r2 = rn * rn - uk * uk;
  const double y2 = w.pdelta[b * NSLICE_MAX];
  const double floor2 = 64.0 * (double)(K + 1) * (1.0 / 9007199254740992.0) * y2;
  const double e2 = (double)eps_b * (double)eps_b;
  if (!(r2 > floor2) || fabs(r2 - e2) <= floor2) {
    const double *Fu = w.V64 + b * w.vstride;
    for (int i = tid; i < K; i += V0_THREADS) {
      double acc = 0.0;
      for (int j = i; j < K; ++j) acc += Fu[(int64_t)j * (j + 1) / 2 + i] * (j == k ? uk : w.u64[b * S + j]);
      zs[i] = acc;
    }
    __syncthreads();
    const float *yb = w.Yp + b * w.Mp;
    double acc = 0.0;
    for (int64_t m = tid; m < d.M; m += V0_THREADS) {
      double rm = (double)yb[m];
      for (int j = 0; j < K; ++j) {
        const int sj = j == k ? nstar : w.sup[b * S + j];
        rm -= zs[j] * (double)d.A32[(int64_t)sj * d.Mp + m];
      }
      acc += rm * rm;
    }
    acc = wave_sum(acc);
    if ((tid & 63) == 0) part4[tid >> 6] = acc;
    __syncthreads();
    r2 = 0.0;
#pragma unroll
    for (int i = 0; i < V0_THREADS / 64; ++i) r2 += part4[i];
  }
  if (tid == 0) {
    w.pnorm[b * NSLICE_MAX] = r2;
    w.sup[b * S + k] = nstar;
    w.u64[b * S + k] = uk;
    w.mask[b * mwords + nstar / 32] = mk[nstar / 32] | (1u << (nstar & 31));
    w.k[b] = K;
    w.flags[b] = fl | (K >= w.Sb[b] ? FLAG_DONE : 0);
  }
}

// x = F u in FP64, rounded once to the FP32 coefficient outputs.
__global__ __launch_bounds__(64) void k_v0_coef64(WorkView w) {
  const int64_t b = blockIdx.x;
  const int k = w.k[b];
  const int S = w.S;
  const double *F = w.V64 + b * w.vstride;
  for (int i = threadIdx.x; i < k; i += 64) {
    double acc = 0.0;
    for (int j = i; j < k; ++j) acc += F[(int64_t)j * (j + 1) / 2 + i] * w.u64[b * S + j];
    w.xh[b * S + i] = (float)acc;
  }
}

// ---------------------------------------------------------------------------
// Residual: r = y - sum_j x_j a_{s_j} on one slice of M for every signal whose
// coefficients changed in this iteration, and that slice's ||r||^2 (FP64).
// Block of 256 lanes; an item (signal, slice) takes LP lanes, 64 / LP items per
// wavefront. Workgroup i handles slice i mod nslice.
// ---------------------------------------------------------------------------
template <bool BF16>
__global__ __launch_bounds__(256) void k_residual(DictView d, WorkView w, int LP, int kbound) {
  extern __shared__ int rsm[];
  const int IPW = 64 / LP;
  const int items = 4 * IPW;
  const int S = w.S;
  // Rows of S + 1 words: the items of a wavefront read their j-th entries from
  // distinct LDS banks (rows of S words would put them all in one bank for S a
  // multiple of 64).
  const int SP = S + 1;
  float *xs = reinterpret_cast<float *>(rsm);  // [items][SP]: -x
  int *ss = rsm + items * SP;                  // [items][SP]: support
  const int slice = blockIdx.x % w.nslice;
  const int64_t group = blockIdx.x / w.nslice;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int item = wave * IPW + lane / LP;
  const int sl = lane % LP;
  const int64_t b = group * items + item;
  // kbound >= k for every signal (the launch knows how many picks have been
  // made at most), so the coefficients and support entries are read in the
  // same memory round as the signal's state instead of after it.
  const int64_t bc = b < w.B ? b : 0;  // padding items read signal 0 and do nothing
  const int fl = w.flags[bc];
  const int kraw = w.k[bc];
  const int kb = kbound < S ? kbound : S;
  for (int j = sl; j < kb; j += LP) {
    xs[item * SP + j] = -w.xh[bc * S + j];
    ss[item * SP + j] = w.sup[bc * S + j];
  }
  const int kk = (b < w.B && (fl & FLAG_NEWX)) ? kraw : 0;
  __syncthreads();
  if (kk == 0) return;  // after the only barrier

  const int64_t nc4 = d.Mp / 4;
  const int64_t sl4 = w.slice_len / 4;
  const int64_t c0 = (int64_t)slice * sl4;
  const float4 *A4 = reinterpret_cast<const float4 *>(d.A32) + c0;
  const float4 *Y4 = reinterpret_cast<const float4 *>(w.Yp) + b * nc4 + c0;
  float4 *R4 = reinterpret_cast<float4 *>(w.R32) + b * nc4 + c0;
  const float *xi = xs + item * SP;
  const int *si = ss + item * SP;
  double nrm = 0.0, dlt = 0.0;
  // FP16 form: the copy is fp16(sigma r) with the scale the solve chose from ||r|| before
  // this update (so |sigma r_m| <= 1)
  const float sig = (BF16 && w.fp16) ? w.rscale_next[b] : 1.f;
  for (int64_t c = sl; c < sl4; c += LP) {
    float4 r = Y4[c];
    int j = 0;
    for (; j + 4 <= kk; j += 4) {
      const float4 a0 = A4[(int64_t)si[j] * nc4 + c];
      const float4 a1 = A4[(int64_t)si[j + 1] * nc4 + c];
      const float4 a2 = A4[(int64_t)si[j + 2] * nc4 + c];
      const float4 a3 = A4[(int64_t)si[j + 3] * nc4 + c];
      const float x0 = xi[j], x1 = xi[j + 1], x2 = xi[j + 2], x3 = xi[j + 3];
      r.x = fmaf(x0, a0.x, r.x); r.y = fmaf(x0, a0.y, r.y); r.z = fmaf(x0, a0.z, r.z); r.w = fmaf(x0, a0.w, r.w);
      r.x = fmaf(x1, a1.x, r.x); r.y = fmaf(x1, a1.y, r.y); r.z = fmaf(x1, a1.z, r.z); r.w = fmaf(x1, a1.w, r.w);
      r.x = fmaf(x2, a2.x, r.x); r.y = fmaf(x2, a2.y, r.y); r.z = fmaf(x2, a2.z, r.z); r.w = fmaf(x2, a2.w, r.w);
      r.x = fmaf(x3, a3.x, r.x); r.y = fmaf(x3, a3.y, r.y); r.z = fmaf(x3, a3.z, r.z); r.w = fmaf(x3, a3.w, r.w);
    }
    for (; j < kk; ++j) {
      const float4 a = A4[(int64_t)si[j] * nc4 + c];
      const float x0 = xi[j];
      r.x = fmaf(x0, a.x, r.x); r.y = fmaf(x0, a.y, r.y); r.z = fmaf(x0, a.z, r.z); r.w = fmaf(x0, a.w, r.w);
    }
    R4[c] = r;
    if (BF16 && w.fp16) {
      ushort4 h;
      h.x = f32_to_f16_rne(r.x * sig);
      h.y = f32_to_f16_rne(r.y * sig);
      h.z = f32_to_f16_rne(r.z * sig);
      h.w = f32_to_f16_rne(r.w * sig);
      reinterpret_cast<ushort4 *>(w.R16)[b * nc4 + c0 + c] = h;
      const double e0 = (double)r.x - f16_used(h.x) / (double)sig;
      const double e1 = (double)r.y - f16_used(h.y) / (double)sig;
      const double e2 = (double)r.z - f16_used(h.z) / (double)sig;
      const double e3 = (double)r.w - f16_used(h.w) / (double)sig;
      dlt += e0 * e0 + e1 * e1 + e2 * e2 + e3 * e3;
    } else if (BF16) {
      ushort4 h;
      h.x = f32_to_bf16_rne(r.x);
      h.y = f32_to_bf16_rne(r.y);
      h.z = f32_to_bf16_rne(r.z);
      h.w = f32_to_bf16_rne(r.w);
      reinterpret_cast<ushort4 *>(w.R16)[b * nc4 + c0 + c] = h;
      const double e0 = (double)r.x - bf16_used(h.x);
      const double e1 = (double)r.y - bf16_used(h.y);
      const double e2 = (double)r.z - bf16_used(h.z);
      const double e3 = (double)r.w - bf16_used(h.w);
      dlt += e0 * e0 + e1 * e1 + e2 * e2 + e3 * e3;
    }
    nrm += (double)r.x * r.x + (double)r.y * r.y + (double)r.z * r.z + (double)r.w * r.w;
  }
  // sum over the item's LP lanes (aligned groups): DPP within rows, then
  // permutes across rows for LP > 16
  if (LP >= 2) { nrm += dppd<DPP_XOR1>(nrm); if (BF16) dlt += dppd<DPP_XOR1>(dlt); }
  if (LP >= 4) { nrm += dppd<DPP_XOR2>(nrm); if (BF16) dlt += dppd<DPP_XOR2>(dlt); }
  if (LP >= 8) { nrm += dppd<DPP_HALF_MIRROR>(nrm); if (BF16) dlt += dppd<DPP_HALF_MIRROR>(dlt); }
  if (LP >= 16) { nrm += dppd<DPP_MIRROR>(nrm); if (BF16) dlt += dppd<DPP_MIRROR>(dlt); }
  for (int o = 16; o < LP; o <<= 1) {
    nrm += __shfl_xor(nrm, o);
    if (BF16) dlt += __shfl_xor(dlt, o);
  }
  if (sl == 0) {
    w.pnorm[b * NSLICE_MAX + slice] = nrm;
    if (BF16) w.pdelta[b * NSLICE_MAX + slice] = dlt;
    if (BF16 && w.fp16 && slice == 0) w.rscale[b] = sig;  // the scale the next product's keys carry
  }
}

// Zero n floats from `row` with the block's threads: 16-byte stores when the
// row is 16-byte aligned and n a multiple of 4, else 4-byte stores.
__device__ inline void zero_row(float *row, int64_t n) {
  if ((n & 3) == 0 && (reinterpret_cast<uintptr_t>(row) & 15) == 0) {
    float4 *r4 = reinterpret_cast<float4 *>(row);
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t c = threadIdx.x; c < n / 4; c += blockDim.x) r4[c] = z;
  } else {
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) row[i] = 0.f;
  }
}

// ---------------------------------------------------------------------------
// Outputs: one 256-thread block per signal. The stop reason follows the
// oracle's order: a NONFINITE, DEPENDENT or EXHAUSTED stop is reported alone;
// otherwise EPS when ||r|| <= eps and SMAX when k reached S.
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
  const int k = __builtin_amdgcn_readfirstlane(w.k[b]);  // wave-uniform: scalar loop bounds
  for (int j = threadIdx.x; j < S; j += blockDim.x) {
    const int sj = j < k ? w.sup[b * S + j] : -1;
    const float xj = j < k ? w.xh[b * S + j] : 0.f;
    ss[j] = sj;
    xs[j] = xj;
    support_out[b * S + j] = sj;
    if (coef_out) coef_out[b * S + j] = xj;
  }
  __syncthreads();
  if (X_out) {  // zero the row, then scatter the k coefficients (the barrier orders the two)
    float *row = X_out + b * N;
    zero_row(row, N);
    __syncthreads();
    for (int j = threadIdx.x; j < k; j += blockDim.x) row[ss[j]] = xs[j];
  }
  if (threadIdx.x == 0) {
    const int fl = w.flags[b];
    const double rn = residual_norm(w, b);
    int st = fl & (OMP_SIG_NONFINITE | OMP_SIG_DEPENDENT | OMP_SIG_EXHAUSTED);
    if (st == 0) {
      if (rn <= (double)w.epsb[b]) st |= OMP_SIG_EPS;
      if (k >= w.Sb[b]) st |= OMP_SIG_SMAX;
    }
    st |= fl & (OMP_SIG_WIDENED | OMP_SIG_NEARTIE);
    if (status_out) status_out[b] = (k << 8) | st;
    if (rnorm_out) rnorm_out[b] = (float)rn;
  }
}

template <class K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

// Dense X [nsig][N] from the compact outputs: one 256-lane block per signal
// zero-fills its row, then scatters the coefficients (the barrier orders the
// two passes' stores within the block).
__global__ __launch_bounds__(256) void k_densify(const int32_t *__restrict__ support, const float *__restrict__ coef,
                                                 int S, int64_t N, float *__restrict__ X_out) {
  const int64_t b = blockIdx.x;
  zero_row(X_out + b * N, N);
  __syncthreads();
  for (int j = threadIdx.x; j < S; j += blockDim.x) {
    const int n = support[b * S + j];
    if (n >= 0 && n < N) X_out[b * N + n] = coef[b * S + j];
  }
}


template <int RPL, bool BF16, bool SLOTS>
hipError_t launch_solve_t(const DictView &d, const WorkView &w, const SlotView &sv, hipStream_t st) {
  const int nw = solve_waves(w);
  if (nw == 0) return hipErrorInvalidValue;  // rejected by the entry points' validation
  const size_t lds = solve_lds_per_wave(w) * nw;
  const unsigned blocks = (unsigned)((w.B + nw - 1) / nw);
  if constexpr (!SLOTS) {
    if (solve_rr(d, w)) {
      if constexpr (RPL == 1) {
        if (w.fuse_res) {
          hipError_t e = allow_lds(k_solve<1, BF16, false, true, true>, lds);
          if (e != hipSuccess) return e;
          hipLaunchKernelGGL((k_solve<1, BF16, false, true, true>), dim3(blocks), dim3(64 * nw), lds, st, d, w, sv);
          return hipGetLastError();
        }
      }
      hipError_t e = allow_lds(k_solve<RPL, BF16, false, true>, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_solve<RPL, BF16, false, true>), dim3(blocks), dim3(64 * nw), lds, st, d, w, sv);
      return hipGetLastError();
    }
  }
  hipError_t e = allow_lds(k_solve<RPL, BF16, SLOTS, false>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_solve<RPL, BF16, SLOTS, false>), dim3(blocks), dim3(64 * nw), lds, st, d, w, sv);
  return hipGetLastError();
}

template <bool SLOTS>
hipError_t launch_solve_any(const DictView &d, const WorkView &w, const SlotView &sv, int precision,
                            hipStream_t st) {
  if (w.B == 0) return hipSuccess;
  const bool bf = is_half(precision);
  if (w.S <= 64)
    return bf ? launch_solve_t<1, true, SLOTS>(d, w, sv, st) : launch_solve_t<1, false, SLOTS>(d, w, sv, st);
  if (w.S <= 128)
    return bf ? launch_solve_t<2, true, SLOTS>(d, w, sv, st) : launch_solve_t<2, false, SLOTS>(d, w, sv, st);
  return bf ? launch_solve_t<4, true, SLOTS>(d, w, sv, st) : launch_solve_t<4, false, SLOTS>(d, w, sv, st);
}

size_t residual_lds(const WorkView &w, int LP) { return (size_t)4 * (64 / LP) * (w.S + 1) * 8; }

// Lanes per signal of the residual kernel: as requested, else by shape (one
// lane per float4 of a slice, at most 16: on the 1024 x 4096 benchmark 16
// lanes with two chunks each beat 32 with one by 0.7% of the whole step, 8 and
// 4 lose); raised until the block's coefficient and support tables fit in LDS.
int residual_lanes(const WorkView &w, int lanes) {
  int LP = 1;
  if (lanes > 0) {
    LP = lanes;
  } else {
    const int sl4 = w.slice_len / 4;
    while (LP < sl4 && LP < 16) LP *= 2;
  }
  while (LP < 64 && residual_lds(w, LP) > (size_t)160 * 1024) LP *= 2;
  return LP;
}

}  // namespace

hipError_t launch_dict_prep(const float *A, int64_t lda, const DictView &d, hipStream_t st) {
  hipLaunchKernelGGL(k_dict_prep, dim3((unsigned)d.Np), dim3(64), 0, st, A, lda, d.M, d.N, d.Mp, d.nu2,
                     d.inv_nu, d.A32, d.A16, d.aerr, d.inv_nu_h);
  hipLaunchKernelGGL(k_dict_aerr_max, dim3(1), dim3(1024), 0, st, d.aerr, d.Np, d.aerr_max);
  return hipGetLastError();
}

hipError_t launch_init(const float *Y, int64_t ldy, const int32_t *S_per, const float *eps_per, float eps,
                       const DictView &d, const WorkView &w, int precision, hipStream_t st) {
  (void)precision;
  hipLaunchKernelGGL(k_init, dim3((unsigned)w.Bp), dim3(64), 0, st, Y, ldy, S_per, eps_per, eps, d.M, w);
  return hipGetLastError();
}

hipError_t launch_solve(const DictView &d, const WorkView &w, int precision, hipStream_t st) {
  SlotView none;
  memset(&none, 0, sizeof(none));
  return launch_solve_any<false>(d, w, none, precision, st);
}

hipError_t launch_solve_slots(const DictView &d, const WorkView &w, const SlotView &sv, int precision,
                              hipStream_t st) {
  return launch_solve_any<true>(d, w, sv, precision, st);
}

hipError_t launch_init_slots(const WorkView &w, const SlotView &sv, hipStream_t st) {
  if (w.B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_slots, dim3((unsigned)w.Bp), dim3(64), 0, st, w, sv);
  return hipGetLastError();
}

hipError_t launch_residual_lp(const DictView &d, const WorkView &w, int precision, int lanes, int kbound,
                              hipStream_t st) {
  if (w.B == 0) return hipSuccess;
  const int LP = residual_lanes(w, lanes);
  if (LP < 1 || LP > 64 || (LP & (LP - 1))) return hipErrorInvalidValue;
  const int items = 4 * (64 / LP);
  const int64_t groups = (w.B + items - 1) / items;
  const size_t lds = residual_lds(w, LP);
  const dim3 grid((unsigned)(groups * w.nslice)), block(256);
  if (is_half(precision)) {
    hipError_t e = allow_lds(k_residual<true>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_residual<true>, grid, block, lds, st, d, w, LP, kbound);
  } else {
    hipError_t e = allow_lds(k_residual<false>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_residual<false>, grid, block, lds, st, d, w, LP, kbound);
  }
  return hipGetLastError();
}

hipError_t launch_gram_select(const DictView &d, const WorkView &w, hipStream_t st) {
  if (!w.gram_dom || !w.P || w.ntile != GSLICE || (w.ncand != 1 && w.ncand != 2) || w.R16 || w.Np != d.Np ||
      w.S > OMP_MAX_S ||
      d.Np % (32 * GSLICE))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gram_select, dim3((unsigned)(w.B * GSLICE)), dim3(64), 0, st, d, w);
  return hipGetLastError();
}

hipError_t launch_v0_first(const DictView &d, const WorkView &w, hipStream_t st) {
  if (!w.v0 || !w.P || !w.D || w.Np != d.Np || w.B == 0) return w.B == 0 ? hipSuccess : hipErrorInvalidValue;
  hipLaunchKernelGGL(k_v0_first, dim3((unsigned)w.B), dim3(V0_THREADS), 0, st, d, w);
  return hipGetLastError();
}

hipError_t launch_v0_step(const DictView &d, const WorkView &w, hipStream_t st) {
  if (!w.v0 || !w.P || !w.D || w.Np != d.Np || d.Np % 4 || w.B == 0) return w.B == 0 ? hipSuccess : hipErrorInvalidValue;
  const size_t lds = (size_t)(w.S + d.Np / 32) * 4;
  hipError_t e = allow_lds(k_v0_step, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_v0_step, dim3((unsigned)w.B), dim3(V0_THREADS), lds, st, d, w);
  return hipGetLastError();
}

hipError_t launch_v0_coef(const WorkView &w, hipStream_t st) {
  if (w.B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_v0_coef, dim3((unsigned)w.B), dim3(64), 0, st, w);
  return hipGetLastError();
}

hipError_t launch_gram64(const DictView &d, hipStream_t st) {
  if (!d.G64 || !d.inv_nu64 || d.Np % G64_T || d.Mp % G64_K) return hipErrorInvalidValue;
  const int nt = (int)(d.Np / G64_T);
  hipLaunchKernelGGL(k_gemm64, dim3((unsigned)(nt * nt)), dim3(256), 0, st, d.A32, d.A32, d.Mp, nt, d.G64, d.Np);
  hipLaunchKernelGGL(k_inv_nu64, dim3((unsigned)((d.Np + 255) / 256)), dim3(256), 0, st, d.nu2, d.Np, d.inv_nu64);
  return hipGetLastError();
}

hipError_t launch_project64(const DictView &d, const WorkView &w, hipStream_t st) {
  if (!w.P64 || w.Bp % G64_T || d.Np % G64_T || w.Mp != d.Mp || d.Mp % G64_K || w.Np != d.Np)
    return hipErrorInvalidValue;
  const int ntr = (int)(w.Bp / G64_T), ntc = (int)(d.Np / G64_T);
  hipLaunchKernelGGL(k_gemm64, dim3((unsigned)(ntr * ntc)), dim3(256), 0, st, w.Yp, d.A32, d.Mp, ntc, w.P64, d.Np);
  return hipGetLastError();
}

hipError_t launch_v0_first64(const DictView &d, const WorkView &w, hipStream_t st) {
  if (w.B == 0) return hipSuccess;
  if (!w.P64 || !d.inv_nu64 || w.Np != d.Np) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_v0_first64, dim3((unsigned)w.B), dim3(V0_THREADS), 0, st, d, w);
  return hipGetLastError();
}

hipError_t launch_v0_step64(const DictView &d, const WorkView &w, hipStream_t st) {
  if (w.B == 0) return hipSuccess;
  if (!w.P64 || !w.D64 || !w.V64 || !w.u64 || !d.G64 || !d.inv_nu64 || w.Np != d.Np) return hipErrorInvalidValue;
  const size_t lds = (size_t)(2 * w.S + d.Np / 32) * 4;
  hipError_t e = allow_lds(k_v0_step64, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_v0_step64, dim3((unsigned)w.B), dim3(V0_THREADS), lds, st, d, w);
  return hipGetLastError();
}

hipError_t launch_v0_coef64(const WorkView &w, hipStream_t st) {
  if (w.B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_v0_coef64, dim3((unsigned)w.B), dim3(64), 0, st, w);
  return hipGetLastError();
}

hipError_t launch_residual(const DictView &d, const WorkView &w, int precision, int kbound, hipStream_t st) {
  return launch_residual_lp(d, w, precision, 0, kbound, st);
}

hipError_t launch_densify(const int32_t *support, const float *coef, int64_t nsig, int S, int64_t N,
                          float *X_out, hipStream_t st) {
  if (nsig == 0 || !X_out) return hipSuccess;
  hipLaunchKernelGGL(k_densify, dim3((unsigned)nsig), dim3(256), 0, st, support, coef, S, N, X_out);
  return hipGetLastError();
}

hipError_t prepare_kernels(const DictView &d, const WorkView &w, int precision, int lanes) {
  const size_t slds = solve_lds_per_wave(w) * (size_t)(solve_waves(w) > 0 ? solve_waves(w) : 1);
  const bool bf = is_half(precision);
  hipError_t e = hipSuccess;
  if (w.S <= 64)
    e = bf ? allow_lds(k_solve<1, true, true, false>, slds) : allow_lds(k_solve<1, false, true, false>, slds);
  else if (w.S <= 128)
    e = bf ? allow_lds(k_solve<2, true, true, false>, slds) : allow_lds(k_solve<2, false, true, false>, slds);
  else e = bf ? allow_lds(k_solve<4, true, true, false>, slds) : allow_lds(k_solve<4, false, true, false>, slds);
  if (e != hipSuccess) return e;
  const size_t rlds = residual_lds(w, residual_lanes(w, lanes));
  e = bf ? allow_lds(k_residual<true>, rlds) : allow_lds(k_residual<false>, rlds);
  if (e != hipSuccess) return e;
  return prepare_corr(d, w, precision);
}

hipError_t launch_finalize(const DictView &d, const WorkView &w, float *X_out, int32_t *support_out,
                           float *coef_out, int32_t *status_out, float *rnorm_out, hipStream_t st) {
  if (w.B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)w.B), dim3(256), 0, st, w, d.N, X_out, support_out, coef_out,
                     status_out, rnorm_out);
  return hipGetLastError();
}

}  // namespace bomp
