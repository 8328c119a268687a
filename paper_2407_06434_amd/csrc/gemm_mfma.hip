// MFMA matrix products of the OMP iteration, for gfx950 (CDNA4).
//
// Both products have the "NT" form C[n][j] = sum_m P[n][m] Q[j][m]: the two
// operands are row-major with the reduction index m contiguous, which is how
// the dictionary (atom-major) and the residuals (signal-major) are stored.
// Storing both operands reduction-contiguous is the layout lesson of the
// paper's Section 3.1; doing the whole batch in one product instead of one
// matrix-vector product per signal is Section 3.2.
//
//   * the Gram matrix G = A^T A (Section 2.2, last paragraph), stored;
//   * the correlation C = A^T R of every atom with every residual (Algorithm 1,
//     argmax step), never stored: the epilogue turns each column into the
//     packed key of its best atom, |c_n| / ||a_n|| over the atoms not yet
//     selected (Section 3.4: argmax without the B x N intermediate).
//
// The tile description and the LDS-staged main loop are in mfma_tile.h.

#include "../../include/batched_omp.h"
#include "mfma_tile.h"
#include "omp_internal.h"

namespace bomp {
namespace {

// ---------------------------------------------------------------------------
// Stored FP32 products C[n][m] = sum_k X[n][k] Z[m][k] (rows of X and Z both
// Mp floats long, ntn tiles of X rows): the Gram matrix G = A32 A32^T, and in
// the Gram-domain form P = R32 A32^T (signal-major, the correlations of every
// signal with every atom). Lanes 0-31 of a fragment row store 32 consecutive
// columns. With several K chunks (split K) workgroup chunk c sums the K slices
// [c * csl, (c + 1) * csl) and stores into its own partial matrix
// G + c * cstride; k_sum_chunks then adds the partials in chunk order.
// ---------------------------------------------------------------------------
using GramTile = Tile<128, 128, 2, 2>;

__global__ __launch_bounds__(GramTile::NTHR) void k_gram(const float *__restrict__ X, const float *__restrict__ Z,
                                                         int64_t Mp, int ntn, int ntm, int csl,
                                                         float *__restrict__ G, int64_t ldg, int64_t cstride) {
  using T = GramTile;
  extern __shared__ u32x4 lds[];
  const int tile = blockIdx.x % (ntn * ntm), chunk = blockIdx.x / (ntn * ntm);
  const int tn = tile % ntn, tm = tile / ntn;
  const int64_t rs = Mp / 4;  // row stride in 16-byte chunks
  const int nsl = (int)(rs / T::CH), s0 = chunk * csl;
  const int cnt = nsl - s0 < csl ? nsl - s0 : csl;  // >= 1 (checked by the launchers)
  const u32x4 *P = reinterpret_cast<const u32x4 *>(X) + (int64_t)tn * T::TN * rs + (int64_t)s0 * T::CH;
  const u32x4 *Q = reinterpret_cast<const u32x4 *>(Z) + (int64_t)tm * T::TB * rs + (int64_t)s0 * T::CH;
  G += (int64_t)chunk * cstride;
  f32x16 acc[T::FN][T::FB];
  mainloop<OpF32, T>(P, rs, Q, rs, cnt, lds, acc);

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wn = wave % T::WN, wb = wave / T::WN;
#pragma unroll
  for (int i = 0; i < T::FN; ++i)
#pragma unroll
    for (int j = 0; j < T::FB; ++j) {
      const int64_t col = (int64_t)tm * T::TB + wb * T::FB * 32 + j * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t row = (int64_t)tn * T::TN + wn * T::FN * 32 + i * 32 + frag_row(lane, r);
        G[row * ldg + col] = acc[i][j][r];
      }
    }
}

// ---------------------------------------------------------------------------
// XCD-aware tile order. Workgroups are handed to the 8 XCDs round robin
// (workgroup b runs on XCD b mod 8), each XCD with its own L2. When the tile
// grid (nta atom tiles x ntb signal tiles) splits into 8 equal rectangles,
// XCD x takes rectangle x, the split chosen to minimise the operand panels one
// XCD reads (nta/px + ntb/py); otherwise the order is plain row-major.
// ---------------------------------------------------------------------------
__device__ inline void xcd_tile(int b, int nta, int ntb, int *tn, int *tb) {
  int px = 0, best = 1 << 30;
  for (int q = 1; q <= 8; q *= 2) {
    const int r = 8 / q;  // q columns of atom tiles, r rows of signal tiles
    if (nta % q == 0 && ntb % r == 0 && nta / q + ntb / r < best) {
      best = nta / q + ntb / r;
      px = q;
    }
  }
  if (px == 0) {
    *tn = b % nta;
    *tb = b / nta;
    return;
  }
  const int x = b % 8, l = b / 8;
  const int lw = nta / px, lh = ntb / (8 / px);
  *tn = (x % px) * lw + l % lw;
  *tb = (x / px) * lh + l / lw;
}

// ---------------------------------------------------------------------------
// Correlation + select. For every signal j of the tile and every atom n of the
// tile, score s = |c_nj| * inv_nu[n]; an atom is a candidate when inv_nu[n] > 0
// (not a zero or padding atom) and its bit in the signal's selected-atom mask
// is clear. A candidate is carried by one 64-bit key,
//   key = (bits(s) << 32) | (0xFFFFFFFF - n),
// whose unsigned maximum is the largest score with ties going to the lowest
// index (bits(s) is monotone for s >= 0); key 0 means "no candidate".
//
// TOP2 = false (FP32 form): one key per (signal, tile), the tile's winner; with
//   SECOND (near-tie flagging) two keys, the tile's best and second best.
// TOP2 = true  (BF16 form): each lane keeps, for each "subgroup" of the atoms
//   it holds for its signal (16 atoms per fragment, SUBF fragments), the three
//   best scores and writes them as three keys. A key is 32 bits: bits(s) with
//   its low 5 bits replaced by 31 - local index, so keeping the best three is a
//   max and two medians of three; the dropped bits change s by less than 2^-18
//   relative, which the certificate accounts for. The key's slot gives the
//   subgroup, its low bits the atom within it. All atoms of the subgroup
//   compete; only when the keys are written are selected, zero-norm and padding
//   atoms marked invalid (bit 31 set; s >= 0 leaves that bit free), so the third
//   key still bounds every atom of the subgroup that is not listed.
// ---------------------------------------------------------------------------
// LDS of the correlation kernel: the main loop's two operand buffers, then (BF16
// and FP16 select) 1/||a|| of the tile's TN atoms and the TN/32 selected-atom
// mask words of each of its TB signals.
template <class T>
struct SelectLds {
  static constexpr int MAIN_CHUNKS = 2 * T::STAGE;
  static constexpr int IV_CHUNKS = T::TN / 4;      // TN floats
  static constexpr int MASK_CPS = T::TN / 128;     // 16-byte chunks of mask words per signal
  static constexpr int MASK_CHUNKS = T::TB * MASK_CPS;
  static constexpr size_t BYTES = (size_t)(MAIN_CHUNKS + IV_CHUNKS + MASK_CHUNKS) * 16;
  static_assert(IV_CHUNKS <= 64 && T::TN % 128 == 0 && MASK_CHUNKS % 64 == 0, "one load per 64 chunks");
};

template <class Op, class T, bool TOP2, bool SECOND = false>
__global__ __launch_bounds__(T::NTHR) void k_corr_select(
    const typename Op::elem *__restrict__ Aop, const typename Op::elem *__restrict__ Rop, int64_t Mp,
    int64_t Np, const float *__restrict__ inv_nu, const uint32_t *__restrict__ mask,
    const int32_t *__restrict__ flags, uint64_t *__restrict__ part, int ntile) {
  extern __shared__ u32x4 lds[];
  int tn, tb;
  xcd_tile(blockIdx.x, ntile, gridDim.x / ntile, &tn, &tb);
  const int64_t b0 = (int64_t)tb * T::TB;
  constexpr int EPC = 16 / sizeof(typename Op::elem);  // elements per 16-byte chunk
  const int64_t rs = Mp / EPC;
  const u32x4 *P = reinterpret_cast<const u32x4 *>(Aop) + (int64_t)tn * T::TN * rs;
  const u32x4 *Q = reinterpret_cast<const u32x4 *>(Rop) + b0 * rs;
  // 16-bit forms: the first K slice is staged before the liveness test below,
  // so that its loads and the test's flag reads are in flight together.
  if (TOP2) stage_first_slice<T>(P, rs, Q, rs, lds);

  // Skip the tile when every signal in it has stopped (keep-in-batch stopping,
  // Section 3.5: finished signals stay in place and are simply not advanced).
  int live = 0;
  for (int t = threadIdx.x; t < T::TB; t += T::NTHR) live |= !(flags[b0 + t] & FLAG_DONE);
  if (!__syncthreads_or(live)) {
    __builtin_amdgcn_s_waitcnt(0);  // no load may still be writing this workgroup's LDS
    return;
  }

  // BF16 / FP16 select: the epilogue's inputs that do not depend on the product,
  // 1/||a|| of the tile's atoms and the tile's selected-atom mask words of every
  // signal, are loaded into LDS behind the operand buffers before the main loop
  // (they land with its first slice), so the epilogue reads them from LDS.
  u32x4 *const ex = lds + SelectLds<T>::MAIN_CHUNKS;
  if (TOP2) {
    using X = SelectLds<T>;
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (wv == 0 && l < X::IV_CHUNKS) dma16(inv_nu + (int64_t)tn * T::TN + 4 * l, (lds_void_t *)ex);
    for (int c0 = wv * 64; c0 < X::MASK_CHUNKS; c0 += T::NW * 64) {
      const int c = c0 + l, t = c / X::MASK_CPS, part16 = c % X::MASK_CPS;
      dma16(mask + (b0 + t) * (Np / 32) + (int64_t)tn * (T::TN / 32) + 4 * part16,
            (lds_void_t *)(ex + X::IV_CHUNKS + c0));
    }
  }
  f32x16 acc[T::FN][T::FB];
  if constexpr (TOP2)
    mainloop_pipelined<Op, T, true>(P, rs, Q, rs, (int)(rs / T::CH), lds, acc);
  else
    mainloop<Op, T>(P, rs, Q, rs, (int)(rs / T::CH), lds, acc);

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wn = wave % T::WN, wb = wave / T::WN;
  const int h = lane >> 5;
  const int64_t mwords = Np / 32;
  const int64_t nw0 = (int64_t)tn * T::TN + wn * T::FN * 32;  // first atom of this wavefront's rows

  if (TOP2) {
    constexpr int SUBF = T::FN >= 2 ? 2 : 1;  // fragments per subgroup
    constexpr int SPH = T::FN / SUBF;         // subgroups per lane
    constexpr int KPT = T::WN * SPH * 2 * NKEEP;
    const float *ivl = reinterpret_cast<const float *>(ex);                            // [TN]
    const uint32_t *mwl = reinterpret_cast<const uint32_t *>(ex + SelectLds<T>::IV_CHUNKS);  // [TB][TN / 32]
    const int a0 = wn * T::FN * 32;  // first atom of this wavefront's rows within the tile
    // 1/||a|| of the lane's rows (the same for every signal column).
    float iv[T::FN][16];
#pragma unroll
    for (int i = 0; i < T::FN; ++i)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const float4 v = *reinterpret_cast<const float4 *>(ivl + a0 + i * 32 + 8 * g + 4 * h);
        iv[i][4 * g + 0] = v.x;
        iv[i][4 * g + 1] = v.y;
        iv[i][4 * g + 2] = v.z;
        iv[i][4 * g + 3] = v.w;
      }
    // When every atom of the wavefront's rows has a non-zero norm (no zero or
    // padding atom), a key's validity needs only the selected-atom mask.
    bool rows_ok = true;
#pragma unroll
    for (int i = 0; i < T::FN; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) rows_ok = rows_ok && iv[i][r] > 0.f;
    const bool all_rows_ok = __builtin_amdgcn_ballot_w64(!rows_ok) == 0;
    // Keys are staged in LDS as [signal of the tile][KPT] (the main loop ends
    // with a barrier, so the LDS is free) and written out row by row below:
    // each signal's KPT keys are contiguous in `part` (32-bit keys).
    uint32_t *stage = reinterpret_cast<uint32_t *>(lds);
#pragma unroll
    for (int j = 0; j < T::FB; ++j) {
      const int jt = wb * T::FB * 32 + j * 32 + (lane & 31);  // signal within the tile
      // selected-atom bits of this signal for the wavefront's FN * 32 atoms
      uint32_t mw[T::FN];
      {
        const uint32_t *mrow = mwl + jt * (T::TN / 32) + (a0 >> 5);
        if (T::FN == 4) {
          const uint4 v = *reinterpret_cast<const uint4 *>(mrow);  // 16-byte aligned: TN / 32 words per signal
          mw[0] = v.x;
          mw[T::FN > 1 ? 1 : 0] = v.y;
          mw[T::FN > 2 ? 2 : 0] = v.z;
          mw[T::FN > 3 ? 3 : 0] = v.w;
        } else {
#pragma unroll
          for (int i = 0; i < T::FN; ++i) mw[i] = mrow[i];
        }
      }
#pragma unroll
      for (int ig = 0; ig < SPH; ++ig) {
        uint32_t k1 = 0, k2 = 0, k3 = 0;
#pragma unroll
        for (int ii = 0; ii < SUBF; ++ii) {
          const int i = ig * SUBF + ii;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const float sc = fabsf(acc[i][j][r]) * iv[i][r];
            const uint32_t key = (__float_as_uint(sc) & ~31u) | (uint32_t)(31 - (ii * 16 + r));
            // insert into k1 >= k2 >= k3: the new second and third are medians of
            // three (v_med3_u32), independent of each other
            const uint32_t n1 = max(k1, key);
            const uint32_t n2 = max(min(k1, k2), min(max(k1, k2), key));
            const uint32_t n3 = max(min(k2, k3), min(max(k2, k3), key));
            k1 = n1;
            k2 = n2;
            k3 = n3;
          }
        }
        const uint32_t ks[3] = {k1, k2, k3};
        const uint32_t w0 = mw[ig * SUBF], w1 = mw[ig * SUBF + SUBF - 1];
#pragma unroll
        for (int q = 0; q < NKEEP; ++q) {
          const int loc = 31 - (int)(ks[q] & 31u);   // ii * 16 + r
          const int ii = loc >> 4, r = loc & 15;
          const int row = 8 * (r >> 2) + 4 * h + (r & 3);
          const int64_t n = nw0 + (ig * SUBF + ii) * 32 + row;
          const uint32_t word = ii ? w1 : w0;
          const bool valid = (all_rows_ok || ivl[n - (int64_t)tn * T::TN] > 0.f) && !((word >> row) & 1u);
          stage[jt * KPT + ((wn * SPH + ig) * 2 + h) * NKEEP + q] = valid ? ks[q] : (ks[q] | 0x80000000u);
        }
      }
    }
    __syncthreads();
    // one signal's KPT keys are 16-byte chunks of `part` (KPT is a multiple of 4)
    static_assert(KPT % 4 == 0, "keys are written in 16-byte chunks");
    constexpr int CPR = KPT / 4;
    uint32_t *dst = reinterpret_cast<uint32_t *>(part) + b0 * ((int64_t)ntile * KPT) + (int64_t)tn * KPT;
    const u32x4 *stg = reinterpret_cast<const u32x4 *>(stage);
    for (int t = threadIdx.x; t < T::TB * CPR; t += T::NTHR)
      reinterpret_cast<u32x4 *>(dst + (int64_t)(t / CPR) * ntile * KPT)[t % CPR] = stg[t];
    return;
  }

  uint64_t *red = reinterpret_cast<uint64_t *>(lds);  // [WN][TB] (x2 with SECOND), LDS is free after the main loop
#pragma unroll
  for (int j = 0; j < T::FB; ++j) {
    const int jt = wb * T::FB * 32 + j * 32 + (lane & 31);  // signal within the tile
    const int64_t b = b0 + jt;
    uint64_t best = 0, sec = 0;  // sec: second best (SECOND only)
#pragma unroll
    for (int i = 0; i < T::FN; ++i) {
      const int64_t nf = nw0 + i * 32;  // first atom of the fragment
      const uint32_t word = mask[b * mwords + nf / 32];
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const float4 iv = *reinterpret_cast<const float4 *>(inv_nu + nf + 8 * g + 4 * h);
        const float ivs[4] = {iv.x, iv.y, iv.z, iv.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = 8 * g + 4 * h + e;
          const float s = fabsf(acc[i][j][4 * g + e]) * ivs[e];
          const bool cand = ivs[e] > 0.f && !((word >> row) & 1u) && s >= 0.f;
          const uint64_t key = cand ? ((uint64_t)__float_as_uint(s) << 32) |
                                          (uint64_t)(0xFFFFFFFFu - (uint32_t)(nf + row))
                                    : 0ull;
          if (SECOND) sec = max(sec, min(best, key));
          best = key > best ? key : best;
        }
      }
    }
    const uint64_t other = __shfl_xor(best, 32);
    if (SECOND) sec = max(max(sec, __shfl_xor(sec, 32)), min(best, other));
    best = other > best ? other : best;
    if (lane < 32) {
      red[wn * T::TB + jt] = best;
      if (SECOND) red[(T::WN + wn) * T::TB + jt] = sec;
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < T::TB; t += T::NTHR) {
    uint64_t best = 0, sec = 0;
#pragma unroll
    for (int w = 0; w < T::WN; ++w) {
      const uint64_t v = red[w * T::TB + t];
      if (SECOND) sec = max(max(sec, red[(T::WN + w) * T::TB + t]), min(best, v));
      best = v > best ? v : best;
    }
    if (SECOND) {
      part[(b0 + t) * ntile * 2 + 2 * tn] = best;
      part[(b0 + t) * ntile * 2 + 2 * tn + 1] = sec;
    } else {
      part[(b0 + t) * ntile + tn] = best;
    }
  }
}

// Tile configurations (atoms x signals, wavefront grid):
//   1: 128 x 128, 2 x 2 wavefronts of 64 x 64
//   2: 256 x 256, 2 x 2 wavefronts of 128 x 128 (accumulators in AGPRs)
//   3: 256 x 256, 2 x 4 wavefronts of 128 x 64
//   4: 256 x 128, 2 x 2 wavefronts of 128 x 64
using Cfg1 = Tile<128, 128, 2, 2>;
using Cfg2 = Tile<256, 256, 2, 2>;
using Cfg3 = Tile<256, 256, 2, 4>;
using Cfg4 = Tile<256, 128, 2, 2>;

template <class K>
hipError_t set_lds(K kernel, size_t bytes) {
  static bool done = false;  // per kernel instantiation
  if (done) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) done = true;
  return e;
}

template <class Op, class T, bool TOP2, bool SECOND = false>
hipError_t launch_corr_t(const typename Op::elem *Aop, const typename Op::elem *Rop, const DictView &d,
                         const WorkView &w, hipStream_t st) {
  auto kern = k_corr_select<Op, T, TOP2, SECOND>;
  const size_t lds_bytes = TOP2 ? SelectLds<T>::BYTES : T::LDS_BYTES;
  hipError_t e = set_lds(kern, lds_bytes);
  if (e != hipSuccess) return e;
  const int ntile = (int)(d.Np / T::TN);
  // the epilogue scores |c| by 1/||a_n|| (FP16 form: divided by the atom's storage scale)
  hipLaunchKernelGGL(kern, dim3((unsigned)(ntile * (w.Bp / T::TB))), dim3(T::NTHR), lds_bytes, st, Aop, Rop,
                     d.Mp, d.Np, d.inv_nu_h ? d.inv_nu_h : d.inv_nu, w.mask, w.flags, w.part, ntile);
  return hipGetLastError();
}

template <class T>
CorrGeom geom(int precision, int cfg, bool ties) {
  CorrGeom g;
  constexpr int SUBF = T::FN >= 2 ? 2 : 1;
  g.cfg = cfg;
  g.tile_atoms = T::TN;
  g.tile_signals = T::TB;
  g.keys_per_tile = is_half(precision) ? T::WN * (T::FN / SUBF) * 2 * NKEEP : (ties ? 2 : 1);
  g.wave_atoms = T::FN * 32;
  g.sub_frags = SUBF;
  g.subs_per_half = T::FN / SUBF;
  return g;
}

}  // namespace

CorrGeom corr_geometry(int precision, int64_t Np, int64_t Bp, int cfg, bool ties) {
  if (cfg == 0) cfg = (Np / 256) * (Bp / 256) >= 192 ? 3 : 1;
  switch (cfg) {
    case 2: return geom<Cfg2>(precision, 2, ties);
    case 3: return geom<Cfg3>(precision, 3, ties);
    case 4: return geom<Cfg4>(precision, 4, ties);
    default: return geom<Cfg1>(precision, 1, ties);
  }
}

hipError_t launch_gram(const DictView &d, hipStream_t st) {
  using T = GramTile;
  hipError_t e = set_lds(k_gram, T::LDS_BYTES);
  if (e != hipSuccess) return e;
  const int nt = (int)(d.Np / T::TN);
  const int nsl = (int)(d.Mp / 4 / T::CH);
  hipLaunchKernelGGL(k_gram, dim3(nt * nt), dim3(T::NTHR), T::LDS_BYTES, st, d.A32, d.A32, d.Mp, nt, nt, nsl,
                     d.G, d.Np, (int64_t)0);
  return hipGetLastError();
}

// P[i] = sum over chunks c, in chunk order, of Pk[c][i]; four floats per lane.
__global__ __launch_bounds__(256) void k_sum_chunks(const float4 *__restrict__ Pk, int chunks, int64_t n4,
                                                    float4 *__restrict__ P) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n4) return;
  float4 a = Pk[i];
  for (int c = 1; c < chunks; ++c) {
    const float4 v = Pk[(int64_t)c * n4 + i];
    a.x += v.x;
    a.y += v.y;
    a.z += v.z;
    a.w += v.w;
  }
  P[i] = a;
}

hipError_t launch_project(const DictView &d, const WorkView &w, hipStream_t st) {
  using T = GramTile;
  static_assert(BPAD % T::TN == 0 && NPAD % T::TB == 0, "padded sizes must be whole tiles");
  if (!w.P || w.Bp % T::TN || d.Np % T::TB || w.Mp != d.Mp || w.Np != d.Np) return hipErrorInvalidValue;
  hipError_t e = set_lds(k_gram, T::LDS_BYTES);
  if (e != hipSuccess) return e;
  const int ntb = (int)(w.Bp / T::TN), nta = (int)(d.Np / T::TB);
  const int nsl = (int)(d.Mp / 4 / T::CH), ks = w.pchunks;
  const int csl = ks >= 1 ? (nsl + ks - 1) / ks : 0;
  if (ks < 1 || (ks > 1 && !w.Pk) || nsl - (ks - 1) * csl < 1) return hipErrorInvalidValue;
  const int64_t n = w.Bp * d.Np;
  hipLaunchKernelGGL(k_gram, dim3(ntb * nta * ks), dim3(T::NTHR), T::LDS_BYTES, st, w.R32, d.A32, d.Mp, ntb, nta,
                     csl, ks > 1 ? w.Pk : w.P, d.Np, n);
  e = hipGetLastError();
  if (e != hipSuccess || ks == 1) return e;
  const int64_t n4 = n / 4;
  hipLaunchKernelGGL(k_sum_chunks, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, st,
                     reinterpret_cast<const float4 *>(w.Pk), ks, n4, reinterpret_cast<float4 *>(w.P));
  return hipGetLastError();
}

template <class T>
hipError_t launch_corr_cfg(const DictView &d, const WorkView &w, int precision, hipStream_t st) {
  if (precision == OMP_PREC_BF16) return launch_corr_t<OpBF16, T, true>(d.A16, w.R16, d, w, st);
  if (precision == OMP_PREC_FP16) return launch_corr_t<OpF16, T, true>(d.A16, w.R16, d, w, st);
  if (w.ncand == 2) return launch_corr_t<OpF32, T, false, true>(d.A32, w.R32, d, w, st);
  return launch_corr_t<OpF32, T, false>(d.A32, w.R32, d, w, st);
}

template <class T>
hipError_t prepare_corr_cfg(int precision, bool second) {
  if (precision == OMP_PREC_BF16) return set_lds(k_corr_select<OpBF16, T, true>, SelectLds<T>::BYTES);
  if (precision == OMP_PREC_FP16) return set_lds(k_corr_select<OpF16, T, true>, SelectLds<T>::BYTES);
  if (second) return set_lds(k_corr_select<OpF32, T, false, true>, T::LDS_BYTES);
  return set_lds(k_corr_select<OpF32, T, false>, T::LDS_BYTES);
}

hipError_t prepare_corr(const DictView &d, const WorkView &w, int precision) {
  (void)d;
  const bool second = w.ncand == 2 && !is_half(precision);
  switch (w.tile_cfg) {
    case 2: return prepare_corr_cfg<Cfg2>(precision, second);
    case 3: return prepare_corr_cfg<Cfg3>(precision, second);
    case 4: return prepare_corr_cfg<Cfg4>(precision, second);
    default: return prepare_corr_cfg<Cfg1>(precision, second);
  }
}

hipError_t launch_corr_select(const DictView &d, const WorkView &w, int precision, hipStream_t st) {
  switch (w.tile_cfg) {
    case 2: return launch_corr_cfg<Cfg2>(d, w, precision, st);
    case 3: return launch_corr_cfg<Cfg3>(d, w, precision, st);
    case 4: return launch_corr_cfg<Cfg4>(d, w, precision, st);
    default: return launch_corr_cfg<Cfg1>(d, w, precision, st);
  }
}

}  // namespace bomp
