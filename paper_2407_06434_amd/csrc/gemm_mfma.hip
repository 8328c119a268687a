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
// Tiling. A workgroup computes a TN x TB tile with WN x WB wavefronts; each
// wavefront owns FN x FB fragments of 32 x 32 (v_mfma_f32_32x32x2f32 for FP32,
// v_mfma_f32_32x32x16_bf16 for BF16). Operands are staged through LDS in
// 128-byte K slices, double buffered; each lane reads 16-byte chunks. Lane l
// of a fragment reads row (l mod 32) at chunk (2q + l/32) of the slice; the
// two halves of the wavefront thus supply the two K sub-blocks an MFMA sums
// over, and both operands use the same K assignment, so the product sums
// every m exactly once (the order of summation inside an MFMA is the
// hardware's).

#include "omp_internal.h"

namespace bomp {
namespace {

typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
// 16-byte chunk as a native vector (HIP's uint4 is a union-based struct that
// can keep arrays of it out of registers).
typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;

struct OpF32 {
  using elem = float;
  // One 16-byte chunk holds 4 FP32 values of K: four 32x32x2 MFMAs.
  __device__ static inline void mma(const u32x4 &a, const u32x4 &b, f32x16 &c) {
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.x), __uint_as_float(b.x), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.y), __uint_as_float(b.y), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.z), __uint_as_float(b.z), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.w), __uint_as_float(b.w), c, 0, 0, 0);
  }
};

struct OpBF16 {
  using elem = uint16_t;
  // One 16-byte chunk holds 8 BF16 values of K: one 32x32x16 MFMA.
  __device__ static inline void mma(const u32x4 &a, const u32x4 &b, f32x16 &c) {
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  }
};

template <int TN_, int TB_, int WN_, int WB_>
struct Tile {
  static constexpr int TN = TN_, TB = TB_, WN = WN_, WB = WB_;
  static constexpr int NTHR = WN * WB * 64;
  static constexpr int FN = TN / (32 * WN);
  static constexpr int FB = TB / (32 * WB);
  static constexpr int CH = 8;       // 16-byte chunks per row per K slice (128 bytes)
  static constexpr int RS = CH + 1;  // LDS row stride in chunks (one chunk of padding)
  static constexpr int A_LD = TN * CH / NTHR;
  static constexpr int B_LD = TB * CH / NTHR;
  static constexpr int STAGE = (TN + TB) * RS;  // chunks per LDS buffer
  static constexpr size_t LDS_BYTES = 2 * STAGE * 16;
  static_assert(FN >= 1 && FB >= 1, "tile too small for the wavefront grid");
  static_assert(TN * CH % NTHR == 0 && TB * CH % NTHR == 0, "loads must divide evenly");
};

// Main loop: acc += P_tile * Q_tile^T over `nslices` K slices of 128 bytes.
// P points at the tile's first row, rows `prs` chunks apart; likewise Q.
template <class Op, class T>
__device__ inline void mainloop(const u32x4 *__restrict__ P, int64_t prs, const u32x4 *__restrict__ Q,
                                int64_t qrs, int nslices, u32x4 *lds, f32x16 (&acc)[T::FN][T::FB]) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wn = wave % T::WN, wb = wave / T::WN;
  const int h = lane >> 5, r32 = lane & 31;

#pragma unroll
  for (int i = 0; i < T::FN; ++i)
#pragma unroll
    for (int j = 0; j < T::FB; ++j) acc[i][j] = f32x16{};

  u32x4 ra[T::A_LD], rb[T::B_LD];
  // Stage 0: global -> registers -> LDS buffer 0.
#pragma unroll
  for (int i = 0; i < T::A_LD; ++i) {
    const int idx = tid + i * T::NTHR;
    ra[i] = P[(int64_t)(idx / T::CH) * prs + (idx % T::CH)];
  }
#pragma unroll
  for (int i = 0; i < T::B_LD; ++i) {
    const int idx = tid + i * T::NTHR;
    rb[i] = Q[(int64_t)(idx / T::CH) * qrs + (idx % T::CH)];
  }
#pragma unroll
  for (int i = 0; i < T::A_LD; ++i) {
    const int idx = tid + i * T::NTHR;
    lds[(idx / T::CH) * T::RS + (idx % T::CH)] = ra[i];
  }
#pragma unroll
  for (int i = 0; i < T::B_LD; ++i) {
    const int idx = tid + i * T::NTHR;
    lds[T::TN * T::RS + (idx / T::CH) * T::RS + (idx % T::CH)] = rb[i];
  }
  __syncthreads();
  for (int s = 0; s < nslices; ++s) {
    const int buf = s & 1;
    const bool more = s + 1 < nslices;
    if (more) {  // prefetch slice s+1 into registers while slice s is multiplied
#pragma unroll
      for (int i = 0; i < T::A_LD; ++i) {
        const int idx = tid + i * T::NTHR;
        ra[i] = P[(int64_t)(idx / T::CH) * prs + (int64_t)(s + 1) * T::CH + (idx % T::CH)];
      }
#pragma unroll
      for (int i = 0; i < T::B_LD; ++i) {
        const int idx = tid + i * T::NTHR;
        rb[i] = Q[(int64_t)(idx / T::CH) * qrs + (int64_t)(s + 1) * T::CH + (idx % T::CH)];
      }
    }
    const u32x4 *la = lds + buf * T::STAGE + (wn * T::FN * 32 + r32) * T::RS + h;
    const u32x4 *lb = lds + buf * T::STAGE + T::TN * T::RS + (wb * T::FB * 32 + r32) * T::RS + h;
#pragma unroll
    for (int q = 0; q < T::CH / 2; ++q) {
      u32x4 af[T::FN], bf[T::FB];
#pragma unroll
      for (int i = 0; i < T::FN; ++i) af[i] = la[i * 32 * T::RS + 2 * q];
#pragma unroll
      for (int j = 0; j < T::FB; ++j) bf[j] = lb[j * 32 * T::RS + 2 * q];
#pragma unroll
      for (int i = 0; i < T::FN; ++i)
#pragma unroll
        for (int j = 0; j < T::FB; ++j) Op::mma(af[i], bf[j], acc[i][j]);
    }
    if (more) {
      u32x4 *nb = lds + (buf ^ 1) * T::STAGE;
#pragma unroll
      for (int i = 0; i < T::A_LD; ++i) {
        const int idx = tid + i * T::NTHR;
        nb[(idx / T::CH) * T::RS + (idx % T::CH)] = ra[i];
      }
#pragma unroll
      for (int i = 0; i < T::B_LD; ++i) {
        const int idx = tid + i * T::NTHR;
        nb[T::TN * T::RS + (idx / T::CH) * T::RS + (idx % T::CH)] = rb[i];
      }
    }
    __syncthreads();
  }
}

// Row of a 32x32 MFMA result held by (lane, register r): the column is lane % 32.
__device__ inline int frag_row(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// ---------------------------------------------------------------------------
// Gram matrix: G[n][m] = sum_k A32[n][k] A32[m][k], FP32 in and out.
// ---------------------------------------------------------------------------
using GramTile = Tile<128, 128, 2, 2>;

__global__ __launch_bounds__(GramTile::NTHR) void k_gram(const float *__restrict__ A32, int64_t Mp,
                                                         int64_t Np, float *__restrict__ G) {
  using T = GramTile;
  extern __shared__ u32x4 lds[];
  const int ntn = (int)(Np / T::TN);
  const int tn = blockIdx.x % ntn, tm = blockIdx.x / ntn;
  const int64_t rs = Mp / 4;  // row stride in 16-byte chunks
  const u32x4 *P = reinterpret_cast<const u32x4 *>(A32) + (int64_t)tn * T::TN * rs;
  const u32x4 *Q = reinterpret_cast<const u32x4 *>(A32) + (int64_t)tm * T::TB * rs;
  f32x16 acc[T::FN][T::FB];
  mainloop<OpF32, T>(P, rs, Q, rs, (int)(rs / T::CH), lds, acc);

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
        G[row * Np + col] = acc[i][j][r];
      }
    }
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
// TOP2 = false (FP32 form): one key per (signal, tile), the tile's winner.
// TOP2 = true  (BF16 form): each lane keeps, for each "subgroup" of the atoms
//   it holds for its signal (16 atoms per fragment, SUBF fragments), the three
//   best scores and writes them as three keys. Inside the loop a candidate is
//   a 32-bit key (bits(s) with its low 5 bits replaced by 31 - local index),
//   so keeping the best three is a min/max sorting network; the dropped bits
//   change s by less than 2^-18 relative, which the certificate accounts for.
//   All atoms of the subgroup compete; only when the keys are written are
//   selected, zero-norm and padding atoms marked invalid (low word 0), so the
//   third key still bounds every atom of the subgroup that is not listed.
// ---------------------------------------------------------------------------
template <class Op, class T, bool TOP2>
__global__ __launch_bounds__(T::NTHR) void k_corr_select(
    const typename Op::elem *__restrict__ Aop, const typename Op::elem *__restrict__ Rop, int64_t Mp,
    int64_t Np, const float *__restrict__ inv_nu, const uint32_t *__restrict__ mask,
    const int32_t *__restrict__ flags, uint64_t *__restrict__ part, int ntile) {
  extern __shared__ u32x4 lds[];
  const int tn = blockIdx.x % ntile, tb = blockIdx.x / ntile;
  const int64_t b0 = (int64_t)tb * T::TB;

  // Skip the tile when every signal in it has stopped (keep-in-batch stopping,
  // Section 3.5: finished signals stay in place and are simply not advanced).
  int live = 0;
  for (int t = threadIdx.x; t < T::TB; t += T::NTHR) live |= !(flags[b0 + t] & FLAG_DONE);
  if (!__syncthreads_or(live)) return;

  constexpr int EPC = 16 / sizeof(typename Op::elem);  // elements per 16-byte chunk
  const int64_t rs = Mp / EPC;
  const u32x4 *P = reinterpret_cast<const u32x4 *>(Aop) + (int64_t)tn * T::TN * rs;
  const u32x4 *Q = reinterpret_cast<const u32x4 *>(Rop) + b0 * rs;
  f32x16 acc[T::FN][T::FB];
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
    // 1/||a|| of the lane's rows (the same for every signal column).
    float iv[T::FN][16];
#pragma unroll
    for (int i = 0; i < T::FN; ++i)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const float4 v = *reinterpret_cast<const float4 *>(inv_nu + nw0 + i * 32 + 8 * g + 4 * h);
        iv[i][4 * g + 0] = v.x;
        iv[i][4 * g + 1] = v.y;
        iv[i][4 * g + 2] = v.z;
        iv[i][4 * g + 3] = v.w;
      }
#pragma unroll
    for (int j = 0; j < T::FB; ++j) {
      const int64_t b = b0 + wb * T::FB * 32 + j * 32 + (lane & 31);
      uint64_t *dst = part + b * ((int64_t)ntile * KPT) + (int64_t)tn * KPT;
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
            const uint32_t lo1 = min(k1, key);
            k1 = max(k1, key);
            const uint32_t lo2 = min(k2, lo1);
            k2 = max(k2, lo1);
            k3 = max(k3, lo2);
          }
        }
        const uint32_t ks[3] = {k1, k2, k3};
#pragma unroll
        for (int q = 0; q < NKEEP; ++q) {
          const int loc = 31 - (int)(ks[q] & 31u);   // ii * 16 + r
          const int ii = loc >> 4, r = loc & 15;
          const int row = 8 * (r >> 2) + 4 * h + (r & 3);
          const int64_t n = nw0 + (ig * SUBF + ii) * 32 + row;
          const bool valid = inv_nu[n] > 0.f && !((mask[b * mwords + (n >> 5)] >> (n & 31)) & 1u);
          const uint64_t score = (uint64_t)(ks[q] & ~31u) << 32;
          dst[((wn * SPH + ig) * 2 + h) * NKEEP + q] =
              score | (valid ? (uint64_t)(0xFFFFFFFFu - (uint32_t)n) : 0ull);
        }
      }
    }
    return;
  }

  uint64_t *red = reinterpret_cast<uint64_t *>(lds);  // [WN][TB], LDS is free after the main loop
#pragma unroll
  for (int j = 0; j < T::FB; ++j) {
    const int jt = wb * T::FB * 32 + j * 32 + (lane & 31);  // signal within the tile
    const int64_t b = b0 + jt;
    uint64_t best = 0;
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
          best = key > best ? key : best;
        }
      }
    }
    const uint64_t other = __shfl_xor(best, 32);
    best = other > best ? other : best;
    if (lane < 32) red[wn * T::TB + jt] = best;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < T::TB; t += T::NTHR) {
    uint64_t best = 0;
#pragma unroll
    for (int w = 0; w < T::WN; ++w) best = red[w * T::TB + t] > best ? red[w * T::TB + t] : best;
    part[(b0 + t) * ntile + tn] = best;
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

template <class Op, class T, bool TOP2>
hipError_t launch_corr_t(const typename Op::elem *Aop, const typename Op::elem *Rop, const DictView &d,
                         const WorkView &w, hipStream_t st) {
  auto kern = k_corr_select<Op, T, TOP2>;
  hipError_t e = set_lds(kern, T::LDS_BYTES);
  if (e != hipSuccess) return e;
  const int ntile = (int)(d.Np / T::TN);
  hipLaunchKernelGGL(kern, dim3((unsigned)(ntile * (w.Bp / T::TB))), dim3(T::NTHR), T::LDS_BYTES, st, Aop, Rop,
                     d.Mp, d.Np, d.inv_nu, w.mask, w.flags, w.part, ntile);
  return hipGetLastError();
}

template <class T>
CorrGeom geom(int precision, int cfg) {
  CorrGeom g;
  constexpr int SUBF = T::FN >= 2 ? 2 : 1;
  g.cfg = cfg;
  g.tile_atoms = T::TN;
  g.tile_signals = T::TB;
  g.keys_per_tile = precision == 1 ? T::WN * (T::FN / SUBF) * 2 * NKEEP : 1;
  g.wave_atoms = T::FN * 32;
  g.sub_frags = SUBF;
  g.subs_per_half = T::FN / SUBF;
  return g;
}

}  // namespace

CorrGeom corr_geometry(int precision, int64_t Np, int64_t Bp, int cfg) {
  if (cfg == 0) cfg = (Np / 256) * (Bp / 256) >= 192 ? 3 : 1;
  switch (cfg) {
    case 2: return geom<Cfg2>(precision, 2);
    case 3: return geom<Cfg3>(precision, 3);
    case 4: return geom<Cfg4>(precision, 4);
    default: return geom<Cfg1>(precision, 1);
  }
}

hipError_t launch_gram(const DictView &d, hipStream_t st) {
  using T = GramTile;
  hipError_t e = set_lds(k_gram, T::LDS_BYTES);
  if (e != hipSuccess) return e;
  const int nt = (int)(d.Np / T::TN);
  hipLaunchKernelGGL(k_gram, dim3(nt * nt), dim3(T::NTHR), T::LDS_BYTES, st, d.A32, d.Mp, d.Np, d.G);
  return hipGetLastError();
}

template <class T>
hipError_t launch_corr_cfg(const DictView &d, const WorkView &w, int precision, hipStream_t st) {
  if (precision == 1) return launch_corr_t<OpBF16, T, true>(d.A16, w.R16, d, w, st);
  return launch_corr_t<OpF32, T, false>(d.A32, w.R32, d, w, st);
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
