// MFMA building blocks shared by the matrix products of libbatched_omp.so
// (gfx950, CDNA4): operand element types, the workgroup tile description and
// the LDS-staged main loop of an "NT" product C[n][j] = sum_k P[n][k] Q[j][k]
// whose operands are both row-major with the reduction index k contiguous.
//
// A workgroup computes a TN x TB tile with WN x WB wavefronts; each wavefront
// owns FN x FB fragments of 32 x 32 (v_mfma_f32_32x32x2f32 for FP32,
// v_mfma_f32_32x32x16_bf16 for BF16). Operands are staged through LDS in
// 128-byte K slices, double buffered; each lane reads 16-byte chunks. Lane l of
// a fragment reads row (l mod 32) at chunk (2q + l/32) of the slice; the two
// halves of the wavefront thus supply the two K sub-blocks an MFMA sums over,
// and both operands use the same K assignment, so the product sums every k
// exactly once (the order of summation inside an MFMA is the hardware's).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

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

}  // namespace
}  // namespace bomp
