// MFMA building blocks shared by the matrix products of libbatched_omp.so
// (gfx950, CDNA4): operand element types, the workgroup tile description and
// the LDS-staged main loop of an "NT" product C[n][j] = sum_k P[n][k] Q[j][k]
// whose operands are both row-major with the reduction index k contiguous.
//
// A workgroup computes a TN x TB tile with WN x WB wavefronts; each wavefront
// owns FN x FB fragments of 32 x 32 (v_mfma_f32_32x32x2f32 for FP32,
// v_mfma_f32_32x32x16_bf16 for BF16, v_mfma_f32_32x32x16_f16 for FP16). Operands are staged through LDS in
// 128-byte K slices, double buffered, with direct global-to-LDS loads (16
// bytes per lane, no register round trip); the 16-bit products also double-buffer
// their fragments in registers (mainloop_pipelined). A staged row is 8 chunks of 16
// bytes; chunk c of row r sits at slot c ^ ((r >> 1) & 7) of the row, so the
// 16 lanes of one LDS read phase (16 consecutive rows, one chunk) hit 16
// distinct 4-bank groups. Lane l of a fragment reads row (l mod 32) at chunk
// (2q + l/32) of the slice; the two halves of the wavefront thus supply the two
// K sub-blocks an MFMA sums over, and both operands use the same K assignment,
// so the product sums every k exactly once (the order of summation inside an
// MFMA is the hardware's).
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

typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;

// FP16 copies of the operands (the FP16 form): one 16-byte chunk holds 8 FP16
// values of K, one 32x32x16 MFMA.
struct OpF16 {
  using elem = uint16_t;
  __device__ static inline void mma(const u32x4 &a, const u32x4 &b, f32x16 &c) {
    c = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0, 0,
                                               0);
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

typedef __attribute__((address_space(3))) void lds_void_t;

template <int TN_, int TB_, int WN_, int WB_>
struct Tile {
  static constexpr int TN = TN_, TB = TB_, WN = WN_, WB = WB_;
  static constexpr int NTHR = WN * WB * 64;
  static constexpr int NW = WN * WB;  // wavefronts
  static constexpr int FN = TN / (32 * WN);
  static constexpr int FB = TB / (32 * WB);
  static constexpr int CH = 8;                 // 16-byte chunks per row per K slice (128 bytes)
  static constexpr int ROWS = TN + TB;         // staged rows per slice (P rows, then Q rows)
  static constexpr int STAGE = ROWS * CH;      // chunks per LDS buffer
  static constexpr int LPW = ROWS / (8 * NW);  // global-to-LDS loads per wavefront per slice (8 rows each)
  static constexpr size_t LDS_BYTES = 2 * STAGE * 16;
  static_assert(FN >= 1 && FB >= 1, "tile too small for the wavefront grid");
  static_assert(ROWS % (8 * NW) == 0 && TN % 8 == 0, "loads must divide evenly");
};

// Slot of chunk c in staged row r.
__device__ inline int lds_slot(int r, int c) { return c ^ ((r >> 1) & 7); }

// One global-to-LDS load of 16 bytes per lane: lane l's 16 bytes from `g` land
// in LDS chunk l after the wave-uniform address `l` (M0 holds that address).
// Written as inline asm on purpose: the compiler counts its own LDS-DMA builtin
// as an LDS access that may complete out of order, and then answers every later
// LDS read with a full lgkmcnt(0) wait, which serialises the fragment reads of
// the main loop against the MFMAs. Hidden from the compiler, these loads are
// waited for explicitly (vmcnt) before the barrier that publishes them. M0 is
// saved and restored around the load (the compiler may hold a value there); the
// only register the asm writes is that scalar save slot, no load destination.
__device__ inline void dma16(const void *g, lds_void_t *l) {
  const uint32_t la = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)l);
  uint32_t saved;
  asm volatile(
      "s_mov_b32 %0, m0\n\t"
      "s_mov_b32 m0, %2\n\t"
      "s_nop 0\n\t"
      "global_load_lds_dwordx4 %1, off\n\t"
      "s_nop 0\n\t"
      "s_mov_b32 m0, %0"
      : "=&s"(saved)
      : "v"(g), "s"(la)
      : "memory");
}

// Pipelined main loop (16-bit operands): acc += P_tile * Q_tile^T over `nslices`
// K slices of 128 bytes. P points at the tile's first row, rows `prs` chunks
// apart; likewise Q. Wavefront w stages rows 8 (i NW + w) .. +7 of every slice
// with its load i: a load writes 64 consecutive LDS chunks (lane l -> chunk l),
// so lane l fetches row 8 (i NW + w) + l/8, chunk lds_slot(row, l mod 8). Two LDS buffers: the
// loads of slice s+2 are issued right after the barrier that ends slice s (its
// buffer is then free). Fragments are double-buffered in registers: the LDS
// reads of step q+1 are issued before the MFMAs of step q, and the slice barrier
// sits between the two halves of a slice's last step, so the MFMA pipe keeps
// working while the wavefronts meet. Loads the caller issued with dma16 before
// the call have landed once the first barrier has passed. Ends with a barrier,
// so the caller may reuse the LDS.
// Source of lane's chunk for load i of the calling wavefront at slice 0 (the
// slot map is an involution, so the chunk that lands in slot l mod 8 is read).
template <class T>
__device__ inline const u32x4 *stage_src(const u32x4 *__restrict__ P, int64_t prs, const u32x4 *__restrict__ Q,
                                         int64_t qrs, int i) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = (i * T::NW + wave) * 8 + (lane >> 3);
  const int c = lds_slot(row, lane & 7);
  return row < T::TN ? P + (int64_t)row * prs + c : Q + (int64_t)(row - T::TN) * qrs + c;
}

// The calling wavefront's loads of K slice 0 into LDS buffer 0 (a caller may
// issue them early and then tell mainloop_pipelined so with FIRST_STAGED).
template <class T>
__device__ inline void stage_first_slice(const u32x4 *__restrict__ P, int64_t prs, const u32x4 *__restrict__ Q,
                                         int64_t qrs, u32x4 *lds) {
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < T::LPW; ++i)
    dma16(reinterpret_cast<const void *>(stage_src<T>(P, prs, Q, qrs, i)),
          (lds_void_t *)(lds + (i * T::NW + wave) * 64));
}

template <class Op, class T, bool FIRST_STAGED = false>
__device__ inline void mainloop_pipelined(const u32x4 *__restrict__ P, int64_t prs, const u32x4 *__restrict__ Q,
                                          int64_t qrs, int nslices, u32x4 *lds, f32x16 (&acc)[T::FN][T::FB]) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wn = wave % T::WN, wb = wave / T::WN;
  const int h = lane >> 5, r32 = lane & 31;
  constexpr int QS = T::CH / 2;         // MFMA steps per slice (32 bytes of K each)
  constexpr int NM = T::FN * T::FB;     // MFMAs (fragment pairs) per step
  constexpr int SPLIT = NM / 2;         // last step: MFMAs issued before the barrier

#pragma unroll
  for (int i = 0; i < T::FN; ++i)
#pragma unroll
    for (int j = 0; j < T::FB; ++j) acc[i][j] = f32x16{};
  if (nslices <= 0) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    return;
  }

  // Source of this lane's chunk for each of its loads, at slice 0.
  const u32x4 *src[T::LPW];
#pragma unroll
  for (int i = 0; i < T::LPW; ++i) src[i] = stage_src<T>(P, prs, Q, qrs, i);
  auto issue = [&](int s, int buf) {
#pragma unroll
    for (int i = 0; i < T::LPW; ++i)
      dma16(reinterpret_cast<const void *>(src[i] + (int64_t)s * T::CH),
            (lds_void_t *)(lds + buf * T::STAGE + (i * T::NW + wave) * 64));
  };

  // LDS offsets (chunks) of this lane's fragment rows and their slot swizzles.
  int aoff[T::FN], asw[T::FN], boff[T::FB], bsw[T::FB];
#pragma unroll
  for (int i = 0; i < T::FN; ++i) {
    const int row = wn * T::FN * 32 + i * 32 + r32;
    aoff[i] = row * T::CH;
    asw[i] = (row >> 1) & 7;
  }
#pragma unroll
  for (int j = 0; j < T::FB; ++j) {
    const int row = T::TN + wb * T::FB * 32 + j * 32 + r32;
    boff[j] = row * T::CH;
    bsw[j] = (row >> 1) & 7;
  }
  u32x4 af[2][T::FN], bf[2][T::FB];
  auto rd = [&](int buf, int q, int set) {
    const u32x4 *L = lds + buf * T::STAGE;
#pragma unroll
    for (int i = 0; i < T::FN; ++i) af[set][i] = L[aoff[i] + ((2 * q + h) ^ asw[i])];
#pragma unroll
    for (int j = 0; j < T::FB; ++j) bf[set][j] = L[boff[j] + ((2 * q + h) ^ bsw[j])];
  };

  if (!FIRST_STAGED) issue(0, 0);
  __builtin_amdgcn_s_waitcnt(0);  // this wavefront's loads of slice 0 have landed ...
  __syncthreads();                // ... and everyone's
  if (nslices > 1) issue(1, 1);
  rd(0, 0, 0);
  for (int s = 0; s < nslices; ++s) {
    const int buf = s & 1;
#pragma unroll
    for (int q = 0; q < QS; ++q) {
      const int cur = q & 1;
      if (q + 1 < QS) {
        rd(buf, q + 1, cur ^ 1);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < NM; ++t) Op::mma(af[cur][t / T::FB], bf[cur][t % T::FB], acc[t / T::FB][t % T::FB]);
        __builtin_amdgcn_sched_barrier(0);
      } else {
#pragma unroll
        for (int t = 0; t < SPLIT; ++t) Op::mma(af[cur][t / T::FB], bf[cur][t % T::FB], acc[t / T::FB][t % T::FB]);
        __builtin_amdgcn_sched_barrier(0);
        if (s + 1 < nslices) {
          // Slice s+1 (the only one in flight) must have landed everywhere, and
          // every wavefront has read all of slice s (its last fragments are in
          // registers), so slice s+2 may overwrite buffer s & 1.
          __builtin_amdgcn_s_waitcnt(0);
          __syncthreads();
          rd(buf ^ 1, 0, cur ^ 1);
          __builtin_amdgcn_sched_barrier(0);
          if (s + 2 < nslices) issue(s + 2, buf);
          __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int t = SPLIT; t < NM; ++t) Op::mma(af[cur][t / T::FB], bf[cur][t % T::FB], acc[t / T::FB][t % T::FB]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  __syncthreads();
}

// Serial main loop (FP32 operands): acc += P_tile * Q_tile^T over `nslices` K
// slices of 128 bytes. P points at the tile's first row, rows `prs` chunks apart; likewise Q.
// Wavefront w stages rows 8 (i NW + w) .. +7 of every slice with its load i: a
// load writes 64 consecutive LDS chunks (lane l -> chunk l), so lane l fetches
// row 8 (i NW + w) + l/8, chunk lds_slot(row, l mod 8). The loads of slice s+1
// are issued right after the barrier that opens slice s and land while slice s
// is multiplied. Each step's fragments are read and then multiplied. The FP32
// product is bound by its MFMAs (four per 16-byte chunk), and there this loop
// is faster than the pipelined one above. Ends with a barrier, so the caller may
// reuse the LDS.
template <class Op, class T>
__device__ inline void mainloop_serial(const u32x4 *__restrict__ P, int64_t prs, const u32x4 *__restrict__ Q,
                                       int64_t qrs, int nslices, u32x4 *lds, f32x16 (&acc)[T::FN][T::FB]) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wn = wave % T::WN, wb = wave / T::WN;
  const int h = lane >> 5, r32 = lane & 31;

#pragma unroll
  for (int i = 0; i < T::FN; ++i)
#pragma unroll
    for (int j = 0; j < T::FB; ++j) acc[i][j] = f32x16{};

  // Source of this lane's chunk for each of its loads, at slice 0.
  const u32x4 *src[T::LPW];
#pragma unroll
  for (int i = 0; i < T::LPW; ++i) {
    const int row = (i * T::NW + wave) * 8 + (lane >> 3);
    const int c = lds_slot(row, lane & 7);  // the slot map is an involution
    src[i] = row < T::TN ? P + (int64_t)row * prs + c : Q + (int64_t)(row - T::TN) * qrs + c;
  }
#pragma unroll
  for (int i = 0; i < T::LPW; ++i)
    __builtin_amdgcn_global_load_lds(reinterpret_cast<const void *>(src[i]),
                                     (lds_void_t *)(lds + (i * T::NW + wave) * 64), 16, 0, 0);

  // LDS offsets (chunks) of this lane's fragment rows and their slot swizzles.
  int aoff[T::FN], asw[T::FN], boff[T::FB], bsw[T::FB];
#pragma unroll
  for (int i = 0; i < T::FN; ++i) {
    const int row = wn * T::FN * 32 + i * 32 + r32;
    aoff[i] = row * T::CH;
    asw[i] = (row >> 1) & 7;
  }
#pragma unroll
  for (int j = 0; j < T::FB; ++j) {
    const int row = T::TN + wb * T::FB * 32 + j * 32 + r32;
    boff[j] = row * T::CH;
    bsw[j] = (row >> 1) & 7;
  }

  for (int s = 0; s < nslices; ++s) {
    const int buf = s & 1;
    __builtin_amdgcn_s_waitcnt(0);  // this wavefront's loads of slice s have landed ...
    __syncthreads();                // ... and everyone's; slice s-1 is no longer read
    if (s + 1 < nslices) {
#pragma unroll
      for (int i = 0; i < T::LPW; ++i)
        __builtin_amdgcn_global_load_lds(reinterpret_cast<const void *>(src[i] + (int64_t)(s + 1) * T::CH),
                                         (lds_void_t *)(lds + (buf ^ 1) * T::STAGE + (i * T::NW + wave) * 64),
                                         16, 0, 0);
    }
    const u32x4 *L = lds + buf * T::STAGE;
#pragma unroll
    for (int q = 0; q < T::CH / 2; ++q) {
      u32x4 af[T::FN], bf[T::FB];
#pragma unroll
      for (int i = 0; i < T::FN; ++i) af[i] = L[aoff[i] + ((2 * q + h) ^ asw[i])];
#pragma unroll
      for (int j = 0; j < T::FB; ++j) bf[j] = L[boff[j] + ((2 * q + h) ^ bsw[j])];
#pragma unroll
      for (int i = 0; i < T::FN; ++i)
#pragma unroll
        for (int j = 0; j < T::FB; ++j) Op::mma(af[i], bf[j], acc[i][j]);
    }
  }
  __syncthreads();
}

// The main loop of every product: pipelined for 16-bit operands, serial for FP32.
template <class Op, class T>
__device__ inline void mainloop(const u32x4 *__restrict__ P, int64_t prs, const u32x4 *__restrict__ Q,
                                int64_t qrs, int nslices, u32x4 *lds, f32x16 (&acc)[T::FN][T::FB]) {
  if constexpr (sizeof(typename Op::elem) == 4)
    mainloop_serial<Op, T>(P, prs, Q, qrs, nslices, lds, acc);
  else
    mainloop_pipelined<Op, T>(P, prs, Q, qrs, nslices, lds, acc);
}

// Row of a 32x32 MFMA result held by (lane, register r): the column is lane % 32.
__device__ inline int frag_row(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

}  // namespace
}  // namespace bomp
