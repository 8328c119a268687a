// Internal declarations shared by the host runtime and the kernels of
// libbatched_omp.so. Not part of the public ABI (see include/batched_omp.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace bomp {

// Padding of the three problem dimensions. The kernels read padded, zero-filled
// copies so that no tile needs a bounds check:
//   Mp  signal length, multiple of the GEMM K stage (64 BF16 / 32 FP32 elements)
//   Np  atoms, multiple of the GEMM atom tile
//   Bp  signals, multiple of the GEMM signal tile
constexpr int KPAD = 64;
constexpr int NPAD = 128;
constexpr int BPAD = 128;

// Squared dependency threshold on the Cholesky pivot: an atom whose distance to
// the span of the support is at most 1e-3 of its norm is not appended.
constexpr double DEP_TOL2 = 1e-6;

// Internal per-signal flag bits (the low byte holds the public OMP_SIG_* bits).
constexpr int FLAG_DONE = 1 << 16;

constexpr uint32_t DICT_MAGIC = 0x4f4d5044u;  // "OMPD"

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Device-side view of a prepared dictionary (all pointers into one allocation).
struct DictView {
  int64_t M, N, Mp, Np;
  double *nu2;     // [Np]   ||a_n||^2 in FP64 (0 for padding atoms)
  float *inv_nu;   // [Np]   1/||a_n|| in FP32 (0 for zero-norm and padding atoms)
  float *A32;      // [Np][Mp] zero-padded FP32 copy of A, atom-major
  float *G;        // [Np][Np] Gram matrix A^T A, FP32, row-major
  uint16_t *A16;   // [Np][Mp] BF16 (round to nearest even) copy of A, or nullptr
};

size_t dict_bytes(int64_t M, int64_t N, int precision);
DictView dict_view(void *mem, int64_t M, int64_t N, int precision);

// Device-side view of the solver workspace.
struct WorkView {
  int64_t B, Bp, Mp, Np;
  int S;          // sparsity cap
  int ntile;      // number of atom tiles of the correlation product
  int ncand;      // keys per (signal, tile) written by the select epilogue
  int sub_atoms;  // BF16 form: wavefront atom stride inside a tile (FN * 32)
  int sub_fn;     // BF16 form: 32-row fragments per wavefront along the atoms
  int tile_atoms; // atoms per tile
  float *Yp;      // [Bp][Mp] zero-padded copy of Y
  float *R32;     // [Bp][Mp] residual, FP32
  uint16_t *R16;  // [Bp][Mp] residual, BF16 (BF16 form only)
  uint64_t *part; // [Bp][ntile*ncand] packed (score, index) keys from the GEMM epilogue
  uint32_t *mask; // [Bp][Np/32] selected-atom bitmask
  int32_t *k;     // [Bp] atoms selected so far
  int32_t *flags; // [Bp] FLAG_DONE | OMP_SIG_* bits
  float *rn;      // [Bp] current ||r||
  int32_t *Sb;    // [Bp] per-signal sparsity cap
  float *epsb;    // [Bp] per-signal tolerance (>= 0)
  int32_t *sup;   // [Bp][S] support in selection order
  float *u;       // [Bp][S] forward-solve vector V^{-1} A_S^T y
  float *xh;      // [Bp][S] current coefficients
  float *V;       // [Bp][S(S+1)/2] packed lower-triangular Cholesky factor, row by row
};

size_t work_bytes(int64_t M, int64_t N, int64_t B, int S, int precision);
WorkView work_view(void *mem, int64_t M, int64_t N, int64_t B, int S, int precision);

// ---- launchers (all enqueue on `st`, return the launch status) -------------

// Atom norms, padded FP32 copy and (optionally) BF16 copy of A.
hipError_t launch_dict_prep(const float *A, int64_t lda, const DictView &d, hipStream_t st);
// G = A32 A32^T through the FP32 MFMA product.
hipError_t launch_gram(const DictView &d, hipStream_t st);

// Start of a solve: padded copies of Y, R = Y, norms, stop tests, state reset.
hipError_t launch_init(const float *Y, int64_t ldy, const int32_t *S_per, const float *eps_per,
                       float eps, const DictView &d, const WorkView &w, int precision,
                       hipStream_t st);
// Correlation A^T R with the fused select epilogue -> w.part.
hipError_t launch_corr_select(const DictView &d, const WorkView &w, int precision, hipStream_t st);
// One OMP step per active signal: merge, Cholesky append, solves, residual, stop test.
hipError_t launch_update(const DictView &d, const WorkView &w, int precision, hipStream_t st);
// Outputs: dense X, support, coefficients, status, residual norm.
hipError_t launch_finalize(const DictView &d, const WorkView &w, float *X_out,
                           int32_t *support_out, float *coef_out, int32_t *status_out,
                           float *rnorm_out, hipStream_t st);

// Shape of the correlation product's output for a precision.
//   FP32: one key per (signal, tile): the tile's best atom.
//   BF16: two keys per (signal, subgroup): the best and second best BF16 scores
//         of the subgroup; subgroup (wn, h) of tile t holds the atoms
//         t*tile_atoms + wn*sub_atoms + 32 i + 8 g + 4 h + e
//         for i < sub_fn, g < 4, e < 4 (the rows one lane holds in the MFMA layout).
struct CorrGeom {
  int tile_atoms;
  int keys_per_tile;
  int sub_atoms;
  int sub_fn;
};
CorrGeom corr_geometry(int precision);

}  // namespace bomp
