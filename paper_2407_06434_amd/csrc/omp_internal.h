// Internal declarations shared by the host runtime and the kernels of
// libbatched_omp.so. Not part of the public ABI (see include/batched_omp.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <functional>
#include <string>

namespace bomp {

// Padding of the three problem dimensions. The kernels read padded, zero-filled
// copies so that no tile needs a bounds check:
//   Mp  signal length, multiple of the GEMM K stage (64 BF16 / 32 FP32 elements)
//   Np  atoms, multiple of the GEMM atom tile
//   Bp  signals, multiple of the GEMM signal tile
constexpr int KPAD = 64;
constexpr int NPAD = 256;
constexpr int BPAD = 256;

// Near-tie flagging: a step is flagged when the second best atom's score is
// within this fraction of the best one's.
constexpr double TIE_REL = 1e-5;

// Squared dependency threshold on the Cholesky pivot: an atom whose distance to
// the span of the support is at most 1e-3 of its norm is not appended.
constexpr double DEP_TOL2 = 1e-6;

// Internal per-signal flag bits (the low byte holds the public OMP_SIG_* bits).
constexpr int FLAG_DONE = 1 << 16;  // the signal takes no further picks
constexpr int FLAG_NEWX = 1 << 17;  // coefficients changed: the residual kernel must run
constexpr int FLAG_EMPTY = 1 << 18; // slot scheduler: the slot holds no signal (its last one is out)

// The residual is computed in up to this many slices of M (one per XCD).
constexpr int NSLICE_MAX = 8;

constexpr uint32_t DICT_MAGIC = 0x4f4d5044u;  // "OMPD"

// Correlation tile configurations 1..MAX_TILE_CFG (0 = chosen by shape).
constexpr int MAX_TILE_CFG = 4;

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Device-side view of a prepared dictionary (all pointers into one allocation).
struct DictView {
  int64_t M, N, Mp, Np;
  double *nu2;     // [Np]   ||a_n||^2 in FP64 (0 for padding atoms)
  float *inv_nu;   // [Np]   1/||a_n|| in FP32 (0 for zero-norm and padding atoms)
  float *A32;      // [Np][Mp] zero-padded FP32 copy of A, atom-major
  float *G;        // [Np][Np] Gram matrix A^T A, FP32, row-major
  uint16_t *A16;   // [Np][Mp] BF16 (round to nearest even) copy of A, or nullptr
  float *aerr;     // [Np]   ||a_n - bf16(a_n)|| / ||a_n|| (BF16 form), 0 for zero atoms
  float *aerr_max; // [1]    max_n aerr[n] (BF16 form)
  double *G64;     // [Np][Np] Gram matrix in FP64 (FP64 form), or nullptr
  double *inv_nu64;// [Np]   1/||a_n|| in FP64 (FP64 form), or nullptr
  // FP16 form: A16 holds fp16(sigma_n a_n), sigma_n a power of two with max |sigma_n a_n|
  // in (1/2, 1], and the product's epilogue scores by inv_nu_h[n] = 1/(sigma_n ||a_n||)
  float *inv_nu_h; // [Np] or nullptr (the other forms score by inv_nu)
};

// The forms whose correlation product runs on 16-bit copies (BF16, FP16) and whose
// pick is the certified exact re-score.
__host__ __device__ inline bool is_half(int precision) { return precision == 1 || precision == 3; }

size_t dict_bytes(int64_t M, int64_t N, int precision);
DictView dict_view(void *mem, int64_t M, int64_t N, int precision);

// Device-side view of the solver workspace.
struct WorkView {
  int64_t B, Bp, Mp, Np;
  int S;          // sparsity cap
  int tile_cfg;      // correlation tile configuration (CorrGeom::cfg)
  int ntile;         // number of atom tiles of the correlation product
  int ncand;         // keys per (signal, tile) written by the select epilogue
  int tile_atoms;    // atoms per tile
  int wave_atoms;    // atom stride between the wavefront rows of a tile (FN * 32)
  int sub_frags;     // BF16 form: 32-row fragments per subgroup
  int subs_per_half; // BF16 form: subgroups per wavefront half
  float *Yp;      // [Bp][Mp] zero-padded copy of Y
  float *R32;     // [Bp][Mp] residual, FP32
  uint16_t *R16;  // [Bp][Mp] residual, BF16 (BF16 form) or FP16 scaled by rscale (FP16 form)
  int fp16;       // 1: R16 and A16 hold FP16 (FP16 form)
  float *rscale;  // [Bp] FP16 form: power-of-two scale of the residual stored in R16 (else nullptr)
  float *rscale_next; // [Bp] FP16 form: the scale the residual kernel stores the next residual with
  uint64_t *part; // [Bp][ntile*ncand] packed (score, index) keys from the GEMM epilogue
  uint32_t *mask; // [Bp][Np/32] selected-atom bitmask
  int32_t *k;     // [Bp] atoms selected so far
  int32_t *flags; // [Bp] FLAG_DONE | OMP_SIG_* bits
  double *pnorm; // [Bp][NSLICE_MAX] ||r||^2 of each slice of the current residual
  double *pdelta;// [Bp][NSLICE_MAX] ||r - bf16(r)||^2 of each slice (BF16 form)
  int nslice;     // slices of M used by the residual kernel (1 or NSLICE_MAX)
  int slice_len;  // floats per slice (Mp / nslice, a multiple of 4)
  int32_t *Sb;    // [Bp] per-signal sparsity cap
  float *epsb;    // [Bp] per-signal tolerance (>= 0)
  int32_t *sup;   // [Bp][S] support in selection order
  float *u;       // [Bp][S] forward-solve vector V^{-1} A_S^T y
  float *xh;      // [Bp][S] current coefficients
  int64_t vstride; // floats per signal in V: S(S+1)/2 rounded up to a multiple of 4
  float *V;       // [Bp][vstride] packed lower-triangular Cholesky factor, row by row
  int gram_fly;   // 1: Gram rows of the picks computed from the atoms (ablation A2)
  int refactor;   // 1: the factor of A_S^T A_S rebuilt from the Gram at every step (ablation A3)
  int gram_dom;   // 1: Gram-domain form (correlations from P and G, no residual vectors)
  float *P;       // [Bp][Np] Gram-domain form: P = Y A^T, the correlations of y (else nullptr)
  float *Pk;      // [pchunks][Bp][Np] split-K partial products of P (pchunks > 1), else nullptr
  int pchunks;    // K chunks of the P product (1: no split)
  int flag_ties;  // 1: near-tie flagging (the select stages keep the second best atom too)
  int v0;         // 1: Algorithm v0 (inverse Cholesky factor F in V, D = A^T Q, correlations in P)
  int fuse_res;   // 1: the solve forms each updated signal's residual itself (norms in slice 0; no residual kernel)
  float *D;       // [Bp][S][Np] v0: D's columns d_j = A^T q_j, each Np long (else nullptr)
  // FP64 form (Algorithm v0 in FP64; else nullptr)
  double *P64;    // [Bp][Np] correlations c = A^T r
  double *D64;    // [Bp][S][Np] columns of D
  double *V64;    // [Bp][vstride] inverse factor F, packed by columns
  double *u64;    // [Bp][S] u = Q^T y
};

// Gram-domain select: the atoms are split into this many contiguous slices, one
// per XCD, each giving one key per signal.
constexpr int GSLICE = 8;

// K chunks of the Gram-domain form's product P = Y A^T on 128 x 128 tiles: split
// until about 512 workgroups run, each chunk keeping at least 16 K slices of 32
// floats (so every chunk is non-empty), at most 8 chunks.
inline int project_chunks(int64_t Bp, int64_t Np, int64_t Mp) {
  const int64_t tiles = (Bp / 128) * (Np / 128), nsl = Mp / 32;
  int ks = 1;
  while (ks < 8 && tiles * ks < 512 && nsl / (ks * 2) >= 16) ks *= 2;
  return ks;
}

// `gram_dom` adds the Gram-domain form's P buffer to the layout; `ties` (near-tie
// flagging) doubles the FP32, Gram-domain and v0 select keys (best and second
// best); `v0` adds P and the D columns of Algorithm v0.
size_t work_bytes(int64_t M, int64_t N, int64_t B, int S, int precision, int cfg, bool gram_dom = false,
                  bool ties = false, bool v0 = false);
WorkView work_view(void *mem, int64_t M, int64_t N, int64_t B, int S, int precision, int cfg,
                   bool gram_dom = false, bool ties = false, bool v0 = false);

// ---- the solve kernel's LDS (shared by its launcher and the entry points'
// validation) ---------------------------------------------------------------
// Subgroups listed as possibly open by the BF16 pick (beyond this the bounding
// keys are scanned).
constexpr int MAYBE_CAP = 32;
// Ints of the BF16 pick's candidate list (room for every key, a multiple of 4).
__host__ __device__ inline int64_t solve_cand_len(int64_t nkeys) { return (nkeys + 3) / 4 * 4; }
// Per wavefront: the packed factor (vstride floats), then in the BF16 form the
// candidate list and the possibly-open list, in 4-byte words.
__host__ __device__ inline int64_t solve_list_words(int64_t nkeys, bool bf16) {
  return bf16 ? solve_cand_len(nkeys) + MAYBE_CAP : 0;
}
__host__ __device__ inline int64_t solve_list_len(const WorkView &w) {
  return solve_list_words((int64_t)w.ntile * w.ncand, w.R16 != nullptr);  // 16-bit forms keep the lists
}
__host__ __device__ inline size_t solve_lds_per_wave(const WorkView &w) {
  return (size_t)(w.vstride + solve_list_len(w)) * 4;
}
constexpr int SOLVE_WAVES = 4;              // wavefronts (signals) per solve block, at most
constexpr size_t LDS_LIMIT = 160 * 1024;    // LDS of one gfx950 workgroup
// Wavefronts per solve block whose LDS fits (0: not even one).
inline int solve_waves_for(int64_t vstride, int64_t nkeys, bool bf16) {
  const size_t per = (size_t)(vstride + solve_list_words(nkeys, bf16)) * 4;
  int nw = SOLVE_WAVES;
  while (nw > 0 && per * (size_t)nw > LDS_LIMIT) --nw;
  return nw;
}
inline int solve_waves(const WorkView &w) {
  return solve_waves_for(w.vstride, (int64_t)w.ntile * w.ncand, w.R16 != nullptr);
}
// Whether one solve wavefront's LDS fits for this problem (else the entry
// points answer OMP_ENOTSUPP before launching anything).
bool solve_fits(int64_t M, int64_t N, int64_t B, int S, int precision, int cfg);

// Slot scheduler (uneven batches): the workspace's B columns are slots that
// signals pass through. When a slot's signal stops, the solve kernel writes that
// signal's outputs and admits the next waiting signal into the slot.
struct SlotView {
  int32_t *sig;          // [slots] signal held by each slot, -1 when empty
  int32_t *ctrl;         // [0] next signal to admit, [1] signals finished
  const float *Y;        // the problem's signals, y_i = Y[i*ldy ..]
  int64_t ldy, M, nsig;
  const int32_t *S_per;  // optional per-signal sparsity caps
  const float *eps_per;  // optional per-signal tolerances
  float eps;
  int32_t *support_out;  // [nsig][S]
  float *coef_out;       // [nsig][S]
  int32_t *status_out;   // optional [nsig]
  float *rnorm_out;      // optional [nsig]
};

// ---- host helpers shared by the entry points --------------------------------
// omp_solve with the workspace given explicitly (omp_solve passes opts'
// workspace, the allocation-free entry point its static scratch). `direct`
// launches the kernels one by one (no graph capture or instantiation).
int solve_impl(const float *A, int64_t M, int64_t N, int64_t lda, const float *Y, int64_t B, int64_t ldy,
               int32_t S, float eps, float *X_out, int32_t *support_out, const struct omp_opts *opts,
               void *stream, void *workspace, size_t workspace_bytes, bool direct);
size_t solve_bytes(int64_t M, int64_t N, int64_t B, int32_t S, const struct omp_opts *opts);
bool aligned(const void *p, size_t a);
bool valid_precision(int precision);         // one of the OMP_PREC_* values
bool dims_ok(int64_t M, int64_t N);          // sizes the padded buffers can hold
int device_error(hipError_t e);              // records e for omp_last_hip_error, returns OMP_EDEVICE
int check_device();                          // OMP_OK on a gfx950 device
constexpr size_t WS_ALIGN = 256;

// Enqueues on `st` the hipGraph cached under `key` for the current device; on
// the first use of a key, `body` enqueues the work on the capture stream it is
// given and is captured. Serialized with the uneven-batch entry points.
hipError_t graph_launch_cached(const std::string &key, const std::function<hipError_t(hipStream_t)> &body,
                               hipStream_t st);

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
// Gram-domain form: P = R32 A32^T (R32 holds y after the init) through the FP32 MFMA product.
hipError_t launch_project(const DictView &d, const WorkView &w, hipStream_t st);
// Gram-domain form: c = P - G[:, S] x for every live signal, its best atom's key -> w.part[b].
hipError_t launch_gram_select(const DictView &d, const WorkView &w, hipStream_t st);
// One OMP step per live signal: stop test, pick, Cholesky append, both solves.
hipError_t launch_solve(const DictView &d, const WorkView &w, int precision, hipStream_t st);
// Whether the solve holds the residual in registers (its own variant, which does not fuse the residual).
bool solve_rr(const DictView &d, const WorkView &w);
bool residual_in_solve(const DictView &d, int64_t B);
// Residual r = y - A_S x (and its BF16 copy and per-slice norms) for the signals just updated;
// kbound is an upper bound on every signal's support size (the number of steps taken so far).
hipError_t launch_residual(const DictView &d, const WorkView &w, int precision, int kbound, hipStream_t st);
// Slot scheduler: fill the slots with the first signals and reset the queue.
hipError_t launch_init_slots(const WorkView &w, const SlotView &sv, hipStream_t st);
// One OMP step per occupied slot; stopped signals are written out and replaced.
hipError_t launch_solve_slots(const DictView &d, const WorkView &w, const SlotView &sv, int precision,
                              hipStream_t st);
// Residual with an explicit number of lanes per signal (power of two, 1..64; 0 = by shape).
hipError_t launch_residual_lp(const DictView &d, const WorkView &w, int precision, int lanes, int kbound,
                              hipStream_t st);
// Dense X [nsig][N] from compact supports and coefficients.
hipError_t launch_densify(const int32_t *support, const float *coef, int64_t nsig, int S, int64_t N,
                          float *X_out, hipStream_t st);
// Raise the LDS limits of every kernel a solve with these views launches (no launch).
hipError_t prepare_kernels(const DictView &d, const WorkView &w, int precision, int lanes);
hipError_t prepare_corr(const DictView &d, const WorkView &w, int precision);

// Algorithm v0 (FP32): each signal's first pick from P = A^T y; one step (pick, pivot,
// new columns of F and D, correlation update, next pick) per live signal; x = F u.
hipError_t launch_v0_first(const DictView &d, const WorkView &w, hipStream_t st);
hipError_t launch_v0_step(const DictView &d, const WorkView &w, hipStream_t st);
hipError_t launch_v0_coef(const WorkView &w, hipStream_t st);
// FP64 form: G64 = A32 A32^T and P64 = Yp A32^T (exact products, FP64 sums), then
// the v0 kernels in FP64.
hipError_t launch_gram64(const DictView &d, hipStream_t st);
hipError_t launch_project64(const DictView &d, const WorkView &w, hipStream_t st);
hipError_t launch_v0_first64(const DictView &d, const WorkView &w, hipStream_t st);
hipError_t launch_v0_step64(const DictView &d, const WorkView &w, hipStream_t st);
hipError_t launch_v0_coef64(const WorkView &w, hipStream_t st);

// Outputs: dense X, support, coefficients, status, residual norm.
hipError_t launch_finalize(const DictView &d, const WorkView &w, float *X_out,
                           int32_t *support_out, float *coef_out, int32_t *status_out,
                           float *rnorm_out, hipStream_t st);

// Keys kept per subgroup by the BF16 epilogue (best, second, third).
constexpr int NKEEP = 3;

// Tile configuration and output structure of the correlation product.
//   FP32: one 64-bit key per (signal, tile): the tile's best atom.
//   BF16: NKEEP 32-bit keys (best BF16 scores, descending) per (signal, subgroup). The
//         lane holding signal j in wavefront row wn, half h (lane / 32) owns,
//         for fragment i, the atoms 32 i + 8 g + 4 h + e (g, e < 4) of its rows;
//         subgroup ig of that lane is fragments ig*sub_frags .. +sub_frags-1.
//         Key slot in the tile: ((wn * subs_per_half + ig) * 2 + h) * NKEEP + {0..NKEEP-1};
//         atom: t*tile_atoms + wn*wave_atoms + 32 (ig*sub_frags + i') + 8 g + 4 h + e.
struct CorrGeom {
  int cfg;  // tile configuration 1..4 (see the correlation kernels)
  int tile_atoms, tile_signals;
  int keys_per_tile;
  int wave_atoms;
  int sub_frags;
  int subs_per_half;
};
// cfg 0 picks by shape: 256 x 256 tiles when that still gives about one tile per CU.
// `ties`: the FP32 epilogue writes two keys per (signal, tile), best and second best.
CorrGeom corr_geometry(int precision, int64_t Np, int64_t Bp, int cfg, bool ties = false);

}  // namespace bomp
