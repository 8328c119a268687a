/*
 * batched_omp.h — C ABI of the MI355X (gfx950) batched Orthogonal Matching
 * Pursuit library, libbatched_omp.so.
 *
 * The problem (Section 1 of Lubonja, Praesius & Tran, "A Practical
 * GPU-Accelerated Implementation of Orthogonal Matching Pursuit"): given a
 * dictionary A (M x N, atoms a_n as columns), a batch of B measurement vectors
 * y_b (length M), a sparsity level S and an optional tolerance eps, find for
 * every b an S-sparse x_b with y_b ~ A x_b by Algorithm 1 (OMP):
 *
 *   r_0 = y, support empty; for k = 1..S:
 *     n* = argmax_n |<r_{k-1}, a_n>| / ||a_n||     (not yet selected atoms)
 *     support_k = support_{k-1} + n*
 *     x_k = argmin_x ||y - A_support x||
 *     r_k = y - A_support x_k
 *   stop as soon as ||r_k|| <= eps.
 *
 * The library runs the whole iteration on the GPU: the correlation A^T R for
 * the batch as one matrix product (Section 3.2), the per-signal argmax fused
 * into that product's epilogue (Section 3.4), the least squares by the
 * progressive Cholesky update of Section 2.2 (Eqs. 4-5) driven by the
 * precomputed Gram matrix A^T A (Section 2.2, last paragraph), and the residual
 * recomputed from y at every step.
 *
 * Conventions for every entry point:
 *   - All array pointers are DEVICE pointers on the caller's current HIP
 *     device, unless a comment says "host".
 *   - The caller allocates and owns every buffer (inputs, outputs, workspace,
 *     dictionary memory). The library allocates no device memory (the one
 *     static array of omp_solve_noalloc aside).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls only enqueue work; results are valid once the stream has reached
 *     the enqueued work (e.g. after hipStreamSynchronize).
 *   - A negative return value means nothing was enqueued, except OMP_EDEVICE,
 *     which means a HIP call failed part-way (omp_last_hip_error() holds the
 *     hipError_t). Per-signal numerical outcomes are status bits, not errors.
 *   - Calls are re-entrant; concurrent calls must use distinct workspaces.
 *   - For fixed inputs, options and device, results are bit-identical from
 *     call to call.
 */
#ifndef BATCHED_OMP_H
#define BATCHED_OMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define OMP_OK 0
#define OMP_EINVAL (-1)     /* invalid argument (sizes, null pointers, alignment, NaN eps) */
#define OMP_EWORKSPACE (-2) /* workspace or dictionary memory missing / too small / misaligned */
#define OMP_EDEVICE (-3)    /* a HIP runtime call failed, or the device is not gfx950 */
#define OMP_ENOTSUPP (-4)   /* valid request beyond the library's limits (e.g. S > OMP_MAX_S) */

/* ---- limits ------------------------------------------------------------ */
#define OMP_MAX_S 256 /* largest sparsity level S (the Cholesky factor lives in LDS) */

/* ---- precision of the correlation product ------------------------------ */
#define OMP_PREC_FP32 0 /* A^T R with FP32 inputs and FP32 accumulation */
#define OMP_PREC_BF16 1 /* A^T R in BF16 with FP32 accumulation; the leading candidates
                           are re-scored in FP32 so that the pick is the FP32 argmax */
#define OMP_PREC_FP16 3 /* as OMP_PREC_BF16 with FP16 copies: each atom stored as fp16(sigma_n a_n) and
                           each residual as fp16(sigma_b r), sigma power-of-two scales that keep
                           every stored value in [-1, 1]; the same certified exact re-score, with
                           FP16's 8x finer rounding in the bound */
#define OMP_PREC_FP64 2 /* everything in FP64 (the FP32 inputs are exact in FP64): the
                           paper's Algorithm v0 (see omp_opts_t.v0) with FP64 correlations,
                           Gram matrix, inverse factor and coefficients; the outputs are the
                           FP64 results rounded once to FP32. Not with gram_domain = 1,
                           refactor or gram_on_the_fly; not in omp_solve_multi. */

/* ---- per-signal status bits (status_out) -------------------------------
 * status_out[b] = (k_b << 8) | bits, k_b = number of atoms selected. */
#define OMP_SIG_EPS 1        /* stopped because ||r|| <= eps_b */
#define OMP_SIG_SMAX 2       /* stopped because k_b reached S_b */
#define OMP_SIG_DEPENDENT 4  /* the picked atom was (numerically) in the span of the support:
                                Cholesky pivot d^2 <= 1e-6 ||a_n*||^2; it was not added */
#define OMP_SIG_NONFINITE 8  /* y_b held a NaN or Inf; nothing was selected, x_b = 0 */
#define OMP_SIG_NEARTIE 16   /* with opts.flag_near_ties: at some step the second best atom
                                scored within 1e-5 (relative) of the picked one */
#define OMP_SIG_EXHAUSTED 32 /* no selectable atom was left (all selected or zero norm) */
#define OMP_SIG_WIDENED 64   /* BF16 form: the FP32 re-score needed the widened candidate set */
#define OMP_SIG_LEARNED 128  /* omp_learned_solve: the network's proposal was accepted (no OMP run) */

/* ---- prepared dictionary ------------------------------------------------
 * Everything about A that does not depend on the signals (Section 2.2: the
 * Gram matrix A^T A is computed once and shared between batches):
 *   atom norms ||a_n||^2 in FP64 and 1/||a_n|| in FP32, a zero-padded FP32
 *   copy of A, the FP32 Gram matrix, and (BF16 form) a BF16 copy of A rounded
 *   to nearest even.
 * The struct lives in host memory and is filled by omp_dict_init; its `mem`
 * points to caller-owned device memory of at least omp_dict_size() bytes. */
typedef struct omp_dict {
  uint32_t magic;    /* set by omp_dict_init */
  int32_t precision; /* OMP_PREC_* the dictionary was prepared for */
  int64_t M, N;      /* dictionary shape */
  int64_t Mp, Np;    /* padded shape used by the kernels */
  const float *A;    /* the caller's A it was prepared from (device) */
  void *mem;         /* device memory holding the prepared data */
  size_t bytes;
} omp_dict_t;

/* Bytes of device memory omp_dict_init needs for an M x N dictionary. */
size_t omp_dict_size(int64_t M, int64_t N, int32_t precision);

/* Prepare a dictionary.
 *   A      device, atom-major: atom n occupies A[n*lda .. n*lda+M-1] (lda >= M).
 *          (Equivalently A is M x N column-major.) Read only.
 *   mem    device, >= omp_dict_size(M, N, precision) bytes, 256-byte aligned.
 *   dict   host struct, filled on success.
 * Enqueued on `stream`. A must stay unchanged while the dictionary is used. */
int omp_dict_init(omp_dict_t *dict, const float *A, int64_t M, int64_t N, int64_t lda,
                  int32_t precision, void *mem, size_t bytes, void *stream);

/* ---- options ------------------------------------------------------------ */
typedef struct omp_opts {
  int32_t precision;            /* OMP_PREC_FP32 (default) or OMP_PREC_BF16 */
  int32_t tile_config;          /* correlation tiles (atoms x signals): 0 = chosen by shape
                                   (default), 1 = 128x128, 2 = 256x256 (4 wavefronts),
                                   3 = 256x256 (8 wavefronts), 4 = 256x128 */
  const int32_t *S_per_signal;  /* device [B], optional: per-signal S_b in 0..S */
  const float *eps_per_signal;  /* device [B], optional: per-signal eps_b (replaces eps) */
  int32_t *status_out;          /* device [B], optional: (k_b << 8) | OMP_SIG_* bits */
  float *rnorm_out;             /* device [B], optional: final ||r_b|| */
  float *coef_out;              /* device [B][S], optional: coefficients aligned with
                                   support_out (0 where support_out is -1) */
  const omp_dict_t *dict;       /* host, optional: a dictionary prepared for the same A, M, N,
                                   and precision; NULL prepares one inside the workspace */
  void *workspace;              /* device, required: >= omp_workspace_size(...) bytes,
                                   256-byte aligned; contents on entry are ignored */
  size_t workspace_bytes;
  float *phase_ms;              /* HOST [OMP_NPHASE], optional profiling: when set, every kernel
                                   launch is bracketed by hipEvents on `stream`, the call waits for
                                   the stream, and phase_ms[p] receives the summed kernel time (ms)
                                   of phase p; NULL (default) keeps the call asynchronous */
  int32_t *phase_launches;      /* HOST [OMP_NPHASE], optional: launches per phase (with phase_ms) */
  int32_t use_graph;            /* 1 (the default of omp_opts_default): the solve's launches are
                                   captured once into a hipGraph, cached per device and per
                                   argument set (every pointer and size of the call), and replayed
                                   with one graph launch; 0: the kernels are launched one by one.
                                   A call with phase_ms set always launches one by one. */
  int32_t gram_on_the_fly;      /* ablation A2 of the paper (measurement only): 1 = the solve
                                   computes the Gram row A_S^T a_n* of each pick from the atoms
                                   (exact products, FP64 sums) instead of reading the prepared
                                   Gram matrix; 0 (default) reads it. Other values: OMP_EINVAL. */
  int32_t refactor;             /* ablation A3 (measurement only): 1 = the solve rebuilds the
                                   Cholesky factor of A_S^T A_S from the Gram entries at every
                                   step (O(k^3)) instead of appending one row to the stored factor
                                   (O(k^2)); u = V^{-1} A_S^T y keeps its incremental form.
                                   0 (default): the progressive update. Other values: OMP_EINVAL. */
  int32_t gram_domain;          /* 1 = Gram-domain form (for tall dictionaries, M >= N, the
                                   scikit-learn Gram solver the paper's Section 2.1 describes):
                                   P = A^T y is formed once per signal by one product, and each
                                   step takes its correlations as c = P - G[:, S] x (O(N k) per
                                   signal, no M-length residual), beta = P[n*], and the residual
                                   norm as ||r||^2 = ||y||^2 - sum_i u_i^2 (FP64 running sum; its
                                   rounding grows as u ||y||^2 / ||r|| when ||r|| << ||y||, so an
                                   eps near the noise floor of y may stop a step apart from the
                                   residual-vector form). Same picks as the default form up to
                                   rounding. FP32 precision only (else OMP_EINVAL); the workspace
                                   grows by (1 + c) * B_pad * N_pad * 4 bytes, c = 0 or the K
                                   chunks (2 to 8) of P's product when the tiles alone would leave
                                   CUs idle (omp_workspace_size with the same opts gives the total).
                                   2 = automatic, FP32 solves only: the Gram-domain form when
                                   4 M >= N, unless B > 4096 and the dictionary is under 1 MiB
                                   in FP32 (4 M N < 2^20 bytes); the residual-vector form
                                   otherwise (the crossover measured on one MI355X; the
                                   scikit-learn choice would be M >= N).
                                   0 (default): residual vectors. Other values: OMP_EINVAL. */
  int32_t flag_near_ties;       /* 1 = record near-ties: status bit OMP_SIG_NEARTIE is set for a
                                   signal when, at any of its steps, the runner-up atom scored
                                   s_2 >= (1 - 1e-5) s_1 (s_1 the picked atom's score; scores as
                                   the form computes them: the FP32 product and the Gram-domain
                                   correlations in FP32, the BF16 form's exact re-score in FP64
                                   sums, which then also re-scores every atom that could come
                                   within 1e-5 of the pick). Two near-tied atoms are ordered by
                                   rounding, so at such a step another implementation may
                                   legitimately pick the other one. Costs a second key per tile
                                   (workspace: omp_workspace_size with the same opts) and wider
                                   re-scoring; for debugging and parity runs. 0 (default): off.
                                   Other values: OMP_EINVAL. */
  int32_t v0;                   /* 1 = the paper's Algorithm v0 (Section 2.3): the inverse
                                   Cholesky factor F_k = V_k^{-T} and D_k = A^T A_k F_k are
                                   updated instead of a Cholesky factor and residual vectors;
                                   c = A^T r is kept per signal from P = A^T y and updated by
                                   one N-long column of D per step (O(N k) bytes per signal and
                                   step, no correlation product); x = F u at the end. FP32 only,
                                   with an FP64 pivot; not with gram_domain = 1, refactor or
                                   gram_on_the_fly (else OMP_EINVAL; gram_domain = 2 is ignored).
                                   The workspace grows by B_pad N_pad (S + 1 + c) 4 bytes (c as
                                   for the Gram-domain form): 4.3 GB for 4096 signals of a
                                   4096-atom dictionary at S = 64. 0 (default): off. */
} omp_opts_t;

/* Phases reported through omp_opts_t.phase_ms. */
#define OMP_PHASE_DICT 0     /* dictionary preparation inside omp_solve (no prepared dictionary) */
#define OMP_PHASE_INIT 1     /* padded copies of Y, norms, stop tests */
#define OMP_PHASE_CORR 2     /* correlation product A^T R with the fused select epilogue */
#define OMP_PHASE_UPDATE 3   /* stop test, pick (BF16: exact re-score), Cholesky append, solves */
#define OMP_PHASE_OUTPUT 4   /* dense X, support, coefficients, status */
#define OMP_PHASE_RESIDUAL 5 /* residual r = y - A_S x, its BF16 copy and norm */
#define OMP_NPHASE 6

/* Fill `opts` with the defaults (FP32, no optional arrays, no workspace). */
void omp_opts_default(omp_opts_t *opts);

/* Bytes of workspace omp_solve needs. `opts` is read for precision and for
 * whether a prepared dictionary is supplied (without one the workspace also
 * holds the dictionary). Returns 0 for invalid sizes. */
size_t omp_workspace_size(int64_t M, int64_t N, int64_t B, int32_t S, const omp_opts_t *opts);

/* Solve B independent OMP problems y_b ~ A x_b (Algorithm 1).
 *   A            device, atom-major [N][lda] FP32 (see omp_dict_init). Must equal opts->dict->A
 *                when a prepared dictionary is given.
 *   M, N         1 <= M, N; S <= min(M, N).
 *   Y            device, signal-major: y_b = Y[b*ldy .. b*ldy+M-1], ldy >= M. Read only.
 *   B            number of signals, B >= 0 (B = 0 enqueues nothing and returns OMP_OK).
 *   S            sparsity level, 1 <= S <= min(M, N, OMP_MAX_S); caps every S_b.
 *   eps          stop signal b when ||r_b|| <= eps (eps <= 0: only when r_b is exactly 0).
 *                Must not be NaN. Ignored when opts->eps_per_signal is given.
 *   X_out        device [B][N] FP32, optional (NULL): the dense solution x_b, zero off the support.
 *   support_out  device [B][S] int32, required: selected atoms in selection order, -1 padded.
 *   opts         host, required (workspace).
 * Ties in the argmax go to the lowest atom index. Atoms of zero norm are never
 * selected. Column norms need not be 1: selection divides by ||a_n||, and x is
 * in the scale of the caller's A (Appendix A of the paper).
 * Returns OMP_OK after enqueueing; OMP_EINVAL / OMP_EWORKSPACE for bad
 * arguments or workspace; OMP_ENOTSUPP when S > OMP_MAX_S or when one signal's
 * solve state (the packed Cholesky factor, S(S+1)/2 floats, plus in the BF16
 * form one word per select key, about 6 N / 64) exceeds the 160 KiB of LDS of
 * a workgroup; OMP_EDEVICE for a HIP error or a device other than gfx950.
 * Nothing is enqueued when the return is not OMP_OK. */
int omp_solve(const float *A, int64_t M, int64_t N, int64_t lda, const float *Y, int64_t B,
              int64_t ldy, int32_t S, float eps, float *X_out, int32_t *support_out,
              const omp_opts_t *opts, void *stream);

/* ---- allocation-free solve ---------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * omp_solve_noalloc is omp_solve (same arguments, same kernels, the same
 * results bit for bit) with the workspace taken from a static device array of
 * OMP_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends. It calls no allocating routine, captures no graph
 * and launches the kernels one by one.
 *   opts->workspace, workspace_bytes and use_graph are ignored; phase_ms and
 *   phase_launches must be NULL (else OMP_EINVAL). Inputs, outputs and the
 *   optional prepared dictionary stay the caller's, as in omp_solve (without a
 *   prepared dictionary the dictionary is prepared inside the array too).
 *   A request whose workspace (omp_workspace_size with the same arguments)
 *   exceeds OMP_NOALLOC_SCRATCH_BYTES returns OMP_ENOTSUPP and enqueues nothing.
 *   Every call on one GPU uses that GPU's one array and leaves its contents
 *   behind (each call initialises what it reads): calls that overlap in time on
 *   one GPU (several streams or host threads) race, and the caller must
 *   serialise them. */
#define OMP_NOALLOC_SCRATCH_BYTES 67108864 /* 64 MiB per GPU */

int omp_solve_noalloc(const float *A, int64_t M, int64_t N, int64_t lda, const float *Y, int64_t B,
                      int64_t ldy, int32_t S, float eps, float *X_out, int32_t *support_out,
                      const omp_opts_t *opts, void *stream);

/* OMP_NOALLOC_SCRATCH_BYTES, as built into the library. */
size_t omp_noalloc_max_bytes(void);

/* ---- uneven batches: several problems, slot scheduling ------------------
 * Batches whose signals stop at very different iterations (per-signal S_b and
 * eps_b, Section 3.5 of the paper: finished signals either stay in the batch or
 * are compacted out) and batches over several dictionaries. Each problem owns
 * `slots` columns of the correlation product. A signal occupies a slot from
 * its admission until it stops; the solve kernel then writes its outputs and
 * admits the next waiting signal into that slot, so the product only spends
 * work on signals still running (plus one iteration per signal for the hand
 * over). The iteration loop of all problems is captured once into a hipGraph
 * (problems on parallel branches) and replayed in chunks until every signal
 * is out; the host reads one counter per problem between chunks.
 * Results per signal are bit-identical to omp_solve with the same precision
 * (a signal's arithmetic does not depend on its slot or neighbours). */
typedef struct omp_problem {
  const omp_dict_t *dict;       /* host, required: prepared dictionary (precision = opts->precision) */
  const float *Y;               /* device [B][ldy]: signals, as in omp_solve */
  int64_t B, ldy;
  int32_t S;                    /* sparsity cap, 1 <= S <= min(M, N, OMP_MAX_S) */
  float eps;                    /* tolerance when eps_per_signal is NULL (not NaN) */
  const int32_t *S_per_signal;  /* device [B], optional */
  const float *eps_per_signal;  /* device [B], optional */
  int32_t *support_out;         /* device [B][S], required */
  float *coef_out;              /* device [B][S], optional */
  float *X_out;                 /* device [B][N], optional: dense x */
  int32_t *status_out;          /* device [B], optional: as in omp_solve */
  float *rnorm_out;             /* device [B], optional */
  /* schedule (0 = chosen by shape; omp_tune writes its choices here) */
  int32_t tile_config;          /* as omp_opts_t.tile_config */
  int32_t slots;                /* signals in flight: a multiple of 256 (rounded up), capped at B */
  int32_t residual_lanes;       /* lanes per signal in the residual kernel: 1, 2, 4, ..., 64 */
} omp_problem_t;

#define OMP_MAX_PROBLEMS 8

typedef struct omp_multi_opts {
  int32_t precision;            /* OMP_PREC_FP32 or OMP_PREC_BF16, for every problem */
  int32_t iters_per_graph;      /* iterations per captured graph chunk; 0 = 8 */
  void *workspace;              /* device, required: >= omp_multi_workspace_size(), 256-byte aligned */
  size_t workspace_bytes;
  float *elapsed_ms;            /* HOST, optional: GPU time of the whole call (events on `stream`) */
  int32_t *iterations;          /* HOST, optional: iterations enqueued (whole chunks) */
} omp_multi_opts_t;

/* Workspace bytes for omp_solve_multi with these problems and schedules
 * (0 for invalid arguments). */
size_t omp_multi_workspace_size(const omp_problem_t *probs, int32_t nprob, const omp_multi_opts_t *opts);

/* Solve nprob (1..OMP_MAX_PROBLEMS) batched OMP problems together (host
 * arrays `probs`). Unlike omp_solve this call WAITS: it returns once every
 * signal is out (the outputs are then complete). Concurrent calls from several
 * host threads are serialized. The library keeps one small pinned host buffer,
 * internal streams at default priority and a cache of captured graphs (keyed
 * by every pointer and size of the call) for the life of the process.
 * Returns OMP_EDEVICE (and leaves the outputs incomplete) if the signals have
 * not all stopped after the bound sum over problems of
 * ceil(B / slots) * (S + 2) + S + 2 iterations, which cannot happen for
 * valid input. */
int omp_solve_multi(const omp_problem_t *probs, int32_t nprob, const omp_multi_opts_t *opts, void *stream);

/* Schedule autotuner: for each problem, times omp_solve_multi on its first
 * `sample` signals (0 = min(B, 8192)) over the candidate tile configurations
 * (1, 3, 4), slot counts (1024 .. 8192) and residual lane counts (by shape and
 * half of it), and writes the fastest choice into probs[p].tile_config, .slots
 * and .residual_lanes. The workspace must hold the largest candidate: size it
 * with omp_multi_workspace_size on problems whose slots field is 8192 (or B).
 * Overwrites the problems' output arrays (sample rows). Waits like
 * omp_solve_multi. */
int omp_tune(omp_problem_t *probs, int32_t nprob, const omp_multi_opts_t *opts, int64_t sample, void *stream);

/* ---- learned support proposal -------------------------------------------
 * An extension of the paper's method: a small network proposes the support
 * and one least-squares solve checks it; plain OMP (omp_solve) takes over for
 * every signal the proposal does not explain.
 *   features  f_n = sqrt(M) |a_n^T y| / (||a_n|| ||y||): Algorithm 1's first
 *             selection statistic, scaled to unit size (BF16 product, so the
 *             dictionary is prepared for OMP_PREC_BF16)
 *   network   h1 = relu(W1 f + b1), h2 = relu(W2 h1 + b2), z = W3 h2 + b3,
 *             BF16 operands, FP32 accumulation, W_l stored [out][in]
 *   proposal  the S atoms with the largest z (ties to the lowest index)
 *   check     least squares on the proposal (Eq. 2) by Cholesky of the Gram
 *             block G[P, P] (Section 2.2), FP64 pivots; accepted when
 *             ||y - A_P x|| <= eps_b and no pivot falls under the dependency
 *             threshold
 *   training  binary cross-entropy with logits against the multi-hot support
 *             of a plain OMP solve, averaged over the batch; Adam (Kingma and
 *             Ba, 2015) on FP32 master weights with BF16 copies.
 * Sizes: n_in = n_out = the dictionary's N, n_hidden; each a multiple of 256. */
typedef struct omp_mlp {
  uint32_t magic;     /* set by omp_mlp_init */
  int32_t n_in, n_hidden, n_out;
  int64_t step;       /* Adam steps taken */
  void *mem;          /* device memory holding weights, BF16 copies and Adam moments */
  size_t bytes;
} omp_mlp_t;

/* Bytes of device memory for a network of these sizes (0 if invalid). */
size_t omp_mlp_size(int32_t n_in, int32_t n_hidden, int32_t n_out);

/* Initialise a network from caller-drawn FP32 parameters (device):
 * params[0..5] = W1 [n_hidden][n_in], b1 [n_hidden], W2 [n_hidden][n_hidden],
 * b2 [n_hidden], W3 [n_out][n_hidden], b3 [n_out]. Adam moments are zeroed and
 * step = 0. `mem` (device, >= omp_mlp_size, 256-byte aligned) is caller-owned. */
int omp_mlp_init(omp_mlp_t *mlp, int32_t n_in, int32_t n_hidden, int32_t n_out, const float *const params[6],
                 void *mem, size_t bytes, void *stream);

/* Copy the FP32 master parameters out (device arrays laid out as in omp_mlp_init). */
int omp_mlp_export(const omp_mlp_t *mlp, float *const params[6], void *stream);

/* Workspace bytes for omp_mlp_features / _forward / _grad / _train_step on B
 * signals of length M (M only matters for omp_mlp_features). */
size_t omp_mlp_workspace_size(const omp_mlp_t *mlp, int64_t M, int64_t B);

/* Features of B signals: F[b][n] (BF16 bits, row stride N) = f_n of y_b; a zero
 * or non-finite y_b gives a zero row. `dict` prepared for OMP_PREC_BF16. */
int omp_mlp_features(const omp_dict_t *dict, const float *Y, int64_t B, int64_t ldy, uint16_t *F,
                     const omp_mlp_t *mlp, void *workspace, size_t workspace_bytes, void *stream);

/* Scores Z[b][n] (FP32, row stride n_out) of B feature rows F (BF16, row stride n_in). */
int omp_mlp_forward(const omp_mlp_t *mlp, const uint16_t *F, int64_t B, float *Z, void *workspace,
                    size_t workspace_bytes, void *stream);

/* Loss and gradients on B feature rows against the supports support[.][S]
 * (-1 entries ignored). rows (device int32 [B], optional): the batch is rows
 * rows[0..B-1] of F and support (a minibatch of a larger set); NULL takes
 * rows 0..B-1. loss_out (device [1], optional): the batch loss.
 * grads_out (host array of 6 device pointers, optional; entries may be NULL):
 * FP32 gradients in the parameter layout of omp_mlp_init. The network is not
 * changed. */
int omp_mlp_grad(const omp_mlp_t *mlp, const uint16_t *F, const int32_t *support, const int32_t *rows, int64_t B,
                 int32_t S, float *loss_out, float *const grads_out[6], void *workspace, size_t workspace_bytes,
                 void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, epsilon 1e-8) with learning rate lr
 * on the batch's gradients (batch selection as in omp_mlp_grad); mlp->step is
 * incremented. */
int omp_mlp_train_step(omp_mlp_t *mlp, const uint16_t *F, const int32_t *support, const int32_t *rows, int64_t B,
                       int32_t S, float lr, float *loss_out, void *workspace, size_t workspace_bytes, void *stream);

/* Workspace bytes for omp_learned_solve (including the fallback omp_solve on
 * up to B signals at opts->precision). */
size_t omp_learned_workspace_size(const omp_dict_t *dict, const omp_mlp_t *mlp, int64_t B, int32_t S,
                                  const omp_opts_t *fallback);

/* Learned solve of B signals: features, network, top-S proposal, least-squares
 * check; the rejected signals are gathered and solved by omp_solve (with
 * `fallback`'s precision and tile configuration; its workspace, dict and
 * optional-array fields are ignored: the dictionary `dict` and this call's
 * workspace are used) and scattered back. Outputs as omp_solve's compact ones:
 * support_out/coef_out [B][S], status_out [B] (accepted: (S << 8) | OMP_SIG_EPS
 * | OMP_SIG_LEARNED), rnorm_out [B]. accepted_out (HOST, optional) receives the
 * number of accepted proposals. S <= 64. This call waits for the stream once
 * (to size the fallback). */
int omp_learned_solve(const omp_dict_t *dict, const omp_mlp_t *mlp, const float *Y, int64_t B, int64_t ldy,
                      int32_t S, float eps, const float *eps_per_signal, int32_t *support_out, float *coef_out,
                      int32_t *status_out, float *rnorm_out, int64_t *accepted_out, const omp_opts_t *fallback,
                      void *workspace, size_t workspace_bytes, void *stream);

/* Human-readable text for a return code (static storage). */
const char *omp_status_string(int status);

/* hipError_t of the most recent OMP_EDEVICE on this thread (0 if none). */
int omp_last_hip_error(void);

/* Library version, e.g. "0.1.0". */
const char *omp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BATCHED_OMP_H */
