/*
 * FP64 CPU oracle for Orthogonal Matching Pursuit.
 *
 * TEST INFRASTRUCTURE ONLY. The solver never loads this file. Only the test
 * suite, the package's smoke check and the benchmark's CPU-baseline leg build,
 * load or call it. It shares no code with the GPU path.
 *
 * What it computes: Algorithm 1 (OMP) of Lubonja, Praesius & Tran, "A Practical
 * GPU-Accelerated Implementation of Orthogonal Matching Pursuit", written out
 * plainly for one signal at a time:
 *
 *   r_0 = y, support empty, k = 0
 *   while k < S and ||r_k|| > eps:
 *       n* = argmax over n not yet selected of |<r_k, a_n>| / ||a_n||
 *       append n* to the support
 *       x_k = argmin_x ||y - A_support x||       (least squares, from scratch)
 *       r_k = y - A_support x_k
 *
 * Everything is float64. The least squares problem is solved from scratch at
 * every step with a Householder QR factorisation of A_support (the textbook
 * algorithm), deliberately not with the progressive Cholesky update of the
 * paper's Section 2.2, so that the oracle and the GPU path reach the same
 * result by different arithmetic.
 *
 * Readings taken where the paper is silent:
 *   - argmax ties go to the lowest atom index;
 *   - atoms already in the support are never re-selected, atoms of zero norm
 *     are never selectable;
 *   - the stop test is on the norm ||r|| <= eps, checked before every pick
 *     (so y = 0 gives an empty support), and eps <= 0 means "stop only on an
 *     exactly zero residual";
 *   - the support is empty at the start (Algorithm 1's initial support set);
 *   - a picked atom whose distance to the span of the support, |R_kk|, is at
 *     most dep_tol * ||a_n*|| is dropped and the signal stops as DEPENDENT;
 *   - a non-finite y stops the signal before any pick (NONFINITE).
 *
 * Forced-prefix mode: for steps k < nprefix the pick is prefix[k] instead of
 * the argmax. The scores are still recorded, so a caller can replay another
 * solver's pick sequence and check, step by step, that each pick was an
 * argmax (or within a near-tie of it) given the same prefix.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EPS 1
#define ORC_SMAX 2
#define ORC_DEPENDENT 4
#define ORC_NONFINITE 8
#define ORC_EXHAUSTED 32

#define ORC_OK 0
#define ORC_EBADPREFIX -1
#define ORC_ENOMEM -2

/* Plain dot product of an atom (float32, contiguous) with a float64 vector. */
static double dot_atom(const float *a, const double *v, int M) {
  double s = 0.0;
  for (int m = 0; m < M; ++m) s += (double)a[m] * v[m];
  return s;
}

static double norm2(const double *v, int M) {
  double s = 0.0;
  for (int m = 0; m < M; ++m) s += v[m] * v[m];
  return sqrt(s);
}

/*
 * Least squares min ||b - W x|| for the M x k matrix W (column-major, columns
 * are the selected atoms in order) by Householder QR. W and b are overwritten.
 * On return x[0..k-1] holds the solution and *rkk = |R[k-1][k-1]|.
 * Returns 0, or 1 when a diagonal entry of R is exactly zero.
 */
static int householder_ls(double *W, double *b, int M, int k, double *x, double *rkk) {
  for (int j = 0; j < k; ++j) {
    double *wj = W + (size_t)j * M;
    /* reflector that maps wj[j..M-1] onto a multiple of e_j */
    double nrm = 0.0;
    for (int i = j; i < M; ++i) nrm += wj[i] * wj[i];
    nrm = sqrt(nrm);
    if (nrm == 0.0) { *rkk = 0.0; return 1; }
    double alpha = (wj[j] > 0.0) ? -nrm : nrm;
    /* v = wj[j..] - alpha e_j, stored in place; beta = 2 / (v^T v) */
    wj[j] -= alpha;
    double vtv = 0.0;
    for (int i = j; i < M; ++i) vtv += wj[i] * wj[i];
    double beta = (vtv > 0.0) ? 2.0 / vtv : 0.0;
    /* apply H = I - beta v v^T to the remaining columns and to b */
    for (int c = j + 1; c < k; ++c) {
      double *wc = W + (size_t)c * M;
      double t = 0.0;
      for (int i = j; i < M; ++i) t += wj[i] * wc[i];
      t *= beta;
      for (int i = j; i < M; ++i) wc[i] -= t * wj[i];
    }
    {
      double t = 0.0;
      for (int i = j; i < M; ++i) t += wj[i] * b[i];
      t *= beta;
      for (int i = j; i < M; ++i) b[i] -= t * wj[i];
    }
    /* R[j][j] = alpha; keep it in wj[j] (v is not needed any more for rows < j+1
       of later columns, and the entries above the diagonal stay in place) */
    wj[j] = alpha;
  }
  *rkk = fabs(W[(size_t)(k - 1) * M + (k - 1)]);
  /* back substitution R x = (Q^T b)[0..k-1]; R[i][c] sits at W[c*M + i] */
  for (int i = k - 1; i >= 0; --i) {
    double s = b[i];
    for (int c = i + 1; c < k; ++c) s -= W[(size_t)c * M + i] * x[c];
    double d = W[(size_t)i * M + i];
    if (d == 0.0) return 1;
    x[i] = s / d;
  }
  return 0;
}

/*
 * One signal.
 *   A        atom-major dictionary, atom n at A + n*lda (lda >= M), float32
 *   y        signal, M float32
 *   S        maximum number of picks (>= 0)
 *   eps      stop when ||r|| <= max(eps, 0)
 *   prefix   forced picks for the first nprefix steps (may be NULL if nprefix == 0)
 *   dep_tol  dependency threshold on |R_kk| / ||a_n*||
 * Outputs (each may be NULL unless stated):
 *   support[S]          picks in order, -1 padded               (required)
 *   coef[S]             final least-squares coefficients, 0 padded (required)
 *   coef_hist[S*S]      row j holds x_{j+1} (coefficients after pick j+1)
 *   rnorm_hist[S+1]     ||r_k|| for k = 0..k_final (rest NaN)
 *   s_best[S], s_second[S], s_pick[S], idx_best[S]
 *                       per step: best score, second best score, score of the
 *                       atom actually picked, index of the best
 *   *k_out, *status_out (required)
 * Returns ORC_OK, ORC_EBADPREFIX (a forced pick was invalid) or ORC_ENOMEM.
 */
int oracle_omp_signal(int M, int N, const float *A, int64_t lda, const float *y, int S, double eps,
                      const int32_t *prefix, int nprefix, double dep_tol,
                      int32_t *support, double *coef, double *coef_hist, double *rnorm_hist,
                      double *s_best, double *s_second, double *s_pick, int32_t *idx_best,
                      int32_t *k_out, int32_t *status_out) {
  int rc = ORC_OK;
  double *nu = (double *)malloc(sizeof(double) * (size_t)N);
  double *r = (double *)malloc(sizeof(double) * (size_t)M);
  double *yd = (double *)malloc(sizeof(double) * (size_t)M);
  double *W = (double *)malloc(sizeof(double) * (size_t)M * (size_t)(S > 0 ? S : 1));
  double *bq = (double *)malloc(sizeof(double) * (size_t)M);
  double *x = (double *)malloc(sizeof(double) * (size_t)(S > 0 ? S : 1));
  char *selected = (char *)calloc((size_t)N, 1);
  if (!nu || !r || !yd || !W || !bq || !x || !selected) { rc = ORC_ENOMEM; goto done; }

  for (int j = 0; j < S; ++j) { support[j] = -1; coef[j] = 0.0; }
  if (coef_hist) for (int j = 0; j < S * S; ++j) coef_hist[j] = 0.0;
  if (rnorm_hist) for (int j = 0; j <= S; ++j) rnorm_hist[j] = NAN;
  if (s_best) for (int j = 0; j < S; ++j) s_best[j] = NAN;
  if (s_second) for (int j = 0; j < S; ++j) s_second[j] = NAN;
  if (s_pick) for (int j = 0; j < S; ++j) s_pick[j] = NAN;
  if (idx_best) for (int j = 0; j < S; ++j) idx_best[j] = -1;

  int k = 0, status = 0;
  double eps_eff = eps > 0.0 ? eps : 0.0;

  int finite = 1;
  for (int m = 0; m < M; ++m) {
    yd[m] = (double)y[m];
    if (!isfinite(yd[m])) finite = 0;
    r[m] = yd[m];
  }
  if (!finite) { status = ORC_NONFINITE; goto finish; }

  for (int n = 0; n < N; ++n) {
    const float *a = A + (size_t)n * (size_t)lda;
    double s = 0.0;
    for (int m = 0; m < M; ++m) s += (double)a[m] * (double)a[m];
    nu[n] = sqrt(s);
  }

  double rn = norm2(r, M);
  if (rnorm_hist) rnorm_hist[0] = rn;

  while (k < S && rn > eps_eff) {
    /* selection: |<r, a_n>| / ||a_n|| over the atoms still selectable */
    double best = -1.0, second = -1.0;
    int ibest = -1;
    for (int n = 0; n < N; ++n) {
      if (selected[n] || nu[n] == 0.0) continue;
      double s = fabs(dot_atom(A + (size_t)n * (size_t)lda, r, M)) / nu[n];
      if (s > best) { second = best; best = s; ibest = n; }
      else if (s > second) second = s;
    }
    int pick = ibest;
    double spick = best;
    if (k < nprefix) {
      pick = prefix[k];
      if (pick < 0 || pick >= N || selected[pick] || nu[pick] == 0.0) { rc = ORC_EBADPREFIX; goto finish; }
      spick = fabs(dot_atom(A + (size_t)pick * (size_t)lda, r, M)) / nu[pick];
    }
    if (pick < 0) { status = ORC_EXHAUSTED; break; }
    if (s_best) s_best[k] = best;
    if (s_second) s_second[k] = second;
    if (s_pick) s_pick[k] = spick;
    if (idx_best) idx_best[k] = ibest;

    /* least squares on the enlarged support, from scratch */
    support[k] = pick;
    for (int j = 0; j <= k; ++j) {
      const float *a = A + (size_t)support[j] * (size_t)lda;
      for (int m = 0; m < M; ++m) W[(size_t)j * M + m] = (double)a[m];
    }
    memcpy(bq, yd, sizeof(double) * (size_t)M);
    double rkk = 0.0;
    int sing = householder_ls(W, bq, M, k + 1, x, &rkk);
    if (sing || rkk <= dep_tol * nu[pick]) {
      support[k] = -1;
      status = ORC_DEPENDENT;
      break;
    }
    selected[pick] = 1;
    k += 1;
    for (int j = 0; j < k; ++j) coef[j] = x[j];
    if (coef_hist) for (int j = 0; j < k; ++j) coef_hist[(size_t)(k - 1) * S + j] = x[j];
    /* r = y - A_support x, explicitly */
    for (int m = 0; m < M; ++m) r[m] = yd[m];
    for (int j = 0; j < k; ++j) {
      const float *a = A + (size_t)support[j] * (size_t)lda;
      for (int m = 0; m < M; ++m) r[m] -= (double)a[m] * x[j];
    }
    rn = norm2(r, M);
    if (rnorm_hist) rnorm_hist[k] = rn;
  }
  if (status == 0) {
    if (rn <= eps_eff) status |= ORC_EPS;
    if (k >= S) status |= ORC_SMAX;
  }

finish:
  *k_out = k;
  *status_out = status;
done:
  free(nu); free(r); free(yd); free(W); free(bq); free(x); free(selected);
  return rc;
}

/*
 * A batch of B independent signals, split over nthreads host threads (one
 * signal per task; the arithmetic per signal is exactly oracle_omp_signal).
 * Per-signal arrays are row-major with row length S (S+1 for rnorm_hist).
 *   S_arr, eps_arr    optional per-signal sparsity / tolerance (NULL: use S, eps);
 *                     S_b is clamped to 0..S (a cap outside that range means no pick
 *                     or the batch's cap)
 *   prefix, nprefix   optional per-signal forced prefixes, prefix row length S
 * Returns the first non-zero per-signal return code, else ORC_OK.
 */
int oracle_omp_batch(int M, int N, const float *A, int64_t lda, int B, const float *Y, int64_t ldy,
                     int S, const int32_t *S_arr, double eps, const float *eps_arr,
                     const int32_t *prefix, const int32_t *nprefix, double dep_tol,
                     int32_t *support, double *coef, double *rnorm_hist,
                     double *s_best, double *s_second, double *s_pick, int32_t *idx_best,
                     int32_t *k_out, int32_t *status_out, int nthreads) {
  int rc_all = ORC_OK;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
  for (int b = 0; b < B; ++b) {
    int Sb = S_arr ? S_arr[b] : S;
    if (Sb > S) Sb = S;
    if (Sb < 0) Sb = 0;
    double eb = eps_arr ? (double)eps_arr[b] : eps;
    size_t o = (size_t)b * (size_t)S;
    /* per-signal outputs live in rows of length S; the signal uses the first Sb */
    int32_t *sup = support + o;
    double *cf = coef + o;
    for (int j = Sb; j < S; ++j) { sup[j] = -1; cf[j] = 0.0; }
    double *rh = rnorm_hist ? rnorm_hist + (size_t)b * (size_t)(S + 1) : NULL;
    if (rh) for (int j = Sb + 1; j <= S; ++j) rh[j] = NAN;
    for (int j = Sb; j < S; ++j) {
      if (s_best) s_best[o + j] = NAN;
      if (s_second) s_second[o + j] = NAN;
      if (s_pick) s_pick[o + j] = NAN;
      if (idx_best) idx_best[o + j] = -1;
    }
    int rc = oracle_omp_signal(M, N, A, lda, Y + (size_t)b * (size_t)ldy, Sb, eb,
                               prefix ? prefix + o : NULL, nprefix ? nprefix[b] : 0, dep_tol,
                               sup, cf, NULL, rh,
                               s_best ? s_best + o : NULL, s_second ? s_second + o : NULL,
                               s_pick ? s_pick + o : NULL, idx_best ? idx_best + o : NULL,
                               k_out + b, status_out + b);
    if (rc != ORC_OK) {
#pragma omp critical
      { if (rc_all == ORC_OK) rc_all = rc; }
    }
  }
  return rc_all;
}
