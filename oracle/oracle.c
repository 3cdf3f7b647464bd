/*
 * oracle.c -- plain, slow, obviously-correct FP64 CPU reference for the
 * envelope (band + arrowhead) Cholesky factorization, solve and
 * log-determinant.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call
 * this file: only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code, header, table or helper with the HIP
 * library.
 *
 * What it computes (sTiles paper, Section II, the three-phase sparse Cholesky
 * and its numerical phase; Algorithm 1 is the tiled form of the same result):
 * for a symmetric positive-definite matrix A, the unique lower-triangular L
 * with positive diagonal and A = L L^T.  The tile algorithm of the paper
 * reaches exactly this L (up to rounding order); here it is computed by the
 * textbook envelope ("skyline") method, element by element, with every dot
 * product summed sequentially in ascending k.
 *
 * Storage ("row profile"): row i holds entries (i, f_i .. i) contiguously,
 * f_i = first structurally nonzero column of row i (f_i <= i).  Arrow rows
 * (the trailing dense rows of a block-arrowhead matrix, Section I) are just
 * rows with f_i = 0.  rp[i] = start of row i, rp[N] = total length.
 * Cholesky preserves the envelope, so L is stored in the same array.
 *
 * Permutations are applied by the caller: the oracle factors whatever
 * symmetric matrix it is given (P A P^T).
 *
 * Pins (tests/test_oracle_pins.py): LAPACK dense Cholesky on small inputs,
 * exactly planted integer factors (bit-exact), closed-form arrowhead and
 * Toeplitz-band determinants, solve backward error, permutation invariance.
 * Selected inversion (tests/test_oracle_selinv.py): the dense inverse on small
 * inputs, the closed-form inverses of the second-difference matrix and of a
 * pure arrowhead, and exactly planted integer inverses (bit-exact).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline int64_t max64(int64_t x, int64_t y) { return x > y ? x : y; }

/* rp[0..N] from f[0..N-1]: row i has (i - f_i + 1) entries. */
void oracle_row_ptr(int64_t N, const int64_t* f, int64_t* rp) {
  rp[0] = 0;
  for (int64_t i = 0; i < N; i++) rp[i + 1] = rp[i] + (i - f[i] + 1);
}

/* Sequential dot product of rows i and j of L over columns [k0, k1). */
static inline double row_dot(const double* v, const int64_t* rp, const int64_t* f,
                             int64_t i, int64_t j, int64_t k0, int64_t k1) {
  const double* ri = v + rp[i] - f[i];
  const double* rj = v + rp[j] - f[j];
  double s = 0.0;
  for (int64_t k = k0; k < k1; k++) s += ri[k] * rj[k];
  return s;
}

/*
 * In-place envelope Cholesky, left-looking by columns (column j is finished
 * from columns 0..j-1, then used), which is the column form of Algorithm 1:
 *   d    = A_jj - sum_{k=f_j}^{j-1} L_jk^2 ;  L_jj = sqrt(d)
 *   L_ij = (A_ij - sum_{k=max(f_i,f_j)}^{j-1} L_ik L_jk) / L_jj   (i > j, f_i <= j)
 * Rows i > j of one column are independent, so they may run in parallel;
 * each dot product stays a plain sequential sum.
 * `wmax` bounds i - f_i over the rows whose f_i > 0 (the band rows); rows with
 * f_i == 0 and i > wmax are scanned separately (the arrow rows), so the
 * candidate rows of column j are (j, j + wmax] plus every row with f_i == 0.
 * Returns 0, or the 1-based index of the first column whose pivot is not
 * positive (LAPACK potrf convention); then L is partial and must not be used.
 */
int64_t oracle_factor(int64_t N, const int64_t* f, double* v, int nthreads) {
  int64_t* rp = (int64_t*)malloc(sizeof(int64_t) * (N + 1));
  oracle_row_ptr(N, f, rp);
  int64_t wmax = 0;
  int64_t nfull = 0;             /* rows with f == 0 beyond the band reach */
  for (int64_t i = 0; i < N; i++) if (i - f[i] > wmax && f[i] > 0) wmax = i - f[i];
  int64_t* full = (int64_t*)malloc(sizeof(int64_t) * (N + 1));
  for (int64_t i = 0; i < N; i++) if (f[i] == 0 && i > wmax) full[nfull++] = i;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  int64_t info = 0;
  for (int64_t j = 0; j < N; j++) {
    double* rowj = v + rp[j] - f[j];
    double d = rowj[j] - row_dot(v, rp, f, j, j, f[j], j);
    if (!(d > 0.0)) { info = j + 1; break; }
    double ljj = sqrt(d);
    rowj[j] = ljj;
    int64_t band_hi = j + wmax < N - 1 ? j + wmax : N - 1;
    #pragma omp parallel
    {
      #pragma omp for schedule(static)
      for (int64_t i = j + 1; i <= band_hi; i++) {
        if (f[i] > j) continue;
        double* rowi = v + rp[i] - f[i];
        double s = rowi[j] - row_dot(v, rp, f, i, j, max64(f[i], f[j]), j);
        rowi[j] = s / ljj;
      }
      #pragma omp for schedule(static)
      for (int64_t q = 0; q < nfull; q++) {
        int64_t i = full[q];
        if (i <= band_hi) continue;
        double* rowi = v + rp[i] - f[i];
        double s = rowi[j] - row_dot(v, rp, f, i, j, max64(f[i], f[j]), j);
        rowi[j] = s / ljj;
      }
    }
  }
  free(full);
  free(rp);
  return info;
}

/* logdet A = 2 sum_i log L_ii, accumulated in long double, rounded once. */
double oracle_logdet(int64_t N, const int64_t* f, const double* L) {
  int64_t* rp = (int64_t*)malloc(sizeof(int64_t) * (N + 1));
  oracle_row_ptr(N, f, rp);
  long double s = 0.0L;
  for (int64_t i = 0; i < N; i++) s += logl((long double)L[rp[i] + (i - f[i])]);
  free(rp);
  return (double)(2.0L * s);
}

/*
 * Solve A X = B with A = L L^T, B column-major N x nrhs (leading dim ldb),
 * overwritten by X.  Forward substitution by rows, backward by columns:
 *   y_i = (b_i - sum_{k=f_i}^{i-1} L_ik y_k) / L_ii
 *   z_i = y_i / L_ii ; y_k -= L_ik z_i for k in [f_i, i)   (i descending)
 */
void oracle_solve(int64_t N, const int64_t* f, const double* L, int64_t nrhs,
                  double* B, int64_t ldb) {
  int64_t* rp = (int64_t*)malloc(sizeof(int64_t) * (N + 1));
  oracle_row_ptr(N, f, rp);
  for (int64_t c = 0; c < nrhs; c++) {
    double* b = B + c * ldb;
    for (int64_t i = 0; i < N; i++) {
      const double* ri = L + rp[i] - f[i];
      double s = b[i];
      for (int64_t k = f[i]; k < i; k++) s -= ri[k] * b[k];
      b[i] = s / ri[i];
    }
    for (int64_t i = N - 1; i >= 0; i--) {
      const double* ri = L + rp[i] - f[i];
      double z = b[i] / ri[i];
      b[i] = z;
      for (int64_t k = f[i]; k < i; k++) b[k] -= ri[k] * z;
    }
  }
  free(rp);
}

/*
 * Selected inversion: the entries of Sigma = A^{-1} inside the envelope of A,
 * from its factor L (A = L L^T), written to S in the same row-profile layout.
 * Inverses of block-arrowhead matrices are one of the tasks the paper's
 * introduction lists for this class (Section I); INLA needs the diagonal of
 * the inverse (posterior marginal variances).
 *
 * Textbook recursion (Takahashi, Fagan and Chen, 1973): from Sigma L = L^{-T},
 * whose lower part below the diagonal is zero and whose diagonal is 1/L_jj,
 * column j of Sigma on the rows R_j = {i > j : f_i <= j} of column j of L is
 *   Sigma_ij = -(1/L_jj) sum_{k in R_j} Sigma_ik L_kj         (i in R_j)
 *   Sigma_jj = (1/L_jj) (1/L_jj - sum_{k in R_j} L_kj Sigma_kj)
 * for j = N-1 down to 0.  Every Sigma_ik used (i, k in R_j) lies in the
 * envelope (row max(i,k) reaches column min(i,k), since f <= j there) and in a
 * column > j, so it is final when column j is computed.  Sums run in
 * ascending k.  Rows of one column are independent (parallel).
 */
void oracle_selinv(int64_t N, const int64_t* f, const double* L, double* S, int nthreads) {
  int64_t* rp = (int64_t*)malloc(sizeof(int64_t) * (N + 1));
  oracle_row_ptr(N, f, rp);
  int64_t wmax = 0;
  for (int64_t i = 0; i < N; i++) if (i - f[i] > wmax && f[i] > 0) wmax = i - f[i];
  int64_t nfull = 0;             /* rows with f == 0 beyond the band reach */
  int64_t* full = (int64_t*)malloc(sizeof(int64_t) * (N + 1));
  for (int64_t i = 0; i < N; i++) if (f[i] == 0 && i > wmax) full[nfull++] = i;
  int64_t* R = (int64_t*)malloc(sizeof(int64_t) * (N + 1));
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  for (int64_t j = N - 1; j >= 0; j--) {
    /* R_j ascending: band candidates (j, j + wmax], then the full rows beyond */
    int64_t nr = 0;
    int64_t band_hi = j + wmax < N - 1 ? j + wmax : N - 1;
    for (int64_t i = j + 1; i <= band_hi; i++) if (f[i] <= j) R[nr++] = i;
    for (int64_t q = 0; q < nfull; q++) if (full[q] > band_hi) R[nr++] = full[q];
    const double ljj = L[rp[j] + (j - f[j])];
    #pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < nr; a++) {
      const int64_t i = R[a];
      double s = 0.0;
      for (int64_t b = 0; b < nr; b++) {
        const int64_t k = R[b];
        const int64_t hi = i > k ? i : k, lo = i > k ? k : i;
        s += S[rp[hi] + (lo - f[hi])] * L[rp[k] + (j - f[k])];
      }
      S[rp[i] + (j - f[i])] = -s / ljj;
    }
    double s = 0.0;
    for (int64_t b = 0; b < nr; b++) {
      const int64_t k = R[b];
      s += L[rp[k] + (j - f[k])] * S[rp[k] + (j - f[k])];
    }
    S[rp[j] + (j - f[j])] = (1.0 / ljj - s) / ljj;
  }
  free(R);
  free(full);
  free(rp);
}

/* Y = A X for symmetric A given by its lower envelope (X, Y column-major). */
void oracle_symv(int64_t N, const int64_t* f, const double* A, int64_t nrhs,
                 const double* X, int64_t ldx, double* Y, int64_t ldy) {
  int64_t* rp = (int64_t*)malloc(sizeof(int64_t) * (N + 1));
  oracle_row_ptr(N, f, rp);
  for (int64_t c = 0; c < nrhs; c++) {
    const double* x = X + c * ldx;
    double* y = Y + c * ldy;
    for (int64_t i = 0; i < N; i++) y[i] = 0.0;
    for (int64_t i = 0; i < N; i++) {
      const double* ri = A + rp[i] - f[i];
      double s = 0.0;
      for (int64_t k = f[i]; k < i; k++) { s += ri[k] * x[k]; y[k] += ri[k] * x[i]; }
      y[i] += s + ri[i] * x[i];
    }
  }
  free(rp);
}

/*
 * Factor residual over selected rows: returns sum over the selected rows i and
 * columns j in [f_i, i] of ((L L^T)_ij - A_ij)^2 in *num and of A_ij^2 in
 * *den (off-diagonal entries counted twice, for the symmetric Frobenius norm).
 * (L L^T)_ij = sum_{k=max(f_i,f_j)}^{j} L_ik L_jk.
 */
void oracle_factor_residual(int64_t N, const int64_t* f, const double* A, const double* L,
                            int64_t nrows, const int64_t* rows, double* num, double* den) {
  int64_t* rp = (int64_t*)malloc(sizeof(int64_t) * (N + 1));
  oracle_row_ptr(N, f, rp);
  long double sn = 0.0L, sd = 0.0L;
  for (int64_t q = 0; q < nrows; q++) {
    int64_t i = rows[q];
    const double* ai = A + rp[i] - f[i];
    const double* li = L + rp[i] - f[i];
    for (int64_t j = f[i]; j <= i; j++) {
      const double* lj = L + rp[j] - f[j];
      double s = 0.0;
      for (int64_t k = max64(f[i], f[j]); k <= j; k++) s += li[k] * lj[k];
      long double r = (long double)s - ai[j];
      long double w = (j == i) ? 1.0L : 2.0L;
      sn += w * r * r;
      sd += w * (long double)ai[j] * ai[j];
    }
  }
  *num = (double)sn;
  *den = (double)sd;
  free(rp);
}
