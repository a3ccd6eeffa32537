/*
 * Householder QR oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the plain, slow, obviously-correct CPU reference that the GPU
 * path is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header, table
 * or helper with the HIP library, and the HIP library never calls it.
 *
 * What it computes (paper, Section 3.1 "Multilevel QR factorization"): the QR
 * factorization A = QR of an m-by-n matrix (m >= n), Q orthogonal, R upper
 * triangular, obtained with Householder reflections.  The multilevel method of
 * Algorithm 1 reaches the same R (a tree of orthogonal eliminations of stacked
 * row blocks preserves A^T A, and R with a positive diagonal is unique for a
 * full-rank A), so the oracle is that definition written out: column-by-column
 * textbook Householder QR with no blocking, no tree and no reordering.
 *
 * Convention (the paper fixes none): the reflector of column j is
 *     H_j = I - beta_j v_j v_j^T,   v_j(j) = 1,
 * chosen so that H_j maps x = A(j:m, j) to +||x|| e_1 (Golub & Van Loan,
 * "Matrix Computations", Householder vector algorithm of Section 5.1.2,
 * including the cancellation-free v(1) formula).  Hence every R_jj >= 0
 * without any later sign fix-up.  When x(2:) == 0 and x(1) < 0 the reflector is
 * H = I - 2 e_1 e_1^T (an exact sign flip), and when x(2:) == 0 and x(1) >= 0 it
 * is the identity.
 *
 * Norms use power-of-two scaling: x is scaled by 2^-e, e = ilogb(max|x|), with
 * ldexp on each element, which is exact for every finite input (subnormals
 * included), so neither overflow nor underflow spoils sigma = ||x(2:)||^2.
 *
 * Storage: R in the upper triangle of A, v_j(j+1:m) below the diagonal,
 * beta_j in beta[j].  Column-major with leading dimension lda.
 *
 * The trailing-column loop is OpenMP-parallel over columns (each column is
 * independent given v_j); it does not change the arithmetic of any column.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define IDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

/* Mutation switch used only by the pin-strength tests: each nonzero value
 * plants one plausible mistake so the tests can show that a pin catches it.
 * The default build has ORACLE_MUTANT == 0 and no mutation is compiled in. */
#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/* Householder vector of x (length len, stride 1), Golub & Van Loan Section
 * 5.1.2.  On return v[0] = 1, v[1:] overwrite x[1:], *beta is the reflector
 * coefficient and *mu is the resulting (non-negative) leading entry. */
static void house(int64_t len, double *x, double *beta, double *mu) {
  double amax = 0.0;
  for (int64_t i = 0; i < len; ++i) {
    double a = fabs(x[i]);
    if (a > amax) amax = a;
  }
  if (amax == 0.0) { /* zero column: H = I, R_jj = 0 */
    *beta = 0.0;
    *mu = 0.0;
    return;
  }
  /* scale by 2^-e elementwise: exact for every finite x, subnormals included
   * (a separate factor 2^-e would overflow for e < -1023) */
  int e = ilogb(amax);
  double x1 = ldexp(x[0], -e);
  double sigma = 0.0; /* ||x(2:)||^2 of the scaled vector */
  for (int64_t i = 1; i < len; ++i) {
    double t = ldexp(x[i], -e);
#if ORACLE_MUTANT == 1
    /* planted mistake: drop the last term of sigma */
    if (i == len - 1) t = 0.0;
#endif
    sigma += t * t;
  }
  if (sigma == 0.0) {
    if (x1 >= 0.0) {
      *beta = 0.0;
      *mu = x[0];
    } else {
      *beta = 2.0; /* H = I - 2 e1 e1^T flips the sign */
      *mu = -x[0];
    }
    /* sigma == 0 means every |x(i)| (i >= 1) is below 2^-537 |x(0)|: those
     * entries are negligible and are set to zero, so v = e_1 exactly. */
    for (int64_t i = 1; i < len; ++i) x[i] = 0.0;
    return;
  }
  double m = sqrt(x1 * x1 + sigma); /* scaled ||x|| */
  double v1;
  if (x1 <= 0.0)
    v1 = x1 - m;
  else
    v1 = -sigma / (x1 + m); /* = x1 - m without cancellation */
#if ORACLE_MUTANT == 2
  v1 = x1 + m; /* planted mistake: wrong sign in v(1) */
#endif
  double b = 2.0 * v1 * v1 / (sigma + v1 * v1);
  for (int64_t i = 1; i < len; ++i) x[i] = ldexp(x[i], -e) / v1;
  *beta = b;
  *mu = ldexp(m, e); /* undo the exact scaling */
}

/* Apply H = I - beta v v^T (v(0) = 1 implicit, v(1:) = vt[1:]) to the column
 * c of length len: c <- c - beta v (v^T c). */
static void apply_reflector(int64_t len, const double *vt, double beta, double *c) {
  double w = c[0];
#if ORACLE_MUTANT == 3
  w = 0.0; /* planted mistake: drop the implicit unit entry of v from v^T c */
#endif
  for (int64_t i = 1; i < len; ++i) w += vt[i] * c[i];
  w *= beta;
  c[0] -= w;
  for (int64_t i = 1; i < len; ++i) c[i] -= w * vt[i];
}

/* In-place Householder QR.  Returns 0, or -1 on invalid arguments. */
int oracle_qr(int64_t m, int64_t n, double *A, int64_t lda, double *beta) {
  if (m < 0 || n < 0 || n > m || lda < (m > 1 ? m : 1)) return -1;
  for (int64_t j = 0; j < n; ++j) {
    double *col = A + IDX(j, j, lda);
    int64_t len = m - j;
    double b, mu;
    house(len, col, &b, &mu);
    beta[j] = b;
    if (b != 0.0) {
#if ORACLE_MUTANT == 4
      int64_t k0 = j + 2; /* planted mistake: skip the first trailing column */
#else
      int64_t k0 = j + 1;
#endif
#pragma omp parallel for schedule(static)
      for (int64_t k = k0; k < n; ++k) apply_reflector(len, col, b, A + IDX(j, k, lda));
    }
    col[0] = mu; /* R_jj; the entries below now hold v(2:) */
  }
  return 0;
}

/* C (m-by-k) <- Q^T C with Q = H_0 H_1 ... H_{n-1} from oracle_qr. */
int oracle_apply_qt(int64_t m, int64_t n, const double *F, int64_t ldf, const double *beta,
                    int64_t k, double *C, int64_t ldc) {
  if (m < 0 || n < 0 || n > m || k < 0) return -1;
#if ORACLE_MUTANT == 5
  for (int64_t j = n - 1; j >= 0; --j) { /* planted mistake: reflectors in the wrong order */
#else
  for (int64_t j = 0; j < n; ++j) {
#endif
    if (beta[j] == 0.0) continue;
    const double *v = F + IDX(j, j, ldf);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < k; ++c) apply_reflector(m - j, v, beta[j], C + IDX(j, c, ldc));
  }
  return 0;
}

/* C (m-by-k) <- Q C. */
int oracle_apply_q(int64_t m, int64_t n, const double *F, int64_t ldf, const double *beta,
                   int64_t k, double *C, int64_t ldc) {
  if (m < 0 || n < 0 || n > m || k < 0) return -1;
#if ORACLE_MUTANT == 6
  for (int64_t j = 0; j < n; ++j) { /* planted mistake: Q applied in Q^T order */
#else
  for (int64_t j = n - 1; j >= 0; --j) {
#endif
    if (beta[j] == 0.0) continue;
    const double *v = F + IDX(j, j, ldf);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < k; ++c) apply_reflector(m - j, v, beta[j], C + IDX(j, c, ldc));
  }
  return 0;
}

/* Explicit thin Q (m-by-n): Q [I_n; 0]. */
int oracle_form_q(int64_t m, int64_t n, const double *F, int64_t ldf, const double *beta,
                  double *Q, int64_t ldq) {
  if (m < 0 || n < 0 || n > m || ldq < (m > 1 ? m : 1)) return -1;
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < m; ++i) Q[IDX(i, j, ldq)] = (i == j) ? 1.0 : 0.0;
  return oracle_apply_q(m, n, F, ldf, beta, n, Q, ldq);
}

/* Back substitution R X = B for the n-by-n upper triangle of F; B is n-by-k.
 * Returns 0, or 1 + (first j with R_jj == 0) if R is exactly singular. */
int oracle_trsm_upper(int64_t n, const double *F, int64_t ldf, int64_t k, double *B, int64_t ldb) {
  for (int64_t j = 0; j < n; ++j)
    if (F[IDX(j, j, ldf)] == 0.0) return (int)(1 + j);
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < k; ++c) {
    double *b = B + IDX(0, c, ldb);
    for (int64_t i = n - 1; i >= 0; --i) {
      double s = b[i];
#if ORACLE_MUTANT == 7
      for (int64_t p = i + 1; p < n; ++p) s -= F[IDX(p, i, ldf)] * b[p]; /* planted: transposed R */
#else
      for (int64_t p = i + 1; p < n; ++p) s -= F[IDX(i, p, ldf)] * b[p];
#endif
      b[i] = s / F[IDX(i, i, ldf)];
    }
  }
  return 0;
}

/* Least squares min ||A x - b||: QR of A (in place), B <- Q^T B, then
 * back-substitution; the solution is left in B(0:n, :).  beta needs n
 * entries.  Returns 0, -1 on bad arguments, or 1 + j for a zero R_jj. */
int oracle_ls(int64_t m, int64_t n, int64_t nrhs, double *A, int64_t lda, double *B, int64_t ldb,
              double *beta) {
  int rc = oracle_qr(m, n, A, lda, beta);
  if (rc) return rc;
  rc = oracle_apply_qt(m, n, A, lda, beta, nrhs, B, ldb);
  if (rc) return rc;
  return oracle_trsm_upper(n, A, lda, nrhs, B, ldb);
}
