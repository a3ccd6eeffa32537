// Launchers of the FP64 refinement kernels of the mixed-precision
// least-squares solve (refine.hip).  Vectors and scalars are device memory;
// A is column-major with leading dimension lda; R is the upper triangle of an
// n x n block with leading dimension ldr.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace caqr {

// out[j] = ||A(:, j)||^2 for j < n.
hipError_t launch_colsq(const double *A, int64_t lda, int64_t m, int64_t n, double *out, hipStream_t s);
// scal[0] = max(||A||_F / sqrt(n), max_j ||A(:, j)||) <= ||A||_2 from colsq.
hipError_t launch_anorm_lower(const double *colsq, int64_t n, double *scal, hipStream_t s);
// r = b - A x (m rows).
hipError_t launch_resid(const double *A, int64_t lda, int64_t m, int64_t n, const double *x, const double *b,
                        double *r, hipStream_t s);
// y = A x.
hipError_t launch_gemv(const double *A, int64_t lda, int64_t m, int64_t n, const double *x, double *y, hipStream_t s);
// u = A^T r.
hipError_t launch_atr(const double *A, int64_t lda, int64_t m, int64_t n, const double *r, double *u, hipStream_t s);
// y <- R^-T y.
hipError_t launch_trsv_upper_t(const double *R, int64_t ldr, int64_t n, double *y, hipStream_t s);
// out[0] = x . y.
hipError_t launch_dot(const double *x, const double *y, int64_t n, double *out, hipStream_t s);
// y += sgn (num[0] / den[0]) x.
hipError_t launch_axpy_ratio(double *y, const double *x, int64_t n, const double *num, const double *den, double sgn,
                             hipStream_t s);
// p = s + (num[0] / den[0]) p.
hipError_t launch_xpby_ratio(double *p, const double *sv, int64_t n, const double *num, const double *den,
                             hipStream_t s);
hipError_t launch_copy(double *dst, const double *src, int64_t n, hipStream_t s);
// out[0] = sqrt(sq[0]) / (a (a sqrt(sq[1]) + sqrt(sq[2]))), a = scal[0].
hipError_t launch_eta_bound(const double *sq, const double *scal, double *out, hipStream_t s);

}  // namespace caqr
