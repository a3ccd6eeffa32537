// Kernels of the mixed-precision least-squares solve: FP64 iterative
// refinement of a solution obtained from a QR factorization whose trailing
// updates ran on FP32 MFMA (paper, Section 3.1: least squares through A = QR).
// The factorization gives R~ (and Q~) of a matrix within about u32 ||A|| of A;
// the refinement is CGLS on min ||b - A R~^-1 y||, x = R~^-1 y (R~ as a right
// preconditioner, so the iteration sees A R~^-1, whose singular values lie
// within about kappa u32 of 1), with every residual, product with A and
// triangular solve in FP64.
//
// All reductions are fixed-order tree sums (results do not depend on timing).
#include <algorithm>

#include "device_common.hpp"
#include "refine.hpp"

namespace caqr {

namespace {

constexpr int kRT = 256;  // threads per workgroup

// Sum over the workgroup of one value per thread, fixed order; every thread
// gets the result.
__device__ __forceinline__ double block_sum(double v, double *red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int h = kRT / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

// out[j] = ||A(:, j)||^2, one workgroup per column.
__global__ void __launch_bounds__(kRT) colsq_kernel(const double *A, int64_t lda, int64_t m, double *out) {
  __shared__ double red[kRT];
  const double *a = A + (int64_t)blockIdx.x * lda;
  double s0 = 0.0, s1 = 0.0;
  int64_t i = threadIdx.x;
  for (; i + kRT < m; i += 2 * kRT) {
    s0 = fma(a[i], a[i], s0);
    s1 = fma(a[i + kRT], a[i + kRT], s1);
  }
  if (i < m) s0 = fma(a[i], a[i], s0);
  const double s = block_sum(s0 + s1, red);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// scal[0] = max(||A||_F / sqrt(n), max_j ||A(:, j)||), a lower bound of ||A||_2.
__global__ void __launch_bounds__(kRT) anorm_kernel(const double *colsq, int64_t n, double *scal) {
  __shared__ double red[kRT];
  double s = 0.0, mx = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += kRT) {
    s += colsq[j];
    mx = fmax(mx, colsq[j]);
  }
  const double tot = block_sum(s, red);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int h = kRT / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) scal[0] = fmax(sqrt(tot / (double)n), sqrt(red[0]));
}

// y = b - A x (RESID) or y = A x, one thread per row; x staged through LDS.
template <bool RESID>
__global__ void __launch_bounds__(kRT) gemv_kernel(const double *A, int64_t lda, int64_t m, int64_t n,
                                                   const double *x, const double *b, double *y) {
  __shared__ double xs[1024];
  const int64_t i = (int64_t)blockIdx.x * kRT + threadIdx.x;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int64_t j0 = 0; j0 < n; j0 += 1024) {
    const int nc = (int)min<int64_t>(1024, n - j0);
    __syncthreads();
    for (int e = threadIdx.x; e < nc; e += kRT) xs[e] = x[j0 + e];
    __syncthreads();
    if (i < m) {
      const double *a = A + i + j0 * lda;
      int j = 0;
      for (; j + 3 < nc; j += 4) {
        s0 = fma(a[(int64_t)j * lda], xs[j], s0);
        s1 = fma(a[(int64_t)(j + 1) * lda], xs[j + 1], s1);
        s2 = fma(a[(int64_t)(j + 2) * lda], xs[j + 2], s2);
        s3 = fma(a[(int64_t)(j + 3) * lda], xs[j + 3], s3);
      }
      for (; j < nc; ++j) s0 = fma(a[(int64_t)j * lda], xs[j], s0);
    }
  }
  if (i < m) {
    const double ax = (s0 + s1) + (s2 + s3);
    y[i] = RESID ? b[i] - ax : ax;
  }
}

// u = A^T r, one workgroup per column.
__global__ void __launch_bounds__(kRT) atr_kernel(const double *A, int64_t lda, int64_t m, const double *r,
                                                  double *u) {
  __shared__ double red[kRT];
  const double *a = A + (int64_t)blockIdx.x * lda;
  double s0 = 0.0, s1 = 0.0;
  int64_t i = threadIdx.x;
  for (; i + kRT < m; i += 2 * kRT) {
    s0 = fma(a[i], r[i], s0);
    s1 = fma(a[i + kRT], r[i + kRT], s1);
  }
  if (i < m) s0 = fma(a[i], r[i], s0);
  const double s = block_sum(s0 + s1, red);
  if (threadIdx.x == 0) u[blockIdx.x] = s;
}

// R^T y = z in place (R upper triangular n x n, ld ldr), forward substitution
// by blocks of 64: the diagonal block staged in LDS and solved by wave 0
// (lane = row), then the rows below by the workgroup,
// y(j1:) -= R(blk, j1:)^T y_blk.
__global__ void __launch_bounds__(kRT) trsv_upper_t_kernel(const double *R, int64_t ldr, int64_t n, double *y) {
  __shared__ double ys[64];
  __shared__ double rd[64][65];  // diagonal block, rd[row][col]
  const int tid = threadIdx.x;
  for (int64_t j0 = 0; j0 < n; j0 += 64) {
    const int nb = (int)min<int64_t>(64, n - j0);
    for (int e = tid; e < 64 * 64; e += kRT) {
      const int row = e % 64, col = e / 64;
      rd[row][col] = (row < nb && col < nb && row <= col) ? R[(j0 + row) + (j0 + col) * ldr] : 0.0;
    }
    __syncthreads();
    if (tid < 64) {
      double yt = (tid < nb) ? y[j0 + tid] : 0.0;
      for (int i = 0; i < nb; ++i) {
        const double yi = __shfl(yt, i) / rd[i][i];
        if (tid == i) yt = yi;
        if (tid > i && tid < nb) yt = fma(-rd[i][tid], yi, yt);
      }
      if (tid < nb) {
        y[j0 + tid] = yt;
        ys[tid] = yt;
      }
    }
    __syncthreads();
    for (int64_t row = j0 + nb + tid; row < n; row += kRT) {
      const double *rc = R + j0 + row * ldr;  // R(j0 .. j0 + nb - 1, row)
      double s0 = y[row], s1 = 0.0;
      int k = 0;
      for (; k + 1 < nb; k += 2) {
        s0 = fma(-rc[k], ys[k], s0);
        s1 = fma(-rc[k + 1], ys[k + 1], s1);
      }
      if (k < nb) s0 = fma(-rc[k], ys[k], s0);
      y[row] = s0 + s1;
    }
    __syncthreads();
  }
}

// out[0] = x . y (one workgroup, fixed-order sum).
__global__ void __launch_bounds__(kRT) dot_kernel(const double *x, const double *y, int64_t n, double *out) {
  __shared__ double red[kRT];
  double s0 = 0.0, s1 = 0.0;
  int64_t i = threadIdx.x;
  for (; i + kRT < n; i += 2 * kRT) {
    s0 = fma(x[i], y[i], s0);
    s1 = fma(x[i + kRT], y[i + kRT], s1);
  }
  if (i < n) s0 = fma(x[i], y[i], s0);
  const double s = block_sum(s0 + s1, red);
  if (threadIdx.x == 0) out[0] = s;
}

// y += sgn (num / den) x
__global__ void axpy_ratio_kernel(double *y, const double *x, int64_t n, const double *num, const double *den,
                                  double sgn) {
  const double a = sgn * (num[0] / den[0]);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = fma(a, x[i], y[i]);
}

// p = s + (num / den) p
__global__ void xpby_ratio_kernel(double *p, const double *s, int64_t n, const double *num, const double *den) {
  const double bta = num[0] / den[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = fma(bta, p[i], s[i]);
}

__global__ void copy_kernel(double *dst, const double *src, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// eta upper bound: sq = {||u||^2, ||x||^2, ||b||^2}, a_lo = scal[0]:
// out = ||u|| / (a_lo (a_lo ||x|| + ||b||)) >= eta(x) (a_lo <= ||A||_2).
__global__ void eta_kernel(const double *sq, const double *scal, double *out) {
  if (threadIdx.x == 0) {
    const double a = scal[0];
    out[0] = sqrt(sq[0]) / (a * (a * sqrt(sq[1]) + sqrt(sq[2])));
  }
}

int grid_for(int64_t n) { return (int)std::min<int64_t>((n + kRT - 1) / kRT, 4096); }

}  // namespace

hipError_t launch_colsq(const double *A, int64_t lda, int64_t m, int64_t n, double *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(colsq_kernel, dim3((unsigned)n), dim3(kRT), 0, s, A, lda, m, out);
  return hipGetLastError();
}

hipError_t launch_anorm_lower(const double *colsq, int64_t n, double *scal, hipStream_t s) {
  hipLaunchKernelGGL(anorm_kernel, dim3(1), dim3(kRT), 0, s, colsq, n, scal);
  return hipGetLastError();
}

hipError_t launch_resid(const double *A, int64_t lda, int64_t m, int64_t n, const double *x, const double *b,
                        double *r, hipStream_t s) {
  hipLaunchKernelGGL(gemv_kernel<true>, dim3((unsigned)((m + kRT - 1) / kRT)), dim3(kRT), 0, s, A, lda, m, n, x, b,
                     r);
  return hipGetLastError();
}

hipError_t launch_gemv(const double *A, int64_t lda, int64_t m, int64_t n, const double *x, double *y,
                       hipStream_t s) {
  hipLaunchKernelGGL(gemv_kernel<false>, dim3((unsigned)((m + kRT - 1) / kRT)), dim3(kRT), 0, s, A, lda, m, n, x,
                     (const double *)nullptr, y);
  return hipGetLastError();
}

hipError_t launch_atr(const double *A, int64_t lda, int64_t m, int64_t n, const double *r, double *u,
                      hipStream_t s) {
  hipLaunchKernelGGL(atr_kernel, dim3((unsigned)n), dim3(kRT), 0, s, A, lda, m, r, u);
  return hipGetLastError();
}

hipError_t launch_trsv_upper_t(const double *R, int64_t ldr, int64_t n, double *y, hipStream_t s) {
  hipLaunchKernelGGL(trsv_upper_t_kernel, dim3(1), dim3(kRT), 0, s, R, ldr, n, y);
  return hipGetLastError();
}

hipError_t launch_dot(const double *x, const double *y, int64_t n, double *out, hipStream_t s) {
  hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(kRT), 0, s, x, y, n, out);
  return hipGetLastError();
}

hipError_t launch_axpy_ratio(double *y, const double *x, int64_t n, const double *num, const double *den, double sgn,
                             hipStream_t s) {
  hipLaunchKernelGGL(axpy_ratio_kernel, dim3(grid_for(n)), dim3(kRT), 0, s, y, x, n, num, den, sgn);
  return hipGetLastError();
}

hipError_t launch_xpby_ratio(double *p, const double *sv, int64_t n, const double *num, const double *den,
                             hipStream_t s) {
  hipLaunchKernelGGL(xpby_ratio_kernel, dim3(grid_for(n)), dim3(kRT), 0, s, p, sv, n, num, den);
  return hipGetLastError();
}

hipError_t launch_copy(double *dst, const double *src, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n)), dim3(kRT), 0, s, dst, src, n);
  return hipGetLastError();
}

hipError_t launch_eta_bound(const double *sq, const double *scal, double *out, hipStream_t s) {
  hipLaunchKernelGGL(eta_kernel, dim3(1), dim3(64), 0, s, sq, scal, out);
  return hipGetLastError();
}

}  // namespace caqr
