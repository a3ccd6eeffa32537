// Least-squares helpers: back substitution with the R of the factorization and
// the numerical checks that ls_solve reports (zero or non-finite R_jj, non-finite
// solution).  The solve is min ||A x - b|| = ||R x - (Q^T b)(0:n)|| for full-rank
// A (paper, Section 3.1 names least squares as a use of A = QR).
#include "device_common.hpp"
#include "kernels.hpp"

namespace caqr {

namespace {

constexpr int kBlk = 64;  // diagonal block of the blocked back substitution

// One workgroup per right-hand side.  Blocks of 64 rows from the bottom: the
// 64x64 diagonal block is staged in LDS (coalesced, one round trip) and solved
// by wave 0 (row by row, lane = row, every R entry an LDS read), then the rows
// above are updated by the whole workgroup, B(0:j0) -= R(0:j0, blk) x_blk.
__global__ void __launch_bounds__(kThreads) trsm_upper_kernel(const double *R, int64_t ldr, int64_t n, double *B,
                                                               int64_t ldb) {
  double *b = B + (int64_t)blockIdx.x * ldb;
  __shared__ double xs[kBlk];
  __shared__ double rd[kBlk][kBlk + 1];  // diagonal block, rd[col][row]
  const int tid = threadIdx.x;
  for (int64_t j1 = n; j1 > 0; j1 -= kBlk) {
    const int64_t j0 = (j1 >= kBlk) ? j1 - kBlk : 0;
    const int nb = (int)(j1 - j0);
    for (int e = tid; e < kBlk * kBlk; e += kThreads) {
      const int row = e % kBlk, col = e / kBlk;
      rd[col][row] = (row < nb && col < nb && row <= col) ? R[(j0 + row) + (j0 + col) * ldr] : 0.0;
    }
    __syncthreads();
    if (tid < 64) {
      // lane t owns row j0 + t of the block
      double bt = (tid < nb) ? b[j0 + tid] : 0.0;
      for (int i = nb - 1; i >= 0; --i) {
        const double bi = __shfl(bt, i);
        const double xi = bi / rd[i][i];
        if (tid == i) bt = xi;
        if (tid < i) bt = fma(-rd[i][tid], xi, bt);
      }
      if (tid < nb) {
        b[j0 + tid] = bt;
        xs[tid] = bt;
      }
    }
    __syncthreads();
    for (int64_t row = tid; row < j0; row += kThreads) {
      double s0 = b[row], s1 = 0.0;
      int k = 0;
      for (; k + 1 < nb; k += 2) {
        s0 = fma(-R[row + (j0 + k) * ldr], xs[k], s0);
        s1 = fma(-R[row + (j0 + k + 1) * ldr], xs[k + 1], s1);
      }
      if (k < nb) s0 = fma(-R[row + (j0 + k) * ldr], xs[k], s0);
      b[row] = s0 + s1;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kThreads) check_kernel(const double *R, int64_t ldr, int64_t n, const double *X,
                                                         int64_t ldx, int64_t nrhs, int64_t *status) {
  __shared__ int64_t first_zero;
  __shared__ int bad;
  if (threadIdx.x == 0) {
    first_zero = n;
    bad = 0;
  }
  __syncthreads();
  for (int64_t j = threadIdx.x; j < n; j += kThreads) {
    const double d = R[j + j * ldr];
    if (d == 0.0) atomicMin((unsigned long long *)&first_zero, (unsigned long long)j);
    if (!isfinite(d)) bad = 1;
  }
  for (int64_t e = threadIdx.x; e < n * nrhs; e += kThreads) {
    const double x = X[(e % n) + (e / n) * ldx];
    if (!isfinite(x)) bad = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    status[0] = (first_zero < n) ? first_zero + 1 : 0;
    status[1] = bad;
  }
}

}  // namespace

hipError_t launch_trsm_upper(const double *R, int64_t ldr, int64_t n, double *B, int64_t ldb, int64_t nrhs,
                             hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(trsm_upper_kernel, dim3((unsigned)nrhs), dim3(kThreads), 0, s, R, ldr, n, B, ldb);
  return hipGetLastError();
}

hipError_t launch_check_solution(const double *R, int64_t ldr, int64_t n, const double *X, int64_t ldx,
                                 int64_t nrhs, int64_t *status, hipStream_t s) {
  hipLaunchKernelGGL(check_kernel, dim3(1), dim3(kThreads), 0, s, R, ldr, n, X, ldx, nrhs, status);
  return hipGetLastError();
}

}  // namespace caqr
