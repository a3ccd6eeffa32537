// Triangular factor T of a block of Householder reflectors, Q = I - Y T Y^T.
//
// T^{-1} = diag(1/tau) + strictly-upper(G) with G = Y^T Y (the product of the
// reflectors written in compact form), so each diagonal 16x16 block of T is
// solved column by column from the bottom up,
//     T(i, j) = -tau_i * sum_{i<k<=j} G(i, k) T(k, j),   T(j, j) = tau_j,
// (which also holds for tau_i = 0), and the blocks above the diagonal follow
// block column by block column, T(0:c0, blk) = -T(0:c0, 0:c0) (G(0:c0, blk) T(blk, blk)).
// Every loop bound is a compile-time constant (masks instead of bounds), so
// the LDS reads are independent and pipelined.
#pragma once

#include "device_common.hpp"

namespace caqr {

// G and T are row-major in LDS with leading dimension ld (>= 64); G's strictly
// upper triangle is read, T's upper triangle is written (zero outside the b x b
// block); T's strictly-lower triangle is used as scratch.  taus[0..63] (zero
// beyond b).  Called by all 256 threads; ends with a barrier.
template <int NQ>
__device__ __forceinline__ void form_t_lds(int b, const double *G, double *T, const double *taus, int ld) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  // diagonal blocks: wave 0, lane = (block a, column jj)
  if (wave == 0) {
    const int a = lane >> 4, jj = lane & 15;
    const int a0 = 16 * a;
    const int j = a0 + jj;
    double t[16];
#pragma unroll
    for (int ii = 15; ii >= 0; --ii) {
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int kk = ii + 1; kk < 16; ++kk) {
        const double g = G[(a0 + ii) * ld + a0 + kk];
        if (kk & 1) s1 = fma(g, t[kk], s1);
        else s0 = fma(g, t[kk], s0);
      }
      const double ti = (a0 + ii < b) ? taus[a0 + ii] : 0.0;
      t[ii] = (ii < jj) ? -ti * (s0 + s1) : ((ii == jj && j < b) ? ti : 0.0);
    }
#pragma unroll
    for (int ii = 0; ii < 16; ++ii) T[(a0 + ii) * ld + j] = t[ii];
  }
  __syncthreads();
  if (NQ == 1) return;
  // X(:, blk) = G(0:c0, blk) T(blk, blk) for every block column, in one pass;
  // X(i, jj) of block column bc is kept in T's free strictly-lower triangle at
  // row c0 + jj, column i (< c0): disjoint for different bc, never read as T.
#pragma unroll
  for (int bc = 1; bc < NQ; ++bc) {
    const int c0 = 16 * bc;
#pragma unroll
    for (int e = 0; e < bc; ++e) {
      const int i = (tid >> 4) + 16 * e;
      const int jj = tid & 15;
      double s0 = 0.0, s1 = 0.0;
#pragma unroll 4
      for (int kk = 0; kk < 16; ++kk) {
        const double g = G[i * ld + c0 + kk];
        const double tv = (kk <= jj) ? T[(c0 + kk) * ld + c0 + jj] : 0.0;
        if (kk & 1) s1 = fma(g, tv, s1);
        else s0 = fma(g, tv, s0);
      }
      T[(c0 + jj) * ld + i] = s0 + s1;
    }
  }
  __syncthreads();
  // T(0:c0, blk) = -T(0:c0, 0:c0) X(:, blk), block column by block column
#pragma unroll
  for (int bc = 1; bc < NQ; ++bc) {
    const int c0 = 16 * bc;
#pragma unroll
    for (int e = 0; e < bc; ++e) {
      const int i = (tid >> 4) + 16 * e;
      const int jj = tid & 15;
      double s0 = 0.0, s1 = 0.0;
#pragma unroll 4
      for (int k = 0; k < c0; ++k) {
        const double tv = (k >= i) ? T[i * ld + k] : 0.0;
        const double xv = T[(c0 + jj) * ld + k];
        if (k & 1) s1 = fma(tv, xv, s1);
        else s0 = fma(tv, xv, s0);
      }
      T[i * ld + c0 + jj] = -(s0 + s1);
    }
    __syncthreads();
  }
}

// T (LDS, row-major, ld) to global as a 64x64 column-major block (ld 64),
// zero outside the upper triangle of the b x b block.
__device__ __forceinline__ void store_t_global(double *Tg, int b, const double *T, int ld) {
  for (int e = threadIdx.x; e < kMaxB * kMaxB; e += kThreads) {
    const int i = e & 63, j = e >> 6;
    Tg[e] = (i <= j && j < b) ? T[i * ld + j] : 0.0;
  }
}

}  // namespace caqr
