// Triangular factor T of a block of Householder reflectors, Q = I - Y T Y^T.
//
// T^{-1} = diag(1/tau) + strictly-upper(G) with G = Y^T Y (the product of the
// reflectors written in compact form), so each diagonal 16x16 block of T is
// solved column by column from the bottom up,
//     T(i, j) = -tau_i * sum_{i<k<=j} G(i, k) T(k, j),   T(j, j) = tau_j,
// (which also holds for tau_i = 0), and the blocks above the diagonal follow
// block column by block column, T(0:c0, blk) = -T(0:c0, 0:c0) (G(0:c0, blk) T(blk, blk)),
// as 16x16 block products on MFMA.
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
  // The blocks above the diagonal, as 16x16 block products on FP64 MFMA (each
  // four 16x16x4 steps): lane (i, k) = (lane % 16, lane / 16) supplies A(i, k)
  // and B(k, i); result (4r + lane / 16, lane % 16) in register r.
  const int li = lane & 15, lk = lane >> 4;
  // X(e, bc) = G(e, bc) T(bc, bc) for every block e < bc (six products over the
  // four waves), kept in T's free strictly-lower triangle: X(i, jj) of block
  // column bc at row 16 bc + jj, column i (< 16 bc); never read as T.
  for (int p = wave; p < NQ * (NQ - 1) / 2; p += 4) {
    int bc = 1, e = p;
    while (e >= bc) {
      e -= bc;
      ++bc;
    }
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int kk = 4 * s4 + lk;
      acc = mfma16x16x4(G[(16 * e + li) * ld + 16 * bc + kk], T[(16 * bc + kk) * ld + 16 * bc + li], acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) T[(16 * bc + li) * ld + 16 * e + 4 * r + lk] = acc[r];
  }
  __syncthreads();
  // T(e, bc) = -sum_{f = e .. bc-1} T(e, f) X(f, bc), block column by block
  // column (each needs the block columns left of it); wave e takes block row e
#pragma unroll
  for (int bc = 1; bc < NQ; ++bc) {
    const int e = wave;
    if (e < bc) {
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int f = e; f < bc; ++f) {
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int kk = 4 * s4 + lk;
          // A(i, k) = T(16e + i, 16f + k) (upper triangular on the diagonal
          // block, zero below it); B(k, j) = X(16f + k, j) = T(16bc + j, 16f + k)
          acc = mfma16x16x4(T[(16 * e + li) * ld + 16 * f + kk], T[(16 * bc + li) * ld + 16 * f + kk], acc);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) T[(16 * e + 4 * r + lk) * ld + 16 * bc + li] = -acc[r];
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
