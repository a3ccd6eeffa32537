// Batched least squares on top of the batched TSQR: for every problem,
// min ||A x - b|| = ||R x - (Q^T b)(0:n)|| (paper, Section 3.1: A = QR with the
// reflectors stored along the reduction tree).  Q^T is applied to each
// right-hand side with the stored reflectors themselves, in the order the
// factorization produced them: the leaves' reflectors (MLUPFACT), then the
// tree nodes' bottom-up (MLUPELIM), each reflector H = I - tau v v^T on its
// own (a right-hand side is one column, so there is no block to form T for).
// Then Q_thin^T b = D (Q_impl^T b)(0:n) and R x = that, by back substitution.
//
// One wave per (problem, leaf or node, right-hand side); the four waves of a
// workgroup are independent (no LDS, no barrier).  Column reductions are the
// 16-lane DPP butterfly followed by the four row sums in a fixed order, so
// results are deterministic.
#include "device_common.hpp"
#include "kernels.hpp"
#include "lsb.hpp"

namespace caqr {

namespace {

constexpr int kLsbWaves = 4;  // waves (items) per workgroup

__device__ __forceinline__ double wave_sum(double x) {
  x = row16_sum(x);
  return (readlane_f64(x, 0) + readlane_f64(x, 16)) + (readlane_f64(x, 32) + readlane_f64(x, 48));
}

// Leaf reflectors of leaf items[w].y of problem items[w].x applied to
// right-hand side items[w].z: rows of the leaf held 1, 2 or 4 per lane
// (row lane + 64 k of the leaf).
__global__ void __launch_bounds__(64 * kLsbWaves) lsb_leaf_kernel(const LsbProb *probs, const int4 *items,
                                                                  int nitems) {
  const int wv = (int)blockIdx.x * kLsbWaves + (int)(threadIdx.x >> 6);
  if (wv >= nitems) return;  // whole wave
  const int lane = threadIdx.x & 63;
  const int4 it = items[wv];
  const LsbProb p = probs[__builtin_amdgcn_readfirstlane(it.x)];
  const int leaf = __builtin_amdgcn_readfirstlane(it.y);
  const int rhs = __builtin_amdgcn_readfirstlane(it.z);
  const int64_t r0 = (int64_t)leaf * p.h;
  const int nk = p.h >> 6;
  double *bc = p.B + (int64_t)rhs * p.ldb;
  double bv[4], yv[4];
  bool ok[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t row = r0 + lane + 64 * k;
    ok[k] = k < nk && row < p.m;
    bv[k] = ok[k] ? bc[row] : 0.0;
    yv[k] = ok[k] ? p.A[row] : 0.0;  // column 0 of Y
  }
  for (int j = 0; j < p.b; ++j) {
    double yn[4];  // next column, loaded while this one is applied
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t row = r0 + lane + 64 * k;
      yn[k] = (ok[k] && j + 1 < p.b) ? p.A[row + (int64_t)(j + 1) * p.lda] : 0.0;
    }
    const double tau = p.tau_leaf[(int64_t)leaf * kMaxB + j];
    double v[4], s = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int rel = lane + 64 * k;
      v[k] = (rel > j) ? yv[k] : (rel == j ? 1.0 : 0.0);
      v[k] = ok[k] ? v[k] : 0.0;
      s = fma(v[k], bv[k], s);
    }
    const double tw = tau * wave_sum(s);
#pragma unroll
    for (int k = 0; k < 4; ++k) bv[k] = fma(-tw, v[k], bv[k]);
#pragma unroll
    for (int k = 0; k < 4; ++k) yv[k] = yn[k];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (ok[k]) bc[r0 + lane + 64 * k] = bv[k];
}

// Node reflectors of the group of survivor slot items[w].y at stride
// items[w].z of problem items[w].x (members g + t s, t < cnt <= arity),
// applied to right-hand side items[w].w: lane i holds row i of every member's
// top b rows.  Reflector j is [e_j ; V_1(0:j, j) ; ... ; V_{cnt-1}(0:j, j)],
// each V_t upper triangular over member t's slot; its dot product sums the
// members' products in each lane first, then over the wave.
__global__ void __launch_bounds__(64 * kLsbWaves) lsb_node_kernel(const LsbProb *probs, const int4 *items,
                                                                  int nitems) {
  constexpr int KMAX = 4;  // largest arity
  const int wv = (int)blockIdx.x * kLsbWaves + (int)(threadIdx.x >> 6);
  if (wv >= nitems) return;
  const int lane = threadIdx.x & 63;
  const int4 it = items[wv];
  const LsbProb p = probs[__builtin_amdgcn_readfirstlane(it.x)];
  const int g = __builtin_amdgcn_readfirstlane(it.y);
  const int s = __builtin_amdgcn_readfirstlane(it.z);
  const int rhs = __builtin_amdgcn_readfirstlane(it.w);
  const int cnt = min(p.arity, (p.L - g + s - 1) / s);
  double *bc = p.B + (int64_t)rhs * p.ldb;
  const int64_t rt = (int64_t)g * p.h + lane;
  const bool okt = lane < p.b && rt < p.m;
  double top = okt ? bc[rt] : 0.0;
  int64_t rc[KMAX - 1];
  bool okc[KMAX - 1];
  double child[KMAX - 1], vv[KMAX - 1];
#pragma unroll
  for (int t = 0; t < KMAX - 1; ++t) {
    rc[t] = (int64_t)(g + (t + 1) * s) * p.h + lane;
    okc[t] = t + 1 < cnt && lane < p.b && rc[t] < p.m;
    child[t] = okc[t] ? bc[rc[t]] : 0.0;
    vv[t] = (okc[t] && lane == 0) ? p.A[rc[t]] : 0.0;  // column 0 of V_t
  }
  for (int j = 0; j < p.b; ++j) {
    double vn[KMAX - 1];
#pragma unroll
    for (int t = 0; t < KMAX - 1; ++t)
      vn[t] = (okc[t] && j + 1 < p.b && lane <= j + 1) ? p.A[rc[t] + (int64_t)(j + 1) * p.lda] : 0.0;
    const double tau = p.tau_node[(int64_t)(g + s) * kMaxB + j];
    double prod = vv[0] * child[0];
#pragma unroll
    for (int t = 1; t < KMAX - 1; ++t) prod = fma(vv[t], child[t], prod);
    const double w = readlane_f64(top, j) + wave_sum(prod);
    const double tw = tau * w;
    if (lane == j) top -= tw;
#pragma unroll
    for (int t = 0; t < KMAX - 1; ++t) {
      child[t] = fma(-tw, vv[t], child[t]);
      vv[t] = vn[t];
    }
  }
  if (okt) bc[rt] = top;
#pragma unroll
  for (int t = 0; t < KMAX - 1; ++t)
    if (okc[t]) bc[rc[t]] = child[t];
}

// Rows 0..n-1 of right-hand side items[w].y of problem items[w].x: scaled by
// the signs D, then solved with the upper triangular R (top n x n of A) by
// back substitution, lane i on row i.  Status pair of (problem, rhs):
// 1 + first j with R_jj == 0 (else 0), and 1 if some R_jj or x_i is not finite.
__global__ void __launch_bounds__(64 * kLsbWaves) lsb_solve_kernel(const LsbProb *probs, const int2 *items,
                                                                   int nitems, int64_t *status) {
  const int wv = (int)blockIdx.x * kLsbWaves + (int)(threadIdx.x >> 6);
  if (wv >= nitems) return;
  const int lane = threadIdx.x & 63;
  const int2 it = items[wv];
  const LsbProb p = probs[__builtin_amdgcn_readfirstlane(it.x)];
  const int rhs = __builtin_amdgcn_readfirstlane(it.y);
  const int n = p.b;
  double *bc = p.B + (int64_t)rhs * p.ldb;
  const bool on = lane < n;
  double c = on ? p.d[lane] * bc[lane] : 0.0;
  const double rd = on ? p.A[lane + (int64_t)lane * p.lda] : 1.0;
  const uint64_t zero = __ballot(on && rd == 0.0);
  bool bad = on && !isfinite(rd);
  for (int j = n - 1; j >= 0; --j) {
    const double xj = readlane_f64(c, j) / readlane_f64(rd, j);
    if (lane == j) c = xj;
    if (lane < j) c = fma(-p.A[lane + (int64_t)j * p.lda], xj, c);
  }
  if (on) bc[lane] = c;
  bad = bad || (on && !isfinite(c));
  const uint64_t nonfinite = __ballot(bad);
  if (lane == 0) {
    int64_t *st = status + 2 * ((int64_t)p.status0 + rhs);
    st[0] = zero ? (int64_t)__builtin_ctzll(zero) + 1 : 0;
    st[1] = nonfinite ? 1 : 0;
  }
}

int waves_grid(int items) { return (items + kLsbWaves - 1) / kLsbWaves; }

}  // namespace

hipError_t launch_lsb_leaves(const LsbProb *probs, const int4 *items, int nitems, hipStream_t s) {
  if (nitems < 1) return hipSuccess;
  hipLaunchKernelGGL(lsb_leaf_kernel, dim3(waves_grid(nitems)), dim3(64 * kLsbWaves), 0, s, probs, items, nitems);
  return hipGetLastError();
}

hipError_t launch_lsb_nodes(const LsbProb *probs, const int4 *items, int nitems, hipStream_t s) {
  if (nitems < 1) return hipSuccess;
  hipLaunchKernelGGL(lsb_node_kernel, dim3(waves_grid(nitems)), dim3(64 * kLsbWaves), 0, s, probs, items, nitems);
  return hipGetLastError();
}

hipError_t launch_lsb_solve(const LsbProb *probs, const int2 *items, int nitems, int64_t *status, hipStream_t s) {
  if (nitems < 1) return hipSuccess;
  hipLaunchKernelGGL(lsb_solve_kernel, dim3(waves_grid(nitems)), dim3(64 * kLsbWaves), 0, s, probs, items, nitems,
                     status);
  return hipGetLastError();
}

}  // namespace caqr
