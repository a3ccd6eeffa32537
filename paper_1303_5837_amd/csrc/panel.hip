// Panel factorization (TSQR) for one tall-skinny panel of width b <= 64.
//
// This is the panel step of ML-CAQR (paper, Section 3.1, Algorithm 1 and items
// 1(a)-1(b) of its description): the panel is split into row blocks, each block
// is factored by Householder QR, and the resulting b-by-b R factors are
// eliminated two by two along a binary reduction tree; each elimination is the
// QR of two stacked upper triangles.  On the GPU the hierarchy levels are:
//
//   level 1  a row block (leaf, h = 16*RPT rows) factored by one workgroup with
//            the block held in registers; column reductions are DPP butterflies
//            inside 16-lane rows (see device_common.hpp for the layout);
//   level 2  the workgroup's own leaves (leaves_per_wg of them) combined in the
//            same workgroup, right after they are factored;
//   level 3  the workgroups' roots combined across the device: the second
//            workgroup to finish below a tree node (an agent-scope atomic
//            ticket) performs that node's elimination, so no workgroup ever
//            waits for another and the pairing is fixed by index, never by
//            arrival order.
//
// The tree is the binary tree over leaves that pairs i with i + 2^(k-1) at
// level k (i a multiple of 2^k), the lower index on top.  Node ids are the
// index of the right (eliminated) child.  The stacked elimination is computed
// once, by one workgroup (the paper computes it at both partners).
//
// Outputs: R (b-by-b, non-negative diagonal) in the top rows of the panel; leaf
// reflectors below each leaf's diagonal; each node's V (upper triangular) over
// the eliminated child's R slot; tau per leaf/node; optionally T per leaf/node
// (compact WY, Q = I - Y T Y^T); the signs D of the root R.
#include <cfloat>

#include "device_common.hpp"
#include "kernels.hpp"

namespace caqr {

namespace {

constexpr int kLdG = kMaxB + 1;  // padded leading dimension of G and T in LDS

template <bool FORM_T>
struct PanelSmem {
  double v[2][16 * 16];  // Householder vector of the current step (by row), double-buffered
  double tau[2];
  double taus[kMaxB];
  double dsign[kMaxB];
  int flag;
  double G[FORM_T ? kMaxB * kLdG : 1];  // strictly upper Y^T Y
  double T[FORM_T ? kMaxB * kLdG : 1];  // T of the current factorization
  double X[FORM_T ? 48 * 16 : 1];       // block product scratch of the T formation
};

// One Householder step per column j = 0..b-1 on the block held in a[][]:
// NACT chunk rows of 16 (LEAF: rows 0..16*NACT-1 of a dense block; STACK: two
// stacked upper triangles, R_top in chunks 0..NQ-1 and R_bot in chunks
// NQ..2NQ-1).  Reflector convention: beta = -sign(alpha) ||x||,
// tau = (beta - alpha) / beta, v = [1; x(2:) / (alpha - beta)]; x(2:) == 0 gives
// tau = 0 (H = I).  The norm is an unscaled sum of squares, recomputed with
// power-of-two scaling when alpha^2 + sigma is zero, subnormal or overflows.
template <int NCH, int NQ, int NACT, bool STACK, bool FORM_T>
__device__ __forceinline__ void householder_steps(double (&a)[NCH][NQ], int b, PanelSmem<FORM_T> &sm) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int r = lane & 15;
  const int c = (tid >> 6) * 4 + (lane >> 4);
#pragma unroll
  for (int Q = 0; Q < NQ; ++Q) {
    for (int cj = 0; cj < 16; ++cj) {
      const int j = 16 * Q + cj;
      if (j >= b) break;
      const int par = j & 1;
      if (c == cj) {
        // ---- owner DPP row: reflector of column j (slot Q of this thread)
        double sig = 0.0;
#pragma unroll
        for (int i = 0; i < NACT; ++i) {
          const bool act = STACK ? (i == Q || (i >= NQ && i <= NQ + Q)) : (i >= Q);
          if (!act) continue;
          const bool below = (i > Q) || (r > cj);
          const double e = a[i][Q];
          sig = below ? fma(e, e, sig) : sig;
        }
        sig = row16_sum(sig);
        const double alpha = readlane_f64(a[Q][Q], (cj & 3) * 16 + cj);
        const double s2 = fma(alpha, alpha, sig);
        // The reflector is formed from x scaled by 2^sh: sh = 0 normally; when
        // alpha^2 + sigma is zero, subnormal, overflowing or NaN, sh = -ilogb(max|x|)
        // (ldexp per element is exact), so that mu, tau and 1 / (alpha - beta)
        // are computed on normal numbers.
        int sh = 0;
        double alpha_s = alpha, sig_s = sig, mu_s;
        if (s2 >= DBL_MIN && s2 <= DBL_MAX) {
          mu_s = sqrt(s2);
        } else {
          double mx = 0.0;
#pragma unroll
          for (int i = 0; i < NACT; ++i) {
            const bool act = STACK ? (i == Q || (i >= NQ && i <= NQ + Q)) : (i >= Q);
            if (!act) continue;
            const bool inx = (i > Q) || (r >= cj);
            mx = inx ? fmax(mx, fabs(a[i][Q])) : mx;
          }
          mx = row16_max(mx);
          if (mx == 0.0 || !(mx <= DBL_MAX)) {  // zero column, or Inf/NaN (propagated)
            mu_s = (mx == 0.0) ? 0.0 : sqrt(s2);
            sig_s = (mx == 0.0) ? 0.0 : sig;
          } else {
            sh = -ilogb(mx);
            double ss = 0.0;
#pragma unroll
            for (int i = 0; i < NACT; ++i) {
              const bool act = STACK ? (i == Q || (i >= NQ && i <= NQ + Q)) : (i >= Q);
              if (!act) continue;
              const bool below = (i > Q) || (r > cj);
              const double e = ldexp(a[i][Q], sh);
              ss = below ? fma(e, e, ss) : ss;
            }
            sig_s = row16_sum(ss);
            alpha_s = ldexp(alpha, sh);
            mu_s = sqrt(fma(alpha_s, alpha_s, sig_s));
          }
        }
        double beta, tau, scal;
        if (sig_s == 0.0) {
          beta = alpha;
          tau = 0.0;
          scal = 0.0;
        } else {
          const double beta_s = -copysign(mu_s, alpha_s);
          tau = (beta_s - alpha_s) / beta_s;
          scal = 1.0 / (alpha_s - beta_s);
          beta = ldexp(beta_s, -sh);
        }
#pragma unroll
        for (int i = 0; i < NACT; ++i) {
          const bool act = STACK ? (i == Q || (i >= NQ && i <= NQ + Q)) : (i >= Q);
          if (!act) continue;
          double vv;
          if (i > Q || r > cj) {
            vv = ldexp(a[i][Q], sh) * scal;
            a[i][Q] = vv;
          } else if (r == cj && i == Q) {
            vv = 1.0;
            a[i][Q] = beta;
          } else {
            vv = 0.0;
          }
          sm.v[par][16 * i + r] = vv;
        }
        if (r == 0) {
          sm.tau[par] = tau;
          sm.taus[j] = tau;
        }
      }
      __syncthreads();
      // ---- every thread: w = v^T A(:, col) for its column slots, then the rank-1 update.
      // v is read from LDS where it is used (not held across the reductions).
      // Slots whose columns are all finished (q < Q) are skipped unless their
      // dot products are needed for T (G = Y^T Y).
      const double tau = sm.tau[par];
      const double *vrow = sm.v[par] + r;
      double p[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) p[q] = 0.0;
#pragma unroll
      for (int i = 0; i < NACT; ++i) {
        const bool act = STACK ? (i == Q || (i >= NQ && i <= NQ + Q)) : (i >= Q);
        if (!act) continue;
        const double vi = vrow[16 * i];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          if (!FORM_T && q < Q) continue;
          p[q] = fma(vi, a[i][q], p[q]);
        }
      }
      double coef[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        if (!FORM_T && q < Q) continue;
        const double w = row16_sum(p[q]);
        const int col = c + 16 * q;
        if (FORM_T) {
          if (r == 0 && col < j) sm.G[col * kLdG + j] = w;
        }
        coef[q] = (col > j && col < b) ? tau * w : 0.0;
      }
#pragma unroll
      for (int i = 0; i < NACT; ++i) {
        const bool act = STACK ? (i == Q || (i >= NQ && i <= NQ + Q)) : (i >= Q);
        if (!act) continue;
        const double vi = vrow[16 * i];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          if (q < Q) continue;  // finished columns are never updated
          a[i][q] = fma(-coef[q], vi, a[i][q]);
        }
      }
    }
  }
}

// T (upper triangular, Q = I - Y T Y^T) from G = strictly-upper(Y^T Y) and tau,
// by the blocked forward recurrence: diagonal 16x16 blocks first
// (T_jj = tau_j, T(0:j, j) = -tau_j T(0:j, 0:j) G(0:j, j)), then each block
// column bc: T(0:16bc, blk) = -T(0:16bc, 0:16bc) G(0:16bc, blk) T(blk, blk).
// Result in sm.T (kLdG-strided, row-major by row index), zero outside 0..b-1.
template <int NQ, bool FORM_T>
__device__ __forceinline__ void form_t(int b, PanelSmem<FORM_T> &sm) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  // diagonal blocks: wave a handles block a, lanes 0..15 own one row each
  if (wave < NQ && lane < 16) {
    const int a0 = 16 * wave;
    const int i = lane;
    double t[16];
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
      const int j = a0 + jj;
      const double tj = (j < b) ? sm.taus[j] : 0.0;
      double s = 0.0;
#pragma unroll
      for (int kk = 0; kk < jj; ++kk) {
        const double g = sm.G[(a0 + kk) * kLdG + j];
        s = (kk >= i) ? fma(t[kk], g, s) : s;
      }
      t[jj] = (i < jj) ? -tj * s : ((i == jj) ? tj : 0.0);
    }
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) sm.T[(a0 + i) * kLdG + a0 + jj] = t[jj];
    // zero the strictly-lower part of this block row outside the diagonal block
    for (int k = 0; k < a0; ++k) sm.T[(a0 + i) * kLdG + k] = 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int bc = 1; bc < NQ; ++bc) {
    const int c0 = 16 * bc;
    // X = G(0:c0, c0:c0+16) * T(c0:c0+16, c0:c0+16)
    for (int e = tid; e < c0 * 16; e += kThreads) {
      const int i = e >> 4, jj = e & 15;
      double s = 0.0;
      for (int kk = 0; kk <= jj; ++kk) s = fma(sm.G[i * kLdG + c0 + kk], sm.T[(c0 + kk) * kLdG + c0 + jj], s);
      sm.X[i * 16 + jj] = s;
    }
    __syncthreads();
    // T(0:c0, c0:c0+16) = -T(0:c0, 0:c0) * X
    for (int e = tid; e < c0 * 16; e += kThreads) {
      const int i = e >> 4, jj = e & 15;
      double s = 0.0;
      for (int k = i; k < c0; ++k) s = fma(sm.T[i * kLdG + k], sm.X[k * 16 + jj], s);
      sm.T[i * kLdG + c0 + jj] = -s;
    }
    __syncthreads();
  }
}

// Write sm.T to global as a 64x64 column-major block (ld 64), zero outside b.
template <bool FORM_T>
__device__ __forceinline__ void store_t(double *Tg, int b, const PanelSmem<FORM_T> &sm) {
  for (int e = threadIdx.x; e < kMaxB * kMaxB; e += kThreads) {
    const int i = e & 63, j = e >> 6;
    Tg[e] = (i <= j && j < b) ? sm.T[i * kLdG + j] : 0.0;
  }
}

template <bool FORM_T>
__device__ __forceinline__ void clear_g(PanelSmem<FORM_T> &sm) {
  if (FORM_T)
    for (int e = threadIdx.x; e < kMaxB * kLdG; e += kThreads) sm.G[e] = 0.0;
}

// Global element (row, col) of the panel, row within [0, m).
__device__ __forceinline__ double *pan(const PanelParams &p, int64_t row, int col) {
  return p.A + row + (int64_t)col * p.lda;
}

// Load the upper triangle of the R stored at slot `leaf` into chunks
// base..base+NQ-1 (zeros elsewhere).
template <int NCH, int NQ>
__device__ __forceinline__ void load_r(double (&a)[NCH][NQ], const PanelParams &p, int64_t slot_row, int base) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15;
  const int c = (threadIdx.x >> 6) * 4 + (lane >> 4);
#pragma unroll
  for (int i = 0; i < NQ; ++i)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int row = 16 * i + r, col = c + 16 * q;
      const int64_t grow = slot_row + row;
      a[base + i][q] = (row <= col && col < p.b && grow < p.m) ? *pan(p, grow, col) : 0.0;
    }
}

// Store the upper triangle (incl. diagonal) held in chunks base..base+NQ-1 to
// the rows starting at slot_row.
template <int NCH, int NQ>
__device__ __forceinline__ void store_upper(const double (&a)[NCH][NQ], const PanelParams &p, int64_t slot_row,
                                            int base) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15;
  const int c = (threadIdx.x >> 6) * 4 + (lane >> 4);
#pragma unroll
  for (int i = 0; i < NQ; ++i)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int row = 16 * i + r, col = c + 16 * q;
      const int64_t grow = slot_row + row;
      if (row <= col && col < p.b && grow < p.m) *pan(p, grow, col) = a[base + i][q];
    }
}

// Eliminate the R at slot `right` against the R at slot `left` (both read from
// global).  Writes V over the right slot, tau/T of node `right`, and the new
// R over the left slot.  The new R stays in chunks 0..NQ-1.
template <int NCH, int NQ, bool FORM_T>
__device__ __forceinline__ void combine(double (&a)[NCH][NQ], const PanelParams &p, int left, int right, int h,
                        PanelSmem<FORM_T> &sm) {
  const int64_t lrow = (int64_t)left * h, rrow = (int64_t)right * h;
  load_r<NCH, NQ>(a, p, lrow, 0);
  load_r<NCH, NQ>(a, p, rrow, NQ);
  clear_g(sm);
  __syncthreads();
  householder_steps<NCH, NQ, 2 * NQ, true, FORM_T>(a, p.b, sm);
  store_upper<NCH, NQ>(a, p, rrow, NQ);  // V of the node
  store_upper<NCH, NQ>(a, p, lrow, 0);   // R of the survivor
  __syncthreads();
  if (threadIdx.x < kMaxB) p.tau_node[(int64_t)right * kMaxB + threadIdx.x] = (threadIdx.x < p.b) ? sm.taus[threadIdx.x] : 0.0;
  if (FORM_T) {
    form_t<NQ, FORM_T>(p.b, sm);
    store_t(p.T_node + (int64_t)right * kMaxB * kMaxB, p.b, sm);
  }
  __syncthreads();
}

// Last-arriver ticket on node `node`; true when this workgroup arrived second
// (and must perform the elimination).  Publishes this workgroup's prior global
// stores before the ticket and acquires the partner's after it.
template <bool FORM_T>
__device__ __forceinline__ bool arrive(const PanelParams &p, int node, PanelSmem<FORM_T> &sm) {
  fence_release();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned old = ticket_add(p.tickets + node);
    sm.flag = (int)old;
    if (old == 1u) ticket_clear(p.tickets + node);
  }
  __syncthreads();
  const bool second = sm.flag == 1;
  if (second) fence_acquire();
  return second;
}

template <int RPT, int NQ, bool FORM_T>
__global__ void __launch_bounds__(kThreads, 2) tsqr_panel_kernel(PanelParams p) {
  constexpr int NCH = (RPT > 2 * NQ) ? RPT : 2 * NQ;
  constexpr int H = 16 * RPT;
  __shared__ PanelSmem<FORM_T> sm;
  double a[NCH][NQ];
  const int lane = threadIdx.x & 63;
  const int r = lane & 15;
  const int c = (threadIdx.x >> 6) * 4 + (lane >> 4);
  const int leaf0 = blockIdx.x * p.lpw;
  const int nleaves = min(p.lpw, p.L - leaf0);

  for (int li = 0; li < nleaves; ++li) {
    const int leaf = leaf0 + li;
    const int64_t row0 = (int64_t)leaf * H;
    // ---- level 1: factor the leaf block in registers
    // uniform fast path: the whole leaf in range and the panel 16*NQ wide
    const bool full = row0 + H <= p.m && p.b == 16 * NQ;
    if (full) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const double *colp = p.A + row0 + r + (int64_t)(c + 16 * q) * p.lda;
#pragma unroll
        for (int i = 0; i < NCH; ++i) a[i][q] = (i < RPT) ? colp[16 * i] : 0.0;
      }
    } else {
#pragma unroll
      for (int i = 0; i < NCH; ++i)
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int64_t grow = row0 + 16 * i + r;
          const int col = c + 16 * q;
          a[i][q] = (i < RPT && grow < p.m && col < p.b) ? *pan(p, grow, col) : 0.0;
        }
    }
    clear_g(sm);
    __syncthreads();
    householder_steps<NCH, NQ, RPT, false, FORM_T>(a, p.b, sm);
    if (full) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        double *colp = p.A + row0 + r + (int64_t)(c + 16 * q) * p.lda;
#pragma unroll
        for (int i = 0; i < RPT; ++i) colp[16 * i] = a[i][q];
      }
    } else {
#pragma unroll
      for (int i = 0; i < RPT; ++i)
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int64_t grow = row0 + 16 * i + r;
          const int col = c + 16 * q;
          if (grow < p.m && col < p.b) *pan(p, grow, col) = a[i][q];
        }
    }
    __syncthreads();
    if (threadIdx.x < kMaxB)
      p.tau_leaf[(int64_t)leaf * kMaxB + threadIdx.x] = (threadIdx.x < p.b) ? sm.taus[threadIdx.x] : 0.0;
    if (FORM_T) {
      form_t<NQ, FORM_T>(p.b, sm);
      store_t(p.T_leaf + (int64_t)leaf * kMaxB * kMaxB, p.b, sm);
    }
    __syncthreads();

    // ---- levels 2 and 3: climb the binary tree from this leaf
    int rt = leaf;  // root of the subtree this workgroup currently holds
    bool go_on = true;
    for (int half = 1; half < p.L; half <<= 1) {
      if ((rt & (2 * half - 1)) == 0) {  // left child at this level
        const int partner = rt + half;
        if (partner >= p.L) continue;                // no sibling: pass through
        if (partner < leaf0 + nleaves) {             // sibling is a later leaf of this workgroup
          go_on = false;
          break;
        }
        if (!arrive(p, partner, sm)) return;         // the sibling's workgroup finishes the node
        combine<NCH, NQ, FORM_T>(a, p, rt, partner, H, sm);
      } else {  // right child: node id rt, left sibling rt - half
        const int left = rt - half;
        if (left < leaf0) {
          if (!arrive(p, rt, sm)) return;
        }
        combine<NCH, NQ, FORM_T>(a, p, left, rt, H, sm);
        rt = left;
      }
    }
    if (!go_on) continue;
    // ---- root: make the diagonal non-negative, R <- D R, record D
    __syncthreads();
    load_r<NCH, NQ>(a, p, 0, 0);
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int row = 16 * i + r;
      if (c == r && row < p.b) sm.dsign[row] = (a[i][i] < 0.0) ? -1.0 : 1.0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NQ; ++i)
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int row = 16 * i + r, col = c + 16 * q;
        if (row <= col && col < p.b) a[i][q] *= sm.dsign[row];
      }
    store_upper<NCH, NQ>(a, p, 0, 0);
    if (threadIdx.x < p.b) p.d[threadIdx.x] = sm.dsign[threadIdx.x];
  }
}

template <int RPT, int NQ, bool FORM_T>
hipError_t launch_panel_t(const PanelParams &p, hipStream_t s) {
  const int grid = (p.L + p.lpw - 1) / p.lpw;
  hipLaunchKernelGGL((tsqr_panel_kernel<RPT, NQ, FORM_T>), dim3(grid), dim3(kThreads), 0, s, p);
  return hipGetLastError();
}

template <int RPT, bool FORM_T>
hipError_t launch_panel_nq(const PanelParams &p, hipStream_t s) {
  switch ((p.b + 15) / 16) {
    case 1: return launch_panel_t<RPT, 1, FORM_T>(p, s);
    case 2: return launch_panel_t<RPT, 2, FORM_T>(p, s);
    case 3: return launch_panel_t<RPT, 3, FORM_T>(p, s);
    case 4: return launch_panel_t<RPT, 4, FORM_T>(p, s);
    default: return hipErrorInvalidValue;
  }
}

template <bool FORM_T>
hipError_t launch_panel_rpt(const PanelParams &p, int leaf_rows, hipStream_t s) {
  switch (leaf_rows) {
    case 64: return launch_panel_nq<4, FORM_T>(p, s);
    case 128: return launch_panel_nq<8, FORM_T>(p, s);
    case 256: return launch_panel_nq<16, FORM_T>(p, s);
    default: return hipErrorInvalidValue;
  }
}

// T of one leaf (blockIdx.x < L) or node (blockIdx.x = L + node id) of a panel
// that was factored without T.  G = strictly-upper(Y^T Y) is computed on FP64
// MFMA (leaf: Y unit lower trapezoidal, h rows; node: [I; V], whose identity
// part contributes nothing off the diagonal), then T by the same blocked
// recurrence as in the panel kernel.
template <int NQ>
__global__ void __launch_bounds__(kThreads) form_t_kernel(FormTParams f) {
  __shared__ PanelSmem<true> sm;
  const bool is_leaf = (int)blockIdx.x < f.L;
  const int idx = is_leaf ? (int)blockIdx.x : (int)blockIdx.x - f.L;
  if (!is_leaf && idx == 0) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t row0 = (int64_t)idx * f.h;
  const int rows = is_leaf ? f.h : 16 * NQ;
  for (int e = threadIdx.x; e < kMaxB * kLdG; e += kThreads) sm.G[e] = 0.0;
  if (threadIdx.x < kMaxB) {
    const double *tau = is_leaf ? f.tau_leaf : f.tau_node;
    sm.taus[threadIdx.x] = (threadIdx.x < f.b) ? tau[(int64_t)idx * kMaxB + threadIdx.x] : 0.0;
  }
  __syncthreads();
  if (wave < NQ) {
    f64x4 g[NQ];
#pragma unroll
    for (int a = 0; a < NQ; ++a) g[a] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < rows / 4; ++s) {
      const int row = 4 * s + lk;
      const int64_t grow = row0 + row;
      // reflector entry (row, col) of this leaf/node
      auto refl = [&](int col) -> double {
        if (col >= f.b) return 0.0;
        if (is_leaf) {
          if (row == col) return 1.0;
          return (row > col && grow < f.m) ? f.Y[grow + (int64_t)col * f.ldy] : 0.0;
        }
        return (row <= col && grow < f.m) ? f.Y[grow + (int64_t)col * f.ldy] : 0.0;
      };
      const double av = refl(16 * wave + li);
#pragma unroll
      for (int a = 0; a < NQ; ++a) g[a] = mfma16x16x4(av, refl(16 * a + li), g[a]);
    }
#pragma unroll
    for (int a = 0; a < NQ; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * wave + 4 * r + lk, k = 16 * a + li;
        if (i < k) sm.G[i * kLdG + k] = g[a][r];
      }
  }
  __syncthreads();
  form_t<NQ, true>(f.b, sm);
  store_t(is_leaf ? f.T_leaf + (int64_t)idx * kMaxB * kMaxB : f.T_node + (int64_t)idx * kMaxB * kMaxB, f.b, sm);
}

template <int NQ>
hipError_t launch_form_t_nq(const FormTParams &f, hipStream_t s) {
  hipLaunchKernelGGL((form_t_kernel<NQ>), dim3(2 * f.L), dim3(kThreads), 0, s, f);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_tsqr_panel(const PanelParams &p, int leaf_rows, bool form_t, hipStream_t s) {
  if (p.b < 1 || p.b > kMaxB || p.L < 1 || p.lpw < 1) return hipErrorInvalidValue;
  return form_t ? launch_panel_rpt<true>(p, leaf_rows, s) : launch_panel_rpt<false>(p, leaf_rows, s);
}

}  // namespace caqr

namespace caqr {

hipError_t launch_form_t(const FormTParams &f, hipStream_t s) {
  if (f.b < 1 || f.b > kMaxB || f.L < 1) return hipErrorInvalidValue;
  switch ((f.b + 15) / 16) {
    case 1: return launch_form_t_nq<1>(f, s);
    case 2: return launch_form_t_nq<2>(f, s);
    case 3: return launch_form_t_nq<3>(f, s);
    case 4: return launch_form_t_nq<4>(f, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace caqr
