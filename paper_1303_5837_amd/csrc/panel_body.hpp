// Device code of the panel factorization (TSQR) of one tall-skinny panel of
// width b <= 64, shared by the translation units that instantiate its kernels
// (panel.hip, panel_ib.hip, panel_batched_f64.hip, panel_batched_f32.hip).
//
// This is the panel step of ML-CAQR (paper, Section 3.1, Algorithm 1 and items
// 1(a)-1(b) of its description): the panel is split into row blocks, each block
// is factored by Householder QR, and the resulting b-by-b R factors are
// eliminated along a reduction tree; each elimination is the QR of the stacked
// upper triangles of one tree node's members.  On the GPU the hierarchy levels
// are:
//
//   level 1  a row block (leaf, h = 16*RPT rows) factored by one workgroup with
//            the block held in registers; column reductions are DPP butterflies
//            inside 16-lane rows (see device_common.hpp for the layout);
//   level 2  the workgroup's own leaves (leaves_per_wg of them) combined in the
//            same workgroup, right after they are factored;
//   level 3  the workgroups' roots combined across the device: the last
//            workgroup to finish below a tree node (an agent-scope atomic
//            ticket) performs that node's elimination, so no workgroup ever
//            waits for another and the grouping is fixed by index, never by
//            arrival order.
//
// The tree has arity K (2 or 4): level s = K^j (j = 0, 1, ...) groups the
// slots g, g + s, ..., g + (K - 1) s, g a multiple of K s, the lowest index on
// top (for K = 2 this pairs i with i + 2^(k-1) at level k).  Node ids are the
// index of the first eliminated member, g + s.  The stacked elimination is
// computed once, by one workgroup (the paper computes it at both partners).  With an
// inner block (the block size of the level below, Section 3.1 item 1(a)),
// leaves and eliminations are factored block by block (InnerBlock below).
//
// Outputs: R (b-by-b, non-negative diagonal) in the top rows of the panel; leaf
// reflectors below each leaf's diagonal; each node's V (upper triangular) over
// each eliminated member's R slot; tau per leaf/node; the signs D of the root R.
// The compact-WY factors T (Q = I - Y T Y^T) of every leaf and node are formed
// afterwards by one separate launch, all of them in parallel, so that the tree
// climb (the critical path of the panel) carries no T work.
#pragma once

#include <cfloat>

#include "device_common.hpp"
#include "kernels.hpp"

namespace caqr {

namespace {

// Waves per panel workgroup.  A workgroup of W wave64s holds a block with
// thread t (wave w = t / 64, lane l = t % 64) owning the elements
//     (row 16 i + l % 16, column c + 4 W s),  c = 4 w + l / 16 = 0 .. 4W - 1,
// for chunk i and column slot s: every column lives in the 16 lanes of one
// DPP row, which hold all its rows, so a column reduction is the same 4-step
// butterfly over the same partial sums whatever W is, and the results do not
// depend on W.  Four waves: eight halve each thread's column slots (and the
// dot products, reductions and updates per step) but were slower on every
// panel shape measured (an eight-wave barrier per step, and one workgroup per
// CU instead of two).
constexpr int kPanelWaves = 4;

template <class T>
struct PanelSmem {
  T v[2][16 * 16];  // Householder vector of the current step (by row), double-buffered
  T tau[2];
  T taus[kMaxB];
  T dsign[kMaxB];
  int flag;
};

// Inner block of a Householder factorization (paper, Section 3.1, item 1(a):
// a level factors its part of a panel of width b_r with the block size
// b_{r-1} of the level below).  With an inner block of KB columns a step
// updates only the columns of its own block; once the block is finished its
// reflectors are applied to the columns right of it as one transformation,
// Q_blk^T c = c - V z with z = T^T (V^T c) obtained by forward substitution,
//     z_k = tau_k (w_k - sum_{l<k} G(l,k) z_l),   w = V^T c,   G = V^T V,
// so T itself is never formed.  G comes for free: at step j the dot products
// of the new reflector with the block's finished columns (which hold the
// earlier reflectors below their diagonals) are G's entries.
// With kShared, w and z of every column right of the block pass through LDS
// so that each reflector is read once for all of them; that takes 16 KB more
// and is used where two workgroups still fit in a CU's 160 KB (with margin
// for the allocation granule).
template <class T, int KB, int ROWS>
struct InnerBlock {
  static constexpr bool kShared =
      sizeof(T) * (KB * ROWS + KB * (KB + 1) + 4 * 16 * KB) + sizeof(PanelSmem<T>) <= 78 * 1024;
  T v[KB][ROWS];    // reflector k of the block, by row of the block in registers
  T g[KB][KB + 1];  // G(l, k), l < k
  T z[kShared ? 4 : 1][16][kShared ? KB : 1];  // w, then z, per (column slot, column group)
};
template <class T, int ROWS>
struct InnerBlock<T, 0, ROWS> {
  static constexpr bool kShared = false;
  T v[1][1];
  T g[1][1];
};

// Range of the normal numbers of T.
template <class T> struct Lim;
template <> struct Lim<double> {
  static constexpr double tiny = DBL_MIN, huge = DBL_MAX;
};
template <> struct Lim<float> {
  static constexpr float tiny = FLT_MIN, huge = FLT_MAX;
};

__device__ __forceinline__ int col_group() { return (threadIdx.x >> 6) * 4 + ((threadIdx.x & 63) >> 4); }

// Chunk rows (16 rows each) that step column block D touches.  A leaf
// (dense block): chunks D and below.  A stack of upper triangles of NB chunks
// each (NACT = K NB, the survivor first): the survivor's diagonal chunk D and
// chunks 0..D of every other triangle; the rest is zero and stays zero.  The
// triangles of members absent from a node (fewer than K at the end of a
// level) are zero-filled rather than skipped, so that the test is a
// compile-time one: zero rows leave every norm, dot product and update
// unchanged (each adds or subtracts an exact zero).
template <bool STACK, int NB, int NACT>
__device__ __forceinline__ bool chunk_act(int i, int D, int cnt) {
  (void)cnt;
  if constexpr (!STACK) {
    return i >= D;
  } else {
    return i == D || (i >= NB && (i % NB) <= D);
  }
}

// Reflectors k0 .. k0 + 4W*IBS - 1 of a finished inner block (stored in ib)
// applied to the column slots right of the block (slots SB0 + IBS and on).
// Reflector by reflector, so that each one's rows are read from LDS once for
// every slot: w = V^T c, then z = T^T w per slot (forward substitution), then
// c -= V z.  w and z pass through ib.z: a column's 16 lanes hold the same
// value, one lane stores it and the same wave reads it back (no barrier).
template <class T, int W, int NCH, int NB, int NS, int NACT, bool STACK, int IBS, int SB0, class IB>
__device__ __forceinline__ void inner_block_update_shared(T (&a)[NCH][NS], int b, const PanelSmem<T> &sm, IB &ib,
                                                          int cnt) {
  static_assert(W == 4 && NS <= 4, "ib.z is laid out for four waves");
  constexpr int KB = 4 * W * IBS;
  constexpr int k0 = 4 * W * SB0;
  constexpr int Q0 = SB0 + IBS;  // first slot right of the block
  const int r = threadIdx.x & 15;
  const int c = col_group();
  __syncthreads();  // the block's last reflector and G entries
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    if (k0 + k >= b) continue;  // reflectors past the panel width were never stored
    const int Dk = (k0 + k) / 16;  // diagonal chunk of reflector k
    T y[NACT];
#pragma unroll
    for (int i = 0; i < NACT; ++i) {
      const bool act = chunk_act<STACK, NB, NACT>(i, Dk, cnt);
      y[i] = act ? ib.v[k][16 * i + r] : T(0);
    }
#pragma unroll
    for (int q = Q0; q < NS; ++q) {
      T s0 = T(0), s1 = T(0);
#pragma unroll
      for (int i = 0; i < NACT; ++i) {
        const bool act = chunk_act<STACK, NB, NACT>(i, Dk, cnt);
        if (!act) continue;
        if (i & 1) s1 = fma(y[i], a[i][q], s1);
        else s0 = fma(y[i], a[i][q], s0);
      }
      const T w = row16_sum(s0 + s1);
      if (r == 0) ib.z[q][c][k] = w;
    }
    // one reflector's rows in flight at a time: hoisting every load of the
    // unrolled loops would need more registers than the block leaves free
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int q = Q0; q < NS; ++q) {
    T z[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) z[k] = ib.z[q][c][k];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      T acc = z[k];
#pragma unroll
      for (int l = 0; l < k; ++l) acc = fma(-ib.g[l][k], z[l], acc);
      z[k] = (k0 + k < b) ? sm.taus[k0 + k] * acc : T(0);
    }
#pragma unroll
    for (int k = 0; k < KB; ++k)
      if (r == 0) ib.z[q][c][k] = z[k];
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    if (k0 + k >= b) continue;
    const int Dk = (k0 + k) / 16;
    T y[NACT];
#pragma unroll
    for (int i = 0; i < NACT; ++i) {
      const bool act = chunk_act<STACK, NB, NACT>(i, Dk, cnt);
      y[i] = act ? ib.v[k][16 * i + r] : T(0);
    }
#pragma unroll
    for (int q = Q0; q < NS; ++q) {
      const T zk = ib.z[q][c][k];
#pragma unroll
      for (int i = 0; i < NACT; ++i) {
        const bool act = chunk_act<STACK, NB, NACT>(i, Dk, cnt);
        if (!act) continue;
        a[i][q] = fma(-y[i], zk, a[i][q]);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  __syncthreads();  // ib is reused by the next block's steps
}

// The same, one column slot at a time with w and z in registers (each
// reflector's rows read again for every slot; no LDS beyond v and G).
template <class T, int W, int NCH, int NB, int NS, int NACT, bool STACK, int IBS, int SB0, class IB>
__device__ __forceinline__ void inner_block_update_slotwise(T (&a)[NCH][NS], int b, const PanelSmem<T> &sm, IB &ib,
                                                            int cnt) {
  constexpr int KB = 4 * W * IBS;
  constexpr int k0 = 4 * W * SB0;
  const int r = threadIdx.x & 15;
  __syncthreads();  // the block's last reflector and G entries
#pragma unroll
  for (int q = SB0 + IBS; q < NS; ++q) {
    T z[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int Dk = (k0 + k) / 16;
      T s0 = T(0), s1 = T(0);
#pragma unroll
      for (int i = 0; i < NACT; ++i) {
        const bool act = chunk_act<STACK, NB, NACT>(i, Dk, cnt);
        if (!act) continue;
        const T y = ib.v[k][16 * i + r];
        if (i & 1) s1 = fma(y, a[i][q], s1);
        else s0 = fma(y, a[i][q], s0);
      }
      z[k] = row16_sum(s0 + s1);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      T acc = z[k];
#pragma unroll
      for (int l = 0; l < k; ++l) acc = fma(-ib.g[l][k], z[l], acc);
      z[k] = (k0 + k < b) ? sm.taus[k0 + k] * acc : T(0);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int Dk = (k0 + k) / 16;
      if (k0 + k < b) {  // reflectors past the panel width were never stored
#pragma unroll
        for (int i = 0; i < NACT; ++i) {
          const bool act = chunk_act<STACK, NB, NACT>(i, Dk, cnt);
          if (!act) continue;
          a[i][q] = fma(-ib.v[k][16 * i + r], z[k], a[i][q]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  __syncthreads();  // ib is reused by the next block's steps
}

template <class T, int W, int NCH, int NB, int NS, int NACT, bool STACK, int IBS, int SB0, class IB>
__device__ __forceinline__ void inner_block_update(T (&a)[NCH][NS], int b, const PanelSmem<T> &sm, IB &ib, int cnt) {
  if constexpr (IB::kShared)
    inner_block_update_shared<T, W, NCH, NB, NS, NACT, STACK, IBS, SB0>(a, b, sm, ib, cnt);
  else
    inner_block_update_slotwise<T, W, NCH, NB, NS, NACT, STACK, IBS, SB0>(a, b, sm, ib, cnt);
}

// One Householder step per column j = 0..b-1 on the block held in a[][]:
// NACT chunk rows of 16 (LEAF: rows 0..16*NACT-1 of a dense block; STACK: two
// stacked upper triangles, R_top in chunks 0..NB-1 and R_bot in chunks
// NB..2NB-1, NB = ceil(b/16)).  Column j has its diagonal in chunk D = j/16 and
// lives in slot S = j / 4W of column group c = j mod 4W.  Reflector convention:
// beta = -sign(alpha) ||x||, tau = (beta - alpha) / beta,
// v = [1; x(2:) / (alpha - beta)]; x(2:) == 0 gives tau = 0 (H = I).  The norm
// is an unscaled sum of squares, recomputed with power-of-two scaling when
// alpha^2 + sigma is zero, subnormal or overflows.  T is double, or float for
// the single-precision batched TSQR (same steps).
// The steps of the 16 columns of diagonal block D.  IBS > 0: inner blocks of
// IBS column slots (16 IBS columns with four waves), ib holding the current
// block's reflectors and G.
template <class T, int W, int NCH, int NB, int NS, int NACT, bool STACK, int IBS, class IB>
__device__ __forceinline__ void diag_block_steps(T (&a)[NCH][NS], int b, PanelSmem<T> &sm, IB *ib, const int D,
                                                 const int cnt) {
  constexpr int CPS = 4 * W;    // columns per slot
  constexpr int BPS = CPS / 16;  // diagonal blocks per slot
  const int r = threadIdx.x & 15;
  const int c = col_group();
  {
    const int S = D / BPS;
    const int SB0 = IBS ? (S / IBS) * IBS : 0;     // first slot of S's inner block
    const int SB1 = IBS ? SB0 + IBS - 1 : NS - 1;  // last slot the steps update
    const int k0 = CPS * SB0;                      // first column of the inner block
    for (int jj = 0; jj < 16; ++jj) {
      const int j = 16 * D + jj;
      if (j >= b) break;
      const int cj = 16 * (D % BPS) + jj;  // column group of column j
      const int par = j & 1;
      if (c == cj) {
        // ---- owner DPP row: reflector of column j (slot S of this thread)
        // sum of squares below the diagonal: four partial sums (short chain)
        T sp[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int i = 0; i < NACT; ++i) {
          const bool act = chunk_act<STACK, NB, NACT>(i, D, cnt);
          if (!act) continue;
          const bool below = (i > D) || (r > jj);
          const T e = a[i][S];
          sp[i & 3] = below ? fma(e, e, sp[i & 3]) : sp[i & 3];
        }
        T sig = row16_sum((sp[0] + sp[1]) + (sp[2] + sp[3]));
        const T alpha = readlane_t(a[D][S], (cj & 3) * 16 + jj);
        const T s2 = fma(alpha, alpha, sig);
        // The reflector is formed from x scaled by 2^sh: sh = 0 normally; when
        // alpha^2 + sigma is zero, subnormal, overflowing or NaN, sh = -ilogb(max|x|)
        // (ldexp per element is exact), so that mu, tau and 1 / (alpha - beta)
        // are computed on normal numbers.
        int sh = 0;
        T alpha_s = alpha, sig_s = sig, mu_s;
        if (s2 >= Lim<T>::tiny && s2 <= Lim<T>::huge) {
          mu_s = sqrt(s2);
        } else {
          T mx = T(0);
#pragma unroll
          for (int i = 0; i < NACT; ++i) {
            const bool act = chunk_act<STACK, NB, NACT>(i, D, cnt);
            if (!act) continue;
            const bool inx = (i > D) || (r >= jj);
            mx = inx ? fmax(mx, fabs(a[i][S])) : mx;
          }
          mx = row16_max(mx);
          if (mx == T(0) || !(mx <= Lim<T>::huge)) {  // zero column, or Inf/NaN (propagated)
            mu_s = (mx == T(0)) ? T(0) : sqrt(s2);
            sig_s = (mx == T(0)) ? T(0) : sig;
          } else {
            sh = -ilogb(mx);
            // the same summation order as the unscaled sum above, so that
            // R(2^k A) = 2^k R(A) holds bitwise on this path too
            T ss[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int i = 0; i < NACT; ++i) {
              const bool act = chunk_act<STACK, NB, NACT>(i, D, cnt);
              if (!act) continue;
              const bool below = (i > D) || (r > jj);
              const T e = ldexp(a[i][S], sh);
              ss[i & 3] = below ? fma(e, e, ss[i & 3]) : ss[i & 3];
            }
            sig_s = row16_sum((ss[0] + ss[1]) + (ss[2] + ss[3]));
            alpha_s = ldexp(alpha, sh);
            mu_s = sqrt(fma(alpha_s, alpha_s, sig_s));
          }
        }
        T beta, tau, scal;
        if (sig_s == T(0)) {
          beta = alpha;
          tau = T(0);
          scal = T(0);
        } else {
          const T beta_s = -copysign(mu_s, alpha_s);
          tau = (beta_s - alpha_s) / beta_s;
          // |alpha - beta| = |alpha| + mu lies in [mu, 2 mu], a normal number:
          // its reciprocal from the hardware estimate refined by Newton steps,
          // independent of the division above so that the two overlap
          scal = rcp_nr(alpha_s - beta_s);
          beta = ldexp(beta_s, -sh);
        }
        // v = x / (alpha - beta) below the diagonal, x taken scaled by 2^sh.
        // sh is the same in the 16 active lanes (this column's row), so the
        // branch is uniform: the scaling is done in place first, and only on
        // the rescue path.
        if (__builtin_amdgcn_readfirstlane(sh) != 0) {
#pragma unroll
          for (int i = 0; i < NACT; ++i) {
            const bool act = chunk_act<STACK, NB, NACT>(i, D, cnt);
            if (act && (i > D || r > jj)) a[i][S] = ldexp(a[i][S], sh);
          }
        }
#pragma unroll
        for (int i = 0; i < NACT; ++i) {
          const bool act = chunk_act<STACK, NB, NACT>(i, D, cnt);
          if (!act) continue;
          T vv;
          if (i > D || r > jj) {
            vv = a[i][S] * scal;
            a[i][S] = vv;
          } else if (r == jj && i == D) {
            vv = T(1);
            a[i][S] = beta;
          } else {
            vv = T(0);
          }
          if constexpr (IBS > 0) ib->v[j - k0][16 * i + r] = vv;
          else sm.v[par][16 * i + r] = vv;
        }
        if (r == 0) {
          sm.tau[par] = tau;
          sm.taus[j] = tau;
        }
      }
      __syncthreads();
      // ---- every thread: w = v^T A(:, col) for its column slots, then the rank-1 update.
      // v is read from LDS where it is used (not held across the reductions).
      // Slots whose columns are all finished (q < S) are skipped.
      // Blocked: only the inner block's slots; its finished columns give G.
      const int q0 = IBS ? SB0 : S;
      const T tau = sm.tau[par];
      const T *vrow = r + [&]() -> const T * {
        if constexpr (IBS > 0) return ib->v[j - k0];
        else return sm.v[par];
      }();
      T p[2][NS];  // two partial sums per slot (half the dependency chain)
#pragma unroll
      for (int q = 0; q < NS; ++q) p[0][q] = p[1][q] = T(0);
#pragma unroll
      for (int i = 0; i < NACT; ++i) {
        const bool act = chunk_act<STACK, NB, NACT>(i, D, cnt);
        if (!act) continue;
        const T vi = vrow[16 * i];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          if (q < q0 || q > SB1) continue;
          p[i & 1][q] = fma(vi, a[i][q], p[i & 1][q]);
        }
      }
      T coef[NS];
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        if (q < q0 || q > SB1) continue;
        const T w = row16_sum(p[0][q] + p[1][q]);
        const int col = c + CPS * q;
        coef[q] = (col > j && col < b) ? tau * w : T(0);
        if constexpr (IBS > 0)
          if (col < j && r == 0) ib->g[col - k0][j - k0] = w;
      }
#pragma unroll
      for (int i = 0; i < NACT; ++i) {
        const bool act = chunk_act<STACK, NB, NACT>(i, D, cnt);
        if (!act) continue;
        const T vi = vrow[16 * i];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          if (q < S || q > SB1) continue;  // finished columns are never updated
          a[i][q] = fma(-coef[q], vi, a[i][q]);
        }
      }
    }
  }
}

// Diagonal blocks D .. NB-1 with inner blocks, each inner block applied to the
// columns right of it once its last column is done (compile-time recursion,
// so that every register index stays a constant).
template <int D, class T, int W, int NCH, int NB, int NS, int NACT, bool STACK, int IBS, class IB>
__device__ __forceinline__ void blocked_steps(T (&a)[NCH][NS], int b, PanelSmem<T> &sm, IB &ib, int cnt) {
  if constexpr (D < NB) {
    constexpr int CPS = 4 * W;
    constexpr int BPS = CPS / 16;
    constexpr int SB0 = (D / BPS / IBS) * IBS;
    diag_block_steps<T, W, NCH, NB, NS, NACT, STACK, IBS>(a, b, sm, &ib, D, cnt);
    if constexpr ((D + 1) % (BPS * IBS) == 0 && SB0 + IBS < NS)
      if (CPS * (SB0 + IBS) < b) inner_block_update<T, W, NCH, NB, NS, NACT, STACK, IBS, SB0>(a, b, sm, ib, cnt);
    blocked_steps<D + 1, T, W, NCH, NB, NS, NACT, STACK, IBS>(a, b, sm, ib, cnt);
  }
}

template <class T, int W, int NCH, int NB, int NS, int NACT, bool STACK, int IBS = 0, class IB = InnerBlock<T, 0, 1>>
__device__ __forceinline__ void householder_steps(T (&a)[NCH][NS], int b, PanelSmem<T> &sm, IB *ib = nullptr,
                                                  int cnt = 2) {
  if constexpr (IBS == 0) {
#pragma unroll
    for (int D = 0; D < NB; ++D) diag_block_steps<T, W, NCH, NB, NS, NACT, STACK, 0>(a, b, sm, ib, D, cnt);
  } else {
    blocked_steps<0, T, W, NCH, NB, NS, NACT, STACK, IBS>(a, b, sm, *ib, cnt);
  }
}

// Global element (row, col) of the panel, row within [0, m).
template <class T>
__device__ __forceinline__ T *pan(const PanelParamsT<T> &p, int64_t row, int col) {
  return p.A + row + (int64_t)col * p.lda;
}

// Load the upper triangle of the R stored at slot_row into chunks
// base..base+NB-1 (zeros elsewhere).
template <class T, int W, int NCH, int NB, int NS>
__device__ __forceinline__ void load_r(T (&a)[NCH][NS], const PanelParamsT<T> &p, int64_t slot_row, int base) {
  const int r = threadIdx.x & 15;
  const int c = col_group();
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const int row = 16 * i + r, col = c + 4 * W * q;
      const int64_t grow = slot_row + row;
      // row blocks below slot q's columns are zero (a compile-time zero, so
      // the register is never live)
      if (i / (4 * W / 16) > q) {
        a[base + i][q] = T(0);
        continue;
      }
      a[base + i][q] = (row <= col && col < p.b && grow < p.m) ? *pan(p, grow, col) : T(0);
    }
}

// Store the upper triangle (incl. diagonal) held in chunks base..base+NB-1 to
// the rows starting at slot_row.
template <class T, int W, int NCH, int NB, int NS>
__device__ __forceinline__ void store_upper(const T (&a)[NCH][NS], const PanelParamsT<T> &p, int64_t slot_row,
                                            int base) {
  const int r = threadIdx.x & 15;
  const int c = col_group();
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const int row = 16 * i + r, col = c + 4 * W * q;
      const int64_t grow = slot_row + row;
      if (i / (4 * W / 16) > q) continue;  // below the diagonal blocks: nothing to store
      if (row <= col && col < p.b && grow < p.m) *pan(p, grow, col) = a[base + i][q];
    }
}

// Stacked elimination of one tree node with arity K: the R factors at slots
// g, g + s, ..., g + (cnt - 1) s (cnt <= K present, read from global) are
// stacked (survivor first) and factored together, with zero triangles in
// place of absent members.  Writes each eliminated slot's part of the node's
// V (upper triangular) over its R, the new R over the survivor's slot, and tau
// of node id g + s.  The new R stays in chunks 0..NB-1.
template <class T, int W, int NCH, int NB, int NS, int K, int IBS = 0, class IB = InnerBlock<T, 0, 1>>
__device__ __forceinline__ void combine_k(T (&a)[NCH][NS], const PanelParamsT<T> &p, int g, int s, int cnt, int h,
                                          PanelSmem<T> &sm, IB *ib = nullptr) {
  static_assert(K * NB <= NCH, "the stack must fit the register block");
  load_r<T, W, NCH, NB, NS>(a, p, (int64_t)g * h, 0);
#pragma unroll
  for (int t = 1; t < K; ++t) {
    if (t < cnt) {
      load_r<T, W, NCH, NB, NS>(a, p, (int64_t)(g + t * s) * h, t * NB);
    } else {  // absent member: an exact zero triangle
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int q = 0; q < NS; ++q) a[t * NB + i][q] = T(0);
    }
  }
  __syncthreads();
  householder_steps<T, W, NCH, NB, NS, K * NB, true, IBS>(a, p.b, sm, ib, cnt);
#pragma unroll
  for (int t = K - 1; t >= 1; --t)
    if (t < cnt) store_upper<T, W, NCH, NB, NS>(a, p, (int64_t)(g + t * s) * h, t * NB);  // V of the node
  store_upper<T, W, NCH, NB, NS>(a, p, (int64_t)g * h, 0);  // R of the survivor
  __syncthreads();
  if (threadIdx.x < kMaxB)
    p.tau_node[(int64_t)(g + s) * kMaxB + threadIdx.x] = (threadIdx.x < p.b) ? sm.taus[threadIdx.x] : T(0);
  __syncthreads();
}

// Last-arriver ticket on node `node` with cnt members; true for the workgroup
// that arrives last (and must perform the elimination).  Publishes this
// workgroup's prior global stores before the ticket and acquires the other
// members' after it; the last arriver leaves the counter at zero.
template <class T>
__device__ __forceinline__ bool arrive_k(const PanelParamsT<T> &p, int node, int cnt, PanelSmem<T> &sm) {
  fence_release();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned old = ticket_add(p.tickets + node);
    const bool last = old + 1u == (unsigned)cnt;
    sm.flag = last ? 1 : 0;
    if (last) ticket_clear(p.tickets + node);
  }
  __syncthreads();
  const bool last = sm.flag == 1;
  if (last) fence_acquire();
  return last;
}

// Members present in the group of survivor g at stride s (slots g + t s < L).
__device__ __forceinline__ int group_count(int g, int s, int K, int L) { return min(K, (L - g + s - 1) / s); }

// combine_k for a node of a K-ary tree with cnt members: a node of two
// members (the last of a level) takes the two-triangle stack, whose steps
// touch half the chunks of the zero-filled K-member one; the node it writes
// (R, V over the one eliminated slot, tau at g + s) is the same.
template <class T, int W, int NCH, int NB, int NS, int K, int IBS = 0, class IB = InnerBlock<T, 0, 1>>
__device__ __forceinline__ void combine_node(T (&a)[NCH][NS], const PanelParamsT<T> &p, int g, int s, int cnt, int h,
                                             PanelSmem<T> &sm, IB *ib = nullptr) {
  if constexpr (K > 2) {
    if (cnt == 2) {
      combine_k<T, W, NCH, NB, NS, 2, IBS>(a, p, g, s, cnt, h, sm, ib);
      return;
    }
  }
  combine_k<T, W, NCH, NB, NS, K, IBS>(a, p, g, s, cnt, h, sm, ib);
}


// Root of the tree: make the diagonal non-negative, R <- D R, record D.
template <class T, int W, int NCH, int NB, int NS>
__device__ __forceinline__ void finish_root(T (&a)[NCH][NS], const PanelParamsT<T> &p, PanelSmem<T> &sm) {
  constexpr int BPS = 4 * W / 16;
  const int r = threadIdx.x & 15;
  const int c = col_group();
  __syncthreads();
  load_r<T, W, NCH, NB, NS>(a, p, 0, 0);
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int row = 16 * i + r;  // its diagonal element: slot i / BPS, column group row mod 4W
    if (c == 16 * (i % BPS) + r && row < p.b) sm.dsign[row] = (a[i][i / BPS] < T(0)) ? T(-1) : T(1);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const int row = 16 * i + r, col = c + 4 * W * q;
      if (row <= col && col < p.b) a[i][q] *= sm.dsign[row];
    }
  store_upper<T, W, NCH, NB, NS>(a, p, 0, 0);
  if (threadIdx.x < p.b) p.d[threadIdx.x] = sm.dsign[threadIdx.x];
}

// Column slots of a W-wave workgroup for NB 16-column blocks.
template <int W, int NB>
struct Slots {
  static constexpr int value = (16 * NB + 4 * W - 1) / (4 * W);
};

// The leaves leaf0 .. leaf0 + lpw - 1 of panel p and the part of its tree
// this workgroup ends up holding (levels 1-3).  The tree has arity K: level
// s = K^j groups the slots g, g + s, ..., g + (K - 1) s (g a multiple of K s),
// and the survivor g holds the node's R.  lpw is a power of K, so the groups
// below lpw lie within one workgroup (eliminated there, no ticket) and those
// above span whole workgroups (the last member to arrive eliminates).
// Without DEVICE_TREE the workgroup stops where its subtree needs another
// workgroup's, and the levels above are eliminated by later launches (one
// per level).
template <class T, int W, int RPT, int NB, bool DEVICE_TREE, int IBS = 0, int K = 2>
__device__ __forceinline__ void panel_body(const PanelParamsT<T> p, int leaf0) {
  __shared__ PanelSmem<T> sm;
  constexpr int NS = Slots<W, NB>::value;
  constexpr int CPS = 4 * W;
  constexpr int NCH = (RPT > K * NB) ? RPT : K * NB;
  constexpr int H = 16 * RPT;
  __shared__ InnerBlock<T, CPS * IBS, 16 * NCH> ib;
  T a[NCH][NS];
  const int r = threadIdx.x & 15;
  const int c = col_group();
  const int nleaves = min(p.lpw, p.L - leaf0);

  for (int li = 0; li < nleaves; ++li) {
    const int leaf = leaf0 + li;
    const int64_t row0 = (int64_t)leaf * H;
    // ---- level 1: factor the leaf block in registers
    // uniform fast path: the whole leaf in range and the panel NS*4W wide
    const bool full = row0 + H <= p.m && p.b == CPS * NS;
    if (full) {
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        const T *colp = p.A + row0 + r + (int64_t)(c + CPS * q) * p.lda;
#pragma unroll
        for (int i = 0; i < NCH; ++i) a[i][q] = (i < RPT) ? colp[16 * i] : T(0);
      }
    } else {
#pragma unroll
      for (int i = 0; i < NCH; ++i)
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          const int64_t grow = row0 + 16 * i + r;
          const int col = c + CPS * q;
          a[i][q] = (i < RPT && grow < p.m && col < p.b) ? *pan(p, grow, col) : T(0);
        }
    }
    __syncthreads();
    householder_steps<T, W, NCH, NB, NS, RPT, false, IBS>(a, p.b, sm, &ib);
    if (full) {
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        T *colp = p.A + row0 + r + (int64_t)(c + CPS * q) * p.lda;
#pragma unroll
        for (int i = 0; i < RPT; ++i) colp[16 * i] = a[i][q];
      }
    } else {
#pragma unroll
      for (int i = 0; i < RPT; ++i)
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          const int64_t grow = row0 + 16 * i + r;
          const int col = c + CPS * q;
          if (grow < p.m && col < p.b) *pan(p, grow, col) = a[i][q];
        }
    }
    __syncthreads();
    if (threadIdx.x < kMaxB)
      p.tau_leaf[(int64_t)leaf * kMaxB + threadIdx.x] = (threadIdx.x < p.b) ? sm.taus[threadIdx.x] : T(0);
    __syncthreads();

    // ---- levels 2 and 3: climb the tree from this leaf
    int rt = leaf;  // root of the subtree this workgroup currently holds
    bool go_on = true;
    for (int s = 1; s < p.L; s *= K) {
      const int g = rt - rt % (K * s);  // survivor of rt's group at this level
      const int cnt = group_count(g, s, K, p.L);
      if (cnt < 2) continue;                          // alone: pass through
      const int last = min(g + K * s, p.L) - 1;       // last leaf under the group
      if (g >= leaf0 && last < leaf0 + nleaves) {     // the group lies within this workgroup's leaves
        if (leaf < last) {                            // a later leaf of this workgroup completes it
          go_on = false;
          break;
        }
      } else if (!DEVICE_TREE || !arrive_k(p, g + s, cnt, sm)) {
        return;  // another workgroup (or a level launch) finishes the node
      }
      combine_node<T, W, NCH, NB, NS, K, IBS>(a, p, g, s, cnt, H, sm, &ib);
      rt = g;
    }
    if (!go_on) continue;
    finish_root<T, W, NCH, NB, NS>(a, p, sm);
  }
}

template <int RPT, int NB, bool DEVICE_TREE, int IBS, int K>
__global__ void __launch_bounds__(64 * kPanelWaves, 2) tsqr_panel_kernel(PanelParams p) {
  panel_body<double, kPanelWaves, RPT, NB, DEVICE_TREE, IBS, K>(p, blockIdx.x * p.lpw);
}

// One device level s of a single panel's tree (when the leaves' launch stops
// at the workgroups' subtrees): workgroup i eliminates the group of survivor
// g = K s i, and normalizes the root at the top level.
template <int NB, int IBS, int K>
__global__ void __launch_bounds__(64 * kPanelWaves, 2) tsqr_level_kernel(PanelParams p, int s, int h) {
  constexpr int NS = Slots<kPanelWaves, NB>::value;
  __shared__ PanelSmem<double> sm;
  __shared__ InnerBlock<double, 4 * kPanelWaves * IBS, 16 * K * NB> ib;
  double a[K * NB][NS];
  const int g = K * s * (int)blockIdx.x;
  const int cnt = group_count(g, s, K, p.L);
  if (cnt < 2) return;  // the launch covers only groups with two or more members
  combine_node<double, kPanelWaves, K * NB, NB, NS, K, IBS>(a, p, g, s, cnt, h, sm, &ib);
  if (K * s >= p.L) finish_root<double, kPanelWaves, K * NB, NB, NS>(a, p, sm);
}

// Many independent panels in one launch: workgroup i takes problem
// items[i].x, leaves from items[i].y on, and the tree levels inside its own
// leaves.  No workgroup waits for or signals another: the levels above are
// eliminated by tsqr_tree_level_kernel launches, whose kernel boundaries
// order them (many thousands of workgroups would otherwise each pay an
// agent-scope fence, an L2 write-back, while the L2s hold the others' data).
template <class T, int RPT, int NB, int K>
__global__ void __launch_bounds__(64 * kPanelWaves, 2) tsqr_panel_batched_kernel(const PanelParamsT<T> *probs,
                                                                                const int2 *items) {
  const int2 it = items[blockIdx.x];
  const PanelParamsT<T> p = probs[__builtin_amdgcn_readfirstlane(it.x)];
  panel_body<T, kPanelWaves, RPT, NB, false, 0, K>(p, __builtin_amdgcn_readfirstlane(it.y));
}

// One device level of the trees of many panels: workgroup i eliminates the
// group of survivor nodes[i].y at stride nodes[i].z of problem nodes[i].x
// (leaf height nodes[i].w & 0xFFF, members present nodes[i].w >> 16), and
// normalizes the root when the node is the top of its tree (bit 12 of
// nodes[i].w).
template <class T, int NB, int K>
__global__ void __launch_bounds__(64 * kPanelWaves, 2) tsqr_tree_level_kernel(const PanelParamsT<T> *probs,
                                                                             const int4 *nodes) {
  constexpr int NS = Slots<kPanelWaves, NB>::value;
  __shared__ PanelSmem<T> sm;
  const int4 nd = nodes[blockIdx.x];
  const PanelParamsT<T> p = probs[__builtin_amdgcn_readfirstlane(nd.x)];
  const int w = __builtin_amdgcn_readfirstlane(nd.w);
  T a[K * NB][NS];
  combine_node<T, kPanelWaves, K * NB, NB, NS, K>(a, p, __builtin_amdgcn_readfirstlane(nd.y),
                                                  __builtin_amdgcn_readfirstlane(nd.z), w >> 16, w & 0xFFF, sm);
  if ((w >> 12) & 1) finish_root<T, kPanelWaves, K * NB, NB, NS>(a, p, sm);
}

constexpr int kPanelThreads = 64 * kPanelWaves;

}  // namespace

}  // namespace caqr
