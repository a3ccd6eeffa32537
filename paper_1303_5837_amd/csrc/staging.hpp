// Staging of 64x64 blocks of reflectors (or T) from global memory through
// registers into LDS, and the LDS reads that feed FP64 MFMA operands.
#pragma once

#include "device_common.hpp"

namespace caqr {

constexpr int kLdb = 68;   // leading dimension (doubles) of a staged 64x64 block in LDS

typedef double f64x2 __attribute__((ext_vector_type(2)));

enum BlockKind { kLeafY = 0, kNodeV = 1, kDense = 2 };

// A 64x64 block staged through registers: thread tid holds 8 row pairs.
// Pair e = s*256 + tid (s = 0..7): column e / 32, block rows 2*(e % 32) and +1.
struct Stage {
  f64x2 v[8];
};

// Load a 64x64 block of reflectors (or T) from global memory into registers:
// block rows 0..63 are the panel rows src0..src0+63.  For KIND kLeafY, `lr_off`
// converts a panel row to the row within the leaf (lr = row - lr_off) and the
// value is the unit lower-trapezoidal leaf reflector; kNodeV: the upper
// triangular V whose row 0 is panel row lr_off; kDense: a dense 64x64
// column-major block, ld 64 (T).
//
// On the uniform fast path (full-width panel, every row in range, 16-byte
// aligned) the loads are issued raw, with no arithmetic on their results, so
// the wait for them falls at stage_store, after the work they overlap.  The
// triangle of a block that holds the diagonal (lr < 64) is then applied by
// stage_fix before the store; the slow path masks as it loads (stage_fix is
// idempotent on its result).
template <int KIND>
__device__ __forceinline__ void stage_load(Stage &st, const double *base, int64_t ld, int64_t src0, int64_t lr_off,
                                           int64_t m, int b, bool vec_ok, int tid) {
  const int row = 2 * (tid & 31);  // block row pair of this thread (same for every s)
  const int colt = tid >> 5;       // block column for s = 0; s adds 8
  if (KIND == kDense) {
#pragma unroll
    for (int s = 0; s < 8; ++s) st.v[s] = *reinterpret_cast<const f64x2 *>(base + row + 64 * (colt + 8 * s));
    return;
  }
  const int64_t g0 = src0 + row;
  const int64_t lr = g0 - lr_off;
  const bool fast = vec_ok && b == kMaxB && src0 + 63 < m;
  if (fast) {
    const double *p = base + g0 + (int64_t)colt * ld;
#pragma unroll
    for (int s = 0; s < 8; ++s) st.v[s] = *reinterpret_cast<const f64x2 *>(p + (int64_t)(8 * s) * ld);
    return;
  }
  const int64_t ga = min(g0, m - 1), gb = min(g0 + 1, m - 1);
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int col = colt + 8 * s;
    const int64_t cc = (int64_t)min(col, b - 1) * ld;
    double x0 = base[ga + cc], x1 = base[gb + cc];
    const bool okc = col < b;
    if (KIND == kLeafY) {
      x0 = (okc && g0 < m && lr > col) ? x0 : ((okc && lr == col) ? 1.0 : 0.0);
      x1 = (okc && g0 + 1 < m && lr + 1 > col) ? x1 : ((okc && lr + 1 == col) ? 1.0 : 0.0);
    } else {  // node V: upper triangle including the diagonal
      x0 = (okc && g0 < m && lr <= col) ? x0 : 0.0;
      x1 = (okc && g0 + 1 < m && lr + 1 <= col) ? x1 : 0.0;
    }
    st.v[s] = f64x2{x0, x1};
  }
}

// Triangle of a block whose first row is row lr0 (< 64) of its leaf or node:
// kLeafY keeps rows below the diagonal and puts 1 on it, kNodeV keeps the
// upper triangle with the diagonal.
template <int KIND>
__device__ __forceinline__ void stage_fix(Stage &st, int lr0, int tid) {
  if (KIND == kDense) return;
  const int lr = lr0 + 2 * (tid & 31);
  const int colt = tid >> 5;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int col = colt + 8 * s;
    double x0 = st.v[s].x, x1 = st.v[s].y;
    if (KIND == kLeafY) {
      x0 = (lr > col) ? x0 : ((lr == col) ? 1.0 : 0.0);
      x1 = (lr + 1 > col) ? x1 : ((lr + 1 == col) ? 1.0 : 0.0);
    } else {
      x0 = (lr <= col) ? x0 : 0.0;
      x1 = (lr + 1 <= col) ? x1 : 0.0;
    }
    st.v[s] = f64x2{x0, x1};
  }
}

__device__ __forceinline__ void stage_store(const Stage &st, double *lds, int tid) {
  double *p = lds + (tid >> 5) * kLdb + 2 * (tid & 31);
#pragma unroll
  for (int s = 0; s < 8; ++s) *reinterpret_cast<f64x2 *>(p + 8 * s * kLdb) = st.v[s];
}

// Four consecutive rows row0..row0+3 of column col of a staged block.
__device__ __forceinline__ f64x4 lds_col4(const double *lds, int col, int row0) {
  const f64x2 lo = *reinterpret_cast<const f64x2 *>(lds + col * kLdb + row0);
  const f64x2 hi = *reinterpret_cast<const f64x2 *>(lds + col * kLdb + row0 + 2);
  return f64x4{lo.x, lo.y, hi.x, hi.y};
}

// Four consecutive columns col0..col0+3 of row `row` of a staged block.
__device__ __forceinline__ f64x4 lds_row4(const double *lds, int row, int col0) {
  return f64x4{lds[col0 * kLdb + row], lds[(col0 + 1) * kLdb + row], lds[(col0 + 2) * kLdb + row],
               lds[(col0 + 3) * kLdb + row]};
}

// ---- split variant: a 64x64 block whose rows 0..31 and 32..63 come from two
// separate 32-row pieces (the two row halves of a leaf), loaded by NT threads.
// Thread tid holds the row pair 2*(tid % 32) of columns tid / 32 + (NT / 32) s.
template <int NT>
struct StageSplit {
  static constexpr int kPer = 64 * 64 / (2 * NT);  // row pairs per thread
  f64x2 v[kPer];
};

// Block row R < 32 is panel row src0 + R (leaf-relative row lr0 + R); block
// row R >= 32 is panel row src1 + R - 32 (leaf-relative lr1 + R - 32).  KIND
// and the fast/slow paths are as for stage_load (kDense: a 64x64 block, ld 64).
template <int KIND, int NT>
__device__ __forceinline__ void stage_load_split(StageSplit<NT> &st, const double *base, int64_t ld, int64_t src0,
                                                 int64_t src1, int64_t lr0, int64_t lr1, int64_t m, int b,
                                                 bool vec_ok, int tid) {
  constexpr int CS = NT / 32;  // column stride between a thread's pairs
  const int R = 2 * (tid & 31);
  const int colt = tid >> 5;
  if (KIND == kDense) {
#pragma unroll
    for (int s = 0; s < StageSplit<NT>::kPer; ++s)
      st.v[s] = *reinterpret_cast<const f64x2 *>(base + R + 64 * (colt + CS * s));
    return;
  }
  const int64_t g0 = (R < 32) ? src0 + R : src1 + (R - 32);
  const int64_t lr = (R < 32) ? lr0 + R : lr1 + (R - 32);
  const bool fast = vec_ok && b == kMaxB && src0 + 31 < m && src1 + 31 < m;
  if (fast) {
    const double *p = base + g0 + (int64_t)colt * ld;
#pragma unroll
    for (int s = 0; s < StageSplit<NT>::kPer; ++s)
      st.v[s] = *reinterpret_cast<const f64x2 *>(p + (int64_t)(CS * s) * ld);
    return;
  }
  const int64_t ga = min(g0, m - 1), gb = min(g0 + 1, m - 1);
#pragma unroll
  for (int s = 0; s < StageSplit<NT>::kPer; ++s) {
    const int col = colt + CS * s;
    const int64_t cc = (int64_t)min(col, b - 1) * ld;
    double x0 = base[ga + cc], x1 = base[gb + cc];
    const bool okc = col < b;
    if (KIND == kLeafY) {
      x0 = (okc && g0 < m && lr > col) ? x0 : ((okc && lr == col) ? 1.0 : 0.0);
      x1 = (okc && g0 + 1 < m && lr + 1 > col) ? x1 : ((okc && lr + 1 == col) ? 1.0 : 0.0);
    } else {
      x0 = (okc && g0 < m && lr <= col) ? x0 : 0.0;
      x1 = (okc && g0 + 1 < m && lr + 1 <= col) ? x1 : 0.0;
    }
    st.v[s] = f64x2{x0, x1};
  }
}

// Triangle of the rows of a split block that lie within the first 64 rows of
// their leaf or node (idempotent on slow-path results).
template <int KIND, int NT>
__device__ __forceinline__ void stage_fix_split(StageSplit<NT> &st, int64_t lr0, int64_t lr1, int tid) {
  if (KIND == kDense) return;
  constexpr int CS = NT / 32;
  const int R = 2 * (tid & 31);
  const int colt = tid >> 5;
  const int64_t lr = (R < 32) ? lr0 + R : lr1 + (R - 32);
  if (lr >= kMaxB) return;
#pragma unroll
  for (int s = 0; s < StageSplit<NT>::kPer; ++s) {
    const int col = colt + CS * s;
    double x0 = st.v[s].x, x1 = st.v[s].y;
    if (KIND == kLeafY) {
      x0 = (lr > col) ? x0 : ((lr == col) ? 1.0 : 0.0);
      x1 = (lr + 1 > col) ? x1 : ((lr + 1 == col) ? 1.0 : 0.0);
    } else {
      x0 = (lr <= col) ? x0 : 0.0;
      x1 = (lr + 1 <= col) ? x1 : 0.0;
    }
    st.v[s] = f64x2{x0, x1};
  }
}

template <int NT>
__device__ __forceinline__ void stage_store_split(const StageSplit<NT> &st, double *lds, int tid) {
  constexpr int CS = NT / 32;
  double *p = lds + (tid >> 5) * kLdb + 2 * (tid & 31);
#pragma unroll
  for (int s = 0; s < StageSplit<NT>::kPer; ++s) *reinterpret_cast<f64x2 *>(p + CS * s * kLdb) = st.v[s];
}

}  // namespace caqr
