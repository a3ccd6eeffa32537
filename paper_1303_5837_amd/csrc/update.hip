// Application of one panel's orthogonal factor to a block of columns.
//
// This is the trailing-matrix update of ML-CAQR (paper, Section 3.1, item 2 of
// the description of Algorithm 1): the updates of the leaves of the reduction
// tree (MLUPFACT), then those of the tree's intermediate eliminations
// (MLUPELIM), walking the tree again in the order it was built.  With the
// reflectors in compact WY form (Q = I - Y T Y^T) every update is two dense
// products around a small triangular one, run on FP64 MFMA:
//
//   leaf   (rows of leaf i, h x 64 tile):  W = Y_i^T C_i,  W <- T_i^T W,  C_i -= Y_i W
//   node   (top b rows of the two leaves): W = C_1 + V^T C_2,  W <- T^T W,
//                                          C_1 -= W,  C_2 -= V W
//
// (T instead of T^T for Q C.)  One workgroup updates one leaf's rows of one
// 64-column tile; wave w owns columns 16w..16w+15 of the tile and keeps them in
// registers between the two products, so C is read and written once.  The
// reflectors are staged through LDS in 64x64 blocks (double-buffered, loaded
// with coalesced 16-byte accesses), and T goes through the same buffers.  For
// Q^T the tree levels follow in the same launch: per (node, tile) an
// agent-scope ticket lets the second workgroup to finish below a node perform
// that node's update on the tile.
//
// Register layout ("contiguous"): a 16-row slab x of a tile is an f64x4 per
// lane holding rows 16x + 4*(lane/16) + r, r = 0..3, of column lane%16.  The
// MFMA result layout holds row 4r + lane/16 in register r, so every product
// whose output uses the contiguous layout reads its A operand at the permuted
// row pi(lane%16) = 4*(lane%4) + (lane%16)/4 of the slab.
#include "device_common.hpp"
#include "kernels.hpp"

namespace caqr {

namespace {

constexpr int kLdb = 68;   // leading dimension (doubles) of a staged 64x64 block in LDS

typedef double f64x2 __attribute__((ext_vector_type(2)));

struct UpdSmem {
  alignas(16) double buf[2][kMaxB * kLdb];
  int flag;
};

__device__ __forceinline__ int pi16(int li) { return 4 * (li & 3) + (li >> 2); }

__device__ __forceinline__ bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// The thread index passed through a register move the compiler cannot see
// through: computations derived from it inside a loop body are redone per
// iteration instead of being hoisted (and kept live) across the whole loop.
__device__ __forceinline__ int opaque_tid() {
  int t;
  asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"((int)threadIdx.x));
  return t;
}

enum BlockKind { kLeafY = 0, kNodeV = 1, kDense = 2 };

// A 64x64 block staged through registers: thread tid holds 8 row pairs.
// Pair e = s*256 + tid (s = 0..7): column e / 32, block rows 2*(e % 32) and +1.
struct Stage {
  f64x2 v[8];
};

// Load a 64x64 block of reflectors (or T) from global memory into registers.
// Block rows 0..31 are source rows src0 + 0..31 and block rows 32..63 are
// source rows src1 + 0..31 (rows relative to the panel; src0 + 32 == src1 for a
// contiguous block).  For KIND kLeafY, `lr_off` converts a panel row to the row
// within the leaf (lr = row - lr_off), and the value is the unit
// lower-trapezoidal leaf reflector; kNodeV: the upper-triangular V whose row 0
// is panel row lr_off; kDense: a dense 64x64 column-major block, ld 64 (T).
template <int KIND>
__device__ __forceinline__ void stage_load(Stage &st, const double *base, int64_t ld, int64_t src0, int64_t src1,
                                           int64_t lr_off, int64_t m, int b, bool vec_ok, int tid) {
  const int row = 2 * (tid & 31);  // block row pair of this thread (same for every s)
  const int colt = tid >> 5;       // block column for s = 0; s adds 8
  if (KIND == kDense) {
#pragma unroll
    for (int s = 0; s < 8; ++s) st.v[s] = *reinterpret_cast<const f64x2 *>(base + row + 64 * (colt + 8 * s));
    return;
  }
  const int64_t g0 = (row < 32) ? src0 + row : src1 + (row - 32);
  const int64_t lr = g0 - lr_off;
  // uniform fast path: full-width panel, every row in range, 16-byte aligned
  const bool fast = vec_ok && b == kMaxB && src0 + 31 < m && src1 + 31 < m;
  if (fast) {
    const double *p = base + g0 + (int64_t)colt * ld;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int col = colt + 8 * s;
      const f64x2 t = *reinterpret_cast<const f64x2 *>(p + (int64_t)(8 * s) * ld);
      double x0 = t.x, x1 = t.y;
      if (KIND == kLeafY) {
        x0 = (lr > col) ? x0 : ((lr == col) ? 1.0 : 0.0);
        x1 = (lr + 1 > col) ? x1 : ((lr + 1 == col) ? 1.0 : 0.0);
      } else {
        x0 = (lr <= col) ? x0 : 0.0;
        x1 = (lr + 1 <= col) ? x1 : 0.0;
      }
      st.v[s] = f64x2{x0, x1};
    }
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

// C slab load/store (contiguous layout) with row/column masking.
__device__ __forceinline__ f64x4 load_slab(const double *C, int64_t ldc, int64_t grow, int64_t col, int64_t m,
                                           bool colok, bool vec_ok) {
  if (colok && vec_ok && grow + 3 < m) {
    const f64x2 lo = *reinterpret_cast<const f64x2 *>(C + grow + col * ldc);
    const f64x2 hi = *reinterpret_cast<const f64x2 *>(C + grow + 2 + col * ldc);
    return f64x4{lo.x, lo.y, hi.x, hi.y};
  }
  f64x4 r;
#pragma unroll
  for (int q = 0; q < 4; ++q) r[q] = (colok && grow + q < m) ? C[grow + q + col * ldc] : 0.0;
  return r;
}

__device__ __forceinline__ void store_slab(double *C, int64_t ldc, int64_t grow, int64_t col, int64_t m, bool colok,
                                           bool vec_ok, f64x4 v) {
  if (!colok) return;
  if (vec_ok && grow + 3 < m) {
    *reinterpret_cast<f64x2 *>(C + grow + col * ldc) = f64x2{v[0], v[1]};
    *reinterpret_cast<f64x2 *>(C + grow + 2 + col * ldc) = f64x2{v[2], v[3]};
    return;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (grow + q < m) C[grow + q + col * ldc] = v[q];
}

// W <- T^T W (TRANS) or T W, in place, with T staged in LDS (64x64, ld kLdb);
// W in the contiguous layout (slab a = reflectors 16a..16a+15).  Block ao of
// T^T W needs blocks a <= ao of W, so the blocks are produced from the last
// one down (from the first one up for T W) and overwrite W as they go.
template <int NQ, bool TRANS>
__device__ __forceinline__ void apply_t_lds(const double *Ts, f64x4 (&w)[NQ]) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int pl = pi16(li);
#pragma unroll
  for (int oo = 0; oo < NQ; ++oo) {
    const int ao = TRANS ? NQ - 1 - oo : oo;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < NQ; ++a) {
      if (TRANS ? (a > ao) : (a < ao)) continue;  // T is upper triangular
      // TRANS: A(i, k) = T(16a + 4lk + r, 16ao + pi(i));  otherwise T(16ao + pi(i), 16a + 4lk + r)
      const f64x4 t = TRANS ? lds_col4(Ts, 16 * ao + pl, 16 * a + 4 * lk) : lds_row4(Ts, 16 * ao + pl, 16 * a + 4 * lk);
#pragma unroll
      for (int r = 0; r < 4; ++r) acc = mfma16x16x4(t[r], w[a][r], acc);
    }
    w[ao] = acc;
  }
}

// The two waves of a column group hold partial sums of W over the two row
// halves; after this call both hold W = P(half 0) + P(half 1) (same order in
// both, so the two copies are bitwise equal).  `xbuf` is a free LDS block.
template <int NQ>
__device__ __forceinline__ void exchange_w(f64x4 (&w)[NQ], double *xbuf) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int cg = wave & 1, rh = wave >> 1;
  f64x4 *x = reinterpret_cast<f64x4 *>(xbuf);
#pragma unroll
  for (int a = 0; a < NQ; ++a) x[((cg * 2 + rh) * NQ + a) * 64 + lane] = w[a];
  __syncthreads();
#pragma unroll
  for (int a = 0; a < NQ; ++a) {
    const f64x4 p0 = x[((cg * 2 + 0) * NQ + a) * 64 + lane];
    const f64x4 p1 = x[((cg * 2 + 1) * NQ + a) * 64 + lane];
    w[a] = p0 + p1;
  }
}

// Update of the top b rows of tree node `node` (eliminated leaf) and of its
// left sibling on this workgroup's tile.  Wave (cg, rh) holds rows
// 32rh..32rh+31 of both row blocks for columns 16cg..16cg+15; the two waves of
// a column group form W = C1 + V^T C2 from partial sums over their rows.
template <int NQ, bool TRANS>
__device__ __forceinline__ void node_update(const UpdateParams &u, int left, int node, int tile, UpdSmem &sm,
                                            bool vec_ok) {
  constexpr int NS = 2;  // 16-row slabs per wave: slab t = 2 rh + x
  const int tid = opaque_tid();
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int cg = wave & 1, rh = wave >> 1;
  const int li = lane & 15, lk = lane >> 4;
  const int pl = pi16(li);
  const int64_t col = (int64_t)tile * kUpdTile + 16 * cg + li;
  const bool colok = col < u.k;
  const int64_t r1 = (int64_t)left * u.h, r2 = (int64_t)node * u.h;
  const int64_t m1 = min<int64_t>(u.m, r1 + u.b), m2 = min<int64_t>(u.m, r2 + u.b);
  Stage st;
  stage_load<kNodeV>(st, u.Y, u.ldy, r2, r2 + 32, r2, u.m, u.b, vec_ok, tid);
  stage_store(st, sm.buf[0], tid);
  stage_load<kDense>(st, u.T_node + (int64_t)node * 64 * 64, 64, 0, 0, 0, 0, 0, true, tid);
  f64x4 c1[NS], c2[NS];
#pragma unroll
  for (int x = 0; x < NS; ++x) {
    c1[x] = load_slab(u.C, u.ldc, r1 + 32 * rh + 16 * x + 4 * lk, col, m1, colok, vec_ok);
    c2[x] = load_slab(u.C, u.ldc, r2 + 32 * rh + 16 * x + 4 * lk, col, m2, colok, vec_ok);
  }
  __syncthreads();
  // partial W over this wave's rows: own slabs of C1 plus V(rows)^T C2(rows)
  f64x4 w[NQ];
#pragma unroll
  for (int a = 0; a < NQ; ++a) {
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int x = 0; x < NS; ++x) {
      const int t = 2 * rh + x;
      if (t > a) continue;  // V upper triangular
      const f64x4 v = lds_col4(sm.buf[0], 16 * a + pl, 16 * t + 4 * lk);
#pragma unroll
      for (int r = 0; r < 4; ++r) acc = mfma16x16x4(v[r], c2[x][r], acc);
    }
#pragma unroll
    for (int x = 0; x < NS; ++x)
      if (2 * rh + x == a) acc += c1[x];
    w[a] = acc;
  }
  exchange_w<NQ>(w, sm.buf[1]);
  __syncthreads();
  stage_store(st, sm.buf[1], tid);  // T
  __syncthreads();
  apply_t_lds<NQ, TRANS>(sm.buf[1], w);
  f64x4 (&w2)[NQ] = w;
  // C1 -= W' (own slabs);  C2 -= V W' (own rows)
#pragma unroll
  for (int x = 0; x < NS; ++x) {
    const int t = 2 * rh + x;
#pragma unroll
    for (int a = 0; a < NQ; ++a)
      if (a == t) c1[x] -= w2[a];
    f64x4 acc = c2[x];
#pragma unroll
    for (int a = 0; a < NQ; ++a) {
      if (a < t) continue;
      const f64x4 v = lds_row4(sm.buf[0], 16 * t + pl, 16 * a + 4 * lk);
#pragma unroll
      for (int r = 0; r < 4; ++r) acc = mfma16x16x4(-v[r], w2[a][r], acc);
    }
    c2[x] = acc;
  }
#pragma unroll
  for (int x = 0; x < NS; ++x) {
    store_slab(u.C, u.ldc, r1 + 32 * rh + 16 * x + 4 * lk, col, m1, colok, vec_ok, c1[x]);
    store_slab(u.C, u.ldc, r2 + 32 * rh + 16 * x + 4 * lk, col, m2, colok, vec_ok, c2[x]);
  }
  __syncthreads();  // LDS buffers free again
}

// Rows 0..b-1 of this workgroup's tile scaled by D.
__device__ __forceinline__ void scale_top_rows(const UpdateParams &u, int tile) {
  for (int e = threadIdx.x; e < u.b * kUpdTile; e += kThreads) {
    const int row = e % u.b;
    const int64_t col = (int64_t)tile * kUpdTile + e / u.b;
    if (col < u.k && row < u.m) u.C[row + col * u.ldc] *= u.d[row];
  }
}

// Q^T update of one leaf on one tile: C_leaf <- C_leaf - Y (T^T (Y^T C_leaf)).
// Wave (cg, rh) holds rows rh*H/2 .. rh*H/2 + H/2 - 1 of the leaf for columns
// 16cg..16cg+15.  Reflector chunks hold 32 rows of each half (block rows
// 0..31: half 0, 32..63: half 1), so every wave works on every chunk.
template <int NQ, int RT, bool TRANS>
__device__ __forceinline__ void leaf_update(const UpdateParams &u, int leaf, int tile, UpdSmem &sm) {
  constexpr int H = 16 * RT;       // leaf rows
  constexpr int HALF = H / 2;      // rows per wave
  constexpr int NX = RT / 2;       // 16-row slabs per wave
  constexpr int NCHUNK = HALF / 32;
  const int tid = opaque_tid();
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int cg = wave & 1, rh = wave >> 1;
  const int li = lane & 15, lk = lane >> 4;
  const int pl = pi16(li);
  const int64_t row0 = (int64_t)leaf * u.h;
  const int64_t col = (int64_t)tile * kUpdTile + 16 * cg + li;
  const bool colok = col < u.k;
  const bool vec_c = aligned16(u.C) && (u.ldc % 2 == 0);
  const bool vec_y = aligned16(u.Y) && (u.ldy % 2 == 0);

  Stage st;
  stage_load<kLeafY>(st, u.Y, u.ldy, row0, row0 + HALF, row0, u.m, u.b, vec_y, tid);
  // uniform fast path for C: the whole leaf x tile block in range and aligned
  const bool cfast = vec_c && row0 + H <= u.m && (int64_t)(tile + 1) * kUpdTile <= u.k;
  double *cptr = u.C + row0 + rh * HALF + 4 * lk + col * u.ldc;
  f64x4 acc[NX];  // rows row0 + rh*HALF + 16x + 4lk + r
  if (cfast) {
#pragma unroll
    for (int x = 0; x < NX; ++x) {
      const f64x2 lo = *reinterpret_cast<const f64x2 *>(cptr + 16 * x);
      const f64x2 hi = *reinterpret_cast<const f64x2 *>(cptr + 16 * x + 2);
      acc[x] = f64x4{lo.x, lo.y, hi.x, hi.y};
    }
  } else {
#pragma unroll
    for (int x = 0; x < NX; ++x)
      acc[x] = load_slab(u.C, u.ldc, row0 + rh * HALF + 16 * x + 4 * lk, col, u.m, colok, vec_c);
  }
  stage_store(st, sm.buf[0], tid);
  __syncthreads();

  // ---- partial W = Y^T C over this wave's rows, chunk by chunk
  f64x4 w[NQ];
#pragma unroll
  for (int a = 0; a < NQ; ++a) w[a] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < NCHUNK; ++c) {
    if (c + 1 < NCHUNK)
      stage_load<kLeafY>(st, u.Y, u.ldy, row0 + 32 * (c + 1), row0 + HALF + 32 * (c + 1), row0, u.m, u.b, vec_y, tid);
    else
      stage_load<kDense>(st, u.T_leaf + (int64_t)leaf * 64 * 64, 64, 0, 0, 0, 0, 0, true, tid);
    const double *ys = sm.buf[c & 1];
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
      const int x = 2 * c + tt;
      const int t = rh * NX + x;  // slab index within the leaf
#pragma unroll
      for (int a = 0; a < NQ; ++a) {
        if (t < a) continue;  // slab rows lie above the reflectors of block a
        const f64x4 y = lds_col4(ys, 16 * a + pl, 32 * rh + 16 * tt + 4 * lk);
#pragma unroll
        for (int r = 0; r < 4; ++r) w[a] = mfma16x16x4(y[r], acc[x][r], w[a]);
      }
    }
    stage_store(st, sm.buf[(c + 1) & 1], tid);
    __syncthreads();
  }
  // ---- W = partial(half 0) + partial(half 1);  W' = T^T W (T in buf[NCHUNK & 1])
  stage_load<kLeafY>(st, u.Y, u.ldy, row0, row0 + HALF, row0, u.m, u.b, vec_y, tid);
  exchange_w<NQ>(w, sm.buf[(NCHUNK + 1) & 1]);
  apply_t_lds<NQ, TRANS>(sm.buf[NCHUNK & 1], w);
  f64x4 (&w2)[NQ] = w;
  __syncthreads();
  stage_store(st, sm.buf[0], tid);
  __syncthreads();
  // ---- C -= Y W', chunk by chunk
#pragma unroll
  for (int c = 0; c < NCHUNK; ++c) {
    if (c + 1 < NCHUNK)
      stage_load<kLeafY>(st, u.Y, u.ldy, row0 + 32 * (c + 1), row0 + HALF + 32 * (c + 1), row0, u.m, u.b, vec_y, tid);
    const double *ys = sm.buf[c & 1];
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
      const int x = 2 * c + tt;
      const int t = rh * NX + x;
#pragma unroll
      for (int a = 0; a < NQ; ++a) {
        if (t < a) continue;
        const f64x4 y = lds_row4(ys, 32 * rh + 16 * tt + pl, 16 * a + 4 * lk);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[x] = mfma16x16x4(-y[r], w2[a][r], acc[x]);
      }
    }
    if (c + 1 < NCHUNK) {
      stage_store(st, sm.buf[(c + 1) & 1], tid);
      __syncthreads();
    }
  }
  if (cfast) {
#pragma unroll
    for (int x = 0; x < NX; ++x) {
      *reinterpret_cast<f64x2 *>(cptr + 16 * x) = f64x2{acc[x][0], acc[x][1]};
      *reinterpret_cast<f64x2 *>(cptr + 16 * x + 2) = f64x2{acc[x][2], acc[x][3]};
    }
  } else {
#pragma unroll
    for (int x = 0; x < NX; ++x)
      store_slab(u.C, u.ldc, row0 + rh * HALF + 16 * x + 4 * lk, col, u.m, colok, vec_c, acc[x]);
  }
  __syncthreads();  // C rows visible to the whole workgroup; LDS free
}

// Q^T of one panel on one tile, for the leaves of group g (u.group leaves,
// a power of two): every leaf update, each followed by the tree levels that
// become complete inside the group (binary pairs i, i + 2^(k-1), the lower
// index on top).  A single group covers the whole tree and also applies D.
// No workgroup depends on another, so no device-scope synchronization is
// needed; the levels above the groups run afterwards, one launch per level.
template <int NQ, int RT>
__global__ void __launch_bounds__(kThreads, 2) qt_group_kernel(UpdateParams u) {
  __shared__ UpdSmem sm;
  const int ngroups = (u.L + u.group - 1) / u.group;
  const int g = blockIdx.x % ngroups;
  const int tile = blockIdx.x / ngroups;
  const bool vec_ok = aligned16(u.C) && (u.ldc % 2 == 0) && aligned16(u.Y) && (u.ldy % 2 == 0);
  const int first = g * u.group, last = min(u.L, first + u.group);
  // all leaves of the group, then the tree levels inside the group bottom-up
#pragma nounroll
  for (int leaf = first; leaf < last; ++leaf) leaf_update<NQ, RT, true>(u, __builtin_amdgcn_readfirstlane(leaf), tile, sm);
  for (int half = 1; half < u.group && half < u.L; half <<= 1)
#pragma nounroll
    for (int node = first + half; node < last; node += 2 * half)
      node_update<NQ, true>(u, node - half, node, tile, sm, vec_ok);
  if (ngroups == 1) scale_top_rows(u, tile);
}

// Q applied (not transposed): leaves only, no tree (the tree runs first, top-down).
template <int NQ, int RT>
__global__ void __launch_bounds__(kThreads, 2) qn_leaf_kernel(UpdateParams u) {
  __shared__ UpdSmem sm;
  const int leaf = blockIdx.x % u.L;
  const int tile = blockIdx.x / u.L;
  leaf_update<NQ, RT, false>(u, leaf, tile, sm);
}

template <int NQ, bool TRANS>
__global__ void __launch_bounds__(kThreads, 2) node_level_kernel(UpdateParams u) {
  __shared__ UpdSmem sm;
  // nodes of this level: ids half, 3*half, 5*half, ... < L
  const int half = 1 << (u.level - 1);
  const int per = (u.L + half - 1) / (2 * half) + 1;
  const int nn = blockIdx.x % per;
  const int tile = blockIdx.x / per;
  const int node = half + 2 * half * nn;
  if (node >= u.L) return;
  const bool vec_ok = aligned16(u.C) && (u.ldc % 2 == 0) && aligned16(u.Y) && (u.ldy % 2 == 0);
  node_update<NQ, TRANS>(u, node - half, node, tile, sm, vec_ok);
}

__global__ void scale_rows_kernel(UpdateParams u) { scale_top_rows(u, blockIdx.x); }

template <int NQ, int RT>
hipError_t launch_qt_t(const UpdateParams &u, hipStream_t s) {
  const int ngroups = (u.L + u.group - 1) / u.group;
  hipLaunchKernelGGL((qt_group_kernel<NQ, RT>), dim3(ngroups * u.tiles), dim3(kThreads), 0, s, u);
  if (ngroups > 1) {
    // levels above the groups, one launch per level (nodes of a level in parallel), then D
    int lev = 1;
    while ((1 << (lev - 1)) < u.group) ++lev;
    for (; (1 << (lev - 1)) < u.L; ++lev) {
      UpdateParams v = u;
      v.level = lev;
      const int half = 1 << (lev - 1);
      const int per = (u.L + half - 1) / (2 * half) + 1;
      hipLaunchKernelGGL((node_level_kernel<NQ, true>), dim3(per * u.tiles), dim3(kThreads), 0, s, v);
    }
    hipLaunchKernelGGL(scale_rows_kernel, dim3(u.tiles), dim3(kThreads), 0, s, u);
  }
  return hipGetLastError();
}

template <int NQ, int RT>
hipError_t launch_qn_t(const UpdateParams &u, hipStream_t s) {
  hipLaunchKernelGGL(scale_rows_kernel, dim3(u.tiles), dim3(kThreads), 0, s, u);
  int levels = 0;
  while ((1 << levels) < u.L) ++levels;
  for (int lev = levels; lev >= 1; --lev) {
    UpdateParams v = u;
    v.level = lev;
    const int half = 1 << (lev - 1);
    const int per = (u.L + half - 1) / (2 * half) + 1;
    hipLaunchKernelGGL((node_level_kernel<NQ, false>), dim3(per * u.tiles), dim3(kThreads), 0, s, v);
  }
  hipLaunchKernelGGL((qn_leaf_kernel<NQ, RT>), dim3(u.L * u.tiles), dim3(kThreads), 0, s, u);
  return hipGetLastError();
}

template <int RT>
hipError_t dispatch_nq(const UpdateParams &u, bool trans, hipStream_t s) {
  switch ((u.b + 15) / 16) {
    case 1: return trans ? launch_qt_t<1, RT>(u, s) : launch_qn_t<1, RT>(u, s);
    case 2: return trans ? launch_qt_t<2, RT>(u, s) : launch_qn_t<2, RT>(u, s);
    case 3: return trans ? launch_qt_t<3, RT>(u, s) : launch_qn_t<3, RT>(u, s);
    case 4: return trans ? launch_qt_t<4, RT>(u, s) : launch_qn_t<4, RT>(u, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t dispatch(const UpdateParams &u, bool trans, hipStream_t s) {
  if (u.b < 1 || u.b > kMaxB || u.L < 1 || u.k < 1 || u.m < 1) return hipErrorInvalidValue;
  switch (u.h) {
    case 64: return dispatch_nq<4>(u, trans, s);
    case 128: return dispatch_nq<8>(u, trans, s);
    case 256: return dispatch_nq<16>(u, trans, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_apply_qt(const UpdateParams &u, hipStream_t s) { return dispatch(u, true, s); }
hipError_t launch_apply_qn(const UpdateParams &u, hipStream_t s) { return dispatch(u, false, s); }

}  // namespace caqr
