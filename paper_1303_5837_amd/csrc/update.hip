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
//   node   (top b rows of the node's members, survivor 0 and eliminated
//           members t = 1 .. cnt-1, cnt <= arity K):
//           W = C_0 + sum_t V_t^T C_t,  W <- T^T W,  C_0 -= W,  C_t -= V_t W
//
// (T instead of T^T for Q C.)  One workgroup of four waves updates the rows
// of one leaf on one 32-column tile: wave (cg, rh) owns columns
// 16cg..16cg+15 of the tile over row half rh of a leaf and keeps them in
// registers between the two products, so C is read and written once per
// leaf; the two halves add their partial W = Y^T C through LDS in a fixed
// order.  Two workgroups share each CU (registers and LDS are sized for it),
// so one issues MFMAs while the other waits for memory or a barrier.  The reflectors are staged through LDS in 64x64 blocks
// (32 rows of each half, double-buffered, loaded with coalesced 16-byte
// accesses), and T goes through the same buffers.  The leaf pass of a wide
// Q^T update (256-row leaves, b = 64) instead keeps a whole leaf's Y and T in
// LDS and gives each of eight waves all 256 rows of 16 columns, one
// workgroup per CU running through many tiles of the same leaf
// (leaf_res_kernel; the same products in the same order).  The tree levels run one
// launch per level (nodes of a level and tiles in parallel), so no workgroup
// ever waits for another; only the single-tile update of the next panel's
// columns climbs the tree inside one launch, with tickets.
//
// Register layout ("contiguous"): a 16-row slab x of a tile is an f64x4 per
// lane holding rows 16x + 4*(lane/16) + r, r = 0..3, of column lane%16.  The
// MFMA result layout holds row 4r + lane/16 in register r, so every product
// whose output uses the contiguous layout reads its A operand at the permuted
// row pi(lane%16) = 4*(lane%4) + (lane%16)/4 of the slab.
#include <hip/hip_ext.h>
#include <algorithm>

#include "device_common.hpp"
#include "kernels.hpp"
#include "staging.hpp"

namespace caqr {

namespace {

constexpr int kUThreads = 256;  // four waves: wave = column group cg (0..1) + 2 * row half rh

struct UpdSmem {
  alignas(32) double buf[2][kMaxB * kLdb];  // reflector chunks, V, T; a free one holds the W partials
};

// LDS of the kernels that apply tree nodes of arity K > 2 with every V_t
// resident (136 KiB for K = 4, one workgroup per CU): buffers 0 .. K-2 hold
// V_1 .. V_{K-1}, buffer K-1 the W partials and then T; a leaf update uses
// buffers 0 and 1 (the layout of UpdSmem).
template <int K>
struct UpdSmemWide {
  alignas(32) double buf[K][kMaxB * kLdb];
  __device__ UpdSmem &leaf() { return *reinterpret_cast<UpdSmem *>(this); }
};

template <int K>
struct NodeSmem {
  using type = UpdSmemWide<K>;
};
template <>
struct NodeSmem<2> {
  using type = UpdSmem;
};
// Workgroups per CU of a kernel that applies tree nodes of arity K.
template <int K>
constexpr int node_wgs_per_cu() {
  return K == 2 ? 2 : 1;
}

// Partial W of (row half, column group, block, lane) in a free staging buffer
// (2 x 2 x 4 x 64 f64x4 = 32 KiB fits in one).
__device__ __forceinline__ f64x4 *xch_at(double *buf, int rh, int cg, int a, int lane) {
  return reinterpret_cast<f64x4 *>(buf) + ((rh * 2 + cg) * 4 + a) * 64 + lane;
}

__device__ __forceinline__ int pi16(int li) { return 4 * (li & 3) + (li >> 2); }

typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 MFMA 16x16x4 with FP32 accumulation (the lower-precision trailing
// update): operands as in the FP64 instruction (A(i, k) in lane i + 16 k,
// B(k, j) in lane j + 16 k), result D(i, j) in lane j + 16 (i / 4), register
// i % 4 -- already the contiguous layout, so its A operand is read at row
// lane % 16 of the slab (no permutation).
__device__ __forceinline__ f32x4 mfma16x16x4_f32(double a, double b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32((float)a, (float)b, c, 0, 0, 0);
}

__device__ __forceinline__ f64x4 to_f64x4(f32x4 v) { return f64x4{v[0], v[1], v[2], v[3]}; }

__host__ __device__ __forceinline__ bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

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

__device__ __forceinline__ f64x4 ld_c4(const double *p) {
  const f64x2 lo = *reinterpret_cast<const f64x2 *>(p);
  const f64x2 hi = *reinterpret_cast<const f64x2 *>(p + 2);
  return f64x4{lo.x, lo.y, hi.x, hi.y};
}

__device__ __forceinline__ void st_c4(double *p, f64x4 v) {
  *reinterpret_cast<f64x2 *>(p) = f64x2{v[0], v[1]};
  *reinterpret_cast<f64x2 *>(p + 2) = f64x2{v[2], v[3]};
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

// The two row halves of a column group hold partial sums of W; afterwards
// both hold W = P(half 0) + P(half 1), added in the same order (bitwise equal).
// xbuf is a free staging buffer; ends with the partials read, so the caller's
// next barrier frees it again.
template <int NQ>
__device__ __forceinline__ void exchange_w(f64x4 (&w)[NQ], double *xbuf) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int cg = wave & 1, rh = wave >> 1;
#pragma unroll
  for (int a = 0; a < NQ; ++a) *xch_at(xbuf, rh, cg, a, lane) = w[a];
  __syncthreads();
#pragma unroll
  for (int a = 0; a < NQ; ++a) w[a] = *xch_at(xbuf, 0, cg, a, lane) + *xch_at(xbuf, 1, cg, a, lane);
}

// Update of the top b rows of tree node `node` (eliminated leaf) and of its
// left sibling on this workgroup's tile.  Wave (cg, rh) holds slabs 2rh and
// 2rh + 1 (16 rows each) of both row blocks for columns 16cg..16cg+15; the two
// halves form W = C1 + V^T C2 from partial sums.  V goes to LDS buffer 0;
// buffer 1 first holds the partial sums, then T.
template <int NQ, bool TRANS>
__device__ __forceinline__ void node_update(const UpdateParams &u, int left, int node, int tile, UpdSmem &sm,
                                            bool vec_ok) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int cg = wave & 1, rh = wave >> 1;
  const int li = lane & 15, lk = lane >> 4;
  const int pl = pi16(li);
  const int64_t col = (int64_t)tile * kUpdTile + 16 * cg + li;
  const bool colok = col < u.k;
  const int64_t r1 = (int64_t)left * u.h, r2 = (int64_t)node * u.h;
  const int64_t m1 = min<int64_t>(u.m, r1 + u.b), m2 = min<int64_t>(u.m, r2 + u.b);
  StageSplit<kUThreads> st;
  stage_load_split<kNodeV>(st, u.Y, u.ldy, r2, r2 + 32, 0, 32, u.m, u.b, vec_ok, tid);
  stage_fix_split<kNodeV>(st, 0, 32, tid);
  stage_store_split(st, sm.buf[0], tid);
  stage_load_split<kDense>(st, u.T_node + (int64_t)node * 64 * 64, 64, 0, 0, 0, 0, 0, 0, true, tid);
  f64x4 c1[2], c2[2];
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    const int t = 2 * rh + x;
    if (t < NQ) {
      c1[x] = load_slab(u.C, u.ldc, r1 + 16 * t + 4 * lk, col, m1, colok, vec_ok);
      c2[x] = load_slab(u.C, u.ldc, r2 + 16 * t + 4 * lk, col, m2, colok, vec_ok);
    }
  }
  __syncthreads();
  // partial W over this wave's slabs: its own slabs of C1 plus V(slab)^T C2(slab)
  f64x4 w[NQ];
#pragma unroll
  for (int a = 0; a < NQ; ++a) {
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const int t = 2 * rh + x;
      if (t > a) continue;  // V upper triangular (also skips t >= NQ)
      const f64x4 v = lds_col4(sm.buf[0], 16 * a + pl, 16 * t + 4 * lk);
#pragma unroll
      for (int r = 0; r < 4; ++r) acc = mfma16x16x4(v[r], c2[x][r], acc);
      if (t == a) acc += c1[x];
    }
    w[a] = acc;
  }
  exchange_w<NQ>(w, sm.buf[1]);
  __syncthreads();  // partials read: buffer 1 takes T
  stage_store_split(st, sm.buf[1], tid);
  __syncthreads();
  apply_t_lds<NQ, TRANS>(sm.buf[1], w);
  // C1 -= W';  C2 -= V W'
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    const int t = 2 * rh + x;
    if (t >= NQ) continue;
#pragma unroll
    for (int a = 0; a < NQ; ++a)
      if (a == t) c1[x] -= w[a];
    f64x4 acc = c2[x];
#pragma unroll
    for (int a = 0; a < NQ; ++a) {
      if (a < t) continue;
      const f64x4 v = lds_row4(sm.buf[0], 16 * t + pl, 16 * a + 4 * lk);
#pragma unroll
      for (int r = 0; r < 4; ++r) acc = mfma16x16x4(-v[r], w[a][r], acc);
    }
    c2[x] = acc;
  }
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    const int t = 2 * rh + x;
    if (t >= NQ) continue;
    store_slab(u.C, u.ldc, r1 + 16 * t + 4 * lk, col, m1, colok, vec_ok, c1[x]);
    store_slab(u.C, u.ldc, r2 + 16 * t + 4 * lk, col, m2, colok, vec_ok, c2[x]);
  }
  __syncthreads();  // LDS buffers free again
}

// The same for a node of up to K members (survivor g, members g + t s,
// t < cnt), K > 2, with every V_t staged once into its own LDS buffer (the
// next one, then T, loading into registers while the previous is stored), so
// that both products with it read LDS: W = C_0 + sum_t V_t^T C_t from the
// two row halves' partial sums (exchanged in buffer K-1, which then takes T),
// then C_0 -= W and C_t -= V_t W.  Members absent from the node (cnt < K) are
// skipped member by member (a uniform branch).
template <int NQ, bool TRANS, int K>
__device__ __forceinline__ void node_update_k(const UpdateParams &u, int g, int s, int cnt, int tile,
                                              UpdSmemWide<K> &sm, bool vec_ok) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int cg = wave & 1, rh = wave >> 1;
  const int li = lane & 15, lk = lane >> 4;
  const int pl = pi16(li);
  const int64_t col = (int64_t)tile * kUpdTile + 16 * cg + li;
  const bool colok = col < u.k;
  auto row_of = [&](int t) { return (int64_t)(g + t * s) * u.h; };
  StageSplit<kUThreads> st;
  stage_load_split<kNodeV>(st, u.Y, u.ldy, row_of(1), row_of(1) + 32, 0, 32, u.m, u.b, vec_ok, tid);
  f64x4 c[K][2];
#pragma unroll
  for (int t = 0; t < K; ++t) {
    if (t >= cnt) break;
    const int64_t rt = row_of(t), mt = min<int64_t>(u.m, rt + u.b);
#pragma unroll
    for (int x = 0; x < 2; ++x)
      if (2 * rh + x < NQ) c[t][x] = load_slab(u.C, u.ldc, rt + 16 * (2 * rh + x) + 4 * lk, col, mt, colok, vec_ok);
  }
#pragma unroll
  for (int t = 1; t < K; ++t) {
    if (t >= cnt) break;
    stage_fix_split<kNodeV>(st, 0, 32, tid);
    stage_store_split(st, sm.buf[t - 1], tid);
    if (t + 1 < cnt)
      stage_load_split<kNodeV>(st, u.Y, u.ldy, row_of(t + 1), row_of(t + 1) + 32, 0, 32, u.m, u.b, vec_ok, tid);
    else
      stage_load_split<kDense>(st, u.T_node + (int64_t)(g + s) * 64 * 64, 64, 0, 0, 0, 0, 0, 0, true, tid);
  }
  __syncthreads();
  // partial W over this wave's slabs: sum_t V_t(slab)^T C_t(slab), then its own slabs of C_0
  f64x4 w[NQ];
#pragma unroll
  for (int a = 0; a < NQ; ++a) w[a] = f64x4{0.0, 0.0, 0.0, 0.0};
  // the NQ accumulations interleaved, every block unconditionally (V's
  // blocks below its diagonal are staged zeros); each one's products in order
#pragma unroll
  for (int t = 1; t < K; ++t) {
    if (t >= cnt) break;
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const int t2 = 2 * rh + x;
      if (t2 >= NQ) continue;  // past the panel's width (slab not loaded)
      f64x4 v[NQ];
#pragma unroll
      for (int a = 0; a < NQ; ++a) v[a] = lds_col4(sm.buf[t - 1], 16 * a + pl, 16 * t2 + 4 * lk);
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int a = 0; a < NQ; ++a) w[a] = mfma16x16x4(v[a][r], c[t][x][r], w[a]);
    }
  }
#pragma unroll
  for (int a = 0; a < NQ; ++a)
#pragma unroll
    for (int x = 0; x < 2; ++x)
      if (2 * rh + x == a) w[a] += c[0][x];
  exchange_w<NQ>(w, sm.buf[K - 1]);
  __syncthreads();  // partials read: buffer K-1 takes T
  stage_store_split(st, sm.buf[K - 1], tid);
  __syncthreads();
  apply_t_lds<NQ, TRANS>(sm.buf[K - 1], w);
  // C_0 -= W';  C_t -= V_t W'
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int a = 0; a < NQ; ++a)
      if (2 * rh + x == a) c[0][x] -= w[a];
#pragma unroll
  for (int t = 1; t < K; ++t) {
    if (t >= cnt) break;
    if constexpr (NQ == 4) {
      // both slabs interleaved, every block unconditionally (V's blocks below
      // its diagonal are staged zeros); each slab's products in order
#pragma unroll
      for (int a = 0; a < NQ; ++a) {
        const f64x4 v0 = lds_row4(sm.buf[t - 1], 32 * rh + pl, 16 * a + 4 * lk);
        const f64x4 v1 = lds_row4(sm.buf[t - 1], 32 * rh + 16 + pl, 16 * a + 4 * lk);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          c[t][0] = mfma16x16x4(-v0[r], w[a][r], c[t][0]);
          c[t][1] = mfma16x16x4(-v1[r], w[a][r], c[t][1]);
        }
      }
    } else {
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const int t2 = 2 * rh + x;
        if (t2 >= NQ) continue;
        f64x4 acc = c[t][x];
#pragma unroll
        for (int a = 0; a < NQ; ++a) {
          if (a < t2) continue;
          const f64x4 v = lds_row4(sm.buf[t - 1], 16 * t2 + pl, 16 * a + 4 * lk);
#pragma unroll
          for (int r = 0; r < 4; ++r) acc = mfma16x16x4(-v[r], w[a][r], acc);
        }
        c[t][x] = acc;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < K; ++t) {
    if (t >= cnt) break;
    const int64_t rt = row_of(t), mt = min<int64_t>(u.m, rt + u.b);
#pragma unroll
    for (int x = 0; x < 2; ++x)
      if (2 * rh + x < NQ) store_slab(u.C, u.ldc, rt + 16 * (2 * rh + x) + 4 * lk, col, mt, colok, vec_ok, c[t][x]);
  }
  __syncthreads();  // LDS buffers free again
}

// Node update of the group of survivor g at stride s with cnt members.
template <int NQ, bool TRANS, int K>
__device__ __forceinline__ void node_update_grp(const UpdateParams &u, int g, int s, int cnt, int tile,
                                                typename NodeSmem<K>::type &sm, bool vec_ok) {
  if constexpr (K == 2)
    node_update<NQ, TRANS>(u, g, g + s, tile, sm, vec_ok);
  else
    node_update_k<NQ, TRANS, K>(u, g, s, cnt, tile, sm, vec_ok);
}

template <int K>
__device__ __forceinline__ UpdSmem &leaf_smem(typename NodeSmem<K>::type &sm) {
  if constexpr (K == 2)
    return sm;
  else
    return sm.leaf();
}

// Members present in the group of survivor g at stride s.
__device__ __forceinline__ int group_members(int g, int s, int K, int L) { return min(K, (L - g + s - 1) / s); }

// Rows 0..b-1 of this workgroup's tile scaled by D (any thread mapping; the
// caller orders it after the tile's last update).
__device__ __forceinline__ void scale_top_rows(const UpdateParams &u, int tile) {
  for (int e = threadIdx.x; e < u.b * kUpdTile; e += blockDim.x) {
    const int row = e % u.b;
    const int64_t col = (int64_t)tile * kUpdTile + e / u.b;
    if (col < u.k && row < u.m) u.C[row + col * u.ldc] *= u.d[row];
  }
}

// Rows 0..b-1 scaled by D, each lane on the rows it wrote itself in
// node_update (or in leaf_update of leaf 0's first slabs): rows
// 16t + 4(lane/16) + r, t = 2rh + x, of column lane%16 of its column group.
template <int NQ>
__device__ __forceinline__ void scale_top_rows_own(const UpdateParams &u, int tile) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int cg = wave & 1, rh = wave >> 1;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t col = (int64_t)tile * kUpdTile + 16 * cg + li;
  if (col >= u.k) return;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * (2 * rh + x) + 4 * lk + r;
      if (row < u.b && row < u.m) u.C[row + col * u.ldc] *= u.d[row];
    }
}

// Q^T (TRANS) or Q update of one leaf on one tile: C_leaf <- C_leaf - Y (T^T (Y^T C_leaf)).
// Wave (cg, rh) holds rows rh*H/2 .. rh*H/2 + H/2 - 1 of the leaf for columns
// 16cg..16cg+15 in registers (RT/2 slabs of 16 rows).  Reflector chunk c holds
// 32 rows of each half (block rows 0..31: half 0 rows 32c.., 32..63: half 1),
// so every wave works on every chunk.  Chunks 0..n-1 for W = Y^T C, then T,
// then chunks n-1..0 for C -= Y W'; chunk c sits in buffer c % 2, T in buffer
// n % 2, and the W partials are exchanged in the last chunk's buffer.
// Every chunk of C is stored as soon as it is final.
// F32: the two products with Y (W = Y^T C and Y W) on FP32 MFMA, each
// accumulated in FP32 from zero (operands rounded to FP32); W' = T^T W, the
// exchange of the partial sums and C itself stay FP64 (C -= the FP32 product).
template <int NQ, int RT, bool TRANS, bool F32 = false>
__device__ __forceinline__ void leaf_update(const UpdateParams &u, int leaf, int tile, UpdSmem &sm) {
  constexpr int H = 16 * RT;       // leaf rows
  constexpr int HALF = H / 2;      // rows per wave
  constexpr int NX = RT / 2;       // 16-row slabs per wave
  constexpr int NCHUNK = HALF / 32;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int cg = wave & 1, rh = wave >> 1;
  const int li = lane & 15, lk = lane >> 4;
  const int pl = F32 ? li : pi16(li);
  const int64_t row0 = (int64_t)leaf * u.h;
  const int64_t col = (int64_t)tile * kUpdTile + 16 * cg + li;
  const bool colok = col < u.k;
  const bool vec_c = aligned16(u.C) && (u.ldc % 2 == 0);
  const bool vec_y = aligned16(u.Y) && (u.ldy % 2 == 0);
  const int xl0 = rh * NX;  // leaf slab index of this wave's slab 0

  StageSplit<kUThreads> st;
  stage_load_split<kLeafY>(st, u.Y, u.ldy, row0, row0 + HALF, 0, HALF, u.m, u.b, vec_y, tid);
  // uniform fast path for C: the whole leaf x tile block in range and aligned
  const bool cfast = vec_c && row0 + H <= u.m && (int64_t)(tile + 1) * kUpdTile <= u.k;
  double *cptr = u.C + row0 + rh * HALF + 4 * lk + col * u.ldc;
  f64x4 acc[NX];  // rows row0 + rh*HALF + 16x + 4lk + r
  if (cfast) {
#pragma unroll
    for (int x = 0; x < NX; ++x) acc[x] = ld_c4(cptr + 16 * x);
  } else {
#pragma unroll
    for (int x = 0; x < NX; ++x)
      acc[x] = load_slab(u.C, u.ldc, row0 + rh * HALF + 16 * x + 4 * lk, col, u.m, colok, vec_c);
  }
  stage_fix_split<kLeafY>(st, 0, HALF, tid);
  stage_store_split(st, sm.buf[0], tid);
  __syncthreads();

  // ---- partial W = Y^T C over this wave's rows, chunk by chunk
  f64x4 w[NQ];
  f32x4 w32[F32 ? NQ : 1];
#pragma unroll
  for (int a = 0; a < NQ; ++a) w[a] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < (F32 ? NQ : 1); ++a) w32[a] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < NCHUNK; ++c) {
    if (c + 1 < NCHUNK)
      stage_load_split<kLeafY>(st, u.Y, u.ldy, row0 + 32 * (c + 1), row0 + HALF + 32 * (c + 1), 32 * (c + 1),
                               HALF + 32 * (c + 1), u.m, u.b, vec_y, tid);
    else
      stage_load_split<kDense>(st, u.T_leaf + (int64_t)leaf * 64 * 64, 64, 0, 0, 0, 0, 0, 0, true, tid);
    const double *ys = sm.buf[c & 1];
    // every block a of the slab unconditionally (rows above block a are
    // staged zeros and add exact zeros), so that the NQ accumulations
    // interleave; each one's products stay in the same order
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
      const int x = 2 * c + tt;
      f64x4 y[NQ];
#pragma unroll
      for (int a = 0; a < NQ; ++a) y[a] = lds_col4(ys, 16 * a + pl, 32 * rh + 16 * tt + 4 * lk);
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int a = 0; a < NQ; ++a) {
          if constexpr (F32)
            w32[F32 ? a : 0] = mfma16x16x4_f32(y[a][r], acc[x][r], w32[F32 ? a : 0]);
          else
            w[a] = mfma16x16x4(y[a][r], acc[x][r], w[a]);
        }
    }
    if (c + 1 < NCHUNK && 32 * (c + 1) < kMaxB)  // rows of the leaf's top triangle
      stage_fix_split<kLeafY>(st, 32 * (c + 1), HALF + 32 * (c + 1), tid);
    stage_store_split(st, sm.buf[(c + 1) & 1], tid);
    __syncthreads();
  }
  // ---- W = P(half 0) + P(half 1), exchanged in the buffer of the last chunk
  // (reloaded below); W' = -T^T W (T in buffer NCHUNK % 2).  The last chunk is
  // loaded again meanwhile for the second pass.
  stage_load_split<kLeafY>(st, u.Y, u.ldy, row0 + 32 * (NCHUNK - 1), row0 + HALF + 32 * (NCHUNK - 1),
                           32 * (NCHUNK - 1), HALF + 32 * (NCHUNK - 1), u.m, u.b, vec_y, tid);
  if constexpr (F32) {
#pragma unroll
    for (int a = 0; a < NQ; ++a) w[a] = to_f64x4(w32[F32 ? a : 0]);
  }
  exchange_w<NQ>(w, sm.buf[(NCHUNK - 1) & 1]);
  apply_t_lds<NQ, TRANS>(sm.buf[NCHUNK & 1], w);
#pragma unroll
  for (int a = 0; a < NQ; ++a) w[a] = -w[a];
  __syncthreads();  // partials read, T used: both buffers free
  if (32 * (NCHUNK - 1) < kMaxB) stage_fix_split<kLeafY>(st, 32 * (NCHUNK - 1), HALF + 32 * (NCHUNK - 1), tid);
  stage_store_split(st, sm.buf[(NCHUNK - 1) & 1], tid);
  if (NCHUNK > 1)
    stage_load_split<kLeafY>(st, u.Y, u.ldy, row0 + 32 * (NCHUNK - 2), row0 + HALF + 32 * (NCHUNK - 2),
                             32 * (NCHUNK - 2), HALF + 32 * (NCHUNK - 2), u.m, u.b, vec_y, tid);
  __syncthreads();
  // ---- C += Y W', chunks NCHUNK-1 .. 0
#pragma unroll
  for (int c = NCHUNK - 1; c >= 0; --c) {
    if (c >= 1) {
      if (32 * (c - 1) < kMaxB)  // rows of the leaf's top triangle
        stage_fix_split<kLeafY>(st, 32 * (c - 1), HALF + 32 * (c - 1), tid);
      stage_store_split(st, sm.buf[(c - 1) & 1], tid);  // into the buffer chunk c + 1 (or T) left
      if (c >= 2)
        stage_load_split<kLeafY>(st, u.Y, u.ldy, row0 + 32 * (c - 2), row0 + HALF + 32 * (c - 2), 32 * (c - 2),
                                 HALF + 32 * (c - 2), u.m, u.b, vec_y, tid);
    }
    const double *ys = sm.buf[c & 1];
    f32x4 prod[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};  // FP32: Y W of this chunk
    // both slabs of the chunk interleaved, every block a unconditionally
    // (rows above block a are staged zeros); each slab's products in order
#pragma unroll
    for (int a = 0; a < NQ; ++a) {
      const f64x4 y0 = lds_row4(ys, 32 * rh + pl, 16 * a + 4 * lk);
      const f64x4 y1 = lds_row4(ys, 32 * rh + 16 + pl, 16 * a + 4 * lk);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if constexpr (F32) {
          prod[0] = mfma16x16x4_f32(y0[r], w[a][r], prod[0]);
          prod[1] = mfma16x16x4_f32(y1[r], w[a][r], prod[1]);
        } else {
          acc[2 * c] = mfma16x16x4(y0[r], w[a][r], acc[2 * c]);
          acc[2 * c + 1] = mfma16x16x4(y1[r], w[a][r], acc[2 * c + 1]);
        }
      }
    }
    if constexpr (F32) {
#pragma unroll
      for (int tt = 0; tt < 2; ++tt) acc[2 * c + tt] += to_f64x4(prod[tt]);
    }
    // rows of chunk c are final
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
      const int x = 2 * c + tt;
      if (cfast)
        st_c4(cptr + 16 * x, acc[x]);
      else
        store_slab(u.C, u.ldc, row0 + rh * HALF + 16 * x + 4 * lk, col, u.m, colok, vec_c, acc[x]);
    }
    if (c >= 1) __syncthreads();
  }
  __syncthreads();  // LDS free for the next update
}

// Workgroups go to the device's eight XCDs round-robin by index, and each XCD
// has its own L2.  This renumbering gives every XCD one contiguous range of
// logical indices (a bijection on [0, n) for any n), so that, with the tile
// index fastest, the workgroups on one XCD share the reflectors and T of few
// leaves or nodes instead of each XCD fetching all of them.
__device__ __forceinline__ int xcd_range_index(int bid, int n) {
  constexpr int kXcd = 8;
  const int q = n / kXcd, r = n % kXcd;
  const int x = bid % kXcd;
  return x * q + min(x, r) + bid / kXcd;
}

// Leaf updates of one panel, one workgroup per (leaf, tile): Q^T (TRANS) runs
// them before the tree levels, Q after them.  No workgroup depends on another.
template <int NQ, int RT, bool TRANS, bool F32 = false>
__global__ void __launch_bounds__(kUThreads, 2) leaf_kernel(UpdateParams u) {
  __shared__ UpdSmem sm;
  const int id = xcd_range_index(blockIdx.x, gridDim.x);
  const int leaf = id / u.tiles;
  const int tile = id % u.tiles;
  leaf_update<NQ, RT, TRANS, F32>(u, leaf, tile, sm);
}

// ---- Q^T leaf updates with the leaf's reflectors resident in LDS (256-row
// leaves, b = 64, FP64): the pass over the leaves of the wide trailing update.
// A workgroup of eight waves (two per SIMD, one workgroup per CU) keeps Y and
// T of one leaf in LDS and takes a contiguous run of jobs (leaf, 128-column
// tile) in leaf-major order (the jobs wholly inside C first, then the edge
// jobs), so Y and T are staged once per leaf it visits.  Wave w holds columns 16w..16w+15 of the tile over all 256 rows (16 slabs in
// the contiguous layout): W = Y^T C needs no exchange between waves, and no
// barrier separates the waves within a job.  Each slab of C is stored as soon
// as it is final and the next job's slab is loaded into its registers, so
// the next job's C is in flight during this job's update (two slabs at a
// time, their accumulations interleaved).  The products are
// formed in the order of leaf_update (partial sums of rows 0..127 and
// 128..255 added, T applied, then C += Y W' slab by slab), so the result is
// bitwise that of leaf_kernel.
constexpr int kResThreads = 512;
constexpr int kResCols = 16 * (kResThreads / 64);  // columns of a job
constexpr int kResRows = 256;                      // leaf rows

// LDS of a workgroup: Y column-major with leading dimension kResLd (the
// 16 columns, or 16 rows, of one MFMA operand read fall in different banks),
// and the ten 16x16 blocks of T on and above the diagonal, each column-major
// with leading dimension 18 (the same property); 151.5 KiB.
constexpr int kResLd = kResRows + 2;
constexpr int kTBlk = 16 * 18;

struct ResSmem {
  alignas(16) double y[kMaxB * kResLd];
  alignas(16) double t[10 * kTBlk];
};

__device__ __forceinline__ int t_block(int a, int ao) { return (ao * (ao + 1) / 2 + a) * kTBlk; }

// Rows row0..row0+3 of column col of Y (row0 even).
__device__ __forceinline__ f64x4 res_col4(const double *y, int col, int row0) {
  const double *p = y + col * kResLd + row0;
  const f64x2 lo = *reinterpret_cast<const f64x2 *>(p);
  const f64x2 hi = *reinterpret_cast<const f64x2 *>(p + 2);
  return f64x4{lo.x, lo.y, hi.x, hi.y};
}

// Columns col0..col0+3 of row `row` of Y.
__device__ __forceinline__ f64x4 res_row4(const double *y, int row, int col0) {
  const double *p = y + col0 * kResLd + row;
  return f64x4{p[0], p[kResLd], p[2 * kResLd], p[3 * kResLd]};
}

// Rows 16a + lr0 .. +3 of column 16ao + lc of T (a <= ao; lr0 even).
__device__ __forceinline__ f64x4 res_t4(const double *t, int a, int ao, int lc, int lr0) {
  const double *p = t + t_block(a, ao) + lc * 18 + lr0;
  const f64x2 lo = *reinterpret_cast<const f64x2 *>(p);
  const f64x2 hi = *reinterpret_cast<const f64x2 *>(p + 2);
  return f64x4{lo.x, lo.y, hi.x, hi.y};
}

// Y (unit lower trapezoidal in its top 64 rows, zero past the panel's last
// row) and T of `leaf` into LDS; every thread of the workgroup takes part.
// Two rounds of eight 16-byte loads per thread keep the staging registers few
// (the next job's C is in flight meanwhile).
__device__ __forceinline__ void res_stage(ResSmem &sm, const UpdateParams &u, int leaf, int tid) {
  // Y: thread tid moves the row pair lr of columns col0 + 4s, s = 0..15, from
  // one base address and a uniform stride (nothing per s to keep live)
  const int64_t row0 = (int64_t)leaf * kResRows;
  const bool full = row0 + kResRows <= u.m;
  const int lr = 2 * (tid & 127), col0 = tid >> 7;
  const int64_t g = row0 + lr;
  const double *src = u.Y + g + (int64_t)col0 * u.ldy;
  const int64_t step = 4 * u.ldy;
  double *dst = sm.y + col0 * kResLd + lr;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    f64x2 v[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const double *q = src + (8 * h + s) * step;
      if (full) {
        v[s] = *reinterpret_cast<const f64x2 *>(q);
      } else {
        v[s].x = (g < u.m) ? q[0] : 0.0;
        v[s].y = (g + 1 < u.m) ? q[1] : 0.0;
      }
    }
    // the row and column as opaque values: the masks below are recomputed at
    // each staging instead of being kept live (spilled) across the job loop
    int lrv = lr, c0v = col0;
    asm volatile("" : "+v"(lrv), "+v"(c0v));
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int col = c0v + 4 * (8 * h + s);
      f64x2 x = v[s];
      if (lrv < kMaxB) {  // the leaf's top triangle: zero above the diagonal, 1 on it
        x.x = (lrv > col) ? x.x : ((lrv == col) ? 1.0 : 0.0);
        x.y = (lrv + 1 > col) ? x.y : ((lrv + 1 == col) ? 1.0 : 0.0);
      }
      *reinterpret_cast<f64x2 *>(dst + 4 * (8 * h + s) * kResLd) = x;
    }
  }
  // T: the row pair tl of columns ct + 16s, kept where the block is on or above the diagonal
  const int tl = 2 * (tid & 31), ct = tid >> 5;
  const double *tg = u.T_leaf + (int64_t)leaf * kMaxB * kMaxB + tl + kMaxB * ct;
  // all four loads unconditional (the 64 x 64 block is whole), the LDS writes masked
  f64x2 tv[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) tv[s] = *reinterpret_cast<const f64x2 *>(tg + 16 * kMaxB * s);
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int a = tl >> 4, ao = s;  // column ct + 16 s lies in block column s
    if (a <= ao) *reinterpret_cast<f64x2 *>(sm.t + t_block(a, ao) + (ct & 15) * 18 + (tl & 15)) = tv[s];
  }
}

// W = Y^T C of one job (partial sums over rows 0..127 and 128..255, then
// added), then W <- -T^T W (blocks from the last one down, in place).
__device__ __forceinline__ void res_form_w(const ResSmem &sm, const f64x4 (&acc)[16], f64x4 (&w)[4], int pl,
                                           int lk) {
  f64x4 p0[4], p1[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) p0[a] = p1[a] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int x = 0; x < 16; ++x) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if (x < a) continue;  // rows above block a are zero
      const f64x4 y = res_col4(sm.y, 16 * a + pl, 16 * x + 4 * lk);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (x < 8) p0[a] = mfma16x16x4(y[r], acc[x][r], p0[a]);
        else p1[a] = mfma16x16x4(y[r], acc[x][r], p1[a]);
      }
    }
    __builtin_amdgcn_sched_barrier(0);  // one slab's operands live at a time
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) w[a] = p0[a] + p1[a];
#pragma unroll
  for (int oo = 0; oo < 4; ++oo) {
    const int ao = 3 - oo;
    f64x4 t4 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if (a > ao) continue;
      const f64x4 t = res_t4(sm.t, a, ao, pl, 4 * lk);
#pragma unroll
      for (int r = 0; r < 4; ++r) t4 = mfma16x16x4(t[r], w[a][r], t4);
    }
    w[ao] = t4;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) w[a] = -w[a];
}

// Slab x of C += Y W'.
__device__ __forceinline__ f64x4 res_apply_slab(const ResSmem &sm, f64x4 c, const f64x4 (&w)[4], int x, int pl,
                                                int lk) {
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    if (x < a) continue;
    const f64x4 y = res_row4(sm.y, 16 * x + pl, 16 * a + 4 * lk);
#pragma unroll
    for (int r = 0; r < 4; ++r) c = mfma16x16x4(y[r], w[a][r], c);
  }
  return c;
}

// Slabs x and x + 1 of C += Y W', their two accumulations interleaved (each
// in the order of res_apply_slab).
__device__ __forceinline__ void res_apply_slab2(const ResSmem &sm, f64x4 &c0, f64x4 &c1, const f64x4 (&w)[4], int x,
                                                int pl, int lk) {
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    if (x + 1 < a) continue;
    const f64x4 y1 = res_row4(sm.y, 16 * (x + 1) + pl, 16 * a + 4 * lk);
    if (x >= a) {
      const f64x4 y0 = res_row4(sm.y, 16 * x + pl, 16 * a + 4 * lk);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        c0 = mfma16x16x4(y0[r], w[a][r], c0);
        c1 = mfma16x16x4(y1[r], w[a][r], c1);
      }
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) c1 = mfma16x16x4(y1[r], w[a][r], c1);
    }
  }
}

__global__ void __launch_bounds__(kResThreads, 1) leaf_res_kernel(UpdateParams u, int ntiles, int jobs) {
  __shared__ ResSmem sm;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int pl = pi16(li);
  const int gw = xcd_range_index(blockIdx.x, gridDim.x);
  const int j0 = (int)((int64_t)jobs * gw / gridDim.x);
  const int j1 = (int)((int64_t)jobs * (gw + 1) / gridDim.x);
  if (j0 >= j1) return;
  // Jobs (leaf, 128-column tile), the ones wholly inside C first, leaf-major
  // (jobs [0, jm): leaf j / ntf, tile j % ntf), then the edge jobs: the last
  // tile of each full leaf when k is not a multiple of 128, and the tiles of
  // the last leaf when it is short.  The first run has no branch around its
  // loads and stores, so the compiler counts the outstanding memory
  // operations exactly: storing a slab, then loading the next job's slab into
  // its registers, waits for nothing, and (with the loop over the job index
  // written as below) the W phase waits for the prefetched slabs one by one
  // rather than for all of them.  The bounds-checked edge jobs run after it,
  // in a loop of their own.
  const int ntf = (int)(u.k / kResCols);
  const int lf = (int)(u.m / kResRows);
  const bool ce = ntf < ntiles;
  const int jm = lf * ntf;
  const int je = jm + (ce ? lf : 0);
  double *const cw = u.C + 4 * lk + (int64_t)(16 * wave + li) * u.ldc;  // this lane's row 4lk of column 16w + li
  auto job_c = [&](int j) { return cw + (int64_t)(j / ntf) * kResRows + (int64_t)(j % ntf) * kResCols * u.ldc; };
  f64x4 acc[16];
  int cur = -1;
  const int jm1 = min(j1, jm);
  int j = (j0 < jm1) ? j0 : -1;
  if (j >= 0) {
    const double *cp = job_c(j);
#pragma unroll
    for (int x = 0; x < 16; ++x) acc[x] = ld_c4(cp + 16 * x);
  }
  while (j >= 0) {
    const int leaf = j / ntf;
    if (leaf != cur) {  // every wave is past the previous leaf's reads
      __syncthreads();
      res_stage(sm, u, leaf, tid);
      __syncthreads();
      cur = leaf;
    }
    double *cp = job_c(j);
    f64x4 w[4];
    res_form_w(sm, acc, w, pl, lk);
    // ---- C += Y W' two slabs at a time; each final slab stored and the next
    // job's slab loaded into its registers (after the last job, a value never
    // used: every slab's load reads this lane's first slab, which stays cached)
    const int jn = (j + 1 < jm1) ? j + 1 : -1;
    const double *np = (jn >= 0) ? job_c(jn) : cp;
    const int ns = (jn >= 0) ? 16 : 0;
#pragma unroll
    for (int x = 0; x < 16; x += 2) {
      res_apply_slab2(sm, acc[x], acc[x + 1], w, x, pl, lk);
      st_c4(cp + 16 * x, acc[x]);
      st_c4(cp + 16 * x + 16, acc[x + 1]);
      acc[x] = ld_c4(np + ns * x);
      acc[x + 1] = ld_c4(np + ns * (x + 1));
      __builtin_amdgcn_sched_barrier(0);
    }
    j = jn;
  }
  for (int j = max(j0, jm); j < j1; ++j) {
    const int leaf = (j < je) ? j - jm : lf;
    const int tile = (j < je) ? ntf : j - je;
    if (leaf != cur) {
      __syncthreads();
      res_stage(sm, u, leaf, tid);
      __syncthreads();
      cur = leaf;
    }
    const int64_t row0 = (int64_t)leaf * kResRows, col = (int64_t)tile * kResCols + 16 * wave + li;
#pragma unroll
    for (int x = 0; x < 16; ++x) acc[x] = load_slab(u.C, u.ldc, row0 + 16 * x + 4 * lk, col, u.m, col < u.k, true);
    f64x4 w[4];
    res_form_w(sm, acc, w, pl, lk);
#pragma unroll
    for (int x = 0; x < 16; ++x) {
      acc[x] = res_apply_slab(sm, acc[x], w, x, pl, lk);
      store_slab(u.C, u.ldc, row0 + 16 * x + 4 * lk, col, u.m, col < u.k, true, acc[x]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// ---- Q^T updates of one tree level's 4-ary nodes with the node's V_1..V_3
// and T resident in LDS (b = 64, FP64), the same scheme as leaf_res_kernel:
// a workgroup of eight waves takes a contiguous run of jobs (node, 128-column
// tile), staging V and T once per node it visits; wave w holds the top 64
// rows of every member for columns 16w..16w+15.  The products are formed in
// the order of node_update_k (partial sums of rows 0..31 and 32..63 of the
// members added, T applied, then C_0 -= W' and C_t -= V_t W'), so the result
// is bitwise that of node_level_kernel.
constexpr int kNodeLd = kMaxB + 2;

struct NodeResSmem {
  alignas(16) double v[3][kMaxB * kNodeLd];  // V_1..V_3, column-major
  alignas(16) double t[10 * kTBlk];
};

__device__ __forceinline__ f64x4 node_col4(const double *v, int col, int row0) {
  const double *p = v + col * kNodeLd + row0;
  const f64x2 lo = *reinterpret_cast<const f64x2 *>(p);
  const f64x2 hi = *reinterpret_cast<const f64x2 *>(p + 2);
  return f64x4{lo.x, lo.y, hi.x, hi.y};
}

__device__ __forceinline__ f64x4 node_row4(const double *v, int row, int col0) {
  const double *p = v + col0 * kNodeLd + row;
  return f64x4{p[0], p[kNodeLd], p[2 * kNodeLd], p[3 * kNodeLd]};
}

// V_t (upper triangular with its diagonal, zero past the panel's last row) of
// members t = 1 .. cnt-1 of the node of survivor g at stride s, and the node's T.
__device__ __forceinline__ void node_res_stage(NodeResSmem &sm, const UpdateParams &u, int g, int s, int cnt,
                                               int tid) {
  const int lr = 2 * (tid & 31), col0 = tid >> 5;  // row pair lr of columns col0 + 16 q, q = 0..3
  int lrv = lr, c0v = col0;
  asm volatile("" : "+v"(lrv), "+v"(c0v));
#pragma unroll
  for (int t = 1; t < 4; ++t) {
    if (t >= cnt) break;
    const int64_t g0 = (int64_t)(g + t * s) * u.h + lr;
    const double *src = u.Y + g0 + (int64_t)col0 * u.ldy;
    const bool full = g0 + 1 < u.m;
    f64x2 v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double *p = src + (int64_t)(16 * q) * u.ldy;
      if (full) {
        v[q] = *reinterpret_cast<const f64x2 *>(p);
      } else {
        v[q].x = (g0 < u.m) ? p[0] : 0.0;
        v[q].y = 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int col = c0v + 16 * q;
      f64x2 x = v[q];
      x.x = (lrv <= col) ? x.x : 0.0;
      x.y = (lrv + 1 <= col) ? x.y : 0.0;
      *reinterpret_cast<f64x2 *>(sm.v[t - 1] + col * kNodeLd + lr) = x;
    }
  }
  const double *tg = u.T_node + (int64_t)(g + s) * kMaxB * kMaxB + lr + kMaxB * col0;
  // T: the row pair lr of columns col0 + 16 q, kept where the block is on or above the diagonal
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int a = lr >> 4, ao = q;
    if (a <= ao)
      *reinterpret_cast<f64x2 *>(sm.t + t_block(a, ao) + col0 * 18 + (lr & 15)) =
          *reinterpret_cast<const f64x2 *>(tg + 16 * kMaxB * q);
  }
}

__global__ void __launch_bounds__(kResThreads, 1) node_res_kernel(UpdateParams u, int ntiles, int jobs) {
  constexpr int K = 4;
  __shared__ NodeResSmem sm;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int pl = pi16(li);
  const int s = u.stride;
  const int gw = xcd_range_index(blockIdx.x, gridDim.x);
  const int j0 = (int)((int64_t)jobs * gw / gridDim.x);
  const int j1 = (int)((int64_t)jobs * (gw + 1) / gridDim.x);
  if (j0 >= j1) return;
  // job j: node j / ntiles (survivor g = K s (j / ntiles)), columns tile * kResCols + 16 wave + li
  auto job_g = [&](int j) { return K * s * (j / ntiles); };
  auto job_col = [&](int j) { return (int64_t)(j % ntiles) * kResCols + 16 * wave + li; };
  auto job_cnt = [&](int j) { return group_members(job_g(j), s, K, u.L); };
  auto job_fast = [&](int j) {
    return (int64_t)(job_g(j) + (job_cnt(j) - 1) * s) * u.h + kMaxB <= u.m &&
           (int64_t)(j % ntiles + 1) * kResCols <= u.k;
  };
  auto load = [&](int j, int t, int x) {
    const int64_t rt = (int64_t)(job_g(j) + t * s) * u.h;
    const int64_t col = job_col(j);
    const int64_t grow = rt + 16 * x + 4 * lk;
    if (job_fast(j)) return ld_c4(u.C + grow + col * u.ldc);
    return load_slab(u.C, u.ldc, grow, col, min<int64_t>(u.m, rt + u.b), col < u.k, true);
  };
  f64x4 c[K][4];
  {
    const int cnt0 = job_cnt(j0);
#pragma unroll
    for (int t = 0; t < K; ++t)
#pragma unroll
      for (int x = 0; x < 4; ++x)
        if (t < cnt0) c[t][x] = load(j0, t, x);
  }
  int cur = -1;
  for (int j = j0; j < j1; ++j) {
    const int node = j / ntiles;
    const int g = job_g(j), cnt = job_cnt(j);
    const int64_t col = job_col(j);
    const bool cfast = job_fast(j);
    const bool next = j + 1 < j1;
    if (cnt >= 2 && node != cur) {  // every wave is past the previous node's reads
      __syncthreads();
      node_res_stage(sm, u, g, s, cnt, tid);
      __syncthreads();
      cur = node;
    }
    if (cnt >= 2) {
      // ---- W = C_0 + sum_t V_t^T C_t: partial sums over rows 0..31 and 32..63
      f64x4 p0[4], p1[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) p0[a] = p1[a] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 1; t < K; ++t) {
        if (t >= cnt) break;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int x = 0; x < 4; ++x) {
            if (x > a) continue;  // V upper triangular
            const f64x4 v = node_col4(sm.v[t - 1], 16 * a + pl, 16 * x + 4 * lk);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              if (x < 2) p0[a] = mfma16x16x4(v[r], c[t][x][r], p0[a]);
              else p1[a] = mfma16x16x4(v[r], c[t][x][r], p1[a]);
            }
          }
        __builtin_amdgcn_sched_barrier(0);
      }
      f64x4 w[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        if (a < 2) p0[a] += c[0][a];
        else p1[a] += c[0][a];
        w[a] = p0[a] + p1[a];
      }
      // ---- W <- T^T W (blocks from the last one down, in place)
#pragma unroll
      for (int oo = 0; oo < 4; ++oo) {
        const int ao = 3 - oo;
        f64x4 t4 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          if (a > ao) continue;
          const f64x4 tt = res_t4(sm.t, a, ao, pl, 4 * lk);
#pragma unroll
          for (int r = 0; r < 4; ++r) t4 = mfma16x16x4(tt[r], w[a][r], t4);
        }
        w[ao] = t4;
      }
      // ---- C_0 -= W';  C_t -= V_t W', each slab stored when final.  At the
      // top level (the root, survivor 0) the panel's top rows also take D.
#pragma unroll
      for (int x = 0; x < 4; ++x) c[0][x] -= w[x];
      if (K * s >= u.L) {
#pragma unroll
        for (int x = 0; x < 4; ++x) c[0][x] *= ld_c4(u.d + 16 * x + 4 * lk);
      }
#pragma unroll
      for (int t = 0; t < K; ++t) {
        if (t >= cnt) break;
        const int64_t rt = (int64_t)(g + t * s) * u.h;
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          if (t > 0) {
            f64x4 acc = c[t][x];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
              if (a < x) continue;
              const f64x4 v = node_row4(sm.v[t - 1], 16 * x + pl, 16 * a + 4 * lk);
#pragma unroll
              for (int r = 0; r < 4; ++r) acc = mfma16x16x4(-v[r], w[a][r], acc);
            }
            c[t][x] = acc;
          }
          const int64_t grow = rt + 16 * x + 4 * lk;
          if (cfast)
            st_c4(u.C + grow + col * u.ldc, c[t][x]);
          else
            store_slab(u.C, u.ldc, grow, col, min<int64_t>(u.m, rt + u.b), col < u.k, true, c[t][x]);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    if (next) {
      const int cn = job_cnt(j + 1);
#pragma unroll
      for (int t = 0; t < K; ++t)
#pragma unroll
        for (int x = 0; x < 4; ++x)
          if (t < cn) c[t][x] = load(j + 1, t, x);
    }
  }
}

// Q^T leaf updates of the K neighbouring leaves of one first-level group
// (leaves g .. g + K - 1) on one tile, then that group's node (its rows were
// just written by this workgroup, so no other workgroup is involved): one
// workgroup per (group, tile), and the level launches start at the second
// level.
template <int NQ, int RT, int K, bool F32 = false>
__global__ void __launch_bounds__(kUThreads, 2) leaf_group_kernel(UpdateParams u) {
  static_assert(K == 2, "wider nodes are applied by their own level launches");
  __shared__ UpdSmem sm;
  const int id = xcd_range_index(blockIdx.x, gridDim.x);
  const int gi = id / u.tiles;
  const int tile = id % u.tiles;
  const int g = K * gi;
  const int cnt = min(K, u.L - g);
  const bool vec_ok = aligned16(u.C) && (u.ldc % 2 == 0) && aligned16(u.Y) && (u.ldy % 2 == 0);
  leaf_update<NQ, RT, true, F32>(u, g, tile, sm);  // each ends with a barrier: the leaf's C stored
  if constexpr (K == 2) {
    if (g + 1 < u.L) {
      leaf_update<NQ, RT, true, F32>(u, g + 1, tile, sm);
      node_update<NQ, true>(u, g, g + 1, tile, sm, vec_ok);
    }
  }
}

// Every node of tree level u.stride = s on every tile: workgroup (group i,
// tile), group survivor g = K s i, for the groups with two or more members.
template <int NQ, bool TRANS, int K>
__global__ void __launch_bounds__(kUThreads, node_wgs_per_cu<K>()) node_level_kernel(UpdateParams u) {
  __shared__ typename NodeSmem<K>::type sm;
  const int s = u.stride;
  const int id = xcd_range_index(blockIdx.x, gridDim.x);
  const int gi = id / u.tiles;
  const int tile = id % u.tiles;
  const int g = K * s * gi;
  const int cnt = group_members(g, s, K, u.L);
  if (cnt < 2) return;
  const bool vec_ok = aligned16(u.C) && (u.ldc % 2 == 0) && aligned16(u.Y) && (u.ldy % 2 == 0);
  node_update_grp<NQ, TRANS, K>(u, g, s, cnt, tile, sm, vec_ok);
}

__global__ void scale_rows_kernel(UpdateParams u) { scale_top_rows(u, blockIdx.x); }

// Last-arriver ticket on node `node` of cnt members; true for the workgroup
// that arrives last (and performs the node's update).  Publishes this
// workgroup's stores to C before the ticket and acquires the other members'
// after it; the last arriver leaves the counter at zero.
__device__ __forceinline__ bool arrive(unsigned *tickets, int node, int cnt, int &flag) {
  fence_release();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned old = ticket_add(tickets + node);
    const bool last = old + 1u == (unsigned)cnt;
    flag = last ? 1 : 0;
    if (last) ticket_clear(tickets + node);
  }
  __syncthreads();
  const bool last = flag == 1;
  if (last) fence_acquire();
  return last;
}

// Q^T of one panel on a few tiles (at most kTreeTiles, e.g. the next panel's
// columns), the whole tree in one launch: workgroup (leaf i, tile t) updates
// leaf i on tile t, then climbs that tile's tree; below every node the last of
// its members' workgroups to arrive (an agent-scope ticket) performs the
// node's update, the others exit.  The grouping is fixed by index, so the
// result does not depend on arrival order.  The workgroup that completes the
// root applies D.
template <int NQ, int RT, int K, bool F32 = false>
__global__ void __launch_bounds__(kUThreads, node_wgs_per_cu<K>()) qt_tree_tile_kernel(UpdateParams u) {
  __shared__ typename NodeSmem<K>::type sm;
  __shared__ int flag;
  const bool vec_ok = aligned16(u.C) && (u.ldc % 2 == 0) && aligned16(u.Y) && (u.ldy % 2 == 0);
  const int leaf = blockIdx.x % u.L;
  const int tile = blockIdx.x / u.L;
  unsigned *tickets = u.tickets + (int64_t)tile * u.L;  // each tile climbs its own tree
  leaf_update<NQ, RT, true, F32>(u, leaf, tile, leaf_smem<K>(sm));
  int rt = leaf;  // root of the subtree this workgroup holds
  for (int s = 1; s < u.L; s *= K) {
    const int g = rt - rt % (K * s);  // survivor of rt's group at this level
    const int cnt = group_members(g, s, K, u.L);
    if (cnt < 2) continue;  // alone: pass through
    if (!arrive(tickets, g + s, cnt, flag)) return;
    node_update_grp<NQ, true, K>(u, g, s, cnt, tile, sm, vec_ok);
    rt = g;
  }
  scale_top_rows_own<NQ>(u, tile);
}

// The resident-reflector leaf pass serves full-width panels of 256-row leaves
// whose C, Y and T allow 16-byte accesses, on at least one full job width.
bool res_ok(const UpdateParams &u) {
  return u.b == kMaxB && u.h == kResRows && u.k >= kResCols && aligned16(u.C) && u.ldc % 2 == 0 && aligned16(u.Y) &&
         u.ldy % 2 == 0 && aligned16(u.T_leaf);
}

// The resident node levels: 4-ary nodes of full-width panels, C, Y and T
// allowing 16-byte accesses, at least one full job width.
bool node_res_ok(const UpdateParams &u) {
  return u.b == kMaxB && u.k >= kResCols && aligned16(u.C) && u.ldc % 2 == 0 && aligned16(u.Y) && u.ldy % 2 == 0 &&
         aligned16(u.T_node) && aligned16(u.d);
}

// Workgroups of the resident-reflector leaf pass (its LDS admits one per CU):
// one per CU of the current device except 3/16 of them, which stay free for
// the panel chain's kernels running beside the wide update (8192^2: 45.7 ms
// with every CU taken, 45.0 with 48 of 256 left, 46.6 with 96); fewer if
// there are fewer jobs.
int res_grid() {
  static int grid[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 208;
  if (!grid[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 256;
    grid[dev] = std::max(1, n - n * 3 / 16);
  }
  return grid[dev];
}

// Trace events of the Q^T call being launched on this thread (set by the
// caller around one call): the start event takes the first launch's start
// time and the stop event the last launch's end time, so timing a call adds
// no packets of its own to the stream.
thread_local hipEvent_t tl_trace_start = nullptr, tl_trace_stop = nullptr;

template <typename Kern, typename... Args>
void launch_traced(Kern kernel, dim3 grid, dim3 block, hipStream_t s, bool last, Args... args) {
  hipEvent_t stop = last ? tl_trace_stop : nullptr;
  if (tl_trace_start || stop) {
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, tl_trace_start, stop, 0, args...);
    tl_trace_start = nullptr;  // the first launch only
  } else {
    hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
  }
}

template <int NQ, int RT, int K, bool F32>
hipError_t launch_qt_t(const UpdateParams &u, hipStream_t s) {
  if (u.tickets && u.tiles <= kTreeTiles && u.L > 1) {
    launch_traced((qt_tree_tile_kernel<NQ, RT, K, F32>), dim3(u.L * u.tiles), dim3(kUThreads), s, true, u);
    return hipGetLastError();
  }
  const bool res_levels = K == 4 && NQ == 4 && node_res_ok(u);  // the top one also applies D
  const bool scale = !(res_levels && u.L > 1);                   // D by its own launch
  // binary trees: leaf pairs with the first level, then the tree bottom-up (one
  // launch per level, nodes of a level in parallel), then D.  Wider nodes: one
  // workgroup per leaf (short workgroups, so that the concurrent panel chain
  // reaches free CUs sooner), then every level by its own launch.
  const int st0 = (K == 2) ? K : 1;  // the first level a level launch takes
  const bool leaf_last = st0 >= u.L && !scale;
  if constexpr (K == 2) {
    launch_traced((leaf_group_kernel<NQ, RT, K, F32>), dim3((u.L + K - 1) / K * u.tiles), dim3(kUThreads),
                  s, leaf_last, u);
  } else if (NQ == 4 && RT == 16 && !F32 && res_ok(u)) {
    const int ntiles = (int)((u.k + kResCols - 1) / kResCols);
    const int jobs = u.L * ntiles;
    const int grid = std::min(jobs, res_grid());
    launch_traced(leaf_res_kernel, dim3(grid), dim3(kResThreads), s, leaf_last, u, ntiles, jobs);
  } else {
    launch_traced((leaf_kernel<NQ, RT, true, F32>), dim3(u.L * u.tiles), dim3(kUThreads), s, leaf_last, u);
  }
  for (int st = st0; st < u.L; st *= K) {
    UpdateParams v = u;
    v.stride = st;
    const int per = (u.L - st + K * st - 1) / (K * st);
    const bool last = st * K >= u.L && !scale;
    if (res_levels) {
      const int ntiles = (int)((u.k + kResCols - 1) / kResCols);
      const int jobs = per * ntiles;
      launch_traced(node_res_kernel, dim3(std::min(jobs, res_grid())), dim3(kResThreads), s, last, v, ntiles, jobs);
    } else {
      launch_traced((node_level_kernel<NQ, true, K>), dim3(per * u.tiles), dim3(kUThreads), s, last, v);
    }
  }
  if (scale) launch_traced(scale_rows_kernel, dim3(u.tiles), dim3(kUThreads), s, true, u);
  return hipGetLastError();
}

template <int NQ, int RT, int K>
hipError_t launch_qn_t(const UpdateParams &u, hipStream_t s) {
  hipLaunchKernelGGL(scale_rows_kernel, dim3(u.tiles), dim3(kUThreads), 0, s, u);
  int top = 1;  // stride of the top level
  while (top * K < u.L) top *= K;
  for (int st = (u.L > 1) ? top : 0; st >= 1; st /= K) {
    UpdateParams v = u;
    v.stride = st;
    const int per = (u.L - st + K * st - 1) / (K * st);
    hipLaunchKernelGGL((node_level_kernel<NQ, false, K>), dim3(per * u.tiles), dim3(kUThreads), 0, s, v);
  }
  hipLaunchKernelGGL((leaf_kernel<NQ, RT, false>), dim3(u.L * u.tiles), dim3(kUThreads), 0, s, u);
  return hipGetLastError();
}

template <int NQ, int RT, int K>
hipError_t launch_qt_p(const UpdateParams &u, hipStream_t s) {
  return u.f32 ? launch_qt_t<NQ, RT, K, true>(u, s) : launch_qt_t<NQ, RT, K, false>(u, s);
}

template <int RT, int K>
hipError_t dispatch_nq(const UpdateParams &u, bool trans, hipStream_t s) {
  switch ((u.b + 15) / 16) {
    case 1: return trans ? launch_qt_p<1, RT, K>(u, s) : launch_qn_t<1, RT, K>(u, s);
    case 2: return trans ? launch_qt_p<2, RT, K>(u, s) : launch_qn_t<2, RT, K>(u, s);
    case 3: return trans ? launch_qt_p<3, RT, K>(u, s) : launch_qn_t<3, RT, K>(u, s);
    case 4: return trans ? launch_qt_p<4, RT, K>(u, s) : launch_qn_t<4, RT, K>(u, s);
    default: return hipErrorInvalidValue;
  }
}

template <int K>
hipError_t dispatch_k(const UpdateParams &u, bool trans, hipStream_t s) {
  switch (u.h) {
    case 64: return dispatch_nq<4, K>(u, trans, s);
    case 128: return dispatch_nq<8, K>(u, trans, s);
    case 256: return dispatch_nq<16, K>(u, trans, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t dispatch(const UpdateParams &u, bool trans, hipStream_t s) {
  if (u.b < 1 || u.b > kMaxB || u.L < 1 || u.k < 1 || u.m < 1) return hipErrorInvalidValue;
  if (u.f32 && !trans) return hipErrorInvalidValue;  // the FP32 products serve the factorization's Q^T only
  if (u.arity == 2) return dispatch_k<2>(u, trans, s);
  if (u.arity == 4) return dispatch_k<4>(u, trans, s);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_apply_qt(const UpdateParams &u, hipStream_t s) { return dispatch(u, true, s); }
hipError_t launch_apply_qn(const UpdateParams &u, hipStream_t s) { return dispatch(u, false, s); }

void set_launch_trace(hipEvent_t start, hipEvent_t stop) {
  tl_trace_start = start;
  tl_trace_stop = stop;
}

}  // namespace caqr
