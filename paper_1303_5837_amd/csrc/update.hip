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
// (T instead of T^T for Q C.)  One workgroup updates the rows of a group of
// leaves on one 64-column tile; wave w owns columns 16w..16w+15 of the tile
// over all rows of a leaf and keeps them in registers between the two
// products, so C is read and written once per leaf and no partial sums cross
// waves.  The reflectors are staged through LDS in 64x64 blocks
// (double-buffered, loaded with coalesced 16-byte accesses), and T goes
// through the same buffers.  For Q^T the tree levels that lie inside a group
// follow in the same launch; the levels above the groups run one launch per
// level, so no workgroup ever waits for another.
//
// Register layout ("contiguous"): a 16-row slab x of a tile is an f64x4 per
// lane holding rows 16x + 4*(lane/16) + r, r = 0..3, of column lane%16.  The
// MFMA result layout holds row 4r + lane/16 in register r, so every product
// whose output uses the contiguous layout reads its A operand at the permuted
// row pi(lane%16) = 4*(lane%4) + (lane%16)/4 of the slab.
#include "device_common.hpp"
#include "kernels.hpp"
#include "staging.hpp"

namespace caqr {

namespace {

struct UpdSmem {
  alignas(16) double buf[2][kMaxB * kLdb];
  int flag;
};

__device__ __forceinline__ int pi16(int li) { return 4 * (li & 3) + (li >> 2); }

__device__ __forceinline__ bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

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

// Update of the top b rows of tree node `node` (eliminated leaf) and of its
// left sibling on this workgroup's tile.  Wave w holds all 16*NQ top rows of
// both row blocks for columns 16w..16w+15, so W = C1 + V^T C2 is complete in
// every wave.  V goes to LDS buffer 0 and T to buffer 1.
template <int NQ, bool TRANS>
__device__ __forceinline__ void node_update(const UpdateParams &u, int left, int node, int tile, UpdSmem &sm,
                                            bool vec_ok) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int pl = pi16(li);
  const int64_t col = (int64_t)tile * kUpdTile + 16 * wave + li;
  const bool colok = col < u.k;
  const int64_t r1 = (int64_t)left * u.h, r2 = (int64_t)node * u.h;
  const int64_t m1 = min<int64_t>(u.m, r1 + u.b), m2 = min<int64_t>(u.m, r2 + u.b);
  Stage st;
  stage_load<kNodeV>(st, u.Y, u.ldy, r2, r2, u.m, u.b, vec_ok, tid);
  stage_fix<kNodeV>(st, 0, tid);
  stage_store(st, sm.buf[0], tid);
  stage_load<kDense>(st, u.T_node + (int64_t)node * 64 * 64, 64, 0, 0, 0, 0, true, tid);
  stage_store(st, sm.buf[1], tid);
  f64x4 c1[NQ], c2[NQ];
#pragma unroll
  for (int t = 0; t < NQ; ++t) {
    c1[t] = load_slab(u.C, u.ldc, r1 + 16 * t + 4 * lk, col, m1, colok, vec_ok);
    c2[t] = load_slab(u.C, u.ldc, r2 + 16 * t + 4 * lk, col, m2, colok, vec_ok);
  }
  __syncthreads();
  // W = C1 + V^T C2 (V upper triangular: slab t reaches blocks a >= t)
  f64x4 w[NQ];
#pragma unroll
  for (int a = 0; a < NQ; ++a) {
    f64x4 acc = c1[a];
#pragma unroll
    for (int t = 0; t <= a; ++t) {
      const f64x4 v = lds_col4(sm.buf[0], 16 * a + pl, 16 * t + 4 * lk);
#pragma unroll
      for (int r = 0; r < 4; ++r) acc = mfma16x16x4(v[r], c2[t][r], acc);
    }
    w[a] = acc;
  }
  apply_t_lds<NQ, TRANS>(sm.buf[1], w);
  // C1 -= W';  C2 -= V W'
#pragma unroll
  for (int t = 0; t < NQ; ++t) {
    c1[t] -= w[t];
    f64x4 acc = c2[t];
#pragma unroll
    for (int a = t; a < NQ; ++a) {
      const f64x4 v = lds_row4(sm.buf[0], 16 * t + pl, 16 * a + 4 * lk);
#pragma unroll
      for (int r = 0; r < 4; ++r) acc = mfma16x16x4(-v[r], w[a][r], acc);
    }
    c2[t] = acc;
  }
#pragma unroll
  for (int t = 0; t < NQ; ++t) {
    store_slab(u.C, u.ldc, r1 + 16 * t + 4 * lk, col, m1, colok, vec_ok, c1[t]);
    store_slab(u.C, u.ldc, r2 + 16 * t + 4 * lk, col, m2, colok, vec_ok, c2[t]);
  }
  __syncthreads();  // LDS buffers free again
}

// Rows 0..b-1 of this workgroup's tile scaled by D (any thread mapping; the
// caller orders it after the tile's last update).
__device__ __forceinline__ void scale_top_rows(const UpdateParams &u, int tile) {
  for (int e = threadIdx.x; e < u.b * kUpdTile; e += kThreads) {
    const int row = e % u.b;
    const int64_t col = (int64_t)tile * kUpdTile + e / u.b;
    if (col < u.k && row < u.m) u.C[row + col * u.ldc] *= u.d[row];
  }
}

// Rows 0..b-1 scaled by D, each lane on the rows it wrote itself in
// node_update / leaf_update (rows 16t + 4(lane/16) + r of column lane%16).
template <int NQ>
__device__ __forceinline__ void scale_top_rows_own(const UpdateParams &u, int tile) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t col = (int64_t)tile * kUpdTile + 16 * wave + li;
  if (col >= u.k) return;
#pragma unroll
  for (int t = 0; t < NQ; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * t + 4 * lk + r;
      if (row < u.b && row < u.m) u.C[row + col * u.ldc] *= u.d[row];
    }
}

// Whether the whole leaf x tile block of C is in range and 16-byte aligned
// (uniform fast path for C).
__device__ __forceinline__ bool leaf_cfast(const UpdateParams &u, int leaf, int tile) {
  return aligned16(u.C) && (u.ldc % 2 == 0) && (int64_t)(leaf + 1) * u.h <= u.m &&
         (int64_t)(tile + 1) * kUpdTile <= u.k;
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

// Q^T (TRANS) or Q update of one leaf on one tile: C_leaf <- C_leaf - Y (T^T (Y^T C_leaf)).
// Wave w holds all H rows of the leaf for columns 16w..16w+15 in registers
// (RT slabs of 16 rows), so both products are complete inside the wave.  The
// reflectors go through LDS in 64-row chunks, double-buffered: chunks 0..n-1
// for W = Y^T C, then T, then chunks n-1..0 for C -= Y W' (the last chunk of
// the first pass is still in LDS and is not reloaded).  Chunk c always sits in
// buffer c % 2; T sits in buffer n % 2.  Inside a chunk the LDS operands of
// the next 16-row slab are read before the products of the current one.
// Every chunk of C is stored as soon as it is final.  `pre` carries the first
// 64 rows of this leaf's tile when the previous call prefetched them
// (has_pre); with next >= 0 this call prefetches those rows of leaf `next`
// during its second pass.
template <int NQ, int RT, bool TRANS>
__device__ __forceinline__ void leaf_update(const UpdateParams &u, int leaf, int tile, UpdSmem &sm, f64x4 (&pre)[4],
                                            bool has_pre, int next) {
  constexpr int H = 16 * RT;       // leaf rows
  constexpr int NCHUNK = H / 64;   // 64-row chunks
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int pl = pi16(li);
  const int64_t row0 = (int64_t)leaf * u.h;
  const int64_t col = (int64_t)tile * kUpdTile + 16 * wave + li;
  const bool colok = col < u.k;
  const bool vec_c = aligned16(u.C) && (u.ldc % 2 == 0);
  const bool vec_y = aligned16(u.Y) && (u.ldy % 2 == 0);

  Stage st;
  stage_load<kLeafY>(st, u.Y, u.ldy, row0, row0, u.m, u.b, vec_y, tid);
  const bool cfast = leaf_cfast(u, leaf, tile);
  double *cptr = u.C + row0 + 4 * lk + col * u.ldc;
  f64x4 acc[RT];  // rows row0 + 16x + 4lk + r
  if (cfast) {
#pragma unroll
    for (int x = 0; x < RT; ++x) {
      if (x < 4 && has_pre)
        acc[x] = pre[x];
      else
        acc[x] = ld_c4(cptr + 16 * x);
    }
  } else {
#pragma unroll
    for (int x = 0; x < RT; ++x) acc[x] = load_slab(u.C, u.ldc, row0 + 16 * x + 4 * lk, col, u.m, colok, vec_c);
  }
  stage_fix<kLeafY>(st, 0, tid);
  stage_store(st, sm.buf[0], tid);
  __syncthreads();

  // ---- W = Y^T C, chunk by chunk
  f64x4 w[NQ];
#pragma unroll
  for (int a = 0; a < NQ; ++a) w[a] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < NCHUNK; ++c) {
    if (c + 1 < NCHUNK)
      stage_load<kLeafY>(st, u.Y, u.ldy, row0 + 64 * (c + 1), row0, u.m, u.b, vec_y, tid);
    else
      stage_load<kDense>(st, u.T_leaf + (int64_t)leaf * 64 * 64, 64, 0, 0, 0, 0, true, tid);
    const double *ys = sm.buf[c & 1];
    f64x4 y[2][NQ];
#pragma unroll
    for (int a = 0; a < NQ; ++a)
      if (4 * c >= a) y[0][a] = lds_col4(ys, 16 * a + pl, 4 * lk);
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
      const int x = 4 * c + tt;  // slab index within the leaf
      if (tt + 1 < 4) {
#pragma unroll
        for (int a = 0; a < NQ; ++a)
          if (x + 1 >= a) y[(tt + 1) & 1][a] = lds_col4(ys, 16 * a + pl, 16 * (tt + 1) + 4 * lk);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int a = 0; a < NQ; ++a)
          if (x >= a) w[a] = mfma16x16x4(y[tt & 1][a][r], acc[x][r], w[a]);  // rows above block a are zero
    }
    stage_store(st, sm.buf[(c + 1) & 1], tid);
    __syncthreads();
  }
  // ---- W' = -T^T W (T in buffer NCHUNK % 2); the next chunk of the second
  // pass (NCHUNK - 2) is loaded meanwhile and goes into T's buffer afterwards
  if (NCHUNK > 1) stage_load<kLeafY>(st, u.Y, u.ldy, row0 + 64 * (NCHUNK - 2), row0, u.m, u.b, vec_y, tid);
  apply_t_lds<NQ, TRANS>(sm.buf[NCHUNK & 1], w);
#pragma unroll
  for (int a = 0; a < NQ; ++a) w[a] = -w[a];
  if (next >= 0) {  // first 64 rows of the next leaf's tile (fast path; the caller checked)
    const double *np = u.C + (int64_t)next * u.h + 4 * lk + col * u.ldc;
#pragma unroll
    for (int x = 0; x < 4; ++x) pre[x] = ld_c4(np + 16 * x);
  }
  __syncthreads();
  // ---- C += Y W', chunks NCHUNK-1 .. 0
#pragma unroll
  for (int c = NCHUNK - 1; c >= 0; --c) {
    if (c >= 1) {
      if (c == 1) stage_fix<kLeafY>(st, 0, tid);   // chunk 0 holds the diagonal
      stage_store(st, sm.buf[(c - 1) & 1], tid);  // chunk c - 1 into the buffer chunk c + 1 (or T) left
      if (c >= 2) stage_load<kLeafY>(st, u.Y, u.ldy, row0 + 64 * (c - 2), row0, u.m, u.b, vec_y, tid);
    }
    const double *ys = sm.buf[c & 1];
    f64x4 y[2][NQ];
#pragma unroll
    for (int a = 0; a < NQ; ++a)
      if (4 * c >= a) y[0][a] = lds_row4(ys, pl, 16 * a + 4 * lk);
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
      const int x = 4 * c + tt;
      if (tt + 1 < 4) {
#pragma unroll
        for (int a = 0; a < NQ; ++a)
          if (x + 1 >= a) y[(tt + 1) & 1][a] = lds_row4(ys, 16 * (tt + 1) + pl, 16 * a + 4 * lk);
      }
#pragma unroll
      for (int a = 0; a < NQ; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (x >= a) acc[x] = mfma16x16x4(y[tt & 1][a][r], w[a][r], acc[x]);
    }
    // rows of chunk c are final
    if (cfast) {
#pragma unroll
      for (int tt = 0; tt < 4; ++tt) st_c4(cptr + 16 * (4 * c + tt), acc[4 * c + tt]);
    } else {
#pragma unroll
      for (int tt = 0; tt < 4; ++tt)
        store_slab(u.C, u.ldc, row0 + 16 * (4 * c + tt) + 4 * lk, col, u.m, colok, vec_c, acc[4 * c + tt]);
    }
    if (c >= 1) __syncthreads();
  }
  __syncthreads();  // LDS free for the next update
}

// One leaf update with no prefetch on either side.
template <int NQ, int RT, bool TRANS>
__device__ __forceinline__ void leaf_update_single(const UpdateParams &u, int leaf, int tile, UpdSmem &sm) {
  f64x4 pre[4];
  leaf_update<NQ, RT, TRANS>(u, leaf, tile, sm, pre, false, -1);
}

// Q^T of one panel on one tile, for the leaves of group g (u.group leaves,
// a power of two): every leaf update, then the tree levels that are complete
// inside the group (binary pairs i, i + 2^(k-1), the lower index on top).  A
// single group covers the whole tree and also applies D.  No workgroup
// depends on another, so no device-scope synchronization is needed; the
// levels above the groups run afterwards, one launch per level.
template <int NQ, int RT>
__global__ void __launch_bounds__(kThreads, 1) qt_group_kernel(UpdateParams u) {
  __shared__ UpdSmem sm;
  const int ngroups = (u.L + u.group - 1) / u.group;
  const int g = blockIdx.x % ngroups;
  const int tile = blockIdx.x / ngroups;
  const bool vec_ok = aligned16(u.C) && (u.ldc % 2 == 0) && aligned16(u.Y) && (u.ldy % 2 == 0);
  const int first = g * u.group, last = min(u.L, first + u.group);
  f64x4 pre[4];
  bool has_pre = false;
#pragma nounroll
  for (int leaf = first; leaf < last; ++leaf) {
    const int lf = __builtin_amdgcn_readfirstlane(leaf);
    const int next = (lf + 1 < last && leaf_cfast(u, lf + 1, tile)) ? lf + 1 : -1;
    leaf_update<NQ, RT, true>(u, lf, tile, sm, pre, has_pre, next);
    has_pre = next >= 0;
  }
  for (int half = 1; half < u.group && half < u.L; half <<= 1)
#pragma nounroll
    for (int node = first + half; node < last; node += 2 * half)
      node_update<NQ, true>(u, node - half, node, tile, sm, vec_ok);
  if (ngroups == 1) scale_top_rows_own<NQ>(u, tile);
}

// Q applied (not transposed): leaves only, no tree (the tree runs first, top-down).
template <int NQ, int RT>
__global__ void __launch_bounds__(kThreads, 1) qn_leaf_kernel(UpdateParams u) {
  __shared__ UpdSmem sm;
  const int leaf = blockIdx.x % u.L;
  const int tile = blockIdx.x / u.L;
  leaf_update_single<NQ, RT, false>(u, leaf, tile, sm);
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

// Last-arriver ticket on node `node`; true when this workgroup arrived second
// (and performs the node's update).  Publishes this workgroup's stores to C
// before the ticket and acquires the partner's after it.
__device__ __forceinline__ bool arrive(unsigned *tickets, int node, int &flag) {
  fence_release();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned old = ticket_add(tickets + node);
    flag = (int)old;
    if (old == 1u) ticket_clear(tickets + node);
  }
  __syncthreads();
  const bool second = flag == 1;
  if (second) fence_acquire();
  return second;
}

// Q^T of one panel on a single tile (at most 64 columns, e.g. the next
// panel's), the whole tree in one launch: workgroup i updates leaf i, then
// climbs the binary tree; below every node the second workgroup to arrive (an
// agent-scope ticket) performs the node's update, the first one exits.  The
// pairing is fixed by index, so the result does not depend on arrival order.
// The workgroup that completes the root applies D.
template <int NQ, int RT>
__global__ void __launch_bounds__(kThreads, 1) qt_tree_tile_kernel(UpdateParams u) {
  __shared__ UpdSmem sm;
  __shared__ int flag;
  const bool vec_ok = aligned16(u.C) && (u.ldc % 2 == 0) && aligned16(u.Y) && (u.ldy % 2 == 0);
  const int leaf = blockIdx.x;
  leaf_update_single<NQ, RT, true>(u, leaf, 0, sm);
  int rt = leaf;  // root of the subtree this workgroup holds
  for (int half = 1; half < u.L; half <<= 1) {
    if ((rt & (2 * half - 1)) == 0) {  // left child at this level
      const int partner = rt + half;
      if (partner >= u.L) continue;      // no sibling: pass through
      if (!arrive(u.tickets, partner, flag)) return;
      node_update<NQ, true>(u, rt, partner, 0, sm, vec_ok);
    } else {  // right child: node id rt, left sibling rt - half
      const int left = rt - half;
      if (!arrive(u.tickets, rt, flag)) return;
      node_update<NQ, true>(u, left, rt, 0, sm, vec_ok);
      rt = left;
    }
  }
  scale_top_rows_own<NQ>(u, 0);
}

template <int NQ, int RT>
hipError_t launch_qt_t(const UpdateParams &u, hipStream_t s) {
  if (u.tickets && u.tiles == 1 && u.L > 1) {
    hipLaunchKernelGGL((qt_tree_tile_kernel<NQ, RT>), dim3(u.L), dim3(kThreads), 0, s, u);
    return hipGetLastError();
  }
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
