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
// 64-column tile, keeping the tile in registers between the two products, so C
// is read and written once.  For Q^T the tree levels follow in the same launch:
// per (node, tile) an agent-scope ticket lets the second workgroup to finish
// below a node perform that node's update on the tile.
#include "device_common.hpp"
#include "kernels.hpp"

namespace caqr {

namespace {

constexpr int kTile = 64;  // columns per workgroup; wave w owns columns 16w..16w+15

// Unit lower-trapezoidal leaf reflector Y(lr, col) of the leaf starting at row0.
__device__ __forceinline__ double y_leaf(const UpdateParams &u, int64_t row0, int lr, int col) {
  const int64_t grow = row0 + lr;
  const bool ok = (lr > col) && (col < u.b) && (grow < u.m);
  double v = ok ? u.Y[grow + (int64_t)col * u.ldy] : 0.0;
  return (lr == col && col < u.b) ? 1.0 : v;
}

// Upper-triangular node reflector block V(row, col) stored at row0 (non-unit diagonal).
__device__ __forceinline__ double v_node(const UpdateParams &u, int64_t row0, int row, int col) {
  const int64_t grow = row0 + row;
  const bool ok = (row <= col) && (col < u.b) && (grow < u.m);
  return ok ? u.Y[grow + (int64_t)col * u.ldy] : 0.0;
}

// W' = T^T W (TRANS) or T W, W in D-layout blocks of 16 reflectors.
template <int NQ, bool TRANS>
__device__ __forceinline__ void apply_t(const double *Tg, const f64x4 (&w)[NQ], f64x4 (&w2)[NQ]) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int ao = 0; ao < NQ; ++ao) {
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < NQ; ++a) {
      if (TRANS ? (a > ao) : (a < ao)) continue;  // T is upper triangular
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int kk = 16 * a + 4 * r + lk;  // reflector index of this k-step
        const int ii = 16 * ao + li;         // output reflector
        // TRANS: A(ii, kk) = T(kk, ii);  otherwise A(ii, kk) = T(ii, kk)
        const double t = TRANS ? Tg[kk + 64 * ii] : Tg[ii + 64 * kk];
        acc = mfma16x16x4(t, w[a][r], acc);
      }
    }
    w2[ao] = acc;
  }
}

// Update of the rows of tree node `node` (eliminated leaf) and its left sibling
// on this workgroup's tile.
template <int NQ, bool TRANS>
__device__ void node_update(const UpdateParams &u, int left, int node, int tile) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t col = (int64_t)tile * kTile + 16 * wave + li;
  const bool colok = col < u.k;
  const int64_t r1 = (int64_t)left * u.h, r2 = (int64_t)node * u.h;
  f64x4 c1[NQ], c2[NQ];
#pragma unroll
  for (int t = 0; t < NQ; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * t + 4 * r + lk;
      const bool ok = colok && row < u.b;
      c1[t][r] = (ok && r1 + row < u.m) ? u.C[r1 + row + col * u.ldc] : 0.0;
      c2[t][r] = (ok && r2 + row < u.m) ? u.C[r2 + row + col * u.ldc] : 0.0;
    }
  // W = C1 + V^T C2
  f64x4 w[NQ];
#pragma unroll
  for (int a = 0; a < NQ; ++a) {
    f64x4 acc = c1[a];
#pragma unroll
    for (int t = 0; t <= a; ++t)  // V upper triangular: rows of block t <= columns of block a
#pragma unroll
      for (int r = 0; r < 4; ++r) acc = mfma16x16x4(v_node(u, r2, 16 * t + 4 * r + lk, 16 * a + li), c2[t][r], acc);
    w[a] = acc;
  }
  f64x4 w2[NQ];
  apply_t<NQ, TRANS>(u.T_node + (int64_t)node * 64 * 64, w, w2);
  // C1 -= W';  C2 -= V W'
#pragma unroll
  for (int t = 0; t < NQ; ++t) {
    c1[t] -= w2[t];
    f64x4 acc = c2[t];
#pragma unroll
    for (int a = t; a < NQ; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc = mfma16x16x4(-v_node(u, r2, 16 * t + li, 16 * a + 4 * r + lk), w2[a][r], acc);
    c2[t] = acc;
  }
#pragma unroll
  for (int t = 0; t < NQ; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * t + 4 * r + lk;
      if (colok && row < u.b) {
        if (r1 + row < u.m) u.C[r1 + row + col * u.ldc] = c1[t][r];
        if (r2 + row < u.m) u.C[r2 + row + col * u.ldc] = c2[t][r];
      }
    }
}

// Rows 0..b-1 of this workgroup's tile scaled by D.
__device__ __forceinline__ void scale_top_rows(const UpdateParams &u, int tile) {
  for (int e = threadIdx.x; e < u.b * kTile; e += kThreads) {
    const int row = e % u.b;
    const int64_t col = (int64_t)tile * kTile + e / u.b;
    if (col < u.k && row < u.m) u.C[row + col * u.ldc] *= u.d[row];
  }
}

template <int NQ, int RT, bool TRANS, bool CLIMB>
__global__ void __launch_bounds__(kThreads, 2) leaf_update_kernel(UpdateParams u) {
  const int leaf = blockIdx.x % u.L;
  const int tile = blockIdx.x / u.L;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t row0 = (int64_t)leaf * u.h;
  const int64_t col = (int64_t)tile * kTile + 16 * wave + li;
  const bool colok = col < u.k;
  const double *Tg = u.T_leaf + (int64_t)leaf * 64 * 64;

  // C tile of this leaf in MFMA D-layout: acc[t][r] = C(row0 + 16t + 4r + lk, col)
  f64x4 acc[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t grow = row0 + 16 * t + 4 * r + lk;
      acc[t][r] = (colok && grow < u.m) ? u.C[grow + col * u.ldc] : 0.0;
    }
  // W = Y^T C   (k-step (t, r) covers rows 16t + 4r + 0..3)
  f64x4 w[NQ];
#pragma unroll
  for (int a = 0; a < NQ; ++a) w[a] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int lr = 16 * t + 4 * r + lk;
#pragma unroll
      for (int a = 0; a < NQ; ++a) {
        if (16 * t + 15 < 16 * a) continue;  // rows of this k-step are above block a's reflectors
        w[a] = mfma16x16x4(y_leaf(u, row0, lr, 16 * a + li), acc[t][r], w[a]);
      }
    }
  f64x4 w2[NQ];
  apply_t<NQ, TRANS>(Tg, w, w2);
  // C -= Y W'
#pragma unroll
  for (int t = 0; t < RT; ++t) {
#pragma unroll
    for (int a = 0; a < NQ; ++a) {
      if (16 * t + 15 < 16 * a) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        acc[t] = mfma16x16x4(-y_leaf(u, row0, 16 * t + li, 16 * a + 4 * r + lk), w2[a][r], acc[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t grow = row0 + 16 * t + 4 * r + lk;
      if (colok && grow < u.m) u.C[grow + col * u.ldc] = acc[t][r];
    }
  if (!CLIMB) return;

  // ---- tree levels for this tile (Q^T order: bottom-up), then D
  __shared__ int flag;
  int rt = leaf;
  for (int half = 1; half < u.L; half <<= 1) {
    int node;
    if ((rt & (2 * half - 1)) == 0) {
      node = rt + half;
      if (node >= u.L) continue;
    } else {
      node = rt;
    }
    fence_release();
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned *tk = u.tickets + (int64_t)node * u.tiles + tile;
      const unsigned old = ticket_add(tk);
      flag = (int)old;
      if (old == 1u) ticket_clear(tk);
    }
    __syncthreads();
    if (flag != 1) return;
    fence_acquire();
    node_update<NQ, TRANS>(u, node - half, node, tile);
    rt = node - half;
    __syncthreads();
  }
  __syncthreads();
  scale_top_rows(u, tile);
}

template <int NQ, bool TRANS>
__global__ void __launch_bounds__(kThreads, 2) node_level_kernel(UpdateParams u) {
  // nodes of this level: ids half, 3*half, 5*half, ... < L
  const int half = 1 << (u.level - 1);
  const int nn = blockIdx.x % ((u.L + half - 1) / (2 * half) + 1);
  const int tile = blockIdx.x / ((u.L + half - 1) / (2 * half) + 1);
  const int node = half + 2 * half * nn;
  if (node >= u.L) return;
  node_update<NQ, TRANS>(u, node - half, node, tile);
}

__global__ void scale_rows_kernel(UpdateParams u) { scale_top_rows(u, blockIdx.x); }

template <int NQ, int RT>
hipError_t launch_qt_t(const UpdateParams &u, hipStream_t s) {
  hipLaunchKernelGGL((leaf_update_kernel<NQ, RT, true, true>), dim3(u.L * u.tiles), dim3(kThreads), 0, s, u);
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
  hipLaunchKernelGGL((leaf_update_kernel<NQ, RT, false, false>), dim3(u.L * u.tiles), dim3(kThreads), 0, s, u);
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
  if (u.b < 1 || u.b > kMaxB || u.L < 1 || u.k < 1) return hipErrorInvalidValue;
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
