// Triangular factors T of the compact WY form (Q = I - Y T Y^T) of every leaf
// and tree node of a factored panel (paper, Section 3.1: the updates of
// Algorithm 1 apply each leaf's and each node's reflectors as one block).
//
// One workgroup per leaf or node, all in one launch.  G = Y^T Y is computed
// on FP64 MFMA from 64-row chunks of the reflectors staged through LDS
// (coalesced loads of every chunk issued at once, then two LDS buffers in
// turn); its 16x16 blocks on and above the
// diagonal are divided among the four waves, so each block is complete in one
// wave.  T then follows from G and tau by the blocked recurrence.
#include "device_common.hpp"
#include "kernels.hpp"
#include "staging.hpp"
#include "tfactor.hpp"

namespace caqr {

namespace {

struct TSmem {
  alignas(16) double buf[2][kMaxB * kLdb];  // reflector chunks; then G (buf 0) and T (buf 1)
  double taus[kMaxB];
};

// Block pair number p (0 .. NQ(NQ+1)/2 - 1) -> (a, c), a <= c, row by row.
template <int NQ>
__device__ constexpr void block_pair(int p, int &a, int &c) {
  a = 0;
  int rem = p;
  while (rem >= NQ - a) {
    rem -= NQ - a;
    ++a;
  }
  c = a + rem;
}

// blockIdx.x < L: leaf blockIdx.x (unit lower-trapezoidal Y of h rows);
// otherwise tree node id blockIdx.x - L = g + s (survivor g, stride s = K^j
// the largest power of the arity dividing the id, whose quotient digit is
// then 1; other ids are not nodes), whose reflectors are [I; V_1; ...;
// V_{cnt-1}] with every V_t upper triangular over member g + t s (the
// identity adds nothing off the diagonal of G = sum_t V_t^T V_t).
template <int NQ>
__global__ void __launch_bounds__(kThreads) form_t_kernel(FormTParams f) {
  constexpr int NP = NQ * (NQ + 1) / 2;  // block pairs
  constexpr int PW = (NP + 3) / 4;       // pairs per wave (at most)
  __shared__ TSmem sm;
  const bool is_leaf = (int)blockIdx.x < f.L;
  const int idx = is_leaf ? (int)blockIdx.x : (int)blockIdx.x - f.L;
  if (!is_leaf && idx == 0) return;
  const int K = f.arity;
  int s = 1;  // node: stride of its level, and its survivor g
  if (!is_leaf) {
    while (idx % (K * s) == 0) s *= K;
    if ((idx / s) % K != 1) return;  // not a node id
  }
  const int g0 = idx - s;  // a node's survivor
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t row0 = (int64_t)idx * f.h;
  // leaf: 64-row chunks of Y; node: one chunk per eliminated member (its V_t)
  const int nch = is_leaf ? (f.h + 63) / 64 : min(K, (f.L - g0 + s - 1) / s) - 1;
  const bool vec_ok = (((uintptr_t)f.Y & 15) == 0) && (f.ldy % 2 == 0);
  if (tid < kMaxB) {
    const double *tau = is_leaf ? f.tau_leaf : f.tau_node;
    sm.taus[tid] = (tid < f.b) ? tau[(int64_t)idx * kMaxB + tid] : 0.0;
  }
  // every chunk's loads issued at once (one round trip instead of one per
  // chunk); a leaf has at most four 64-row chunks
  Stage st[4];
  if (is_leaf) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c < nch) stage_load<kLeafY>(st[c], f.Y, f.ldy, row0 + 64 * c, row0, f.m, f.b, vec_ok, tid);
    stage_fix<kLeafY>(st[0], 0, tid);
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c < nch) {
        const int64_t r = (int64_t)(g0 + (c + 1) * s) * f.h;
        stage_load<kNodeV>(st[c], f.Y, f.ldy, r, r, f.m, f.b, vec_ok, tid);
      }
    stage_fix<kNodeV>(st[0], 0, tid);
  }
  stage_store(st[0], sm.buf[0], tid);
  __syncthreads();
  // The wave's block pairs (a, c), fixed for the whole loop; a wave with fewer
  // than PW pairs repeats its last one (result unused).  Every product is
  // issued unconditionally -- slabs of zeros (a leaf's top chunk is unit lower
  // trapezoidal, every V_t upper triangular) add exact zeros -- so that the
  // PW independent accumulations interleave instead of running as one
  // dependent MFMA chain after another.
  int pa[PW], pc[PW];
#pragma unroll
  for (int q = 0; q < PW; ++q) block_pair<NQ>(min(wave + 4 * q, NP - 1), pa[q], pc[q]);
  f64x4 g[PW];
#pragma unroll
  for (int q = 0; q < PW; ++q) g[q] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (c >= nch) break;
    const double *ys = sm.buf[c & 1];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
      f64x4 ya[PW], yc[PW];
#pragma unroll
      for (int q = 0; q < PW; ++q) {
        ya[q] = lds_col4(ys, 16 * pa[q] + li, 16 * tt + 4 * lk);
        yc[q] = lds_col4(ys, 16 * pc[q] + li, 16 * tt + 4 * lk);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < PW; ++q) g[q] = mfma16x16x4(ya[q][r], yc[q][r], g[q]);
    }
    if (c + 1 < 4 && c + 1 < nch) {
      if (!is_leaf) stage_fix<kNodeV>(st[c + 1 < 4 ? c + 1 : 3], 0, tid);  // each V_t is a triangle
      stage_store(st[c + 1 < 4 ? c + 1 : 3], sm.buf[(c + 1) & 1], tid);
    }
    __syncthreads();
  }
  // strictly upper G into buffer 0: register r of lane (li, lk) of pair (a, c)
  // holds G(16a + 4r + lk, 16c + li)
  double *G = sm.buf[0];
  double *T = sm.buf[1];
#pragma unroll
  for (int q = 0; q < PW; ++q) {
    const int p = wave + 4 * q;
    if (p >= NP) continue;
    int a, cc;
    block_pair<NQ>(p, a, cc);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * a + 4 * r + lk, k = 16 * cc + li;
      if (i < k) G[i * kLdb + k] = g[q][r];
    }
  }
  __syncthreads();
  form_t_lds<NQ>(f.b, G, T, sm.taus, kLdb);
  store_t_global(is_leaf ? f.T_leaf + (int64_t)idx * kMaxB * kMaxB : f.T_node + (int64_t)idx * kMaxB * kMaxB, f.b, T,
                 kLdb);
}

template <int NQ>
hipError_t launch_form_t_nq(const FormTParams &f, hipStream_t s) {
  hipLaunchKernelGGL((form_t_kernel<NQ>), dim3(2 * f.L), dim3(kThreads), 0, s, f);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_form_t(const FormTParams &f, hipStream_t s) {
  if (f.b < 1 || f.b > kMaxB || f.L < 1 || f.h < 1) return hipErrorInvalidValue;
  if (f.arity != 2 && f.arity != 4) return hipErrorInvalidValue;
  switch ((f.b + 15) / 16) {
    case 1: return launch_form_t_nq<1>(f, s);
    case 2: return launch_form_t_nq<2>(f, s);
    case 3: return launch_form_t_nq<3>(f, s);
    case 4: return launch_form_t_nq<4>(f, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace caqr
