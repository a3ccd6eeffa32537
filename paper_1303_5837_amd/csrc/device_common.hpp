// Device helpers shared by the gfx950 kernels of the library.
//
// Workgroup layout of a row block ("tile") used by the panel kernels: 256
// threads = 4 wave64s.  Thread t has wave w = t / 64 and lane l = t % 64;
// within the wave, the 16-lane DPP row d = l / 16 and the position r = l % 16.
// The thread owns column group c = 4 w + d and row lane r, i.e. the elements
//     (row 16 i + r, column c + 16 q)   for chunk i and column slot q.
// A column is therefore held by the 16 lanes of one DPP row, so every column
// reduction (norm, dot product) is a 4-step DPP butterfly inside that row and
// needs neither LDS nor a barrier.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace caqr {

constexpr int kThreads = 256;  // threads per panel workgroup
constexpr int kMaxB = 64;      // widest panel

typedef double f64x4 __attribute__((ext_vector_type(4)));

// DPP controls (gfx9 encoding).
constexpr int kDppQuadXor1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int kDppRowHalfMirror = 0x141;  // lane r <-> 7 - r within each 8
constexpr int kDppRowMirror = 0x140;      // lane r <-> 15 - r within each 16

// Every pattern used here reads a lane of the same row, so every lane is
// written and the move needs no "old" value.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp_f32(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, false));
}

// 1/x from the hardware estimate refined by Newton steps (within about one
// ulp; used only where x is a normal number well inside the range).
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float rcp_nr(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  const float e = fmaf(-x, r, 1.0f);
  return fmaf(r, e, r);
}

// Sum over the 16 lanes of a DPP row.  Every lane of the row ends with the
// bitwise-same value: each step adds a pair in both orders, and IEEE addition
// is commutative.
__device__ __forceinline__ double row16_sum(double x) {
  x += dpp_f64<kDppQuadXor1>(x);
  x += dpp_f64<kDppQuadXor2>(x);
  x += dpp_f64<kDppRowHalfMirror>(x);
  x += dpp_f64<kDppRowMirror>(x);
  return x;
}

__device__ __forceinline__ double row16_max(double x) {
  x = fmax(x, dpp_f64<kDppQuadXor1>(x));
  x = fmax(x, dpp_f64<kDppQuadXor2>(x));
  x = fmax(x, dpp_f64<kDppRowHalfMirror>(x));
  x = fmax(x, dpp_f64<kDppRowMirror>(x));
  return x;
}

__device__ __forceinline__ float row16_sum(float x) {
  x += dpp_f32<kDppQuadXor1>(x);
  x += dpp_f32<kDppQuadXor2>(x);
  x += dpp_f32<kDppRowHalfMirror>(x);
  x += dpp_f32<kDppRowMirror>(x);
  return x;
}

__device__ __forceinline__ float row16_max(float x) {
  x = fmaxf(x, dpp_f32<kDppQuadXor1>(x));
  x = fmaxf(x, dpp_f32<kDppQuadXor2>(x));
  x = fmaxf(x, dpp_f32<kDppRowHalfMirror>(x));
  x = fmaxf(x, dpp_f32<kDppRowMirror>(x));
  return x;
}

// Value of x in lane `lane` (wave-uniform) broadcast to the whole wave.
__device__ __forceinline__ double readlane_f64(double x, int lane) {
  int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double readlane_t(double x, int lane) { return readlane_f64(x, lane); }
__device__ __forceinline__ float readlane_t(float x, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}

// Agent-scope release/acquire around the last-arriver tickets of the device
// tree.  Every thread fences its own prior global stores before the barrier
// that precedes the ticket, and every thread fences before reading data
// published by another workgroup.
__device__ __forceinline__ void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

__device__ __forceinline__ unsigned ticket_add(unsigned *p) {
  return __hip_atomic_fetch_add(p, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void ticket_clear(unsigned *p) {
  __hip_atomic_store(p, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// FP64 MFMA 16x16x4: D(16x16) += A(16x4) B(4x16).  Operand lane layout on
// gfx950 (checked on the device): A(i, k) in lane i + 16 k, B(k, j) in lane
// j + 16 k, and D(i, j) in lane j + 16 (i % 4), register i / 4.
__device__ __forceinline__ f64x4 mfma16x16x4(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

}  // namespace caqr
