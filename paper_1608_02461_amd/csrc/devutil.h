// Device helpers shared by the FMM translation units (inline, header-only).
#pragma once

#include "common.h"

namespace hfmm {

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ float rcpT(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcpT(double x) { return 1.0 / x; }

// acc += a * b (complex; V is float2 or double2)
template <class V>
__device__ __forceinline__ void cmac(V& acc, V a, V b) {
  acc.x = fmaT(a.x, b.x, acc.x);
  acc.x = fmaT(-a.y, b.y, acc.x);
  acc.y = fmaT(a.x, b.y, acc.y);
  acc.y = fmaT(a.y, b.x, acc.y);
}
// acc += a * conj(b)
template <class V>
__device__ __forceinline__ void cmacc(V& acc, V a, V b) {
  acc.x = fmaT(a.x, b.x, acc.x);
  acc.x = fmaT(a.y, b.y, acc.x);
  acc.y = fmaT(a.y, b.x, acc.y);
  acc.y = fmaT(-a.x, b.y, acc.y);
}

// Bessel functions of order n at x through J_n(x) = (x/2)^n / n! S_n(x^2/4),
// S_n(y) = sum_j (-y)^j n! / (j! (n+j)!) (DLMF 10.2.2), which has no
// division by x:
//   sseries: S_n(y) from its first K + 1 terms by Horner, with the term
//            ratios -y / (j (n + j)) formed in registers (no table loads);
//   sdown:   S_{n-1} = S_n - y S_{n+1} / (n (n + 1)), the three-term
//            recurrence J_{n-1} + J_{n+1} = (2n/x) J_n in this scaling, run
//            downward (the stable direction) from two series values.
template <class T>
__device__ __forceinline__ T sseries(int n, int K, T y) {
  T S = T(1);
  for (int j = K; j >= 1; --j) S = fmaT(-y * rcpT(T(j) * T(n + j)), S, T(1));
  return S;
}
template <class T>
__device__ __forceinline__ T sdown(int n, T y, T Sn, T Sn1) {
  return fmaT(-y * rcpT(T(n) * T(n + 1)), Sn1, Sn);
}

// The LDS stores and loads of one wave are performed in order; this keeps
// the compiler from moving them across the point, so lanes of the wave see
// each other's stores (waves that share no LDS need no block barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The far-field chain runs beside the near field, whose waves keep every
// SIMD busy.  Its kernels raise their waves' issue priority so that the
// chain, which is short of parallelism, advances at close to its own speed
// while the near field takes the issue slots it leaves.
__device__ __forceinline__ void chain_priority() { __builtin_amdgcn_s_setprio(3); }

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2);
// this maps hardware block b to a logical block so that every XCD walks one
// contiguous range of the Morton order, and neighbouring blocks, which read
// the same data, share an L2.  Identity when the grid is not a multiple of 8.
__device__ __forceinline__ int xcd_swizzle(int b, int n) {
  if (n & 7) return b;
  return (b & 7) * (n >> 3) + (b >> 3);
}

}  // namespace hfmm
