// Leaf far field of the FMM (Sec. 5.1.2): the last levels of the downward
// pass (L2L) and the L2P at every point, plus the final sum of the near and
// far fields.  Included once, by fmm.hip, inside its anonymous namespace.
#pragma once

#include "devutil.h"
#include "p2p.h"

// L2P at one target, d = position relative to its leaf centre: the local
// expansion sum_m L_m J_m(k rho) e^{i m theta} of the leaf (Sec. 5.1.2), for
// every column.  With w = (k/2)(dx + i dy) (in the level's scaling) and
// J_m e^{i m theta} = w^m / m! S_m, the positive orders are a Horner sum in
// w and the negative ones, J_{-m} e^{-i m theta} = (-1)^m conj(w)^m / m! S_m,
// one in conj(w); S_m runs downward alongside (sseries, sdown).
template <class T, int NR>
__device__ __forceinline__ void far_field(const P2PArgs<T>& a, const cplx<T>* Lleaf, cplx<T> d, cplx<T> (&F)[NR]) {
  const int pL = a.pL, P = 2 * pL + 1;
  const cplx<T>* Lf = Lleaf + pL;  // Lf[r P + m], m in [-pL, pL]
  const T wr = a.wscale * d.x, wi = a.wscale * d.y;
  const T y = a.yscale * (d.x * d.x + d.y * d.y);
  T s1 = sseries(pL + 1, a.K, y), s0 = sseries(pL, a.K, y);
  cplx<T> A[NR], B[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) A[r] = B[r] = mk<T>(0, 0);
  cplx<T> lp[NR], lm[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    lp[r] = Lf[r * P + pL];
    lm[r] = Lf[r * P - pL];
  }
  for (int n = pL; n >= 0; --n) {
    // s0 = S_n, s1 = S_{n+1}; lp, lm = L_n, L_{-n}; the next pair loads ahead
    cplx<T> lpn[NR], lmn[NR];
    const int n1 = n > 0 ? n - 1 : 0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      lpn[r] = Lf[r * P + n1];
      lmn[r] = Lf[r * P - n1];
    }
    const T inv = rcpT(T(n + 1));
    const T sgs = (n & 1) ? -s0 : s0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      // A <- S_n L_n + (w / (n+1)) A;  B <- (-1)^n S_n L_{-n} + (conj(w) / (n+1)) B  (n >= 1)
      const T ar = (A[r].x * wr - A[r].y * wi) * inv, ai = (A[r].x * wi + A[r].y * wr) * inv;
      A[r] = mk<T>(fmaT(s0, lp[r].x, ar), fmaT(s0, lp[r].y, ai));
      if (n > 0) {
        const T br = (B[r].x * wr + B[r].y * wi) * inv, bi = (B[r].y * wr - B[r].x * wi) * inv;
        B[r] = mk<T>(fmaT(sgs, lm[r].x, br), fmaT(sgs, lm[r].y, bi));
      }
      lp[r] = lpn[r];
      lm[r] = lmn[r];
    }
    if (n > 0) {
      const T sm = sdown(n, y, s0, s1);
      s1 = s0;
      s0 = sm;
    }
  }
  // F = A_0 + conj(w) B_1
#pragma unroll
  for (int r = 0; r < NR; ++r)
    F[r] = mk<T>(A[r].x + wr * B[r].x + wi * B[r].y, A[r].y + wr * B[r].y - wi * B[r].x);
}

// The last d = L - r levels of the downward pass below one box b of level r
// and the L2P at every point of its 4^d leaves, one block of 256 threads per
// box: L (level r+1) = its M2L part + L2L from L_b; L (level r+2, d = 2) the
// same from level r+1; then far[i] = (i/4) sum_m L_m J_m(k rho) e^{i m theta}
// for every point i of the leaves, stored at a.operm[i] when set (the
// caller's order), else at i.  The intermediate levels stay in LDS.
template <class T>
struct DownTreeArgs {
  P2PArgs<T> a;          // points, columns, far-field scales (far_field)
  const cplx<T>* Lr;     // level r: final local expansions
  const cplx<T>* L1;     // level r+1: M2L parts (d >= 1)
  const cplx<T>* L2;     // level r+2: M2L parts (d = 2)
  const cplx<T>* W1;     // L2L table level r -> r+1: [c][P0][P1]
  const cplx<T>* W2;     // L2L table level r+1 -> r+2: [c][P1][P2]
  cplx<T>* far;          // N x nrhs, written through a.operm when set
  int d, P0, P1, P2;
};

template <class T, int NR>
__global__ __launch_bounds__(256) void k_down_tree(DownTreeArgs<T> g) {
  extern __shared__ unsigned char smem_raw[];
  chain_priority();
  const P2PArgs<T>& a = g.a;
  if (a.alive && !a.alive[0]) return;
  const int b = blockIdx.x, tid = threadIdx.x;
  const int P0 = g.P0, P1 = g.P1, P2 = g.P2, nrhs = a.nrhs, r0 = a.r0;
  cplx<T>* s1 = reinterpret_cast<cplx<T>*>(smem_raw);  // [4][NR][P1]
  cplx<T>* s2 = s1 + 4 * NR * P1;                        // [16][NR][P2]
  if (g.d >= 1) {
    for (int it = tid; it < 4 * NR * P1; it += 256) {
      const int c = it / (NR * P1), rem = it - c * NR * P1, r = rem / P1, lo = rem - r * P1;
      cplx<T> acc = g.L1[((size_t)(4 * b + c) * nrhs + r0 + r) * P1 + lo];
      const cplx<T>* src = g.Lr + ((size_t)b * nrhs + r0 + r) * P0;
      const cplx<T>* W = g.W1 + (size_t)c * P0 * P1 + lo;
      for (int m = 0; m < P0; ++m) cmac(acc, W[(size_t)m * P1], src[m]);
      s1[it] = acc;
    }
    __syncthreads();
  }
  if (g.d == 2) {
    for (int it = tid; it < 16 * NR * P2; it += 256) {
      const int c2 = it / (NR * P2), rem = it - c2 * NR * P2, r = rem / P2, lo = rem - r * P2;
      cplx<T> acc = g.L2[((size_t)(16 * b + c2) * nrhs + r0 + r) * P2 + lo];
      const cplx<T>* src = s1 + ((c2 >> 2) * NR + r) * P1;
      const cplx<T>* W = g.W2 + (size_t)(c2 & 3) * P1 * P2 + lo;
      for (int m = 0; m < P1; ++m) cmac(acc, W[(size_t)m * P2], src[m]);
      s2[it] = acc;
    }
    __syncthreads();
  }
  // L2P: 256 / 4^d threads per leaf
  const int nleaf = 1 << (2 * g.d), tpl = 256 >> (2 * g.d);
  const int lf = tid / tpl, sub = tid - lf * tpl;
  const int leaf = nleaf * b + lf;
  const int PL = g.d == 2 ? P2 : (g.d == 1 ? P1 : P0);
  const cplx<T>* Lleaf = g.d == 2 ? s2 + (size_t)lf * NR * PL
                                  : (g.d == 1 ? s1 + (size_t)lf * NR * PL : g.Lr + ((size_t)b * nrhs + r0) * PL);
  const int t0 = a.leaf_off[leaf], t1 = a.leaf_off[leaf + 1];
  for (int i = t0 + sub; i < t1; i += tpl) {
    cplx<T> F[NR];
    far_field<T, NR>(a, Lleaf, a.rel[i], F);
    const int64_t o = a.operm ? a.operm[i] : i;
#pragma unroll
    for (int r = 0; r < NR; ++r) g.far[(size_t)(r0 + r) * a.N + o] = mk<T>(T(-0.25) * F[r].y, T(0.25) * F[r].x);
  }
}

// phi += far over columns [r0, r0 + NR): both in the same point order.
template <class T, int NR>
__global__ __launch_bounds__(256) void k_combine(cplx<T>* __restrict__ phi, const cplx<T>* __restrict__ far,
                                                 int64_t N, int r0, const int* alive) {
  if (alive && !alive[0]) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const size_t j = (size_t)(r0 + r) * N + i;
    const cplx<T> f = far[j], v = phi[j];
    phi[j] = mk<T>(v.x + f.x, v.y + f.y);
  }
}
