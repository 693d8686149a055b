// FMM kernels and driver for the 2-D Helmholtz kernel (i/4) H0(k r).
//
// Work decomposition (one 64-lane wavefront per block throughout):
//   P2M   one wave per leaf; lanes build the per-point basis into LDS, then
//         lanes own coefficients and reduce over the leaf's points.
//   M2M   one wave per parent box; lanes own output coefficients.
//   down  one wave per box at level l: L2L from the parent plus M2L over the
//         interaction list (children of the parent's neighbours that are not
//         neighbours), lanes own output coefficients.
//   L2P   one wave per leaf; the leaf's local expansion sits in LDS, lanes own
//         target points.
//   P2P   one wave per target leaf; the 3 x 3 neighbour leaves are staged in
//         LDS (positions relative to the target leaf centre, scaled by k),
//         G lanes share a target and split its sources, shuffles reduce.
// No floating-point atomics: every output has one owner, so results are
// deterministic run to run.
#include <algorithm>
#include <cmath>
#include <complex>
#include <type_traits>

#include "fmm.h"

namespace hfmm {

namespace {

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float log2T(float x) { return __log2f(x); }
__device__ __forceinline__ double log2T(double x) { return log2(x); }

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

template <class T> const cplx<T>* rel_of(const Tree& t);
template <> const float2* rel_of<float>(const Tree& t) { return t.rel32.p; }
template <> const double2* rel_of<double>(const Tree& t) { return t.rel64.p; }

// Series S_n(y) = sum_j (-y)^j n! / (j! (n+j)!) by Horner, so that
// J_n(x) = (x/2)^n / n! * S_n(x^2/4).
template <class T>
__device__ __forceinline__ T jseries(const T* __restrict__ sr, int K, T y) {
  T S = T(1);
  for (int j = K; j >= 1; --j) S = fmaT(-y * sr[j], S, T(1));
  return S;
}

// ------------------------------------------------------------------ P2M
template <class T, int NR>
__global__ __launch_bounds__(64) void k_p2m(const int32_t* __restrict__ leaf_off, const cplx<T>* __restrict__ rel,
                                            const cplx<T>* __restrict__ q, int64_t N, int nrhs, int r0,
                                            cplx<T>* __restrict__ Mout, int pL, T wscale, T yscale,
                                            const T* __restrict__ series, int K, const uint8_t* __restrict__ flags,
                                            const int* __restrict__ alive) {
  extern __shared__ unsigned char smem_raw[];
  const int leaf = blockIdx.x;
  if (alive && !alive[0]) return;
  if (flags && !flags[leaf]) return;
  cplx<T>* sb = reinterpret_cast<cplx<T>*>(smem_raw);  // [(pL+1)][64]
  cplx<T>* sq = sb + (pL + 1) * 64;                     // [NR][64]
  const int lane = threadIdx.x;
  const int P = 2 * pL + 1;
  const int t0 = leaf_off[leaf], t1 = leaf_off[leaf + 1];
  cplx<T> accP[NR], accN[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) accP[r] = accN[r] = mk<T>(0, 0);
  for (int c0 = t0; c0 < t1; c0 += 64) {
    const int cnt = min(64, t1 - c0);
    if (lane < cnt) {
      const cplx<T> d = rel[c0 + lane];
      const T wr = wscale * d.x, wi = -wscale * d.y;  // w = (k / 2s) (dx - i dy)
      const T y = yscale * (d.x * d.x + d.y * d.y);   // (k rho)^2 / 4
      T ur = T(1), ui = T(0);
      for (int n = 0; n <= pL; ++n) {
        const T* sr = series + n * (K + 1);
        const T S = jseries(sr, K, y);
        sb[n * 64 + lane] = mk<T>(ur * S, ui * S);
        const T inv = sr[0];
        const T nr = (ur * wr - ui * wi) * inv, ni = (ur * wi + ui * wr) * inv;
        ur = nr;
        ui = ni;
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) sq[r * 64 + lane] = q[(size_t)(r0 + r) * N + c0 + lane];
    }
    __syncthreads();
    if (lane <= pL) {
      for (int j = 0; j < cnt; ++j) {
        const cplx<T> b = sb[lane * 64 + j];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const cplx<T> qq = sq[r * 64 + j];
          cmac(accP[r], qq, b);
          cmacc(accN[r], qq, b);
        }
      }
    }
    __syncthreads();
  }
  if (lane <= pL) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const size_t base = ((size_t)leaf * nrhs + r0 + r) * P;
      Mout[base + pL + lane] = accP[r];
      if (lane > 0) {
        const T sg = (lane & 1) ? T(-1) : T(1);
        Mout[base + pL - lane] = mk<T>(sg * accN[r].x, sg * accN[r].y);
      }
    }
  }
}

// ------------------------------------------------------------------ M2M
template <class T, int NR>
__global__ __launch_bounds__(64) void k_m2m(const cplx<T>* __restrict__ Mc, cplx<T>* __restrict__ Mp,
                                            const cplx<T>* __restrict__ W, int Pc, int Pp, int nrhs, int r0,
                                            const uint8_t* __restrict__ fc, const uint8_t* __restrict__ fp,
                                            const int* __restrict__ alive) {
  const int b = blockIdx.x;
  if (alive && !alive[0]) return;
  if (fp && !fp[b]) return;
  for (int lo = threadIdx.x; lo < Pp; lo += 64) {
    cplx<T> acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = mk<T>(0, 0);
    for (int c = 0; c < 4; ++c) {
      const int child = 4 * b + c;
      if (fc && !fc[child]) continue;
      const cplx<T>* Wc = W + (size_t)c * Pc * Pp;
      const cplx<T>* src = Mc + ((size_t)child * nrhs + r0) * Pc;
      for (int n = 0; n < Pc; ++n) {
        const cplx<T> w = Wc[(size_t)n * Pp + lo];
#pragma unroll
        for (int r = 0; r < NR; ++r) cmac(acc[r], w, src[(size_t)r * Pc + n]);
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) Mp[((size_t)b * nrhs + r0 + r) * Pp + lo] = acc[r];
  }
}

// ------------------------------------------------------------------ L2L + M2L
template <class T, int NR>
__global__ __launch_bounds__(64) void k_down(const cplx<T>* __restrict__ M, cplx<T>* __restrict__ Lc,
                                             const cplx<T>* __restrict__ Lp, const cplx<T>* __restrict__ Tm,
                                             const cplx<T>* __restrict__ W2, int P, int Pp, int l, int nrhs,
                                             int r0, const uint8_t* __restrict__ fsrc,
                                             const int* __restrict__ alive) {
  const int b = blockIdx.x;
  if (alive && !alive[0]) return;
  int bx, by;
  demorton((uint32_t)b, bx, by);
  const int np = 1 << (l - 1);
  const int cpos = b & 3;
  const int pbx = bx >> 1, pby = by >> 1;
  for (int lo = threadIdx.x; lo < P; lo += 64) {
    cplx<T> acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = mk<T>(0, 0);
    if (Lp) {
      const cplx<T>* Wc = W2 + (size_t)cpos * Pp * P;
      const cplx<T>* src = Lp + ((size_t)(b >> 2) * nrhs + r0) * Pp;
      for (int m = 0; m < Pp; ++m) {
        const cplx<T> w = Wc[(size_t)m * P + lo];
#pragma unroll
        for (int r = 0; r < NR; ++r) cmac(acc[r], w, src[(size_t)r * Pp + m]);
      }
    }
    for (int px = pbx - 1; px <= pbx + 1; ++px) {
      if (px < 0 || px >= np) continue;
      for (int py = pby - 1; py <= pby + 1; ++py) {
        if (py < 0 || py >= np) continue;
        for (int c = 0; c < 4; ++c) {
          const int sx = 2 * px + (c & 1), sy = 2 * py + (c >> 1);
          const int ox = sx - bx, oy = sy - by;
          if (ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1) continue;
          const uint32_t s = morton((uint32_t)sx, (uint32_t)sy);
          if (fsrc && !fsrc[s]) continue;
          const cplx<T>* To = Tm + (size_t)((ox + 3) * 7 + (oy + 3)) * P * P;
          const cplx<T>* src = M + ((size_t)s * nrhs + r0) * P;
          for (int n = 0; n < P; ++n) {
            const cplx<T> tv = To[(size_t)n * P + lo];
#pragma unroll
            for (int r = 0; r < NR; ++r) cmac(acc[r], tv, src[(size_t)r * P + n]);
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) Lc[((size_t)b * nrhs + r0 + r) * P + lo] = acc[r];
  }
}

// ------------------------------------------------------------------ L2P
template <class T, int NR>
__global__ __launch_bounds__(64) void k_l2p(const int32_t* __restrict__ leaf_off, const cplx<T>* __restrict__ rel,
                                            const cplx<T>* __restrict__ Lc, cplx<T>* __restrict__ phi, int64_t N,
                                            int nrhs, int r0, int pL, T wscale, T yscale,
                                            const T* __restrict__ series, int K, int accumulate,
                                            const int* __restrict__ alive) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* sL = reinterpret_cast<cplx<T>*>(smem_raw);  // [NR][P]
  const int leaf = blockIdx.x;
  if (alive && !alive[0]) return;
  const int t0 = leaf_off[leaf], t1 = leaf_off[leaf + 1];
  if (t0 == t1) return;
  const int P = 2 * pL + 1;
  for (int i = threadIdx.x; i < NR * P; i += 64) {
    const int r = i / P, n = i - r * P;
    sL[i] = Lc[((size_t)leaf * nrhs + r0 + r) * P + n];
  }
  __syncthreads();
  for (int i = t0 + (int)threadIdx.x; i < t1; i += 64) {
    const cplx<T> d = rel[i];
    const T wr = wscale * d.x, wi = wscale * d.y;  // (k / 2s)(dx + i dy)
    const T y = yscale * (d.x * d.x + d.y * d.y);
    cplx<T> acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = mk<T>(0, 0);
    T ur = T(1), ui = T(0);
    for (int n = 0; n <= pL; ++n) {
      const T* sr = series + n * (K + 1);
      const T S = jseries(sr, K, y);
      const cplx<T> c = mk<T>(ur * S, ui * S);
      const T sg = (n & 1) ? T(-1) : T(1);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        cmac(acc[r], sL[r * P + pL + n], c);
        if (n > 0) {
          const cplx<T> lm = sL[r * P + pL - n];
          cmacc(acc[r], mk<T>(sg * lm.x, sg * lm.y), c);
        }
      }
      const T inv = sr[0];
      const T nr = (ur * wr - ui * wi) * inv, ni = (ur * wi + ui * wr) * inv;
      ur = nr;
      ui = ni;
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const size_t idx = (size_t)(r0 + r) * N + i;
      cplx<T> v = mk<T>(T(-0.25) * acc[r].y, T(0.25) * acc[r].x);
      if (accumulate) {
        const cplx<T> o = phi[idx];
        v.x += o.x;
        v.y += o.y;
      }
      phi[idx] = v;
    }
  }
}

// ------------------------------------------------------------------ P2P
template <class T>
struct P2PArgs {
  const int32_t* leaf_off;
  const cplx<T>* rel;
  const cplx<T>* q;
  cplx<T>* phi;
  const uint8_t* flags;  // leaf-level source flags or NULL
  const int* alive;      // device flag: 0 skips the launch's work, or NULL
  int64_t N;
  int nrhs, r0, L, G, accumulate;
  T k, kls;  // k and k * leaf side
  T cJ[32], cY[32];
  T ua, ub, c1, c0;
};

template <class T, int NR>
struct P2PCfg {
  static constexpr int SCH = (2 * sizeof(T) * (1 + NR) * 512 <= 16384) ? 512 : 256;
};

// One pair: t = (k r)^2.  FAST uses the fitted polynomial (D coefficients),
// otherwise the full-range FP64 routine.
template <class T, int D, bool FAST, bool MASK>
__device__ __forceinline__ void h0_pair(const P2PArgs<T>& a, T t, T& J, T& Y) {
  bool valid = true;
  if (MASK) {
    valid = t > T(0);
    t = valid ? t : T(1);
  }
  if constexpr (FAST) {
    const T u = fmaT(t, a.ua, a.ub);
    T j = a.cJ[D - 1], yh = a.cY[D - 1];
#pragma unroll
    for (int i = D - 2; i >= 0; --i) {
      j = fmaT(j, u, a.cJ[i]);
      yh = fmaT(yh, u, a.cY[i]);
    }
    const T lg = log2T(t);
    Y = fmaT(j, fmaT(lg, a.c1, a.c0), yh);
    J = j;
  } else {
    const double2 h = h0_general(sqrt((double)t));
    J = (T)h.x;
    Y = (T)h.y;
  }
  if (MASK) {
    J = valid ? J : T(0);
    Y = valid ? Y : T(0);
  }
}

template <class T, int NR, int D, bool FAST>
__global__ __launch_bounds__(64) void k_p2p(P2PArgs<T> a) {
  constexpr int SCH = P2PCfg<T, NR>::SCH;
  __shared__ cplx<T> spos[SCH];
  __shared__ cplx<T> sq[NR][SCH];
  __shared__ int s_lo[9], s_pre[10], s_n, s_total, s_nonown;
  __shared__ T s_ox[9], s_oy[9];
  const int leaf = blockIdx.x;
  if (a.alive && !a.alive[0]) return;
  const int t0 = a.leaf_off[leaf], t1 = a.leaf_off[leaf + 1];
  if (t0 == t1) return;
  const int lane = threadIdx.x;
  if (lane == 0) {
    int bx, by;
    demorton((uint32_t)leaf, bx, by);
    const int nb = 1 << a.L;
    int n = 0, pos = 0;
    for (int pass = 0; pass < 2; ++pass) {  // neighbours first, own leaf last
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy) {
          const bool own = (dx == 0 && dy == 0);
          if (own != (pass == 1)) continue;
          const int sx = bx + dx, sy = by + dy;
          if (sx < 0 || sy < 0 || sx >= nb || sy >= nb) continue;
          const uint32_t sl = morton((uint32_t)sx, (uint32_t)sy);
          if (a.flags && !a.flags[sl]) continue;
          const int lo = a.leaf_off[sl], hi = a.leaf_off[sl + 1];
          if (lo == hi) continue;
          s_lo[n] = lo;
          s_pre[n] = pos;
          s_ox[n] = T(dx) * a.kls;
          s_oy[n] = T(dy) * a.kls;
          pos += hi - lo;
          ++n;
        }
      if (pass == 0) s_nonown = pos;
    }
    s_pre[n] = pos;
    s_n = n;
    s_total = pos;
  }
  __syncthreads();
  const int total = s_total, nonown = s_nonown, nseg = s_n;
  if (total == 0 && a.accumulate) return;
  const int G = a.G, TPR = 64 / G;
  const int g = lane & (G - 1), tl = lane / G;
  for (int rb = t0; rb < t1; rb += TPR) {
    const int ti = rb + tl;
    const bool act = ti < t1;
    T xt = 0, yt = 0;
    if (act) {
      const cplx<T> d = a.rel[ti];
      xt = a.k * d.x;
      yt = a.k * d.y;
    }
    T A[NR], B[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) A[r] = B[r] = T(0);
    for (int c0 = 0; c0 < total; c0 += SCH) {
      const int cnt = min(SCH, total - c0);
      __syncthreads();
      for (int idx = lane; idx < cnt; idx += 64) {
        const int gi = c0 + idx;
        int sg = 0;
        while (sg + 1 < nseg && gi >= s_pre[sg + 1]) ++sg;
        const int slot = s_lo[sg] + gi - s_pre[sg];
        const cplx<T> d = a.rel[slot];
        spos[idx] = mk<T>(fmaT(a.k, d.x, s_ox[sg]), fmaT(a.k, d.y, s_oy[sg]));
#pragma unroll
        for (int r = 0; r < NR; ++r) sq[r][idx] = a.q[(size_t)(a.r0 + r) * a.N + slot];
      }
      __syncthreads();
      const int split = min(max(nonown - c0, 0), cnt);
#pragma unroll 2
      for (int j = g; j < split; j += G) {
        const cplx<T> s = spos[j];
        const T dx = xt - s.x, dy = yt - s.y;
        const T t = fmaT(dx, dx, dy * dy);
        T J, Y;
        h0_pair<T, D, FAST, false>(a, t, J, Y);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const cplx<T> qq = sq[r][j];
          A[r] = fmaT(qq.x, J, A[r]);
          A[r] = fmaT(-qq.y, Y, A[r]);
          B[r] = fmaT(qq.x, Y, B[r]);
          B[r] = fmaT(qq.y, J, B[r]);
        }
      }
      for (int j = split + g; j < cnt; j += G) {
        const cplx<T> s = spos[j];
        const T dx = xt - s.x, dy = yt - s.y;
        const T t = fmaT(dx, dx, dy * dy);
        T J, Y;
        h0_pair<T, D, FAST, true>(a, t, J, Y);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const cplx<T> qq = sq[r][j];
          A[r] = fmaT(qq.x, J, A[r]);
          A[r] = fmaT(-qq.y, Y, A[r]);
          B[r] = fmaT(qq.x, Y, B[r]);
          B[r] = fmaT(qq.y, J, B[r]);
        }
      }
    }
    for (int off = 1; off < G; off <<= 1) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        A[r] += __shfl_xor(A[r], off);
        B[r] += __shfl_xor(B[r], off);
      }
    }
    if (g == 0 && act) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const size_t idx = (size_t)(a.r0 + r) * a.N + ti;
        // q (i/4) H0 summed: (i/4)(A + iB) = (-B/4, A/4)
        cplx<T> v = mk<T>(T(-0.25) * B[r], T(0.25) * A[r]);
        if (a.accumulate) {
          const cplx<T> o = a.phi[idx];
          v.x += o.x;
          v.y += o.y;
        }
        a.phi[idx] = v;
      }
    }
  }
}

// ------------------------------------------------------------------ misc
template <class T>
__global__ void k_gather(const cplx<T>* __restrict__ q, cplx<T>* __restrict__ qs, const int32_t* __restrict__ perm,
                         int64_t N, int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int64_t r = i / N, j = i - r * N;
  qs[i] = q[r * N + perm[j]];
}

template <class T>
__global__ void k_scatter(const cplx<T>* __restrict__ phis, cplx<T>* __restrict__ phi,
                          const int32_t* __restrict__ perm, int64_t N, int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int64_t r = i / N, j = i - r * N;
  phi[r * N + perm[j]] = phis[i];
}

__global__ void k_leaf_flags(const int32_t* __restrict__ leaf_off, const int32_t* __restrict__ perm,
                             int64_t nleaves, int64_t lo, int64_t hi, uint8_t* __restrict__ f) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nleaves) return;
  uint8_t s = 0;
  for (int i = leaf_off[b]; i < leaf_off[b + 1]; ++i) {
    const int o = perm[i];
    if (o >= lo && o < hi) {
      s = 1;
      break;
    }
  }
  f[b] = s;
}

__global__ void k_flags_up(const uint8_t* __restrict__ fc, uint8_t* __restrict__ fp, int64_t np) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= np) return;
  fp[b] = (uint8_t)(fc[4 * b] | fc[4 * b + 1] | fc[4 * b + 2] | fc[4 * b + 3]);
}

inline int blocks_for(int64_t n, int t = 256) { return (int)((n + t - 1) / t); }

// ------------------------------------------------------------------ plan
std::complex<double> cyl_in(int nu, const std::vector<double>& J, double th) {
  const int a = nu < 0 ? -nu : nu;
  double v = J[a];
  if (nu < 0 && (a & 1)) v = -v;
  return v * std::exp(std::complex<double>(0, nu * th));
}

std::complex<double> cyl_out(int nu, const std::vector<std::complex<double>>& H, double th) {
  const int a = nu < 0 ? -nu : nu;
  std::complex<double> v = H[a];
  if (nu < 0 && (a & 1)) v = -v;
  return v * std::exp(std::complex<double>(0, nu * th));
}

template <class T>
std::unique_ptr<FmmPlan<T>> make_plan(const Tree& t, double k, int p) {
  constexpr bool F32 = std::is_same<T, float>::value;
  auto pl = std::make_unique<FmmPlan<T>>();
  pl->k = k;
  pl->p = p;
  pl->L = t.L;
  const int L = t.L;
  pl->lv.resize(L + 1);
  int64_t coef = 0, box0 = 0;
  for (int l = 0; l <= L; ++l) {
    LevelInfo& li = pl->lv[l];
    const double sl = t.side / double(1 << l);
    li.p = p + (int)std::floor(k * std::sqrt(2.0) * sl / 2.0);
    li.P = 2 * li.p + 1;
    li.s = std::min(1.0, k * sl);
    li.box0 = box0;
    box0 += int64_t(1) << (2 * l);
    if (l >= 2) {
      li.coef = coef;
      coef += (int64_t(1) << (2 * l)) * li.P;
    }
  }
  pl->coef_total = coef;
  pl->flag_total = box0;

  // near field: pair arguments k r are bounded by the 3 x 3 leaf block
  const double lside = t.leaf_side();
  const double X = (L == 0) ? k * std::sqrt(2.0) * t.side : k * 2.0 * std::sqrt(2.0) * lside;
  static const int candF[] = {6, 8, 10, 12, 16};
  static const int candD[] = {12, 16, 20, 24, 28};
  pl->near_fast = fit_near_poly(X * X * (1 + 1e-9), F32, F32 ? candF : candD, 5, F32 ? 5e-7 : 2e-13, pl->poly);
  const double mean = double(t.n) / double(t.nleaves);
  pl->G = mean >= 40 ? 1 : (mean >= 20 ? 2 : 4);

  if (L >= 2) {
    const LevelInfo& lf = pl->lv[L];
    const double xmax = k * lside / std::sqrt(2.0);
    HFMM_REQUIRE(xmax <= 6.0,
                 "fmm: leaf boxes are too large for this wavenumber (k * leaf_side / sqrt(2) = " +
                     std::to_string(xmax) + "); use a smaller leaf_size");
    HFMM_REQUIRE(lf.p <= 40, "fmm: leaf-level order above 40");
    // series terms: y^K / (K!)^2 below eps at y = xmax^2 / 4
    const double y = xmax * xmax / 4, eps = F32 ? 1e-9 : 1e-18;
    int K = 1;
    double term = y;
    while (term > eps && K < 60) {
      ++K;
      term *= y / (double(K) * K);
    }
    pl->K = K;
    std::vector<T> ser((size_t)(lf.p + 1) * (K + 1));
    for (int n = 0; n <= lf.p; ++n) {
      ser[(size_t)n * (K + 1)] = T(1.0 / (n + 1));
      for (int j = 1; j <= K; ++j) ser[(size_t)n * (K + 1) + j] = T(1.0 / (double(j) * (n + j)));
    }
    pl->series.upload(ser);

    double maxabs = 0;
    auto put = [&](std::vector<cplx<T>>& v, size_t i, std::complex<double> z) {
      maxabs = std::max(maxabs, std::abs(z));
      v[i] = mk<T>(T(z.real()), T(z.imag()));
    };
    // M2M and L2L tables, levels 2..L-1 (parent level l)
    std::vector<cplx<T>> hm2m, hl2l;
    pl->m2m_off.assign(L + 1, 0);
    pl->l2l_off.assign(L + 1, 0);
    std::vector<double> J;
    for (int l = 2; l < L; ++l) {
      const LevelInfo &lp = pl->lv[l], &lc = pl->lv[l + 1];
      const double sch = t.side / double(1 << (l + 1));
      pl->m2m_off[l] = hm2m.size();
      pl->l2l_off[l] = hl2l.size();
      hm2m.resize(hm2m.size() + (size_t)4 * lp.P * lc.P);
      hl2l.resize(hl2l.size() + (size_t)4 * lp.P * lc.P);
      for (int c = 0; c < 4; ++c) {
        const double cx = (c & 1) - 0.5, cy = (c >> 1) - 0.5;
        const std::complex<double> d(cx * sch, cy * sch);  // child centre - parent centre
        const double r = std::abs(d);
        besselj_seq(lp.p + lc.p, k * r, J);
        const double th_pc = std::arg(-d), th_cp = std::arg(d);
        for (int n = -lc.p; n <= lc.p; ++n)
          for (int lo = -lp.p; lo <= lp.p; ++lo) {
            std::complex<double> v = cyl_in(n - lo, J, th_pc) * std::pow(lc.s, std::abs(n)) / std::pow(lp.s, std::abs(lo));
            put(hm2m, pl->m2m_off[l] + ((size_t)c * lc.P + (n + lc.p)) * lp.P + (lo + lp.p), v);
          }
        for (int m = -lp.p; m <= lp.p; ++m)
          for (int lo = -lc.p; lo <= lc.p; ++lo) {
            std::complex<double> v = cyl_in(m - lo, J, th_cp) * std::pow(lc.s, std::abs(lo)) / std::pow(lp.s, std::abs(m));
            put(hl2l, pl->l2l_off[l] + ((size_t)c * lp.P + (m + lp.p)) * lc.P + (lo + lc.p), v);
          }
      }
    }
    if (hm2m.empty()) hm2m.resize(1);
    if (hl2l.empty()) hl2l.resize(1);
    // M2L tables, levels 2..L, 49 offset slots (40 used)
    std::vector<cplx<T>> hm2l;
    pl->m2l_off.assign(L + 1, 0);
    std::vector<std::complex<double>> H;
    for (int l = 2; l <= L; ++l) {
      const LevelInfo& li = pl->lv[l];
      const int P = li.P, pp = li.p;
      const double sl = t.side / double(1 << l);
      pl->m2l_off[l] = hm2l.size();
      hm2l.resize(hm2l.size() + (size_t)49 * P * P, mk<T>(0, 0));
      for (int ox = -3; ox <= 3; ++ox)
        for (int oy = -3; oy <= 3; ++oy) {
          if (std::max(std::abs(ox), std::abs(oy)) < 2) continue;
          const std::complex<double> z(-ox * sl, -oy * sl);  // target centre - source centre
          hankel_seq(2 * pp, k * std::abs(z), H);
          const double th = std::arg(z);
          const size_t o = (size_t)((ox + 3) * 7 + (oy + 3));
          for (int n = -pp; n <= pp; ++n)
            for (int m = -pp; m <= pp; ++m) {
              std::complex<double> v = cyl_out(n - m, H, th) * std::pow(li.s, std::abs(m) + std::abs(n));
              put(hm2l, pl->m2l_off[l] + (o * P + (n + pp)) * P + (m + pp), v);
            }
        }
    }
    pl->max_table = maxabs;
    HFMM_REQUIRE(std::isfinite(maxabs), "fmm: translation table overflow (order too high for this tree)");
    if (F32)
      HFMM_REQUIRE(maxabs < 1e36, "fmm: FP32 translation tables would overflow; lower p or use FP64");
    pl->m2m.upload(hm2m);
    pl->l2l.upload(hl2l);
    pl->m2l.upload(hm2l);
  }
  return pl;
}

template <class T, int NR>
void run_cols(const Tree& t, FmmPlan<T>& pl, const cplx<T>* q, cplx<T>* phi, int nrhs, int r0,
              const uint8_t* flags, bool accumulate, hipStream_t st, const int* alive, StageTimer* tm) {
  const int L = t.L;
  const int64_t N = t.n;
  const cplx<T>* rel = rel_of<T>(t);
  cplx<T>* M = pl.M.p;
  cplx<T>* Lc = pl.Lc.p;
  const double k = pl.k;
  if (L >= 2) {
    const LevelInfo& lf = pl.lv[L];
    const size_t sh = (size_t)(lf.p + 1 + NR) * 64 * sizeof(cplx<T>);
    k_p2m<T, NR><<<(int)t.nleaves, 64, sh, st>>>(t.leaf_off.p, rel, q, N, nrhs, r0, M + lf.coef * nrhs, lf.p,
                                                 T(k / (2 * lf.s)), T(k * k / 4), pl.series.p, pl.K,
                                                 flags ? flags + lf.box0 : nullptr, alive);
    HFMM_LAUNCH_CHECK();
    for (int l = L - 1; l >= 2; --l) {
      const LevelInfo &lp = pl.lv[l], &lc = pl.lv[l + 1];
      k_m2m<T, NR><<<1 << (2 * l), 64, 0, st>>>(M + lc.coef * nrhs, M + lp.coef * nrhs, pl.m2m.p + pl.m2m_off[l],
                                                lc.P, lp.P, nrhs, r0, flags ? flags + lc.box0 : nullptr,
                                                flags ? flags + lp.box0 : nullptr, alive);
      HFMM_LAUNCH_CHECK();
    }
    if (tm) tm->mark(1, st);
    for (int l = 2; l <= L; ++l) {
      const LevelInfo& li = pl.lv[l];
      const LevelInfo& lp = pl.lv[l - 1];
      k_down<T, NR><<<1 << (2 * l), 64, 0, st>>>(M + li.coef * nrhs, Lc + li.coef * nrhs,
                                                 l > 2 ? Lc + lp.coef * nrhs : nullptr, pl.m2l.p + pl.m2l_off[l],
                                                 l > 2 ? pl.l2l.p + pl.l2l_off[l - 1] : nullptr, li.P, lp.P, l,
                                                 nrhs, r0, flags ? flags + li.box0 : nullptr, alive);
      HFMM_LAUNCH_CHECK();
    }
    if (tm) tm->mark(2, st);
    k_l2p<T, NR><<<(int)t.nleaves, 64, (size_t)NR * lf.P * sizeof(cplx<T>), st>>>(
        t.leaf_off.p, rel, Lc + lf.coef * nrhs, phi, N, nrhs, r0, lf.p, T(k / (2 * lf.s)), T(k * k / 4),
        pl.series.p, pl.K, accumulate ? 1 : 0, alive);
    HFMM_LAUNCH_CHECK();
    if (tm) tm->mark(3, st);
  }
  P2PArgs<T> a{};
  a.leaf_off = t.leaf_off.p;
  a.rel = rel;
  a.q = q;
  a.phi = phi;
  a.flags = flags ? flags + pl.lv[L].box0 : nullptr;
  a.alive = alive;
  a.N = N;
  a.nrhs = nrhs;
  a.r0 = r0;
  a.L = L;
  a.G = pl.G;
  a.accumulate = (L >= 2 || accumulate) ? 1 : 0;
  a.k = T(k);
  a.kls = T(k * t.leaf_side());
  const NearPoly& P = pl.poly;
  for (int i = 0; i < 32; ++i) {
    a.cJ[i] = T(P.cJ[i]);
    a.cY[i] = T(P.cY[i]);
  }
  a.ua = T(P.ua);
  a.ub = T(P.ub);
  a.c1 = T(P.c1);
  a.c0 = T(P.c0);
  const int grid = (int)t.nleaves;
  if (!pl.near_fast) {
    k_p2p<T, NR, 1, false><<<grid, 64, 0, st>>>(a);
  } else {
    switch (P.deg) {
#define HFMM_P2P_CASE(DD) \
  case DD: k_p2p<T, NR, DD, true><<<grid, 64, 0, st>>>(a); break;
      HFMM_P2P_CASE(6)
      HFMM_P2P_CASE(8)
      HFMM_P2P_CASE(10)
      HFMM_P2P_CASE(12)
      HFMM_P2P_CASE(16)
      HFMM_P2P_CASE(20)
      HFMM_P2P_CASE(24)
      HFMM_P2P_CASE(28)
#undef HFMM_P2P_CASE
      default: throw Error(HFMM_ERR_INTERNAL, "fmm: unexpected near-field degree");
    }
  }
  HFMM_LAUNCH_CHECK();
  if (tm) tm->mark(4, st);
}

}  // namespace

template <class T>
FmmPlan<T>& get_plan(Tree& t, double k, int p) {
  HFMM_REQUIRE(std::isfinite(k) && k > 0, "fmm: k must be finite and > 0");
  HFMM_REQUIRE(p >= 1 && p <= 40, "fmm: p must be in [1, 40]");
  const auto key = std::make_tuple(k, p, std::is_same<T, float>::value ? 1 : 0);
  auto it = t.plans.find(key);
  if (it == t.plans.end()) it = t.plans.emplace(key, make_plan<T>(t, k, p)).first;
  return *static_cast<FmmPlan<T>*>(it->second.get());
}

template <class T>
void fmm_sorted(const Tree& t, FmmPlan<T>& pl, const cplx<T>* q, cplx<T>* phi, int nrhs, const uint8_t* flags,
                bool accumulate, hipStream_t st, const int* alive, StageTimer* tm) {
  pl.ensure_work(nrhs);
  for (int r0 = 0; r0 < nrhs;) {
    const int left = nrhs - r0;
    if (left >= 4) {
      run_cols<T, 4>(t, pl, q, phi, nrhs, r0, flags, accumulate, st, alive, tm);
      r0 += 4;
    } else if (left >= 2) {
      run_cols<T, 2>(t, pl, q, phi, nrhs, r0, flags, accumulate, st, alive, tm);
      r0 += 2;
    } else {
      run_cols<T, 1>(t, pl, q, phi, nrhs, r0, flags, accumulate, st, alive, tm);
      r0 += 1;
    }
  }
}

void source_flags(const Tree& t, int64_t lo, int64_t hi, uint8_t* d_flags, hipStream_t st) {
  const int L = t.L;
  int64_t off = 0;
  std::vector<int64_t> box0(L + 1);
  for (int l = 0; l <= L; ++l) {
    box0[l] = off;
    off += int64_t(1) << (2 * l);
  }
  k_leaf_flags<<<blocks_for(t.nleaves), 256, 0, st>>>(t.leaf_off.p, t.perm.p, t.nleaves, lo, hi, d_flags + box0[L]);
  HFMM_LAUNCH_CHECK();
  for (int l = L - 1; l >= 0; --l) {
    const int64_t np = int64_t(1) << (2 * l);
    k_flags_up<<<blocks_for(np), 256, 0, st>>>(d_flags + box0[l + 1], d_flags + box0[l], np);
    HFMM_LAUNCH_CHECK();
  }
}

template <class T>
void fmm_apply(Tree& t, double k, int p, const cplx<T>* q, cplx<T>* phi, int nrhs, hipStream_t st,
               StageTimer* tm) {
  HFMM_REQUIRE(nrhs >= 1, "fmm_apply: nrhs must be >= 1");
  HFMM_REQUIRE(q != nullptr && phi != nullptr, "fmm_apply: NULL array");
  FmmPlan<T>& pl = get_plan<T>(t, k, p);
  const int64_t total = t.n * nrhs;
  pl.qs.ensure(total);
  pl.phis.ensure(total);
  if (tm) tm->mark(-1, st);
  k_gather<T><<<blocks_for(total), 256, 0, st>>>(q, pl.qs.p, t.perm.p, t.n, total);
  HFMM_LAUNCH_CHECK();
  if (tm) tm->mark(0, st);
  fmm_sorted<T>(t, pl, pl.qs.p, pl.phis.p, nrhs, nullptr, false, st, nullptr, tm);
  k_scatter<T><<<blocks_for(total), 256, 0, st>>>(pl.phis.p, phi, t.perm.p, t.n, total);
  HFMM_LAUNCH_CHECK();
  if (tm) tm->mark(5, st);
}

template FmmPlan<float>& get_plan<float>(Tree&, double, int);
template FmmPlan<double>& get_plan<double>(Tree&, double, int);
template void fmm_sorted<float>(const Tree&, FmmPlan<float>&, const float2*, float2*, int, const uint8_t*, bool,
                                hipStream_t, const int*, StageTimer*);
template void fmm_sorted<double>(const Tree&, FmmPlan<double>&, const double2*, double2*, int, const uint8_t*, bool,
                                 hipStream_t, const int*, StageTimer*);
template void fmm_apply<float>(Tree&, double, int, const float2*, float2*, int, hipStream_t, StageTimer*);
template void fmm_apply<double>(Tree&, double, int, const double2*, double2*, int, hipStream_t, StageTimer*);

StageTimer::~StageTimer() {
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
}

void StageTimer::mark(int s, hipStream_t st) {
  hipEvent_t e;
  HFMM_HIP(hipEventCreate(&e));
  ev.push_back(e);
  stage.push_back(s);
  HFMM_HIP(hipEventRecord(e, st));
}

void StageTimer::collect(float* ms, int nstage) {
  for (int i = 0; i < nstage; ++i) ms[i] = 0;
  if (ev.empty()) return;
  HFMM_HIP(hipEventSynchronize(ev.back()));
  for (size_t i = 1; i < ev.size(); ++i) {
    float d = 0;
    HFMM_HIP(hipEventElapsedTime(&d, ev[i - 1], ev[i]));
    if (stage[i] >= 0 && stage[i] < nstage) ms[stage[i]] += d;
  }
}

}  // namespace hfmm
