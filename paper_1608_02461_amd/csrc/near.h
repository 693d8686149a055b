// Near-field (P2P) kernels of the FMM: the direct sum of G(x - y) q(y) over
// the sources in a target leaf's 3 x 3 leaf neighbourhood (the near part of
// the FMM calculation flow, Sec. 5.1.2), G = (i/4) H0^(1)(k r) (Sec. 5.2, the
// 2-D Green's function).  Included only by near.hip, inside an anonymous
// namespace; kept in a file of its own so that its source identifies the
// measured kernel.
#pragma once

#include "devutil.h"
#include "p2p.h"
#include "special.h"

// log2 of the pair argument t = (k r)^2 > 0.
// FP32: v_log_f32 without the denormal-input rescaling: every argument here
// is (k r)^2 of two distinct FP32 positions, far above the denormal range.
// FP64: a table-driven reduction (the method of P. T. P. Tang, "Table-driven
// implementation of the logarithm function in IEEE floating-point
// arithmetic", ACM TOMS 16, 1990, with the table inverted instead of exact
// products): t = m 2^e with m in [1/2, 1) (frexp); the top 7 fraction bits i
// of m pick c_i = 1/2 + (i + 1/2)/256, and
//     log2 t = e + log2 c_i + log2(1 + r),   r = m (1/c_i) - 1,  |r| <= 1/256,
// with log2(1 + r) = r (1/ln 2)(1 - r/2 + r^2/3 - r^3/4 + r^4/5) + O(r^6).
// The table (1/c_i, log2 c_i) is staged in LDS by the kernel.  Absolute
// error below 1e-14 (the near-field fit tolerates 2e-13).
constexpr double kInvLn2 = 1.4426950408889634074;
__device__ __forceinline__ double log2_tab(double t, const double2* __restrict__ tab) {
  const double m = __builtin_amdgcn_frexp_mant(t);
  const int e = __builtin_amdgcn_frexp_exp(t);
  const double2 c = tab[(__double2hiint(m) >> 13) & 127];
  const double r = fma(m, c.x, -1.0);
  double P = kInvLn2 / 5.0;
  P = fma(P, r, -kInvLn2 / 4.0);
  P = fma(P, r, kInvLn2 / 3.0);
  P = fma(P, r, -kInvLn2 / 2.0);
  P = fma(P, r, kInvLn2);
  return fma(r, P, (double)e + c.y);
}
__device__ __forceinline__ float log2T(float x, const double2*) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ double log2T(double x, const double2* tab) { return log2_tab(x, tab); }

// Running sums of q (J0 + i Y0) over one target's sources, J0 carried as
// Jc = c1 J0:  Re = sum (qx J0 - qy Y0) = jinv aj - ay,
//              Im = sum (qx Y0 + qy J0) = by + jinv bj.
template <class T, int NR>
struct PairSum {
  T aj[NR], ay[NR], by[NR], bj[NR];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int r = 0; r < NR; ++r) aj[r] = ay[r] = by[r] = bj[r] = T(0);
  }
  __device__ __forceinline__ void add(int r, cplx<T> q, T Jc, T Y) {
    aj[r] = fmaT(q.x, Jc, aj[r]);
    ay[r] = fmaT(q.y, Y, ay[r]);
    by[r] = fmaT(q.x, Y, by[r]);
    bj[r] = fmaT(q.y, Jc, bj[r]);
  }
  // sum over the G lanes (a power of two) that share a target
  __device__ __forceinline__ void reduce(int G) {
    for (int off = 1; off < G; off <<= 1) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        aj[r] += __shfl_xor(aj[r], off);
        ay[r] += __shfl_xor(ay[r], off);
        by[r] += __shfl_xor(by[r], off);
        bj[r] += __shfl_xor(bj[r], off);
      }
    }
  }
  // (i/4) times the sum: (i/4)(Re + i Im) = (-Im/4, Re/4)
  __device__ __forceinline__ cplx<T> phi(int r, T jinv) const {
    const T re = fmaT(jinv, aj[r], -ay[r]), im = fmaT(jinv, bj[r], by[r]);
    return mk<T>(T(-0.25) * im, T(0.25) * re);
  }
};

template <class T, int NR>
struct P2PCfg {
  static constexpr int SCH = (2 * sizeof(T) * (1 + NR) * 512 <= 16384) ? 512 : 256;
};

// Coefficient counts below this are fitted as polynomials in t itself (the
// first two candidates of each precision's list).
template <class T> struct kPlainDeg;
template <> struct kPlainDeg<float> { static constexpr int below = 9; };
template <> struct kPlainDeg<double> { static constexpr int below = 12; };

// A wave-uniform value held in a VGPR for the whole kernel: the first Horner
// step has two constant operands and one of them must sit in a VGPR; pinned
// once here, the compiler does not copy it into one inside every loop trip.
__device__ __forceinline__ float pin_vgpr(float x) {
  float r;
  asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
  return r;
}
__device__ __forceinline__ double pin_vgpr(double x) { return x; }

// One pair: t = (k r)^2; returns Jc = c1 J0(sqrt t) and Y = Y0(sqrt t).
// FAST uses the fitted polynomials (D coefficients each), otherwise the
// full-range FP64 routine.  MASK zeroes the pair at t = 0 (a point with
// itself, or a coincident point).
template <class T, int D, bool FAST, bool MASK>
__device__ __forceinline__ void h0_pair(const P2PArgs<T>& a, T t, T& J, T& Y, T cj2, T cy2,
                                        const double2* __restrict__ l2tab) {
  // cj2, cy2: a.cJ[D - 2], a.cY[D - 2] (pinned in VGPRs by the caller);
  // l2tab: the FP64 log2 table in LDS (unused in FP32)
  bool valid = true;
  if (MASK) {
    valid = t > T(0);
    t = valid ? t : T(1);
  }
  if constexpr (FAST) {
    // the low degrees are polynomials in t itself, the others in u = ua t + ub
    const T u = D < kPlainDeg<T>::below ? t : fmaT(t, a.ua, a.ub);
    T j = fmaT(a.cJ[D - 1], u, cj2), yh = fmaT(a.cY[D - 1], u, cy2);
#pragma unroll
    for (int i = D - 3; i >= 0; --i) {
      j = fmaT(j, u, a.cJ[i]);
      yh = fmaT(yh, u, a.cY[i]);
    }
    Y = fmaT(j, log2T(t, l2tab), yh);
    J = j;
  } else {
    const double2 h = h0_general(sqrt((double)t));
    J = (T)h.x * a.c1;
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
  __shared__ double2 s_l2[sizeof(T) == 8 ? 128 : 1];
  const int leaf = blockIdx.x;
  if (a.alive && !a.alive[0]) return;
  const int t0 = a.leaf_off[leaf], t1 = a.leaf_off[leaf + 1];
  if (t0 == t1) return;
  const int lane = threadIdx.x;
  if constexpr (sizeof(T) == 8 && FAST) {
    s_l2[lane] = a.l2tab[lane];
    s_l2[lane + 64] = a.l2tab[lane + 64];
  }
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
    PairSum<T, NR> acc;
    acc.zero();
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
        h0_pair<T, D, FAST, false>(a, t, J, Y, a.cJ[D >= 2 ? D - 2 : 0], a.cY[D >= 2 ? D - 2 : 0], s_l2);
#pragma unroll
        for (int r = 0; r < NR; ++r) acc.add(r, sq[r][j], J, Y);
      }
      for (int j = split + g; j < cnt; j += G) {
        const cplx<T> s = spos[j];
        const T dx = xt - s.x, dy = yt - s.y;
        const T t = fmaT(dx, dx, dy * dy);
        T J, Y;
        h0_pair<T, D, FAST, true>(a, t, J, Y, a.cJ[D >= 2 ? D - 2 : 0], a.cY[D >= 2 ? D - 2 : 0], s_l2);
#pragma unroll
        for (int r = 0; r < NR; ++r) acc.add(r, sq[r][j], J, Y);
      }
    }
    acc.reduce(G);
    if (g == 0 && act) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const size_t idx = (size_t)(a.r0 + r) * a.N + (a.operm ? a.operm[ti] : ti);
        cplx<T> v = acc.phi(r, a.jinv);
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

// leaves) is staged in LDS once, positions relative to the parent centre and
// scaled by k.  In row-major leaf order each wave's sources are 3 contiguous
// runs (one per row) and the own leaf splits the middle run: 4 unmasked
// segments plus one masked.  G lanes share a target (template), each taking
// every G-th source; a shuffle tree sums the G partial sums.
template <class T, int NR>
struct P2P4Cfg {
  static constexpr int kBytes = 2 * (int)sizeof(T) * (1 + NR);
  static constexpr int SCAP = (sizeof(T) == 4 ? 32768 : 49152) / kBytes;
};

template <class T, int D, bool FAST, bool MASK, int NR, int G>
__device__ __forceinline__ void p2p_run(const P2PArgs<T>& a, const cplx<T>* __restrict__ spos,
                                        const cplx<T> (*sq)[P2P4Cfg<T, NR>::SCAP], int lo, int hi, int g, T xt,
                                        T yt, PairSum<T, NR>& acc, T cj2, T cy2, const double2* __restrict__ l2) {
#pragma unroll 4
  for (int j = lo + g; j < hi; j += G) {
    const cplx<T> s = spos[j];
    const T dx = xt - s.x, dy = yt - s.y;
    const T t = fmaT(dx, dx, dy * dy);
    T J, Y;
    h0_pair<T, D, FAST, MASK>(a, t, J, Y, cj2, cy2, l2);
#pragma unroll
    for (int r = 0; r < NR; ++r) acc.add(r, sq[r][j], J, Y);
  }
}

template <class T, int NR, int D, bool FAST, int G>
__global__ __launch_bounds__(256) void k_p2p4(P2PArgs<T> a) {
  constexpr int SCAP = P2P4Cfg<T, NR>::SCAP;
  __shared__ cplx<T> spos[SCAP];
  __shared__ cplx<T> sq[NR][SCAP];
  __shared__ int s_pre[17], s_lo[16], s_rounds[4];
  __shared__ T s_ox[16], s_oy[16];
  __shared__ double2 s_l2[sizeof(T) == 8 ? 128 : 1];
  if (a.alive && !a.alive[0]) return;
  const int parent = xcd_swizzle((int)blockIdx.x, (int)gridDim.x);
  if constexpr (sizeof(T) == 8 && FAST) {
    if (threadIdx.x < 128) s_l2[threadIdx.x] = a.l2tab[threadIdx.x];
  }
  int px, py;
  demorton((uint32_t)parent, px, py);
  const int nb = 1 << a.L;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  if (tid < 16) {
    const int rx = tid & 3, ry = tid >> 2;
    const int lx = 2 * px - 1 + rx, ly = 2 * py - 1 + ry;
    int cnt = 0, lo = 0;
    if (lx >= 0 && ly >= 0 && lx < nb && ly < nb) {
      const uint32_t sl = morton((uint32_t)lx, (uint32_t)ly);
      if (!a.flags || a.flags[sl]) {
        lo = a.leaf_off[sl];
        cnt = a.leaf_off[sl + 1] - lo;
      }
    }
    s_lo[tid] = lo;
    s_pre[tid + 1] = cnt;
    s_ox[tid] = T(rx - 1.5) * a.kls;
    s_oy[tid] = T(ry - 1.5) * a.kls;
  }
  __syncthreads();
  if (tid == 0) {
    s_pre[0] = 0;
    for (int i = 1; i <= 16; ++i) s_pre[i] += s_pre[i - 1];
  }
  __syncthreads();
  const int total = s_pre[16];
  if (total == 0 && a.accumulate) return;
  // this wave's target leaf (child position w of the parent) and its segments
  const int cx = w & 1, cy = w >> 1;
  const uint32_t tleaf = 4u * (uint32_t)parent + (uint32_t)w;
  const int t0 = a.leaf_off[tleaf], t1 = a.leaf_off[tleaf + 1];
  const T txo = T(cx - 0.5) * a.kls, tyo = T(cy - 0.5) * a.kls;
  const int r0 = cy * 4 + cx, r1 = (cy + 1) * 4 + cx, r2 = (cy + 2) * 4 + cx, io = r1 + 1;
  const int sg_lo[4] = {s_pre[r0], s_pre[r2], s_pre[r1], s_pre[io + 1]};
  const int sg_hi[4] = {s_pre[r0 + 3], s_pre[r2 + 3], s_pre[io], s_pre[r1 + 3]};
  const int own_lo = s_pre[io], own_hi = s_pre[io + 1];
  constexpr int TPR = 64 / G;
  const int g = lane & (G - 1), tl = lane / G;
  const T cj2 = pin_vgpr(a.cJ[D >= 2 ? D - 2 : 0]), cy2 = pin_vgpr(a.cY[D >= 2 ? D - 2 : 0]);
  auto stage = [&](int c0, int cnt) {
    for (int idx = tid; idx < cnt; idx += 256) {
      const int gi = c0 + idx;
      int lf = 0;
      while (lf < 15 && gi >= s_pre[lf + 1]) ++lf;
      const int slot = s_lo[lf] + gi - s_pre[lf];
      const cplx<T> d = a.rel[slot];
      spos[idx] = mk<T>(fmaT(a.k, d.x, s_ox[lf]), fmaT(a.k, d.y, s_oy[lf]));
#pragma unroll
      for (int r = 0; r < NR; ++r) sq[r][idx] = a.q[(size_t)(a.r0 + r) * a.N + slot];
    }
  };
  // whole region: 16 threads per leaf of the 4 x 4 block, no search
  auto stage_all = [&]() {
    const int lf = tid >> 4, sub = tid & 15;
    const int lo = s_lo[lf], dst = s_pre[lf], n = s_pre[lf + 1] - dst;
    const T ox = s_ox[lf], oy = s_oy[lf];
#pragma unroll 2
    for (int i = sub; i < n; i += 16) {
      const cplx<T> d = a.rel[lo + i];
      spos[dst + i] = mk<T>(fmaT(a.k, d.x, ox), fmaT(a.k, d.y, oy));
#pragma unroll
      for (int r = 0; r < NR; ++r) sq[r][dst + i] = a.q[(size_t)(a.r0 + r) * a.N + lo + i];
    }
  };
  auto finish = [&](int ti, bool act, PairSum<T, NR>& acc, int gw, int gl) {
    acc.reduce(gw);
    if (gl == 0 && act) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const size_t idx = (size_t)(a.r0 + r) * a.N + (a.operm ? a.operm[ti] : ti);
        cplx<T> v = acc.phi(r, a.jinv);
        if (a.accumulate) {
          const cplx<T> o = a.phi[idx];
          v.x += o.x;
          v.y += o.y;
        }
        a.phi[idx] = v;
      }
    }
  };
  if (total <= SCAP) {
    stage_all();
    __syncthreads();
    // one pass = 64 / GG targets, GG lanes each; the last pass of a leaf
    // widens GG to 2 G or 4 G when few targets are left, so that fewer
    // lanes idle
    auto pass = [&](auto gc, int rb) {
      constexpr int GG = decltype(gc)::value;
      const int gl = lane & (GG - 1), ti = rb + lane / GG;
      const bool act = ti < t1;
      T xt = 0, yt = 0;
      if (act) {
        const cplx<T> d = a.rel[ti];
        xt = fmaT(a.k, d.x, txo);
        yt = fmaT(a.k, d.y, tyo);
      }
      PairSum<T, NR> acc;
      acc.zero();
#pragma unroll
      for (int sgi = 0; sgi < 4; ++sgi)
        p2p_run<T, D, FAST, false, NR, GG>(a, spos, sq, sg_lo[sgi], sg_hi[sgi], gl, xt, yt, acc, cj2, cy2, s_l2);
      p2p_run<T, D, FAST, true, NR, GG>(a, spos, sq, own_lo, own_hi, gl, xt, yt, acc, cj2, cy2, s_l2);
      finish(ti, act, acc, GG, gl);
      return 64 / GG;
    };
    for (int rb = t0; rb < t1;) {
      const int rem = t1 - rb;
      if (rem <= TPR / 4)
        rb += pass(std::integral_constant<int, 4 * G>{}, rb);
      else if (rem <= TPR / 2)
        rb += pass(std::integral_constant<int, 2 * G>{}, rb);
      else
        rb += pass(std::integral_constant<int, G>{}, rb);
    }
  } else {
    // the region does not fit: uniform rounds across the block, sources in chunks
    if (lane == 0) s_rounds[w] = (t1 - t0 + TPR - 1) / TPR;
    __syncthreads();
    const int R = max(max(s_rounds[0], s_rounds[1]), max(s_rounds[2], s_rounds[3]));
    for (int round = 0; round < R; ++round) {
      const int ti = t0 + round * TPR + tl;
      const bool act = ti < t1;
      T xt = 0, yt = 0;
      if (act) {
        const cplx<T> d = a.rel[ti];
        xt = fmaT(a.k, d.x, txo);
        yt = fmaT(a.k, d.y, tyo);
      }
      PairSum<T, NR> acc;
      acc.zero();
      for (int c0 = 0; c0 < total; c0 += SCAP) {
        const int cnt = min(SCAP, total - c0);
        __syncthreads();
        stage(c0, cnt);
        __syncthreads();
#pragma unroll
        for (int sgi = 0; sgi < 4; ++sgi) {
          const int lo = max(sg_lo[sgi], c0) - c0, hi = min(sg_hi[sgi], c0 + cnt) - c0;
          p2p_run<T, D, FAST, false, NR, G>(a, spos, sq, lo, hi, g, xt, yt, acc, cj2, cy2, s_l2);
        }
        const int lo = max(own_lo, c0) - c0, hi = min(own_hi, c0 + cnt) - c0;
        p2p_run<T, D, FAST, true, NR, G>(a, spos, sq, lo, hi, g, xt, yt, acc, cj2, cy2, s_l2);
      }
      finish(ti, act, acc, G, g);
    }
  }
}

// Double-layer near field: phi_i += sum_j q_j dG/dn_j(x_i, y_j) over the
// sources of the 3 x 3 leaf neighbourhood, with the normal derivative of the
// 2-D Green's function taken at the source (Sec. 5.2):
//   dG/dn_y = (i k / 4) H1(k r) (x - y).n_y / r = (k/4) (i J1 - Y1) c,
//   c = (k (x - y)).n / (k r).
// One wave per target leaf; the pair arithmetic runs in FP64 with the
// full-range H1 routine (the boundary carries few sources, so this kernel
// is small next to the volume near field).  Pairs at zero distance add
// nothing (a flat element exerts no double-layer field on its own midpoint).
template <class T, int NR>
__global__ __launch_bounds__(64) void k_p2p_dipole(P2PArgs<T> a) {
  constexpr int SCH = 256;
  __shared__ double2 spos[SCH], snrm[SCH];
  __shared__ cplx<T> sq[NR][SCH];
  __shared__ int s_lo[9], s_pre[10], s_n;
  __shared__ double s_ox[9], s_oy[9];
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
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy) {
        const int sx = bx + dx, sy = by + dy;
        if (sx < 0 || sy < 0 || sx >= nb || sy >= nb) continue;
        const uint32_t sl = morton((uint32_t)sx, (uint32_t)sy);
        if (a.flags && !a.flags[sl]) continue;
        const int lo = a.leaf_off[sl], hi = a.leaf_off[sl + 1];
        if (lo == hi) continue;
        s_lo[n] = lo;
        s_pre[n] = pos;
        s_ox[n] = double(dx) * (double)a.kls;
        s_oy[n] = double(dy) * (double)a.kls;
        pos += hi - lo;
        ++n;
      }
    s_pre[n] = pos;
    s_n = n;
  }
  __syncthreads();
  const int nseg = s_n, total = s_pre[nseg];
  if (total == 0 && a.accumulate) return;
  const double k = (double)a.k;
  for (int rb = t0; rb < t1; rb += 64) {
    const int ti = rb + lane;
    const bool act = ti < t1;
    double xt = 0, yt = 0;
    if (act) {
      const cplx<T> d = a.rel[ti];
      xt = k * (double)d.x;
      yt = k * (double)d.y;
    }
    double accr[NR], acci[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) accr[r] = acci[r] = 0.0;
    for (int c0 = 0; c0 < total; c0 += SCH) {
      const int cnt = min(SCH, total - c0);
      __syncthreads();
      for (int idx = lane; idx < cnt; idx += 64) {
        const int gi = c0 + idx;
        int sg = 0;
        while (sg + 1 < nseg && gi >= s_pre[sg + 1]) ++sg;
        const int slot = s_lo[sg] + gi - s_pre[sg];
        const cplx<T> d = a.rel[slot];
        spos[idx] = make_double2(fma(k, (double)d.x, s_ox[sg]), fma(k, (double)d.y, s_oy[sg]));
        const cplx<T> nv = a.dn[slot];
        snrm[idx] = make_double2((double)nv.x, (double)nv.y);
#pragma unroll
        for (int r = 0; r < NR; ++r) sq[r][idx] = a.q[(size_t)(a.r0 + r) * a.N + slot];
      }
      __syncthreads();
      if (act) {
        for (int j = 0; j < cnt; ++j) {
          const double dx = xt - spos[j].x, dy = yt - spos[j].y;
          const double kr = sqrt(dx * dx + dy * dy);
          if (!(kr > 0.0)) continue;
          const double2 h = h1_general(kr);
          const double c = 0.25 * k * (dx * snrm[j].x + dy * snrm[j].y) / kr;
          const double vr = -c * h.y, vi = c * h.x;  // (k/4) c (i J1 - Y1)
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const double qr = (double)sq[r][j].x, qi = (double)sq[r][j].y;
            accr[r] += qr * vr - qi * vi;
            acci[r] += qr * vi + qi * vr;
          }
        }
      }
    }
    if (act) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const size_t idx = (size_t)(a.r0 + r) * a.N + (a.operm ? a.operm[ti] : ti);
        cplx<T> v = mk<T>(T(accr[r]), T(acci[r]));
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
