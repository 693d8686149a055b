// Near-field (P2P) kernels of the FMM: the direct sum of G(x - y) q(y) over
// the sources in a target leaf's 3 x 3 leaf neighbourhood (Sec. 3, the near
// part of the FMM sum), G = (i/4) H0^(1)(k r).  Included once, by fmm.hip,
// inside its anonymous namespace, after the fmaT/log2T/cmac helpers; kept in
// a file of its own so that its source identifies the measured kernel.
#pragma once

template <class T>
struct P2PArgs {
  const int32_t* leaf_off;
  const cplx<T>* rel;
  const cplx<T>* q;
  cplx<T>* phi;
  const uint8_t* flags;  // leaf-level source flags or NULL
  const int* alive;      // device flag: 0 skips the launch's work, or NULL
  const int32_t* operm;  // NULL: phi in Morton order; else phi[operm[i]] (caller order)
  int64_t N;
  int nrhs, r0, L, G, accumulate;
  T k, kls;  // k and k * leaf side
  T cJ[32], cY[32];
  T ua, ub;  // centred polynomial variable u = ua t + ub
  T c1, jinv;  // J0 is carried as Jc = c1 J0; jinv = 1 / c1
  // far field (L2P) of the target leaves, or Lc = NULL for none: local
  // expansions [leaf][nrhs][2 pL + 1] of the leaf level, the Bessel series
  // length and the scales (as in P2M)
  const cplx<T>* Lc;
  int pL, K;
  T wscale, yscale;
};

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
__device__ __forceinline__ void h0_pair(const P2PArgs<T>& a, T t, T& J, T& Y, T cj2, T cy2) {
  // cj2, cy2: a.cJ[D - 2], a.cY[D - 2] (pinned in VGPRs by the caller)
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
    Y = fmaT(j, log2T(t), yh);
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
        h0_pair<T, D, FAST, false>(a, t, J, Y, a.cJ[D >= 2 ? D - 2 : 0], a.cY[D >= 2 ? D - 2 : 0]);
#pragma unroll
        for (int r = 0; r < NR; ++r) acc.add(r, sq[r][j], J, Y);
      }
      for (int j = split + g; j < cnt; j += G) {
        const cplx<T> s = spos[j];
        const T dx = xt - s.x, dy = yt - s.y;
        const T t = fmaT(dx, dx, dy * dy);
        T J, Y;
        h0_pair<T, D, FAST, true>(a, t, J, Y, a.cJ[D >= 2 ? D - 2 : 0], a.cY[D >= 2 ? D - 2 : 0]);
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

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2);
// this maps hardware block b to a logical block so that every XCD walks one
// contiguous range of the Morton order, and neighbouring blocks, which read
// the same leaves, share an L2.  Identity when the grid is not a multiple of 8.
__device__ __forceinline__ int xcd_swizzle(int b, int n) {
  if (n & 7) return b;
  return (b & 7) * (n >> 3) + (b >> 3);
}

// P2P, one block per parent box: its 4 waves are the 4 sibling target
// leaves, and the union of their 3 x 3 neighbourhoods (a 4 x 4 block of
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
                                        T yt, PairSum<T, NR>& acc, T cj2, T cy2) {
#pragma unroll 4
  for (int j = lo + g; j < hi; j += G) {
    const cplx<T> s = spos[j];
    const T dx = xt - s.x, dy = yt - s.y;
    const T t = fmaT(dx, dx, dy * dy);
    T J, Y;
    h0_pair<T, D, FAST, MASK>(a, t, J, Y, cj2, cy2);
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
  if (a.alive && !a.alive[0]) return;
  const int parent = xcd_swizzle((int)blockIdx.x, (int)gridDim.x);
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
        p2p_run<T, D, FAST, false, NR, GG>(a, spos, sq, sg_lo[sgi], sg_hi[sgi], gl, xt, yt, acc, cj2, cy2);
      p2p_run<T, D, FAST, true, NR, GG>(a, spos, sq, own_lo, own_hi, gl, xt, yt, acc, cj2, cy2);
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
          p2p_run<T, D, FAST, false, NR, G>(a, spos, sq, lo, hi, g, xt, yt, acc, cj2, cy2);
        }
        const int lo = max(own_lo, c0) - c0, hi = min(own_hi, c0 + cnt) - c0;
        p2p_run<T, D, FAST, true, NR, G>(a, spos, sq, lo, hi, g, xt, yt, acc, cj2, cy2);
      }
      finish(ti, act, acc, G, g);
    }
  }
}
