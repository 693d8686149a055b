// FMM driver for the 2-D Helmholtz kernel (i/4) H0(k r) (Sec. 5.1.2, Sec.
// 5.2): plans (level orders, translation tables, MFMA fragments, near-field
// polynomial), the launch schedule of one apply, the autotuner and its cache.
// Kernels: P2M here; the MFMA translations (M2M, M2L, L2L) in translate.h;
// the last L2L levels and the L2P in farfield.h; the near field (P2P) in
// near.h (built separately, near.hip).  The VALU M2M / M2L + L2L kernels
// here are the reference path selected by the tree option m2l_valu.
// Schedule of an apply on a tree of depth >= 2: P2M (gathering the charges
// into Morton order), then the near field on the caller's stream beside the
// far-field chain on the tree's second stream, then one kernel that adds the
// two.  No floating-point atomics: every output has one owner, so results
// are deterministic run to run.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <type_traits>

#include "devutil.h"
#include "fmm.h"
#include "p2p.h"

namespace hfmm {

namespace {

template <class T> const cplx<T>* rel_of(const Tree& t);
template <> const float2* rel_of<float>(const Tree& t) { return t.rel32.p; }
template <> const double2* rel_of<double>(const Tree& t) { return t.rel64.p; }

// ------------------------------------------------------------------ P2M
// DIP: the sources are dipoles with unit normals dn (sorted order) and
// density q, whose field is q dG/dn_y (the double layer of Sec. 5.2).  With
// c_m = J_m(k rho) e^{-i m phi} / s^m the scaled basis and n = nx + i ny,
// the directional derivative of J_m e^{-i m phi} along n at the source,
// (k/2)[conj(n) J_{m-1} e^{-i(m-1)phi} - n J_{m+1} e^{-i(m+1)phi}] (the
// ladder relations of the cylinder functions, DLMF 10.6.2), gives
//   Mt_m     += q (k/2)[conj(n) c_{m-1} / s - n c_{m+1} s],
//   Mt_{-m}  += (-1)^m q (-(k/2))[conj(n) conj(c_{m+1}) s - n conj(c_{m-1}) / s]
// (from J_{-j} e^{i j phi} = (-1)^j conj(J_j e^{-i j phi})),
// with c_{-1} = -conj(c_1) s^2 (J_{-1} = -J_1).
template <class T, int NR, int LPW, bool DIP>
__global__ __launch_bounds__(256) void k_p2m(const int32_t* __restrict__ leaf_off, const cplx<T>* __restrict__ rel,
                                            const cplx<T>* __restrict__ q, int64_t N, int nrhs, int r0,
                                            cplx<T>* __restrict__ Mout, int pL, T wscale, T yscale, int K,
                                            const uint8_t* __restrict__ flags, const int* __restrict__ alive,
                                            const int32_t* __restrict__ gperm, cplx<T>* __restrict__ qs_out,
                                            const cplx<T>* __restrict__ dn, T hk, T sl) {
  extern __shared__ unsigned char smem_raw[];
  // blockDim / 64 waves per block, LPW consecutive leaves per wave (small
  // leaves share a wave so that its lanes stay busy); every wave has its own
  // LDS region.  The basis of a chunk of 64 points is leaf-independent (the
  // positions are relative to their own leaf); the sums then take lanes
  // (leaf l, group g, order n).
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int leaf0 = ((int)(blockDim.x >> 6) * blockIdx.x + w) * LPW;
  if (alive && !alive[0]) return;
  if (LPW == 1 && flags && !flags[leaf0]) return;
  constexpr int NB = DIP ? 2 : 1;  // basis arrays: c_m, or the dipole's positive and negative orders
  cplx<T>* sb = reinterpret_cast<cplx<T>*>(smem_raw) + (size_t)w * max(NB * (pL + 1) + NR, 2 * NR) * 64;  // [(pL+1)][64]
  cplx<T>* sbn = sb + (pL + 1) * 64;                    // DIP: [(pL+1)][64]
  cplx<T>* sq = sb + NB * (pL + 1) * 64;                // [NR][64]
  const int P = 2 * pL + 1;
  const int per = pL + 1, G = 64 / (LPW * per);  // groups per (leaf, order)
  const int l = lane / (G * per), lr = lane - l * G * per, g = lr / per, n = lr - g * per;
  const bool accl = l < LPW;
  const int t0 = leaf_off[leaf0], t1 = leaf_off[leaf0 + LPW];
  const int lo_l = accl ? leaf_off[leaf0 + l] : 0, hi_l = accl ? leaf_off[leaf0 + l + 1] : 0;
  cplx<T> accP[NR], accN[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) accP[r] = accN[r] = mk<T>(0, 0);
  for (int c0 = t0; c0 < t1; c0 += 64) {
    const int cnt = min(64, t1 - c0);
    if (lane < cnt) {
      const cplx<T> d = rel[c0 + lane];
      const T wr = wscale * d.x, wi = -wscale * d.y;  // w = (k / 2s) (dx - i dy)
      const T y = yscale * (d.x * d.x + d.y * d.y);   // (k rho)^2 / 4
      // S_n downward into the lane's column, then times w^n / n! upward
      T s1 = sseries(pL + 1, K, y), s0 = sseries(pL, K, y);
      const T stop = s1;  // S_{pL+1}
      for (int m = pL; m >= 0; --m) {
        sb[m * 64 + lane].x = s0;
        if (m > 0) {
          const T sm = sdown(m, y, s0, s1);
          s1 = s0;
          s0 = sm;
        }
      }
      T ur = T(1), ui = T(0);
      for (int m = 0; m <= pL; ++m) {
        const T S = sb[m * 64 + lane].x;
        sb[m * 64 + lane] = mk<T>(ur * S, ui * S);
        const T inv = rcpT(T(m + 1));
        const T nr = (ur * wr - ui * wi) * inv, ni = (ur * wi + ui * wr) * inv;
        ur = nr;
        ui = ni;
      }
      if constexpr (DIP) {
        // (ur, ui) = w^{pL+1} / (pL+1)!, so c_{pL+1} = (ur, ui) S_{pL+1}
        const cplx<T> nv = dn[c0 + lane];
        const T isl = rcpT(sl);
        const cplx<T> c1 = pL >= 1 ? sb[64 + lane] : mk<T>(ur * stop, ui * stop);
        cplx<T> cp = mk<T>(-c1.x * sl * sl, c1.y * sl * sl);  // c_{-1}
        for (int m = 0; m <= pL; ++m) {
          const cplx<T> cm = sb[m * 64 + lane];
          const cplx<T> cn = m < pL ? sb[(m + 1) * 64 + lane] : mk<T>(ur * stop, ui * stop);
          // conj(n) c_{m-1} / s - n c_{m+1} s
          const T ar = (nv.x * cp.x + nv.y * cp.y) * isl, ai = (nv.x * cp.y - nv.y * cp.x) * isl;
          const T br = (nv.x * cn.x - nv.y * cn.y) * sl, bi = (nv.x * cn.y + nv.y * cn.x) * sl;
          sb[m * 64 + lane] = mk<T>(hk * (ar - br), hk * (ai - bi));
          // -(conj(n) conj(c_{m+1}) s - n conj(c_{m-1}) / s)
          const T er = (nv.x * cn.x - nv.y * cn.y) * sl, ei = -(nv.x * cn.y + nv.y * cn.x) * sl;
          const T fr = (nv.x * cp.x + nv.y * cp.y) * isl, fi = (nv.y * cp.x - nv.x * cp.y) * isl;
          sbn[m * 64 + lane] = mk<T>(hk * (fr - er), hk * (fi - ei));
          cp = cm;
        }
      }
      // charges in Morton order; with gperm, q is in caller order and the
      // sorted copy is written to qs_out for the near field
      const int j = c0 + lane;
      const int src = gperm ? gperm[j] : j;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const cplx<T> v = q[(size_t)(r0 + r) * N + src];
        sq[r * 64 + lane] = v;
        if (gperm) qs_out[(size_t)(r0 + r) * N + j] = v;
      }
    }
    wave_lds_sync();
    // lane = (leaf l, group g, order n): the G groups split the chunk's
    // points of leaf l
    if (accl) {
      const int jl = max(lo_l, c0) - c0, jh = min(hi_l, c0 + cnt) - c0;
      for (int j = jl + g; j < jh; j += G) {
        const cplx<T> b = sb[n * 64 + j];
        if constexpr (DIP) {
          const cplx<T> bn = sbn[n * 64 + j];
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const cplx<T> qq = sq[r * 64 + j];
            cmac(accP[r], qq, b);
            cmac(accN[r], qq, bn);
          }
        } else {
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const cplx<T> qq = sq[r * 64 + j];
            cmac(accP[r], qq, b);
            cmacc(accN[r], qq, b);
          }
        }
      }
    }
    wave_lds_sync();
  }
  // sum the G partial sums of each (leaf, order) (sb is free again)
  cplx<T>* red = sb;  // [NR][2][64]
  if (accl) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      red[(r * 2 + 0) * 64 + lane] = accP[r];
      red[(r * 2 + 1) * 64 + lane] = accN[r];
    }
  }
  wave_lds_sync();
  const int leaf = leaf0 + l;
  if (accl && g == 0 && (LPW == 1 || !flags || flags[leaf])) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      cplx<T> sp = accP[r], sn = accN[r];
      for (int gg = 1; gg < G; ++gg) {
        const cplx<T> a = red[(r * 2 + 0) * 64 + lane + gg * per];
        const cplx<T> b = red[(r * 2 + 1) * 64 + lane + gg * per];
        sp.x += a.x;
        sp.y += a.y;
        sn.x += b.x;
        sn.y += b.y;
      }
      const size_t base = ((size_t)leaf * nrhs + r0 + r) * P;
      Mout[base + pL + n] = sp;
      if (n > 0) {
        const T sg = (n & 1) ? T(-1) : T(1);
        Mout[base + pL - n] = mk<T>(sg * sn.x, sg * sn.y);
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

#include "translate.h"
#include "farfield.h"

// ------------------------------------------------------------------ misc
template <class T>
__global__ void k_gather(const cplx<T>* __restrict__ q, cplx<T>* __restrict__ qs, const int32_t* __restrict__ perm,
                         int64_t N) {  // grid: (points, columns)
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const size_t col = (size_t)blockIdx.y * N;
  qs[col + j] = q[col + perm[j]];
}

template <class T>
__global__ void k_scatter(const cplx<T>* __restrict__ phis, cplx<T>* __restrict__ phi,
                          const int32_t* __restrict__ perm, int64_t N) {  // grid: (points, columns)
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const size_t col = (size_t)blockIdx.y * N;
  phi[col + perm[j]] = phis[col + j];
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
// A table entry rounded to FP16 (1) or BF16 (2), round to nearest even, and
// back (the host side of the M2L rounding experiment).
inline float round_host(float v, int mode) {
  if (mode == 1) return (float)(_Float16)v;
  if (mode == 2) {
    uint32_t b;
    std::memcpy(&b, &v, 4);
    b += 0x7fffu + ((b >> 16) & 1u);
    b &= 0xffff0000u;
    std::memcpy(&v, &b, 4);
  }
  return v;
}
inline double round_host(double v, int) { return v; }

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

// Launch shape of the MFMA M2L at level l: the 8 x 8 target tile, or the
// 4 x 4 one (on request, or where the 8 x 8 window does not fit in LDS).
// A level of few blocks whose waves each walk a long chain of dependent
// table loads (10 offset classes of ceil(KS / 4) MFMA chunks) splits its 40
// classes over S = 2, 5 or 10 blocks per target tile and row tile, so that
// more waves share the level and each walks 10 / S classes; the partial sums
// meet in a last-block reduction.
struct M2LShape {
  bool use = false;
  int tile = 0, KSL = 0, gx = 0, NP = 1, S = 1;
  size_t lds = 0;
};
M2LShape m2l_shape(const MfmaLevel& mf, int l, bool small_pref, bool split) {
  M2LShape s;
  const bool small = (small_pref && mf.fit4) || !mf.on;
  s.use = small ? mf.fit4 : mf.on;
  if (!s.use) return s;
  const int nb = 1 << l;
  s.tile = small ? std::min(4, nb) : mf.tile;
  s.KSL = small ? mf.KSL4 : mf.KSL;
  s.lds = small ? mf.lds4 : mf.lds;
  s.gx = (nb / s.tile) * (nb / s.tile);
  s.NP = s.tile == 8 ? 4 : 1;
  int nch = 0;  // MFMA chunks of one class
  for (int k0 = 0; k0 < mf.KS; k0 += s.KSL) nch += (std::min(s.KSL, mf.KS - k0) + 3) / 4;
  if (split && s.gx * mf.RT < kM2LSplitBlocks && 10 * nch > kM2LChain) {
    s.S = 10;
    for (int S : {2, 5})
      if (10 * nch / S <= kM2LChain) {
        s.S = S;
        break;
      }
  }
  return s;
}
// partial-sum elements of one launch with NR columns
inline size_t m2l_part_elems(const M2LShape& s, const MfmaLevel& mf, int nr) {
  return s.S > 1 ? (size_t)nr * s.gx * mf.RT * s.S * s.NP * 256 : 0;
}

template <class T>
std::unique_ptr<FmmPlan<T>> make_plan(const Tree& t, double k, int p) {
  constexpr bool F32 = std::is_same<T, float>::value;
  auto pl = std::make_unique<FmmPlan<T>>();
  pl->npts = t.n;
  pl->k = k;
  pl->p = p;
  pl->L = t.L;
  const int L = t.L;
  pl->lv.resize(L + 1);
  int64_t coef = 0, box0 = 0;
  for (int l = 0; l <= L; ++l) {
    LevelInfo& li = pl->lv[l];
    const double sl = t.side_len / double(1 << l);
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
  // the tree's option selects the VALU downward kernels at every level (reference, ablation)
  pl->use_mfma = !t.m2l_valu;
  pl->m2l_round = F32 ? t.m2l_round : 0;

  // near field: pair arguments k r are bounded by the 3 x 3 leaf block
  const double lside = t.leaf_side();
  const double X = (L == 0) ? k * std::sqrt(2.0) * t.side_len : k * 2.0 * std::sqrt(2.0) * lside;
  // FP32: 1e-6 absolute on J0 and Yf, below the rounding of a complex64 sum
  // over the few hundred pairs of a leaf neighbourhood
  static const int candF[] = {5, 7, 9, 12, 16};
  static const int candD[] = {8, 10, 12, 16, 24};  // (both lists match the launch_p2p switches)
  // the first two candidates of each are polynomials in t itself (kPlainDeg)
  pl->near_fast = fit_near_poly(X * X * (1 + 1e-9), F32, F32 ? candF : candD, 5, 2, F32 ? 1e-6 : 2e-13, pl->poly);
  if (!F32) {
    // the near field's FP64 log2 table: c_i = 1/2 + (i + 1/2)/256, i = 0..127
    std::vector<double2> tab(128);
    for (int i = 0; i < 128; ++i) {
      const long double c = 0.5L + (i + 0.5L) / 256.0L;
      tab[i] = make_double2((double)(1.0L / c), (double)log2l(c));
    }
    pl->l2tab.upload(tab);
  }
  const double mean = double(t.n) / double(t.nleaves);
  const int G0 = mean >= 40 ? 1 : (mean >= 20 ? 2 : 4);
  for (int g = 0; g < 3; ++g) pl->G[g] = G0;

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
      const double sch = t.side_len / double(1 << (l + 1));
      pl->m2m_off[l] = hm2m.size();
      pl->l2l_off[l] = hl2l.size();
      hm2m.resize(hm2m.size() + (size_t)4 * lp.P * lc.P);
      hl2l.resize(hl2l.size() + (size_t)4 * lp.P * lc.P);
      for (int c = 0; c < 4; ++c) {
        const double cx = (c & 1) - 0.5, cy = (c >> 1) - 0.5;
        const std::complex<double> d(cx * sch, cy * sch);  // child centre - parent centre
        const double r = std::abs(d);
        const int D = lp.p + lc.p;
        besselj_seq(D, k * r, J);
        const double th_pc = std::arg(-d), th_cp = std::arg(d);
        // entries depend on the index difference and on |index| through the
        // scales: tabulate both once per child
        std::vector<std::complex<double>> cpc(2 * D + 1), ccp(2 * D + 1);
        for (int nu = -D; nu <= D; ++nu) {
          cpc[nu + D] = cyl_in(nu, J, th_pc);
          ccp[nu + D] = cyl_in(nu, J, th_cp);
        }
        std::vector<double> sc(D + 1), sp(D + 1);
        for (int a = 0; a <= D; ++a) {
          sc[a] = std::pow(lc.s, a);
          sp[a] = std::pow(lp.s, a);
        }
        for (int n = -lc.p; n <= lc.p; ++n)
          for (int lo = -lp.p; lo <= lp.p; ++lo) {
            std::complex<double> v = cpc[n - lo + D] * sc[std::abs(n)] / sp[std::abs(lo)];
            put(hm2m, pl->m2m_off[l] + ((size_t)c * lc.P + (n + lc.p)) * lp.P + (lo + lp.p), v);
          }
        for (int m = -lp.p; m <= lp.p; ++m)
          for (int lo = -lc.p; lo <= lc.p; ++lo) {
            std::complex<double> v = ccp[m - lo + D] * sc[std::abs(lo)] / sp[std::abs(m)];
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
      const double sl = t.side_len / double(1 << l);
      pl->m2l_off[l] = hm2l.size();
      hm2l.resize(hm2l.size() + (size_t)49 * P * P, mk<T>(0, 0));
      for (int ox = -3; ox <= 3; ++ox)
        for (int oy = -3; oy <= 3; ++oy) {
          if (std::max(std::abs(ox), std::abs(oy)) < 2) continue;
          const std::complex<double> z(-ox * sl, -oy * sl);  // target centre - source centre
          hankel_seq(2 * pp, k * std::abs(z), H);
          const double th = std::arg(z);
          const size_t o = (size_t)((ox + 3) * 7 + (oy + 3));
          std::vector<std::complex<double>> cv(4 * pp + 1);
          std::vector<double> sv(2 * pp + 1);
          for (int nu = -2 * pp; nu <= 2 * pp; ++nu) cv[nu + 2 * pp] = cyl_out(nu, H, th);
          for (int a = 0; a <= 2 * pp; ++a) sv[a] = std::pow(li.s, a);
          for (int n = -pp; n <= pp; ++n)
            for (int m = -pp; m <= pp; ++m) {
              std::complex<double> v = cv[n - m + 2 * pp] * sv[std::abs(m) + std::abs(n)];
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

    // MFMA fragments: frag[..][rt][ks][lane] = A[16 rt + lane%16][4 ks + lane/16]
    // with A the real form of a complex (P_out x P_in) block (see k_m2l_mfma)
    auto embed = [](const cplx<T>& z, int i, int kk, int Pout, int Pin) -> T {
      if (i >= 2 * Pout || kk >= 2 * Pin) return T(0);
      const bool io = i >= Pout, ki = kk >= Pin;
      if (!io && !ki) return z.x;
      if (!io && ki) return -z.y;
      if (io && !ki) return z.y;
      return z.x;
    };
    pl->mf.assign(L + 1, MfmaLevel{});
    std::vector<T> haf, hwf, hmf;
    auto frag = [&](std::vector<T>& dst, int64_t base, int nterm, int RT, int KS, int Pout, int Pin,
                    auto&& value) {  // value(term, m_out, n_in) -> complex entry
      dst.resize(dst.size() + (size_t)nterm * RT * KS * 64, T(0));
      for (int tm = 0; tm < nterm; ++tm)
        for (int rt = 0; rt < RT; ++rt)
          for (int ks = 0; ks < KS; ++ks)
            for (int ln = 0; ln < 64; ++ln) {
              const int i = rt * 16 + (ln & 15), kk = ks * 4 + (ln >> 4);
              if (i < 2 * Pout && kk < 2 * Pin)
                dst[base + (((size_t)tm * RT + rt) * KS + ks) * 64 + ln] = embed(value(tm, i % Pout, kk % Pin), i, kk, Pout, Pin);
            }
    };
    for (int l = 2; l <= L; ++l) {
      MfmaLevel& m = pl->mf[l];
      const int P = pl->lv[l].P, nb = 1 << l;
      m.RT = (2 * P + 15) / 16;
      m.KS = (2 * P + 3) / 4;      // k steps of 4 (the padding is zero)
      m.KSA = (m.KS + 3) / 4 * 4;  // table stride: whole chunks of 4 k steps
      // M2L window: a tile of 8 x 8 targets (4 x 4 on a 4 x 4 grid, or by
      // the autotuner): the window plus one zero box in at most kM2LLds bytes
      // of LDS (the block also needs room for the partial sums of 4 waves);
      // when the whole k range does not fit, the kernel stages it in slices
      // of KSL k steps
      auto window = [&](int tile, int ksl) {
        const int win = std::min(nb, std::min(tile, nb) + 4);
        return (size_t)(win * win + 1) * (4 * ((ksl + 3) / 4 * 4) + 2) * sizeof(T);
      };
      auto lds_for = [&](int tile, int ksl) {
        const int np = tile >= 8 && nb >= 8 ? 4 : 1;
        return std::max(window(tile, ksl), (size_t)4 * np * 4 * 64 * sizeof(T));
      };
      auto slice = [&](int tile) {
        int ksl = m.KS;
        while (ksl > 4 && window(tile, ksl) > kM2LLds) ksl = std::max(4, (ksl / 2 + 3) / 4 * 4);
        return ksl;
      };
      m.tile = std::min(8, nb);
      m.KSL = slice(m.tile);
      m.lds = lds_for(m.tile, m.KSL);
      m.KSL4 = slice(4);
      m.lds4 = lds_for(4, m.KSL4);
      m.on = m.lds <= 65536;
      m.fit4 = m.lds4 <= 65536;
      if (!m.on && m.fit4) {
        m.tile = 4;
        m.KSL = m.KSL4;
        m.lds = m.lds4;
        m.on = true;
      }
      m.gx = (nb / m.tile) * (nb / m.tile);
      m.gy = m.RT;
      if (m.on || m.fit4) {
        m.af = (int64_t)haf.size();
        frag(haf, m.af, 49, m.RT, m.KSA, P, P, [&](int o, int mo, int ni) -> cplx<T> {
          const int ox = o / 7 - 3, oy = o % 7 - 3;
          if (std::max(std::abs(ox), std::abs(oy)) < 2) return mk<T>(0, 0);
          return hm2l[pl->m2l_off[l] + ((size_t)o * P + ni) * P + mo];
        });
      }
      if (l > 2) {  // L2L into level l from its parent level
        const int Pp = pl->lv[l - 1].P;
        m.KSp = (2 * Pp + 3) / 4;
        m.wf = (int64_t)hwf.size();
        frag(hwf, m.wf, 4, m.RT, m.KSp, P, Pp, [&](int c, int mo, int ni) -> cplx<T> {
          return hl2l[pl->l2l_off[l - 1] + ((size_t)c * Pp + ni) * P + mo];
        });
      }
      if (l < L) {  // M2M into level l from its child level
        const int Pc = pl->lv[l + 1].P;
        m.KSc = (2 * Pc + 3) / 4;
        m.mm = (int64_t)hmf.size();
        frag(hmf, m.mm, 4, m.RT, m.KSc, P, Pc, [&](int c, int mo, int ni) -> cplx<T> {
          return hm2m[pl->m2m_off[l] + ((size_t)c * Pc + ni) * P + mo];
        });
      }
    }
    pl->m2l_oscale.assign(L + 1, 1.0);
    if (pl->m2l_round) {  // accuracy experiment: 16-bit M2L matrices
      for (int l = 2; l <= L; ++l) {
        const MfmaLevel& m = pl->mf[l];
        if (!(m.on || m.fit4)) continue;
        T* A = haf.data() + m.af;
        const size_t cnt = (size_t)49 * m.RT * m.KSA * 64;
        double amax = 0;
        for (size_t i = 0; i < cnt; ++i) amax = std::max(amax, std::fabs((double)A[i]));
        // FP16: scale the level's table by a power of two into range (the
        // kernel scales its output back); BF16 has FP32's exponent range
        double sc = 1.0;
        if (pl->m2l_round == 1)
          while (amax / sc > 16384.0) sc *= 2.0;
        for (size_t i = 0; i < cnt; ++i) A[i] = round_host(T(A[i] / sc), pl->m2l_round);
        pl->m2l_oscale[l] = sc;
      }
    }
    if (haf.empty()) haf.resize(1);
    if (hwf.empty()) hwf.resize(1);
    if (hmf.empty()) hmf.resize(1);
    pl->afrag.upload(haf);
    pl->wfrag.upload(hwf);
    pl->mfrag.upload(hmf);
    // class-group storage for either tile choice, up to 4 columns
    size_t part = 1, cnt = 1;
    for (int sm = 0; sm < 2; ++sm) {
      size_t pp = 0, cc = 0;
      for (int l = 2; l <= L; ++l) {
        const M2LShape s = m2l_shape(pl->mf[l], l, sm == 1, true);
        if (!s.use || s.S == 1) continue;
        pp += m2l_part_elems(s, pl->mf[l], 4);
        cc += (size_t)s.gx * pl->mf[l].RT;
      }
      part = std::max(part, pp);
      cnt = std::max(cnt, cc);
    }
    pl->m2l_part.alloc(part);
    pl->m2l_cnt.upload(std::vector<unsigned>(cnt, 0u));
  }
  return pl;
}


template <class T>
P2PArgs<T> p2p_args(const Tree& t, const FmmPlan<T>& pl, const cplx<T>* q, cplx<T>* phi, int nrhs, int r0, int nr,
                    const uint8_t* flags, bool accumulate, const int* alive, const int32_t* operm = nullptr,
                    const cplx<T>* Lleaf = nullptr, const cplx<T>* dn = nullptr) {
  P2PArgs<T> a{};
  a.operm = operm;
  a.leaf_off = t.leaf_off.p;
  a.rel = rel_of<T>(t);
  a.q = q;
  a.phi = phi;
  a.flags = flags ? flags + pl.lv[t.L].box0 : nullptr;
  a.alive = alive;
  a.N = t.n;
  a.nrhs = nrhs;
  a.r0 = r0;
  a.L = t.L;
  a.G = pl.G[nr_group(nr)];
  a.accumulate = accumulate ? 1 : 0;
  a.k = T(pl.k);
  a.kls = T(pl.k * t.leaf_side());
  const NearPoly& P = pl.poly;
  for (int i = 0; i < 32; ++i) {
    a.cJ[i] = T(P.cJ[i]);
    a.cY[i] = T(P.cY[i]);
  }
  a.ua = T(P.ua);
  a.ub = T(P.ub);
  a.c1 = T(P.c1);
  a.jinv = T(1.0 / P.c1);
  a.Lc = nullptr;
  a.dn = dn;
  a.l2tab = pl.l2tab.p;
  if (Lleaf && t.L >= 2) {  // the leaf level's local expansions, for the L2P kernel
    const LevelInfo& lf = pl.lv[t.L];
    a.Lc = Lleaf;
    a.pL = lf.p;
    a.K = pl.K;
    a.wscale = T(pl.k / (2 * lf.s));
    a.yscale = T(pl.k * pl.k / 4);
  }
  return a;
}

// M2L of all levels in one launch (the VALU kernel for a level whose LDS
// window does not fit).  pl.m2l_small selects the 4 x 4 target tile.
template <class T, int NR>
void launch_m2l(const Tree& t, const FmmPlan<T>& pl, cplx<T>* M, cplx<T>* Lc, int nrhs, int r0,
                const uint8_t* flags, const int* alive, hipStream_t st) {
  const int L = t.L;
  M2LAllArgs<T> ma{};
  ma.alive = alive;
  ma.round = pl.m2l_round;
  ma.nrhs = nrhs;
  ma.r0 = r0;
  ma.nr = NR;
  int blocks = 0;
  size_t lds = 0, part = 0, cnt = 0;
  for (int l = 2; l <= L; ++l) {
    const LevelInfo& li = pl.lv[l];
    const MfmaLevel& mf = pl.mf[l];
    const M2LShape s = m2l_shape(mf, l, pl.m2l_small, pl.m2l_split);
    if (!s.use) {
      k_down<T, NR><<<1 << (2 * l), 64, 0, st>>>(M + li.coef * nrhs, Lc + li.coef * nrhs, nullptr,
                                                 pl.m2l.p + pl.m2l_off[l], nullptr, li.P, 1, l, nrhs, r0,
                                                 flags ? flags + li.box0 : nullptr, alive);
      HFMM_LAUNCH_CHECK();
      continue;
    }
    M2LLevel<T>& v = ma.lv[ma.nlev++];
    v.M = M + li.coef * nrhs;
    v.Lc = Lc + li.coef * nrhs;
    v.Af = pl.afrag.p + mf.af;
    v.fsrc = flags ? flags + li.box0 : nullptr;
    v.nb = 1 << l;
    v.P = li.P;
    v.RT = mf.RT;
    v.KS = mf.KS;
    v.KSL = s.KSL;
    v.KSA = mf.KSA;
    v.tile = s.tile;
    v.gx = s.gx;
    v.block0 = blocks;
    v.oscale = T(pl.m2l_oscale.empty() ? 1.0 : pl.m2l_oscale[l]);
    v.S = s.S;
    v.part = nullptr;
    v.cnt = nullptr;
    if (s.S > 1) {
      v.part = pl.m2l_part.p + part;
      v.cnt = pl.m2l_cnt.p + cnt;
      part += m2l_part_elems(s, mf, NR);
      cnt += (size_t)s.gx * mf.RT;
    }
    blocks += v.gx * mf.RT * s.S;
    lds = std::max(lds, s.lds);
  }
  HFMM_REQUIRE(part <= pl.m2l_part.n && cnt <= pl.m2l_cnt.n, "fmm: internal: M2L class-group storage too small");
  if (ma.nlev) {
    k_m2l_mfma<T><<<blocks, kM2LThreads, lds, st>>>(ma);
    HFMM_LAUNCH_CHECK();
  }
}

// Far-field chain of one column group: M2M levels L-1 .. 2, M2L of every
// level, L2L levels 3 .. r (MFMA kernels, or the VALU ones on request),
// then k_down_tree: L2L of the last levels r+1 .. L and the L2P into w.far,
// r = max(2, L - 2).  `fa` carries the points and far-field scales.
// Stage timing (tm set): [6] the M2M levels, [7] the M2L, [8] the L2L
// levels with the down tree, all on `st`.
template <class T, int NR>
void far_chain(const Tree& t, FmmPlan<T>& pl, const FmmWork<T>& w, int nrhs, int r0, const uint8_t* flags,
               hipStream_t st, const int* alive, const P2PArgs<T>& fa, StageTimer* tm) {
  const int L = t.L;
  const int rl = std::max(2, L - 2);  // the down tree starts below this level
  cplx<T>* M = w.M;
  cplx<T>* Lc = w.Lc;
  const int e0 = tm ? tm->mark(-1, st) : -1;
  int e_up = -1, e_m2l = -1;
  if (pl.use_mfma) {
    for (int l = L - 1; l >= 2; --l) {
      const LevelInfo &lp = pl.lv[l], &lc = pl.lv[l + 1];
      const MfmaLevel& mf = pl.mf[l];
      TTArgs<T> ta{};
      ta.in = M + lc.coef * nrhs;
      ta.out = M + lp.coef * nrhs;
      ta.Wf = pl.mfrag.p + mf.mm;
      ta.fin = flags ? flags + lc.box0 : nullptr;
      ta.fout = flags ? flags + lp.box0 : nullptr;
      ta.alive = alive;
      ta.mode = 1;
      ta.nparents = 1 << (2 * l);
      ta.Pin = lc.P;
      ta.Pout = lp.P;
      ta.RT = mf.RT;
      ta.KS = mf.KSc;
      ta.nrhs = nrhs;
      ta.r0 = r0;
      ta.nr = NR;
      k_tt_mfma<T><<<dim3((ta.nparents + 15) / 16, mf.RT), 256, 0, st>>>(ta);
      HFMM_LAUNCH_CHECK();
    }
    if (tm) e_up = tm->mark(6, st, e0);
    launch_m2l<T, NR>(t, pl, M, Lc, nrhs, r0, flags, alive, st);
    if (tm) e_m2l = tm->mark(7, st, e_up);
    for (int l = 3; l <= rl; ++l) {
      const LevelInfo &li = pl.lv[l], &lp = pl.lv[l - 1];
      const MfmaLevel& mf = pl.mf[l];
      TTArgs<T> ta{};
      ta.in = Lc + lp.coef * nrhs;
      ta.out = Lc + li.coef * nrhs;
      ta.Wf = pl.wfrag.p + mf.wf;
      ta.alive = alive;
      ta.mode = 0;
      ta.nparents = 1 << (2 * (l - 1));
      ta.Pin = lp.P;
      ta.Pout = li.P;
      ta.RT = mf.RT;
      ta.KS = mf.KSp;
      ta.nrhs = nrhs;
      ta.r0 = r0;
      ta.nr = NR;
      k_tt_mfma<T><<<dim3((ta.nparents + 15) / 16, mf.RT), 256, 0, st>>>(ta);
      HFMM_LAUNCH_CHECK();
    }
  } else {
    for (int l = L - 1; l >= 2; --l) {
      const LevelInfo &lp = pl.lv[l], &lc = pl.lv[l + 1];
      k_m2m<T, NR><<<1 << (2 * l), 64, 0, st>>>(M + lc.coef * nrhs, M + lp.coef * nrhs, pl.m2m.p + pl.m2m_off[l],
                                                lc.P, lp.P, nrhs, r0, flags ? flags + lc.box0 : nullptr,
                                                flags ? flags + lp.box0 : nullptr, alive);
      HFMM_LAUNCH_CHECK();
    }
    for (int l = 2; l <= L; ++l) {
      const LevelInfo& li = pl.lv[l];
      const LevelInfo& lp = pl.lv[l - 1];
      k_down<T, NR><<<1 << (2 * l), 64, 0, st>>>(M + li.coef * nrhs, Lc + li.coef * nrhs,
                                                 l > 2 && l <= rl ? Lc + lp.coef * nrhs : nullptr, pl.m2l.p + pl.m2l_off[l],
                                                 l > 2 && l <= rl ? pl.l2l.p + pl.l2l_off[l - 1] : nullptr, li.P, lp.P, l,
                                                 nrhs, r0, flags ? flags + li.box0 : nullptr, alive);
      HFMM_LAUNCH_CHECK();
    }
  }
  // the last levels and the L2P
  DownTreeArgs<T> g{};
  g.a = fa;
  g.d = L - rl;
  g.Lr = Lc + pl.lv[rl].coef * nrhs;
  g.P0 = pl.lv[rl].P;
  if (g.d >= 1) {
    g.L1 = Lc + pl.lv[rl + 1].coef * nrhs;
    g.W1 = pl.l2l.p + pl.l2l_off[rl];
    g.P1 = pl.lv[rl + 1].P;
  }
  if (g.d == 2) {
    g.L2 = Lc + pl.lv[rl + 2].coef * nrhs;
    g.W2 = pl.l2l.p + pl.l2l_off[rl + 1];
    g.P2 = pl.lv[rl + 2].P;
  }
  g.far = w.far;
  const size_t sh = (size_t)(4 * NR * g.P1 + 16 * NR * g.P2) * sizeof(cplx<T>);
  k_down_tree<T, NR><<<1 << (2 * rl), 256, sh, st>>>(g);
  HFMM_LAUNCH_CHECK();
  // the VALU path's M2L and L2L share launches: both count under [8]
  if (tm) tm->mark(8, st, e_m2l >= 0 ? e_m2l : e0);
}

// One column group (NR columns from r0).  P2M (which also gathers the
// charges into Morton order when `perm` is given) comes first.  On a tree
// of depth >= 2 (and 2^18 points or more) the far-field chain then runs on
// the tree's side stream while the near field runs on `st` (smaller trees
// run both on `st`, near field first).  The near field writes (or adds to)
// phi, the chain ends with the L2P into the far-field array w.far, both
// through `perm` when given, and a last streaming kernel adds the far
// field to phi.  Stage timing: [1] P2M, [2] the far-field chain including
// the L2P (side stream, beside [4]; its parts in [6], [7], [8]), [4] the
// near field, [3] the sum, including the wait for [2].  With dn the sources are dipoles (sorted I/O).
template <class T, int NR>
void run_cols(const Tree& t, FmmPlan<T>& pl, const FmmWork<T>& w, const cplx<T>* q, cplx<T>* phi, int nrhs, int r0,
              const uint8_t* flags, bool accumulate, hipStream_t st, const int* alive, StageTimer* tm,
              const int32_t* perm, cplx<T>* qs, const cplx<T>* dn) {
  const int L = t.L;
  const int64_t N = t.n;
  const cplx<T>* rel = rel_of<T>(t);
  const double k = pl.k;
  const cplx<T>* qnear = perm ? qs : q;
  const int G = pl.G[nr_group(NR)];
  auto near = [&](const P2PArgs<T>& a) {
    if (dn)
      launch_p2p_dipole<T, NR>(L, t.nleaves, a, st);
    else
      launch_p2p<T, NR>(L, t.nleaves, pl.near_fast, pl.poly.deg, a, G, st);
  };
  if (L >= 2) {
    HFMM_REQUIRE(t.side != nullptr, "fmm: internal: tree without a side stream");
    // small trees: the chain on `st` itself (two events would cost more
    // than the overlap gains)
    const bool overlap = t.n >= (int64_t(1) << 18);
    hipStream_t cs = overlap ? t.side : st;
    const LevelInfo& lf = pl.lv[L];
    const int nb = dn ? 2 : 1;
    // basis [nb (p+1)][64] and charges [NR][64], reused as the [NR][2][64] partial sums
    const size_t sh = (size_t)std::max(nb * (lf.p + 1) + NR, 2 * NR) * 64 * sizeof(cplx<T>);
    const int lpb = 4 * sh <= 65536 ? 4 : (2 * sh <= 65536 ? 2 : 1);  // waves per block
    // leaves per wave: small leaves share a wave
    const double mean = double(N) / double(t.nleaves);
    const int lpw = (mean <= 20 && 4 * (lf.p + 1) <= 64) ? 4 : ((mean <= 40 && 2 * (lf.p + 1) <= 64) ? 2 : 1);
    const T hk = T(k / 2), sl = T(lf.s);
    auto p2m = [&](auto lc, auto dc) {
      constexpr int LPW = decltype(lc)::value;
      constexpr bool DIP = decltype(dc)::value;
      k_p2m<T, NR, LPW, DIP><<<(int)(t.nleaves / (lpb * LPW)), 64 * lpb, lpb * sh, st>>>(
          t.leaf_off.p, rel, q, N, nrhs, r0, w.M + lf.coef * nrhs, lf.p, T(k / (2 * lf.s)), T(k * k / 4), pl.K,
          flags ? flags + lf.box0 : nullptr, alive, perm, qs, dn, hk, sl);
    };
    if (dn) {
      HFMM_REQUIRE(perm == nullptr, "fmm: internal: dipole sources need sorted input");
      p2m(std::integral_constant<int, 1>{}, std::true_type{});
    } else if (lpw == 4) {
      p2m(std::integral_constant<int, 4>{}, std::false_type{});
    } else if (lpw == 2) {
      p2m(std::integral_constant<int, 2>{}, std::false_type{});
    } else {
      p2m(std::integral_constant<int, 1>{}, std::false_type{});
    }
    HFMM_LAUNCH_CHECK();
    const int e_p2m = tm ? tm->mark(1, st) : -1;
    if (overlap) {
      HFMM_HIP(hipEventRecord(t.fork, st));
      HFMM_HIP(hipStreamWaitEvent(t.side, t.fork, 0));
    }
    // the near field is queued first: when the host is not ahead of the
    // device, the chain's many launches would otherwise delay its start
    const P2PArgs<T> a = p2p_args<T>(t, pl, qnear, phi, nrhs, r0, NR, flags, accumulate, alive, perm, nullptr, dn);
    near(a);
    const int e_p2p = tm ? tm->mark(4, st, e_p2m) : -1;
    const P2PArgs<T> b =
        p2p_args<T>(t, pl, qnear, phi, nrhs, r0, NR, flags, false, alive, perm, w.Lc + lf.coef * nrhs);
    far_chain<T, NR>(t, pl, w, nrhs, r0, flags, cs, alive, b, tm);
    if (tm) tm->mark(2, cs, overlap ? e_p2m : e_p2p);
    if (overlap) {
      HFMM_HIP(hipEventRecord(t.join, t.side));
      HFMM_HIP(hipStreamWaitEvent(st, t.join, 0));
    }
    k_combine<T, NR><<<(int)((N + 255) / 256), 256, 0, st>>>(phi, w.far, N, r0, alive);
    HFMM_LAUNCH_CHECK();
    if (tm) tm->mark(3, st, overlap ? e_p2p : -1);
    return;
  }
  // a single leaf: the near field is the whole sum
  const P2PArgs<T> a = p2p_args<T>(t, pl, qnear, phi, nrhs, r0, NR, flags, accumulate, alive, perm, nullptr, dn);
  near(a);
  if (tm) tm->mark(4, st);
}

// ------------------------------------------------------------------ tuning
struct TuneVal {
  int G = 1;
  int m2l_small = 0;
  int m2l_split = 1;
};

std::mutex& tune_mutex() {
  static std::mutex m;
  return m;
}
std::map<std::string, TuneVal>& tune_table() {
  static std::map<std::string, TuneVal> t;
  return t;
}

std::string device_arch() {
  int dev = 0;
  HFMM_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HFMM_HIP(hipGetDeviceProperties(&prop, dev));
  std::string a(prop.gcnArchName);
  for (char& c : a)
    if (c == ' ') c = '_';
  return a;
}

// Key of a plan's launch shapes: device architecture, precision, depth,
// mean leaf occupancy, near-field polynomial and the level orders.
template <class T>
std::string plan_key(const Tree& t, const FmmPlan<T>& pl) {
  std::ostringstream os;
  os << device_arch() << ":" << (std::is_same<T, float>::value ? "fp32" : "fp64") << ":L" << t.L;
  char mean[32];
  std::snprintf(mean, sizeof mean, ":m%.1f", double(t.n) / double(t.nleaves));
  os << mean << ":d" << (pl.near_fast ? pl.poly.deg : 0) << ":p";
  for (int l = 0; l <= t.L; ++l) os << (l ? "," : "") << pl.lv[l].p;
  return os.str();
}

// Launch-shape autotuner for one column-group width (the kernels' cost does
// not depend on the charges, so zeros are used): the P2P lanes per target
// G in {1, 2, 4} and, for one column, the M2L target tile (8 x 8 or 4 x 4)
// and then, with that tile, whether the coarse levels split into class
// groups (only when 5 % faster than without, so that timing noise does not
// flip the choice from one process to the next where the two are close).
template <class T, int NR>
void autotune_group(const Tree& t, FmmPlan<T>& pl) {
  constexpr int g = NR >= 4 ? 2 : (NR >= 2 ? 1 : 0);
  hipStream_t st;
  HFMM_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  hipEvent_t e0, e1;
  HFMM_HIP(hipEventCreate(&e0));
  HFMM_HIP(hipEventCreate(&e1));
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(st);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(st);
  };
  try {
    pl.ensure_work(NR);
    pl.qs.ensure((size_t)t.n * NR);
    pl.phis.ensure((size_t)t.n * NR);
    HFMM_HIP(hipMemsetAsync(pl.qs.p, 0, (size_t)t.n * NR * sizeof(cplx<T>), st));
    HFMM_HIP(hipMemsetAsync(pl.M.p, 0, (size_t)pl.coef_total * NR * sizeof(cplx<T>), st));
    auto timed = [&](auto&& fn) {
      float best = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        HFMM_HIP(hipEventRecord(e0, st));
        fn();
        HFMM_HIP(hipEventRecord(e1, st));
        HFMM_HIP(hipEventSynchronize(e1));
        float ms = 0;
        HFMM_HIP(hipEventElapsedTime(&ms, e0, e1));
        best = std::min(best, ms);
      }
      return best;
    };
    const P2PArgs<T> a = p2p_args<T>(t, pl, pl.qs.p, pl.phis.p, NR, 0, NR, nullptr, false, nullptr);
    // the fastest G; a larger G within 5 % of it wins (the choice stays
    // the same from one plan to the next when two are that close)
    float ms[3];
    const int Gs[3] = {1, 2, 4};
    float bestms = 1e30f;
    for (int i = 0; i < 3; ++i) {
      ms[i] = timed([&] { launch_p2p<T, NR>(t.L, t.nleaves, pl.near_fast, pl.poly.deg, a, Gs[i], st); });
      bestms = std::min(bestms, ms[i]);
    }
    int bestG = pl.G[g];
    for (int i = 0; i < 3; ++i)
      if (ms[i] <= 1.05f * bestms) bestG = Gs[i];
    pl.G[g] = bestG;
    if (g == 0) {
      for (int i = 0; i < 3; ++i) pl.tune_ms[i] = ms[i];
      bool any_choice = false;
      for (int l = 2; l <= t.L; ++l) any_choice = any_choice || (pl.mf[l].fit4 && pl.mf[l].tile == 8);
      if (pl.use_mfma && any_choice) {
        pl.m2l_small = false;
        const float big = timed([&] { launch_m2l<T, 1>(t, pl, pl.M.p, pl.Lc.p, 1, 0, nullptr, nullptr, st); });
        pl.m2l_small = true;
        const float small = timed([&] { launch_m2l<T, 1>(t, pl, pl.M.p, pl.Lc.p, 1, 0, nullptr, nullptr, st); });
        pl.tune_ms[3] = big;
        pl.tune_ms[4] = small;
        pl.m2l_small = small < big;
      }
      bool any_split = false;
      for (int l = 2; l <= t.L; ++l) any_split = any_split || m2l_shape(pl.mf[l], l, pl.m2l_small, true).S > 1;
      if (pl.use_mfma && any_split) {
        pl.m2l_split = false;
        const float whole = timed([&] { launch_m2l<T, 1>(t, pl, pl.M.p, pl.Lc.p, 1, 0, nullptr, nullptr, st); });
        pl.m2l_split = true;
        const float parts = timed([&] { launch_m2l<T, 1>(t, pl, pl.M.p, pl.Lc.p, 1, 0, nullptr, nullptr, st); });
        pl.tune_ms[5] = whole;
        pl.tune_ms[6] = parts;
        pl.m2l_split = parts < 0.95f * whole;
      }
    }
  } catch (...) {
    cleanup();
    throw;
  }
  cleanup();
}

}  // namespace

template <class T>
void ensure_tuned(Tree& t, FmmPlan<T>& pl, int nrhs) {
  if (t.L < 2) {  // nothing to choose on a single leaf
    for (int g = 0; g < 3; ++g) pl.tuned[g] = true;
    return;
  }
  bool need[3] = {false, false, false};
  for (int r0 = 0; r0 < nrhs;) {
    const int left = nrhs - r0, w = left >= 4 ? 4 : (left >= 2 ? 2 : 1);
    need[nr_group(w)] = true;
    r0 += w;
  }
  if (pl.tune_key.empty()) pl.tune_key = plan_key<T>(t, pl);
  for (int g = 0; g < 3; ++g) {
    if (!need[g] || pl.tuned[g]) continue;
    const std::string key = pl.tune_key + ":c" + std::to_string(1 << g) + (pl.use_mfma ? "" : ":valu");
    {
      std::lock_guard<std::mutex> lk(tune_mutex());
      auto it = tune_table().find(key);
      if (it != tune_table().end()) {
        pl.G[g] = it->second.G;
        if (g == 0) {
          pl.m2l_small = it->second.m2l_small != 0;
          pl.m2l_split = it->second.m2l_split != 0;
        }
        pl.tuned[g] = true;
        pl.tune_source = 2;
        continue;
      }
    }
    if (t.autotune) {
      if (g == 0)
        autotune_group<T, 1>(t, pl);
      else if (g == 1)
        autotune_group<T, 2>(t, pl);
      else
        autotune_group<T, 4>(t, pl);
      pl.tune_source = 1;
      std::lock_guard<std::mutex> lk(tune_mutex());
      TuneVal v;
      v.G = pl.G[g];
      v.m2l_small = pl.m2l_small ? 1 : 0;
      v.m2l_split = pl.m2l_split ? 1 : 0;
      tune_table()[key] = v;
    }
    pl.tuned[g] = true;
  }
}

void tune_cache_save(const std::string& path) {
  std::lock_guard<std::mutex> lk(tune_mutex());
  std::ofstream f(path);
  HFMM_REQUIRE(f.good(), "tune_cache_save: cannot open " + path);
  f << "# hfmm tuning cache: key G m2l_small m2l_split\n";
  for (const auto& kv : tune_table())
    f << kv.first << " " << kv.second.G << " " << kv.second.m2l_small << " " << kv.second.m2l_split << "\n";
  HFMM_REQUIRE(f.good(), "tune_cache_save: write failed on " + path);
}

int tune_cache_load(const std::string& path) {
  std::ifstream f(path);
  HFMM_REQUIRE(f.good(), "tune_cache_load: cannot open " + path);
  std::lock_guard<std::mutex> lk(tune_mutex());
  std::string line;
  int n = 0;
  while (std::getline(f, line)) {
    if (line.empty() || line[0] == '#') continue;
    std::istringstream is(line);
    std::string key;
    TuneVal v;
    if (!(is >> key >> v.G >> v.m2l_small)) throw Error(HFMM_ERR_ARG, "tune_cache_load: bad line: " + line);
    if (!(is >> v.m2l_split)) v.m2l_split = 1;  // files written before the class-group choice
    HFMM_REQUIRE(v.G == 1 || v.G == 2 || v.G == 4, "tune_cache_load: lanes per target must be 1, 2 or 4");
    tune_table()[key] = v;
    ++n;
  }
  return n;
}

int tune_cache_size() {
  std::lock_guard<std::mutex> lk(tune_mutex());
  return (int)tune_table().size();
}

void tune_cache_clear() {
  std::lock_guard<std::mutex> lk(tune_mutex());
  tune_table().clear();
}

template <class T>
FmmPlan<T>* find_plan(Tree& t, double k, int p) {
  auto it = t.plans.find(std::make_tuple(k, p, std::is_same<T, float>::value ? 1 : 0));
  return it == t.plans.end() ? nullptr : static_cast<FmmPlan<T>*>(it->second.get());
}

template <class T>
FmmPlan<T>& get_plan(Tree& t, double k, int p) {
  HFMM_REQUIRE(std::isfinite(k) && k > 0, "fmm: k must be finite and > 0");
  HFMM_REQUIRE(p >= 1 && p <= 40, "fmm: p must be in [1, 40]");
  const auto key = std::make_tuple(k, p, std::is_same<T, float>::value ? 1 : 0);
  auto it = t.plans.find(key);
  if (it == t.plans.end()) {
    auto pl = make_plan<T>(t, k, p);
    ensure_tuned<T>(t, *pl, 1);
    it = t.plans.emplace(key, std::move(pl)).first;
  }
  return *static_cast<FmmPlan<T>*>(it->second.get());
}

template <class T>
void fmm_sorted(const Tree& t, FmmPlan<T>& pl, const cplx<T>* q, cplx<T>* phi, int nrhs, const uint8_t* flags,
                bool accumulate, hipStream_t st, const int* alive, StageTimer* tm, const int32_t* perm,
                cplx<T>* qs, const FmmWork<T>* w, const cplx<T>* dn) {
  HFMM_REQUIRE(!perm || (t.L >= 2 && qs && !flags), "fmm: internal: permuted I/O needs a tree of depth >= 2");
  FmmWork<T> own;
  if (!w) {
    pl.ensure_work(nrhs);
    own.M = pl.M.p;
    own.Lc = pl.Lc.p;
    own.far = pl.far.p;
    w = &own;
  }
  for (int r0 = 0; r0 < nrhs;) {
    const int left = nrhs - r0;
    if (left >= 4) {
      run_cols<T, 4>(t, pl, *w, q, phi, nrhs, r0, flags, accumulate, st, alive, tm, perm, qs, dn);
      r0 += 4;
    } else if (left >= 2) {
      run_cols<T, 2>(t, pl, *w, q, phi, nrhs, r0, flags, accumulate, st, alive, tm, perm, qs, dn);
      r0 += 2;
    } else {
      run_cols<T, 1>(t, pl, *w, q, phi, nrhs, r0, flags, accumulate, st, alive, tm, perm, qs, dn);
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

namespace {
bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HFMM_HIP(hipStreamIsCapturing(st, &cs));
  return cs != hipStreamCaptureStatusNone;
}

// Sorted unit normals (the point order of the tree) in the working precision.
template <class T>
__global__ void k_gather_normals(const double2* __restrict__ nrm, const int32_t* __restrict__ perm, int64_t N,
                                 cplx<T>* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const double2 v = nrm[perm[j]];
  out[j] = mk<T>(T(v.x), T(v.y));
}
}  // namespace

template <class T>
void fmm_apply(Tree& t, double k, int p, const cplx<T>* q, cplx<T>* phi, int nrhs, hipStream_t st,
               StageTimer* tm) {
  HFMM_REQUIRE(nrhs >= 1, "fmm_apply: nrhs must be >= 1");
  HFMM_REQUIRE(q != nullptr && phi != nullptr, "fmm_apply: NULL array");
  FmmPlan<T>& pl = get_plan<T>(t, k, p);
  if (!capturing(st)) ensure_tuned<T>(t, pl, nrhs);
  const int64_t total = t.n * nrhs;
  pl.qs.ensure(total);
  pl.phis.ensure(total);
  if (tm) tm->mark(-1, st);
  if (t.L >= 2) {
    // the P2M kernel gathers the charges into Morton order and the near-field
    // kernel writes the potentials back in caller order
    fmm_sorted<T>(t, pl, q, phi, nrhs, nullptr, false, st, nullptr, tm, t.perm.p, pl.qs.p);
  } else {
    k_gather<T><<<dim3(blocks_for(t.n), nrhs), 256, 0, st>>>(q, pl.qs.p, t.perm.p, t.n);
    HFMM_LAUNCH_CHECK();
    if (tm) tm->mark(0, st);
    fmm_sorted<T>(t, pl, pl.qs.p, pl.phis.p, nrhs, nullptr, false, st, nullptr, tm);
    k_scatter<T><<<dim3(blocks_for(t.n), nrhs), 256, 0, st>>>(pl.phis.p, phi, t.perm.p, t.n);
    HFMM_LAUNCH_CHECK();
    if (tm) tm->mark(5, st);
  }
}

template <class T>
void fmm_apply_dipole(Tree& t, double k, int p, const cplx<T>* q, const double* normals, cplx<T>* phi, int nrhs,
                      hipStream_t st) {
  HFMM_REQUIRE(nrhs >= 1, "fmm_apply_dipole: nrhs must be >= 1");
  HFMM_REQUIRE(q != nullptr && phi != nullptr && normals != nullptr, "fmm_apply_dipole: NULL array");
  FmmPlan<T>& pl = get_plan<T>(t, k, p);
  const int64_t total = t.n * nrhs;
  pl.qs.ensure(total);
  pl.phis.ensure(total);
  pl.dns.ensure(t.n);
  k_gather<T><<<dim3(blocks_for(t.n), nrhs), 256, 0, st>>>(q, pl.qs.p, t.perm.p, t.n);
  HFMM_LAUNCH_CHECK();
  k_gather_normals<T><<<blocks_for(t.n), 256, 0, st>>>(reinterpret_cast<const double2*>(normals), t.perm.p, t.n,
                                                      pl.dns.p);
  HFMM_LAUNCH_CHECK();
  fmm_sorted<T>(t, pl, pl.qs.p, pl.phis.p, nrhs, nullptr, false, st, nullptr, nullptr, nullptr, nullptr, nullptr,
                pl.dns.p);
  k_scatter<T><<<dim3(blocks_for(t.n), nrhs), 256, 0, st>>>(pl.phis.p, phi, t.perm.p, t.n);
  HFMM_LAUNCH_CHECK();
}

template <class T>
size_t fmm_apply_scratch(Tree& t, double k, int p, const cplx<T>* q, cplx<T>* phi, int nrhs, void* scratch,
                         size_t bytes, hipStream_t st) {
  HFMM_REQUIRE(nrhs >= 1, "fmm_apply: nrhs must be >= 1");
  HFMM_REQUIRE(q != nullptr && phi != nullptr, "fmm_apply: NULL array");
  FmmPlan<T>* pl = find_plan<T>(t, k, p);
  if (!pl)
    throw Error(HFMM_ERR_STATE,
                "fmm_apply (no allocation): no plan for this (k, p, precision) on the tree; make it first "
                "(hfmm_fmm_plan_info or one hfmm_fmm_apply)");
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t cb = sizeof(cplx<T>);
  const size_t nq = (size_t)t.n * nrhs * cb;
  const size_t nexp = t.L >= 2 ? (size_t)pl->coef_total * nrhs * cb : 0;
  // regions: M, Lc, far, qs (depth >= 2); qs, phis (a single leaf)
  const size_t need = t.L >= 2 ? 2 * up(nexp) + 2 * up(nq) : 2 * up(nq);
  if (need > bytes) return need;
  char* base = static_cast<char*>(scratch);
  if (t.L >= 2) {
    FmmWork<T> w;
    w.M = reinterpret_cast<cplx<T>*>(base);
    w.Lc = reinterpret_cast<cplx<T>*>(base + up(nexp));
    w.far = reinterpret_cast<cplx<T>*>(base + 2 * up(nexp));
    cplx<T>* qs = reinterpret_cast<cplx<T>*>(base + 2 * up(nexp) + up(nq));
    fmm_sorted<T>(t, *pl, q, phi, nrhs, nullptr, false, st, nullptr, nullptr, t.perm.p, qs, &w);
  } else {
    cplx<T>* qs = reinterpret_cast<cplx<T>*>(base);
    cplx<T>* phis = reinterpret_cast<cplx<T>*>(base + up(nq));
    k_gather<T><<<dim3(blocks_for(t.n), nrhs), 256, 0, st>>>(q, qs, t.perm.p, t.n);
    HFMM_LAUNCH_CHECK();
    FmmWork<T> w;  // unused on a single leaf
    fmm_sorted<T>(t, *pl, qs, phis, nrhs, nullptr, false, st, nullptr, nullptr, nullptr, nullptr, &w);
    k_scatter<T><<<dim3(blocks_for(t.n), nrhs), 256, 0, st>>>(phis, phi, t.perm.p, t.n);
    HFMM_LAUNCH_CHECK();
  }
  return 0;
}

template FmmPlan<float>& get_plan<float>(Tree&, double, int);
template FmmPlan<double>& get_plan<double>(Tree&, double, int);
template FmmPlan<float>* find_plan<float>(Tree&, double, int);
template FmmPlan<double>* find_plan<double>(Tree&, double, int);
template void ensure_tuned<float>(Tree&, FmmPlan<float>&, int);
template void ensure_tuned<double>(Tree&, FmmPlan<double>&, int);
template void fmm_sorted<float>(const Tree&, FmmPlan<float>&, const float2*, float2*, int, const uint8_t*, bool,
                                hipStream_t, const int*, StageTimer*, const int32_t*, float2*,
                                const FmmWork<float>*, const float2*);
template void fmm_sorted<double>(const Tree&, FmmPlan<double>&, const double2*, double2*, int, const uint8_t*, bool,
                                 hipStream_t, const int*, StageTimer*, const int32_t*, double2*,
                                 const FmmWork<double>*, const double2*);
template void fmm_apply<float>(Tree&, double, int, const float2*, float2*, int, hipStream_t, StageTimer*);
template void fmm_apply<double>(Tree&, double, int, const double2*, double2*, int, hipStream_t, StageTimer*);
template void fmm_apply_dipole<float>(Tree&, double, int, const float2*, const double*, float2*, int, hipStream_t);
template void fmm_apply_dipole<double>(Tree&, double, int, const double2*, const double*, double2*, int,
                                       hipStream_t);
template size_t fmm_apply_scratch<float>(Tree&, double, int, const float2*, float2*, int, void*, size_t,
                                         hipStream_t);
template size_t fmm_apply_scratch<double>(Tree&, double, int, const double2*, double2*, int, void*, size_t,
                                          hipStream_t);

StageTimer::~StageTimer() {
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
}

int StageTimer::mark(int s, hipStream_t st, int from_ev) {
  hipEvent_t e;
  HFMM_HIP(hipEventCreate(&e));
  ev.push_back(e);
  stage.push_back(s);
  from.push_back(from_ev >= 0 ? from_ev : (int)ev.size() - 2);
  HFMM_HIP(hipEventRecord(e, st));
  return (int)ev.size() - 1;
}

void StageTimer::collect(float* ms, int nstage) {
  for (int i = 0; i < nstage; ++i) ms[i] = 0;
  for (hipEvent_t e : ev) HFMM_HIP(hipEventSynchronize(e));
  for (size_t i = 1; i < ev.size(); ++i) {
    float d = 0;
    HFMM_HIP(hipEventElapsedTime(&d, ev[from[i]], ev[i]));
    if (stage[i] >= 0 && stage[i] < nstage) ms[stage[i]] += d;
  }
}

}  // namespace hfmm
