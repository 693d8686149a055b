// 3-D Helmholtz FMM on the oct-tree (Sec. 5.1.1 in 3-D, the kernel
// exp(i k r) / (4 pi r) of Sec. 5.2, the flow of Sec. 5.1.2).
//
// Expansions (the paper defers its 3-D expansions to a library; these follow
// from the addition theorem of the spherical Hankel function):
//   R_n^m(x) = j_n(k|x|) Y_n^m(x/|x|),  S_n^m(x) = h_n(k|x|) Y_n^m(x/|x|),
//   Y_n^m orthonormal with the Condon-Shortley phase, n <= p_l, all m;
//   P2M  M_nm = i k sum_j q_j conj(R_n^m(y_j - c)),  far field sum M_nm S_n^m(x - c)
//   L2P  phi(x) = sum L_nm R_n^m(x - c)
//   translations  T_{n'm',nm}(t) = 4 pi sum_l i^(n'+l-n) f_l(k|t|) conj(Y_l^(m'-m)(t/|t|))
//                                  * integral(conj(Y_n'^m') Y_l^(m'-m) Y_n^m),
//   f_l = j_l (M2M with t = parent - child centre, L2L with t = child -
//   parent centre) or h_l (M2L with t = target - source centre).
//
// Data layout in HBM: the expansions of a level are [box (Morton)][Kp] reals,
// Re of coefficient n^2+n+m at n^2+n+m, Im at P2 + n^2+n+m (P2 = (p_l+1)^2),
// zero up to Kp = 2 P2 rounded up to 16.  Every translation is then a real
// matrix product on the matrix cores, A = [[Re T, -Im T], [Im T, Re T]]:
//   M2M  parent = [A_0 .. A_7] x (its 8 children's vectors, contiguous in
//        Morton order): one product with K = 8 Kp_child;
//   L2L  (the 8 children's vectors, contiguous) += [A_0; ..; A_7] x parent;
//   M2L  for the 8 parity classes of target boxes, the 189 offsets of the
//        class's interaction list, each a product over all targets of the
//        class (sources outside the domain read zero).
// The leaf kernels build R_n^m from solid harmonics: with u = k (x - c),
// s = |u|, j_n(s) = s^n jh_n(s) and s^n Y_n^m = Rh_n^m(u_z, s^2) (u_x + i u_y)^m,
// where jh_n (a power series in s^2, then the downward three-term
// recurrence) and Rh_n^m (the normalised Legendre recurrence times powers of
// s) are polynomials: no division, no special case at the box centre.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "devutil.h"
#include "fmm3.h"
#include "special.h"
#include "tree.h"

namespace hfmm {

namespace {

constexpr double kPi3 = 3.14159265358979323846;
constexpr int kMaxP3 = 20;  // largest order of any level
// Taylor terms of the FP64 near-field cosine and sine: 7, 10 or 13, the
// fewest whose first omitted term is below 1e-17 at the largest k r (<= 2)
constexpr int kTaylorMax3 = 13;

typedef float f32x4_3 __attribute__((ext_vector_type(4)));
typedef double f64x4_3 __attribute__((ext_vector_type(4)));
template <class T> struct Acc3;
template <> struct Acc3<float> { typedef f32x4_3 type; };
template <> struct Acc3<double> { typedef f64x4_3 type; };
__device__ __forceinline__ f32x4_3 mfma3(float a, float b, f32x4_3 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4_3 mfma3(double a, double b, f64x4_3 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// row of the 16x16 accumulator in register q of lane group kq = lane/16
template <class T> __device__ __forceinline__ int acc_row(int kq, int q);
template <> __device__ __forceinline__ int acc_row<float>(int kq, int q) { return 4 * kq + q; }
template <> __device__ __forceinline__ int acc_row<double>(int kq, int q) { return 4 * q + kq; }

template <class T> struct Vec4;
template <> struct Vec4<float> { typedef float4 type; };
template <> struct Vec4<double> { typedef double4 type; };

__device__ __forceinline__ void sincosT(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void sincosT(double x, double* s, double* c) { sincos(x, s, c); }

// ------------------------------------------------------------------ tree
__global__ void k3_morton(const double* __restrict__ xyz, int n, double x0, double y0, double z0, double side,
                          int L, uint32_t* __restrict__ keys, int32_t* __restrict__ vals, int* __restrict__ bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
  const bool ok = isfinite(x) && isfinite(y) && isfinite(z) && x >= x0 && x <= x0 + side && y >= y0 &&
                  y <= y0 + side && z >= z0 && z <= z0 + side;
  if (!ok) bad[0] = 1;
  const int nb = 1 << L;
  int ix = 0, iy = 0, iz = 0;
  if (ok) {
    ix = min(max((int)floor((x - x0) / side * nb), 0), nb - 1);
    iy = min(max((int)floor((y - y0) / side * nb), 0), nb - 1);
    iz = min(max((int)floor((z - z0) / side * nb), 0), nb - 1);
  }
  keys[i] = morton3((uint32_t)ix, (uint32_t)iy, (uint32_t)iz);
  vals[i] = i;
}

__global__ void k3_finalize(const double* __restrict__ xyz, const uint32_t* __restrict__ skeys,
                            const int32_t* __restrict__ perm, int n, double x0, double y0, double z0, double lside,
                            double4* __restrict__ rel64, float4* __restrict__ rel32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int o = perm[i];
  const uint32_t key = skeys[i];
  const double cx = x0 + (compact3(key) + 0.5) * lside;
  const double cy = y0 + (compact3(key >> 1) + 0.5) * lside;
  const double cz = z0 + (compact3(key >> 2) + 0.5) * lside;
  const double rx = xyz[3 * o] - cx, ry = xyz[3 * o + 1] - cy, rz = xyz[3 * o + 2] - cz;
  rel64[i] = make_double4(rx, ry, rz, 0.0);
  rel32[i] = make_float4((float)rx, (float)ry, (float)rz, 0.f);
}

// ------------------------------------------------------------------ leaf kernels
template <class T>
struct Leaf3Args {
  const typename Vec4<T>::type* rel;  // sorted points minus leaf centre
  const cplx<T>* qs;                  // sorted charges (P2M, P2P)
  const cplx<T>* near;                // near field, sorted (L2P)
  cplx<T>* near_out;                  // (P2P)
  const int32_t* perm;                // (L2P)
  const int32_t* off;                 // leaf offsets
  T* E;                               // leaf-level M (P2M) or L (L2P)
  cplx<T>* out;                       // caller order (L2P)
  const T* rec;                       // (a, b) of the Legendre recurrence, then Q_m^m
  int p, P2, Kp, nser, L;
  int cp;                             // P2M: points per LDS chunk
  T k, h;                             // wavenumber, leaf side (P2P)
  // FP64 P2P: when every near pair has k r <= 2, cos(k r) and sin(k r)/(k r)
  // as Taylor polynomials in y = (k r)^2 with ntay terms (0: library sincos)
  int ntay;
  double tc[16], ts[16];
};

// jh_n(s) = j_n(s) / s^n for n = 0..p into col[n * 64]: the power series
// jh_n = 1/(2n+1)!! sum_t (-s^2/2)^t / (t! (2n+3)(2n+5)...(2n+2t+1)) at n = p
// and p - 1 (K terms, by Horner), then jh_{n-1} = (2n+1) jh_n - s^2 jh_{n+1}.
template <class T>
__device__ __forceinline__ T jh_series(int n, int K, T s2) {
  const T y = T(0.5) * s2;
  T S = T(1);
  for (int t = K; t >= 1; --t) S = fmaT(-y / (T(t) * T(2 * n + 2 * t + 1)), S, T(1));
  T df = T(1);
  for (int i = 3; i <= 2 * n + 1; i += 2) df *= T(i);
  return S / df;
}
template <class T>
__device__ __forceinline__ void jh_all(int p, int K, T s2, T* col) {
  col[p * 64] = jh_series<T>(p, K, s2);
  if (p >= 1) col[(p - 1) * 64] = jh_series<T>(p - 1, K, s2);
  for (int n = p - 1; n >= 1; --n) col[(n - 1) * 64] = T(2 * n + 1) * col[n * 64] - s2 * col[(n + 1) * 64];
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// P2M: one wave per leaf, in chunks of CP points, two phases.
// 1. A lane per point writes its column of a table in LDS (row stride CP + 1):
//    jh_n (n <= p), jh_n Rh_n^m for m <= n (so that R_n^m = that times
//    (u_x + i u_y)^m), the powers (u_x + i u_y)^m and the charge.
// 2. A lane per coefficient pair (n, m) and (n, -m), m >= 0 (G lanes per pair
//    when the pairs are few, G a power of two), sums over the chunk's points:
//    M_nm += q conj(R_n^m), M_n,-m += (-1)^m q R_n^m; the G lanes of a pair
//    add up by shuffles and one of them adds to the leaf's sums in LDS.
template <class T>
__global__ __launch_bounds__(64) void k3_p2m(Leaf3Args<T> a) {
  extern __shared__ __align__(16) unsigned char p2m_smem[];
  T* acc = reinterpret_cast<T*>(p2m_smem);   // 2 P2
  T* tab = acc + 2 * a.P2;                    // [E][CP + 1]
  const int p = a.p, CP = a.cp, S = CP + 1;
  const int npair = (p + 1) * (p + 2) / 2;
  T* tjh = tab;                               // rows 0..p
  T* tjr = tab + (p + 1) * S;                 // rows tri(n, m)
  T* twr = tjr + npair * S;                   // rows m
  T* twi = twr + (p + 1) * S;
  T* tq = twi + (p + 1) * S;                  // 2 rows
  const int leaf = blockIdx.x, lane = threadIdx.x;
  const int b0 = a.off[leaf], b1 = a.off[leaf + 1];
  for (int c = lane; c < 2 * a.P2; c += 64) acc[c] = T(0);
  const T* qmm = a.rec + (p + 1) * (p + 2);
  int G = 1;
  while (G * 2 * npair <= 64) G *= 2;
  for (int base = b0; base < b1; base += CP) {
    const int cnt = min(CP, b1 - base);
    __syncthreads();
    if (lane < cnt) {
      const int i = base + lane;
      const typename Vec4<T>::type r = a.rel[i];
      const cplx<T> q = a.qs[i];
      const T ux = a.k * r.x, uy = a.k * r.y, uz = a.k * r.z;
      const T s2 = ux * ux + uy * uy + uz * uz;
      // jh_n by the series at p and p - 1, then downward
      tjh[p * S + lane] = jh_series<T>(p, a.nser, s2);
      if (p >= 1) tjh[(p - 1) * S + lane] = jh_series<T>(p - 1, a.nser, s2);
      for (int n = p - 1; n >= 1; --n)
        tjh[(n - 1) * S + lane] = T(2 * n + 1) * tjh[n * S + lane] - s2 * tjh[(n + 1) * S + lane];
      cplx<T> wm = mk<T>(1, 0);
      for (int m = 0; m <= p; ++m) {
        if (m > 0) wm = mk<T>(wm.x * ux - wm.y * uy, wm.x * uy + wm.y * ux);
        twr[m * S + lane] = wm.x;
        twi[m * S + lane] = wm.y;
        T r2 = 0, r1 = qmm[m];
        for (int n = m; n <= p; ++n) {
          if (n > m) {
            const T* ab = a.rec + 2 * (n * (n + 1) / 2 + m);
            const T rn = ab[0] * (uz * r1 - ab[1] * s2 * r2);
            r2 = r1;
            r1 = rn;
          }
          tjr[(n * (n + 1) / 2 + m) * S + lane] = tjh[n * S + lane] * r1;
        }
      }
      tq[lane] = q.x;
      tq[S + lane] = q.y;
    }
    __syncthreads();
    for (int base_pair = 0; base_pair < npair; base_pair += 64 / G) {
      const int pr = base_pair + lane / G, part = lane % G;
      const bool on = pr < npair;
      int n = 0;
      if (on)
        while ((n + 1) * (n + 2) / 2 <= pr) ++n;
      const int m = on ? pr - n * (n + 1) / 2 : 0;
      T pr_r = 0, pr_i = 0, ng_r = 0, ng_i = 0;
      if (on) {
        const T* jr = tjr + pr * S;
        const T* wr = twr + m * S;
        const T* wi = twi + m * S;
        for (int j = part; j < cnt; j += G) {
          const T b = jr[j];
          const T bx = b * wr[j], by = b * wi[j];
          const T qx = tq[j], qy = tq[S + j];
          pr_r += qx * bx + qy * by;
          pr_i += qy * bx - qx * by;
          ng_r += qx * bx - qy * by;
          ng_i += qx * by + qy * bx;
        }
      }
      for (int o = 1; o < G; o <<= 1) {
        pr_r += __shfl_xor(pr_r, o);
        pr_i += __shfl_xor(pr_i, o);
        ng_r += __shfl_xor(ng_r, o);
        ng_i += __shfl_xor(ng_i, o);
      }
      if (on && part == 0) {
        const int c = n * n + n + m;
        acc[c] += pr_r;
        acc[a.P2 + c] += pr_i;
        if (m > 0) {
          const T sg = (m & 1) ? T(-1) : T(1);
          acc[c - 2 * m] += sg * ng_r;
          acc[a.P2 + c - 2 * m] += sg * ng_i;
        }
      }
    }
  }
  __syncthreads();
  T* out = a.E + (size_t)leaf * a.Kp;
  for (int c = lane; c < a.Kp; c += 64) {
    // times i k
    T v = T(0);
    if (c < a.P2) v = -a.k * acc[a.P2 + c];
    else if (c < 2 * a.P2) v = a.k * acc[c - a.P2];
    out[c] = v;
  }
}

// L2P: one wave per leaf, one lane per point; the leaf's local expansion in
// LDS; adds the near field and writes caller order.
template <class T>
__global__ __launch_bounds__(64) void k3_l2p(Leaf3Args<T> a) {
  __shared__ T jh[(kMaxP3 + 1) * 64];
  __shared__ T Ls[2 * (kMaxP3 + 1) * (kMaxP3 + 1)];
  const int leaf = blockIdx.x, lane = threadIdx.x;
  const int b0 = a.off[leaf], b1 = a.off[leaf + 1];
  if (b0 == b1) return;
  const T* src = a.E + (size_t)leaf * a.Kp;
  for (int c = lane; c < 2 * a.P2; c += 64) Ls[c] = src[c];
  __syncthreads();
  const T* qmm = a.rec + (a.p + 1) * (a.p + 2);
  for (int base = b0; base < b1; base += 64) {
    const int i = base + lane;
    const bool v = i < b1;
    typename Vec4<T>::type r = a.rel[v ? i : b0];
    const T ux = a.k * r.x, uy = a.k * r.y, uz = a.k * r.z;
    const T s2 = ux * ux + uy * uy + uz * uz;
    jh_all<T>(a.p, a.nser, s2, jh + lane);
    T ar = 0, ai = 0;
    cplx<T> wm = mk<T>(1, 0);
    for (int m = 0; m <= a.p; ++m) {
      if (m > 0) wm = mk<T>(wm.x * ux - wm.y * uy, wm.x * uy + wm.y * ux);
      T r2 = 0, r1 = qmm[m];
      const T sg = (m & 1) ? T(-1) : T(1);
      for (int n = m; n <= a.p; ++n) {
        if (n > m) {
          const T* ab = a.rec + 2 * (n * (n + 1) / 2 + m);
          const T rn = ab[0] * (uz * r1 - ab[1] * s2 * r2);
          r2 = r1;
          r1 = rn;
        }
        const T jr = jh[n * 64 + lane] * r1;
        const T bx = jr * wm.x, by = jr * wm.y;
        const int c = n * n + n + m;
        const T lr = Ls[c], li = Ls[a.P2 + c];
        ar += lr * bx - li * by;
        ai += lr * by + li * bx;
        if (m > 0) {
          // R_n^-m = (-1)^m conj(R_n^m)
          const T mr = Ls[c - 2 * m], mi = Ls[a.P2 + c - 2 * m];
          ar += sg * (mr * bx + mi * by);
          ai += sg * (mi * bx - mr * by);
        }
      }
    }
    if (v) {
      const cplx<T> nf = a.near[i];
      a.out[a.perm[i]] = mk<T>(nf.x + ar, nf.y + ai);
    }
  }
}

// One pair of the near field: G(r) r 4 pi = (cos k r + i sin k r) / r, zero
// at r = 0.  FP32: the hardware reciprocal square root and the hardware sine
// and cosine (arguments in turns, k r / 2 pi below a few turns here); FP64:
// IEEE square root, division and sincos.
__device__ __forceinline__ void pair3(float r2, float k, float k2pi, float& gr, float& gi) {
  const float inv = r2 > 0.f ? __builtin_amdgcn_rsqf(r2) : 0.f;
  const float t = r2 * inv * k2pi;
  gr = __builtin_amdgcn_cosf(t) * inv;
  gi = __builtin_amdgcn_sinf(t) * inv;
}
__device__ __forceinline__ void pair3(double r2, double k, double, double& gr, double& gi) {
  const double r = sqrt(r2);
  const double inv = r2 > 0.0 ? 1.0 / r : 0.0;
  double sn, cs;
  sincos(k * r, &sn, &cs);
  gr = cs * inv;
  gi = sn * inv;
}
// FP64 with the Taylor form: 1/r from the hardware reciprocal square root and
// two Newton steps, cos(k r) = C(y) and sin(k r)/r = k S(y), y = k^2 r^2.
template <int NT>
__device__ __forceinline__ void pair3_taylor(double r2, double k, double k2, const double* tc, const double* ts,
                                             double& gr, double& gi) {
  double y0 = __builtin_amdgcn_rsq(r2);
  y0 = y0 * (1.5 - 0.5 * r2 * y0 * y0);
  y0 = y0 * (1.5 - 0.5 * r2 * y0 * y0);
  const bool nz = r2 > 0.0;
  const double inv = nz ? y0 : 0.0;
  const double y = k2 * r2;
  double c = tc[NT - 1], sv = ts[NT - 1];
#pragma unroll
  for (int n = NT - 2; n >= 0; --n) {
    c = fma(c, y, tc[n]);
    sv = fma(sv, y, ts[n]);
  }
  gr = c * inv;
  gi = nz ? k * sv : 0.0;
}

// P2P: one wave per target leaf; a leaf of at most 32 points gives each
// target 2 lanes (even and odd sources, summed by a lane swap at the end),
// a larger one a lane per target, 64 targets per pass.  The 27
// neighbouring leaves' points are staged through LDS 64 at a time.  Offsets
// between leaf centres are whole multiples of the leaf side, so the
// difference of two points is formed from leaf-relative coordinates.
template <class T, int NT>
__global__ __launch_bounds__(64) void k3_p2p(Leaf3Args<T> a) {
  typedef typename Vec4<T>::type V;
  __shared__ V sp[64];
  __shared__ cplx<T> sq[64];
  const int leaf = xcd_swizzle(blockIdx.x, gridDim.x), lane = threadIdx.x;
  const int t0 = a.off[leaf], t1 = a.off[leaf + 1];
  if (t0 == t1) return;
  const int bx = (int)compact3((uint32_t)leaf), by = (int)compact3((uint32_t)leaf >> 1),
            bz = (int)compact3((uint32_t)leaf >> 2);
  const int nb = 1 << a.L;
  const T inv4pi = T(1.0 / (4.0 * kPi3)), k2pi = T(double(a.k) / (2.0 * kPi3));
  const bool two = t1 - t0 <= 32;
  const int G = two ? 2 : 1, sub = two ? (lane & 1) : 0, tl = two ? (lane >> 1) : lane;
  const int per = 64 / G;
  for (int tb = t0; tb < t1; tb += per) {
    const int i = tb + tl;
    const bool v = i < t1;
    const V rt = a.rel[v ? i : t0];
    T ar = 0, ai = 0;
    for (int nbi = 0; nbi < 27; ++nbi) {
      const int dx = nbi % 3 - 1, dy = (nbi / 3) % 3 - 1, dz = nbi / 9 - 1;
      const int sx = bx + dx, sy = by + dy, sz = bz + dz;
      if (sx < 0 || sy < 0 || sz < 0 || sx >= nb || sy >= nb || sz >= nb) continue;
      const int s = (int)morton3((uint32_t)sx, (uint32_t)sy, (uint32_t)sz);
      const int s0 = a.off[s], s1 = a.off[s + 1];
      // target centre minus source centre
      const T ox = T(-dx) * a.h, oy = T(-dy) * a.h, oz = T(-dz) * a.h;
      const T cx = rt.x + ox, cy = rt.y + oy, cz = rt.z + oz;
      for (int sb = s0; sb < s1; sb += 64) {
        __syncthreads();
        const int j = sb + lane;
        if (j < s1) {
          sp[lane] = a.rel[j];
          sq[lane] = a.qs[j];
        }
        __syncthreads();
        const int cnt = min(64, s1 - sb);
        for (int jj = sub; jj < cnt; jj += G) {
          const V ps = sp[jj];
          const T ddx = cx - ps.x, ddy = cy - ps.y, ddz = cz - ps.z;
          const T r2 = ddx * ddx + ddy * ddy + ddz * ddz;
          T gr, gi;
          if constexpr (NT > 0)
            pair3_taylor<NT>(r2, a.k, a.k * a.k, a.tc, a.ts, gr, gi);
          else
            pair3(r2, a.k, k2pi, gr, gi);
          const cplx<T> qq = sq[jj];
          ar += qq.x * gr - qq.y * gi;
          ai += qq.x * gi + qq.y * gr;
        }
      }
    }
    if (two) {
      ar += __shfl_xor(ar, 1);
      ai += __shfl_xor(ai, 1);
    }
    if (v && sub == 0) a.near_out[i] = mk<T>(ar * inv4pi, ai * inv4pi);
  }
}

template <class T>
__global__ void k3_gather(const cplx<T>* __restrict__ q, const int32_t* __restrict__ perm, int n,
                          cplx<T>* __restrict__ qs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) qs[i] = q[perm[i]];
}

// ------------------------------------------------------------------ translations on MFMA
// C[:, col] (+)= A x B[:, col] over 16-row tiles of A (RT of them) and 4-k
// steps (KS), A laid out per lane: A_frag[rt][ks][lane] = A[16 rt + lane%16][4 ks + lane/16].
// A block has 4 waves, each with kNC3 column tiles of 16 and up to RG row
// tiles (grid.y walks the row groups; RG = 8 in FP32, 4 in FP64).  M2L mode:
// grid.z is the parity class of the target boxes, a column is a class
// member, and the 189 offsets of the class's interaction list are summed
// (table slot (dx+3)*49 + (dy+3)*7 + dz+3, the offsets from `offs`).
// The (offset, 4-k chunk) iterations are one flat loop: the 4 waves share
// each A chunk through LDS (double-buffered), and the next chunk's A and B
// loads are in flight while the current chunk's MFMAs run.
constexpr int kNC3 = 2, kColsPerBlock3 = 4 * kNC3 * 16;
// row tiles per block: FP32 8; FP64 7 for launches of 7 or 14 row tiles
// (Kp = 112: one row group, so the sources are gathered once; 2 waves per
// SIMD, yet 4.23 -> 3.49 ms for the M2L of the 2^20 apply), else 4
template <class T>
int pick_rg(int RT) {
  return sizeof(T) == 8 ? (RT % 7 == 0 ? 7 : 4) : 8;
}

template <class T>
struct Tr3Args {
  const T* A;
  const T* B;
  T* C;
  const int* offs;  // M2L: [8][189] packed (dx+3) | (dy+3) << 4 | (dz+3) << 8
  int RT, KS, ncols, crows, accumulate;
  int KSe;  // k steps that hold data (<= KS; the rest of A and B is zero padding)
  int64_t ldb, ldc, aslot;  // column strides; M2L: table stride per offset slot
  int m2l, nb, h;           // M2L: boxes per axis, nb / 2
  // groups: grid.z = 8 S (M2L) or S; group g takes iterations [n g / S,
  // n (g + 1) / S) of the flat (offset, k chunk) loop of n iterations and,
  // for S > 1, stores its partial sum at part + g pstride (a later pass
  // adds the S partials)
  int S;
  T* part;
  int64_t pstride;
};

template <class T, int RG>
__global__ __launch_bounds__(256) void k3_trans(Tr3Args<T> a) {
  typedef typename Acc3<T>::type V4;
  constexpr int ACH = RG * 4 * 64;    // A values per chunk
  constexpr int APT = ACH / 256;      // per thread
  __shared__ __align__(32) T abuf[2][ACH];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, j = lane & 15, kq = lane >> 4;
  const int rg0 = blockIdx.y * RG;
  const int nrt = min(RG, a.RT - rg0);
  const int par = a.m2l ? (blockIdx.z & 7) : 0, grp = a.m2l ? (blockIdx.z >> 3) : blockIdx.z;
  const int px = par & 1, py = (par >> 1) & 1, pz = (par >> 2) & 1;
  int tx[kNC3], ty[kNC3], tz[kNC3], obox[kNC3];
  bool colv[kNC3];
#pragma unroll
  for (int c = 0; c < kNC3; ++c) {
    const int col = (blockIdx.x * 4 + wave) * (kNC3 * 16) + c * 16 + j;
    colv[c] = col < a.ncols;
    const int cc = colv[c] ? col : 0;
    if (a.m2l) {
      tx[c] = 2 * (cc % a.h) + px;
      ty[c] = 2 * ((cc / a.h) % a.h) + py;
      tz[c] = 2 * (cc / (a.h * a.h)) + pz;
      obox[c] = (int)morton3((uint32_t)tx[c], (uint32_t)ty[c], (uint32_t)tz[c]);
    } else {
      tx[c] = ty[c] = tz[c] = 0;
      obox[c] = cc;
    }
  }
  const int nch = (a.KSe + 3) >> 2;
  const int nall = (a.m2l ? 189 : 1) * nch;
  const int it_lo = (int)((int64_t)nall * grp / a.S), it_hi = (int)((int64_t)nall * (grp + 1) / a.S);
  const int* po = a.offs + par * 189;
  // source columns of offset oi (recomputed only when the offset changes)
  const T* Ab;
  const T* bc[kNC3];
  bool bv[kNC3];
  auto locate = [&](int oi) {
    if (a.m2l) {
      const int e = po[oi];
      const int dx = (e & 15) - 3, dy = ((e >> 4) & 15) - 3, dz = (e >> 8) - 3;
      Ab = a.A + (size_t)((dx + 3) * 49 + (dy + 3) * 7 + (dz + 3)) * a.aslot;
#pragma unroll
      for (int c = 0; c < kNC3; ++c) {
        const int sx = tx[c] - dx, sy = ty[c] - dy, sz = tz[c] - dz;
        bv[c] = colv[c] && sx >= 0 && sy >= 0 && sz >= 0 && sx < a.nb && sy < a.nb && sz < a.nb;
        const int sb = bv[c] ? (int)morton3((uint32_t)sx, (uint32_t)sy, (uint32_t)sz) : 0;
        bc[c] = a.B + (size_t)sb * a.ldb;
      }
    } else {
      Ab = a.A;
#pragma unroll
      for (int c = 0; c < kNC3; ++c) {
        bv[c] = colv[c];
        bc[c] = a.B + (size_t)obox[c] * a.ldb;
      }
    }
  };
  // A chunk element e = i * 256 + tid of this thread: row tile i, k step
  // u = tid / 64, lane ln = tid % 64; it goes to LDS at (i * 64 + ln) * 4 + u,
  // so that a lane reads its 4 k steps of a row tile with one 16-byte load
  const int lbase = (tid & 63) * 4 + (tid >> 6);
  const size_t abase = (size_t)rg0 * a.KS * 64 + tid;
  const size_t astride = (size_t)a.KS * 64;
  auto loadA = [&](int k0, T (&ra)[APT]) {
    const T* p0 = Ab + abase + (size_t)k0 * 64;
#pragma unroll
    for (int i = 0; i < APT; ++i) ra[i] = i < nrt ? p0[i * astride] : T(0);
  };
  auto loadB = [&](int k0, T (&rb)[4][kNC3]) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int c = 0; c < kNC3; ++c) rb[u][c] = bv[c] ? bc[c][(k0 + u) * 4 + kq] : T(0);
  };
  typedef typename Vec4<T>::type A4;
  V4 acc[RG][kNC3];
#pragma unroll
  for (int r = 0; r < RG; ++r)
#pragma unroll
    for (int c = 0; c < kNC3; ++c) acc[r][c] = V4{0, 0, 0, 0};

  T ra[APT], rb[4][kNC3], rbn[4][kNC3];
  int oi = it_lo / nch, ch = it_lo - oi * nch, chc = ch;
  locate(oi);
  // a wave none of whose columns has a source in this iteration skips its
  // MFMAs (it still stages A with the block)
  bool wv = __ballot(bv[0] | bv[1]) != 0;
  loadA(ch * 4, ra);
  loadB(ch * 4, rb);
#pragma unroll
  for (int i = 0; i < APT; ++i) abuf[0][i * 256 + lbase] = ra[i];
  __syncthreads();
  for (int it = it_lo; it < it_hi; ++it) {
    const int cur = (it - it_lo) & 1;
    const bool more = it + 1 < it_hi;
    bool wvn = false;
    if (more) {
      if (++ch == nch) {
        ch = 0;
        locate(++oi);
      }
      wvn = __ballot(bv[0] | bv[1]) != 0;
      loadA(ch * 4, ra);
      loadB(ch * 4, rbn);
    }
    // k steps of this chunk that hold data (the last chunk of a K that is
    // not a multiple of 16 skips the padding)
    const int lim = min(4, a.KSe - 4 * chc);
    if (wv) {
      const A4* ab4 = reinterpret_cast<const A4*>(abuf[cur]);
#pragma unroll
      for (int r = 0; r < RG; ++r)
        if (r < nrt) {
          const A4 av = ab4[r * 64 + lane];
          const T avu[4] = {av.x, av.y, av.z, av.w};
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (u < lim) {
#pragma unroll
              for (int c = 0; c < kNC3; ++c) acc[r][c] = mfma3(avu[u], rb[u][c], acc[r][c]);
            }
        }
    }
    wv = wvn;
    chc = ch;
    if (more) {
#pragma unroll
      for (int i = 0; i < APT; ++i) abuf[cur ^ 1][i * 256 + lbase] = ra[i];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < kNC3; ++c) rb[u][c] = rbn[u][c];
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < RG; ++r) {
    if (r >= nrt) continue;
#pragma unroll
    for (int c = 0; c < kNC3; ++c) {
      if (!colv[c]) continue;
      T* dst = (a.S > 1 ? a.part + grp * a.pstride : a.C) + (size_t)obox[c] * a.ldc;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = 16 * (rg0 + r) + acc_row<T>(kq, q);
        if (row < a.crows) dst[row] = a.accumulate ? dst[row] + acc[r][c][q] : acc[r][c][q];
      }
    }
  }
}

// C (+)= sum of the S partial sums (fixed order)
template <class T>
__global__ void k3_sum_parts(const T* __restrict__ part, int S, int64_t pstride, int accumulate, T* __restrict__ C) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= pstride) return;
  T s = part[i];
  for (int g = 1; g < S; ++g) s += part[g * pstride + i];
  C[i] = accumulate ? C[i] + s : s;
}

// Blocks of a translation launch (one group) and the groups that bring the
// launch to about 3 waves per SIMD (at most one per iteration, at most 63).
// (A 7-tile FP32 instance that fits 4 waves per SIMD, with 1024 blocks, was
// slower: 3.39 against 3.31 ms for the 2^20 apply.)
template <class T>
int trans_groups(int ncols, int RT, int nall, bool m2l) {
  const int rg = pick_rg<T>(RT);
  const int base = (m2l ? 8 : 1) * ((ncols + kColsPerBlock3 - 1) / kColsPerBlock3) * ((RT + rg - 1) / rg);
  int S = (768 + base - 1) / base;
  return std::max(1, std::min(S, std::min(63, nall)));
}

template <class T>
void launch_trans(Tr3Args<T> a, T* part, size_t part_n, hipStream_t stream) {
  HFMM_REQUIRE(a.KSe >= 1 && a.KSe <= a.KS, "fmm3: bad k-step count");
  const int nall = (a.m2l ? 189 : 1) * ((a.KSe + 3) / 4);
  a.S = trans_groups<T>(a.ncols, a.RT, nall, a.m2l != 0);
  a.part = part;
  const int rg = pick_rg<T>(a.RT);
  dim3 g((a.ncols + kColsPerBlock3 - 1) / kColsPerBlock3, (a.RT + rg - 1) / rg, (a.m2l ? 8 : 1) * a.S);
  const int acc = a.accumulate;
  if (a.S > 1) a.accumulate = 0;  // partials are stored
  HFMM_REQUIRE(a.S == 1 || (part != nullptr && (size_t)a.S * a.pstride <= part_n), "fmm3: partial-sum buffer too small");
  if constexpr (sizeof(T) == 8) {
    if (rg == 7)
      k3_trans<T, 7><<<g, 256, 0, stream>>>(a);
    else
      k3_trans<T, 4><<<g, 256, 0, stream>>>(a);
  }
  else
    k3_trans<T, 8><<<g, 256, 0, stream>>>(a);
  HFMM_LAUNCH_CHECK();
  if (a.S > 1) {
    k3_sum_parts<T><<<(unsigned)((a.pstride + 255) / 256), 256, 0, stream>>>(part, a.S, a.pstride, acc, a.C);
    HFMM_LAUNCH_CHECK();
  }
}

// ------------------------------------------------------------------ host tables
inline int tri(int n, int m) { return n * (n + 1) / 2 + m; }
inline int kpad(int P2) { return (2 * P2 + 15) / 16 * 16; }

// Theta_n^m(x), m >= 0, of Y_n^m = Theta_n^m(cos th) e^{i m ph} (orthonormal,
// Condon-Shortley phase) for n <= nmax: Q_m^m = (-1)^m sqrt((2m+1)!!/(4 pi (2m)!!)),
// Q_n^m = a_n^m (x Q_{n-1}^m - b_n^m Q_{n-2}^m), Theta = Q (1 - x^2)^(m/2).
void theta_table(int nmax, double x, std::vector<double>& out) {
  out.assign((size_t)tri(nmax, nmax) + 1, 0.0);
  const double s = std::sqrt(std::max(0.0, 1.0 - x * x));
  double qmm = 1.0 / std::sqrt(4.0 * kPi3), smm = 1.0;
  for (int m = 0; m <= nmax; ++m) {
    if (m > 0) {
      qmm *= -std::sqrt((2.0 * m + 1.0) / (2.0 * m));
      smm *= s;
    }
    double q2 = 0.0, q1 = qmm;
    out[tri(m, m)] = qmm * smm;
    for (int n = m + 1; n <= nmax; ++n) {
      const double an = std::sqrt((4.0 * n * n - 1.0) / (double(n) * n - double(m) * m));
      const double bn = std::sqrt(std::max(0.0, ((n - 1.0) * (n - 1.0) - double(m) * m) / (4.0 * (n - 1.0) * (n - 1.0) - 1.0)));
      const double qn = an * (x * q1 - bn * q2);
      out[tri(n, m)] = qn * smm;
      q2 = q1;
      q1 = qn;
    }
  }
}

inline double theta_signed(const std::vector<double>& th, int n, int m) {
  // Theta_n^-m = (-1)^m Theta_n^m
  return m >= 0 ? th[tri(n, m)] : ((-m) & 1 ? -th[tri(n, -m)] : th[tri(n, -m)]);
}

// Integrals of conj(Y_n'^m') Y_l^(m'-m) Y_n^m over the sphere by Gauss-Legendre
// in cos(theta) (exact: the integrand is a polynomial of degree <= 2 (po + pi))
// after the azimuthal integral (2 pi).
struct GauntTab {
  int po = 0, pi = 0, lmax = 0;
  std::vector<double> g;  // [(a * P2i + b) * (lmax + 1) + l]
};

GauntTab gaunt_table(int po, int pi) {
  GauntTab G;
  G.po = po;
  G.pi = pi;
  G.lmax = po + pi;
  const int P2o = (po + 1) * (po + 1), P2i = (pi + 1) * (pi + 1), nl = G.lmax + 1;
  G.g.assign((size_t)P2o * P2i * nl, 0.0);
  const int nq = G.lmax + 2;
  std::vector<double> xs, ws;
  gauss_legendre(nq, xs, ws);
  std::vector<std::vector<double>> th(nq);
  for (int q = 0; q < nq; ++q) theta_table(G.lmax, xs[q], th[q]);
  for (int n1 = 0; n1 <= po; ++n1)
    for (int m1 = -n1; m1 <= n1; ++m1)
      for (int n = 0; n <= pi; ++n)
        for (int m = -n; m <= n; ++m) {
          const int mu = m1 - m;
          for (int l = std::abs(n1 - n); l <= n1 + n; ++l) {
            if (((n1 + n + l) & 1) || std::abs(mu) > l) continue;
            double s = 0.0;
            for (int q = 0; q < nq; ++q)
              s += ws[q] * theta_signed(th[q], n1, m1) * theta_signed(th[q], l, mu) * theta_signed(th[q], n, m);
            G.g[((size_t)(n1 * n1 + n1 + m1) * P2i + (n * n + n + m)) * nl + l] = 2.0 * kPi3 * s;
          }
        }
  return G;
}

// T (P2o x P2i, row-major) for the shift t: f_l = j_l (regular) or h_l (singular).
void translation3(const GauntTab& G, double k, const double t[3], bool singular,
                  std::vector<std::complex<double>>& T) {
  const int P2o = (G.po + 1) * (G.po + 1), P2i = (G.pi + 1) * (G.pi + 1), nl = G.lmax + 1;
  const double r = std::sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
  const double kr = k * r, ph = std::atan2(t[1], t[0]);
  std::vector<double> th;
  theta_table(G.lmax, t[2] / r, th);
  std::vector<std::complex<double>> f(nl);
  for (int l = 0; l < nl; ++l)
    f[l] = std::complex<double>(std::sph_bessel(l, kr), singular ? std::sph_neumann(l, kr) : 0.0);
  // conj(Y_l^mu(t)) for all l, mu
  auto ycj = [&](int l, int mu) {
    const std::complex<double> e = std::polar(1.0, -mu * ph);
    return theta_signed(th, l, mu) * e;
  };
  const std::complex<double> ipow[4] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
  T.assign((size_t)P2o * P2i, 0.0);
  for (int n1 = 0; n1 <= G.po; ++n1)
    for (int m1 = -n1; m1 <= n1; ++m1)
      for (int n = 0; n <= G.pi; ++n)
        for (int m = -n; m <= n; ++m) {
          const int a = n1 * n1 + n1 + m1, b = n * n + n + m, mu = m1 - m;
          const double* g = &G.g[((size_t)a * P2i + b) * nl];
          std::complex<double> s = 0.0;
          for (int l = std::abs(n1 - n); l <= n1 + n; ++l) {
            if (g[l] == 0.0) continue;
            s += ipow[((n1 + l - n) % 4 + 4) % 4] * f[l] * ycj(l, mu) * g[l];
          }
          T[(size_t)a * P2i + b] = 4.0 * kPi3 * s;
        }
}

// Real form of T into the per-lane fragment layout, at (row0, col0) of a
// matrix with KS k-steps.
template <class T>
void put_frag(const std::vector<std::complex<double>>& Tm, int P2o, int P2i, int row0, int col0, int KS, T* dst,
              double& amax) {
  auto set = [&](int r, int c, double v) {
    dst[((size_t)(r >> 4) * KS + (c >> 2)) * 64 + (r & 15) + 16 * (c & 3)] = T(v);
    amax = std::max(amax, std::fabs(v));
  };
  for (int i = 0; i < P2o; ++i)
    for (int jj = 0; jj < P2i; ++jj) {
      const std::complex<double> z = Tm[(size_t)i * P2i + jj];
      set(row0 + i, col0 + jj, z.real());
      set(row0 + i, col0 + P2i + jj, -z.imag());
      set(row0 + P2o + i, col0 + jj, z.imag());
      set(row0 + P2o + i, col0 + P2i + jj, z.real());
    }
}

template <class T>
struct Plan3 : Plan3Base {
  int L = 0, pl = 0, nser = 0;
  std::vector<int> ord, P2, Kp;
  std::vector<size_t> eoff, m2l_off, m2m_off, l2l_off;
  DevBuf<T> M, Lc, A, rec;
  DevBuf<int> offs;
  DevBuf<T> part;
  DevBuf<cplx<T>> qs, near;
  hipEvent_t ev[6] = {};
  ~Plan3() override {
    for (auto e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

template <class T>
Plan3<T>& get_plan3(Tree3& t, double k, int p) {
  const auto key = std::make_tuple(k, p, sizeof(T) == 4 ? 1 : 0);
  auto it = t.plans.find(key);
  if (it != t.plans.end()) return static_cast<Plan3<T>&>(*it->second);
  auto pl = std::make_unique<Plan3<T>>();
  Plan3<T>& P = *pl;
  const int L = t.L;
  P.L = L;
  P.ord = fmm3_orders(t, k, p);
  P.P2.assign(L + 1, 0);
  P.Kp.assign(L + 1, 0);
  for (int l = 2; l <= L; ++l) {
    HFMM_REQUIRE(P.ord[l] <= kMaxP3, "fmm3_apply: an expansion order above 20 (lower p or k)");
    P.P2[l] = (P.ord[l] + 1) * (P.ord[l] + 1);
    P.Kp[l] = kpad(P.P2[l]);
  }
  P.pl = P.ord[L];
  // the leaf series: |k (y - c)| <= k sqrt(3)/2 h
  const double smax = k * std::sqrt(3.0) / 2.0 * t.leaf_side();
  HFMM_REQUIRE(smax <= 6.0, "fmm3_apply: k times the leaf half-diagonal must be <= 6");
  {
    const double y = 0.5 * smax * smax;
    double term = 1.0;
    int K = 0;
    while (K < 60) {
      ++K;
      term *= y / (K * (2.0 * K + 1.0));
      if (term < 1e-18) break;
    }
    P.nser = K + 1;
  }
  // expansions
  P.eoff.assign(L + 2, 0);
  size_t tot = 0;
  for (int l = 2; l <= L; ++l) {
    P.eoff[l] = tot;
    tot += ((size_t)1 << (3 * l)) * P.Kp[l];
  }
  P.M.alloc(tot);
  P.Lc.alloc(tot);
  // tables
  P.m2l_off.assign(L + 1, 0);
  P.m2m_off.assign(L + 1, 0);
  P.l2l_off.assign(L + 1, 0);
  size_t at = 0;
  for (int l = 2; l <= L; ++l) {
    P.m2l_off[l] = at;
    at += (size_t)343 * P.Kp[l] * P.Kp[l];
  }
  for (int l = 2; l < L; ++l) {
    P.m2m_off[l] = at;
    at += (size_t)P.Kp[l] * 8 * P.Kp[l + 1];
  }
  for (int l = 3; l <= L; ++l) {
    P.l2l_off[l] = at;
    at += (size_t)8 * P.Kp[l] * P.Kp[l - 1];
  }
  std::vector<T> hA(at, T(0));
  double amax = 0.0;
  std::vector<std::complex<double>> Tm;
  for (int l = 2; l <= L; ++l) {
    const double s = t.side_len / double(1 << l);
    const GauntTab G = gaunt_table(P.ord[l], P.ord[l]);
    const int KS = P.Kp[l] / 4;
    for (int dz = -3; dz <= 3; ++dz)
      for (int dy = -3; dy <= 3; ++dy)
        for (int dx = -3; dx <= 3; ++dx) {
          if (std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz))) <= 1) continue;
          const double tv[3] = {dx * s, dy * s, dz * s};
          translation3(G, k, tv, true, Tm);
          put_frag<T>(Tm, P.P2[l], P.P2[l], 0, 0, KS,
                      hA.data() + P.m2l_off[l] + (size_t)((dx + 3) * 49 + (dy + 3) * 7 + (dz + 3)) * P.Kp[l] * P.Kp[l],
                      amax);
        }
  }
  for (int l = 2; l < L; ++l) {
    const double sc = t.side_len / double(1 << (l + 1));
    const GauntTab G = gaunt_table(P.ord[l], P.ord[l + 1]);
    const int KS = 8 * P.Kp[l + 1] / 4;
    for (int oc = 0; oc < 8; ++oc) {
      // parent centre minus child centre
      const double tv[3] = {-((oc & 1) - 0.5) * sc, -(((oc >> 1) & 1) - 0.5) * sc, -(((oc >> 2) & 1) - 0.5) * sc};
      translation3(G, k, tv, false, Tm);
      put_frag<T>(Tm, P.P2[l], P.P2[l + 1], 0, oc * P.Kp[l + 1], KS, hA.data() + P.m2m_off[l], amax);
    }
  }
  for (int l = 3; l <= L; ++l) {
    const double sc = t.side_len / double(1 << l);
    const GauntTab G = gaunt_table(P.ord[l], P.ord[l - 1]);
    const int KS = P.Kp[l - 1] / 4;
    for (int oc = 0; oc < 8; ++oc) {
      // child centre minus parent centre
      const double tv[3] = {((oc & 1) - 0.5) * sc, (((oc >> 1) & 1) - 0.5) * sc, (((oc >> 2) & 1) - 0.5) * sc};
      translation3(G, k, tv, false, Tm);
      put_frag<T>(Tm, P.P2[l], P.P2[l - 1], oc * P.Kp[l], 0, KS, hA.data() + P.l2l_off[l], amax);
    }
  }
  HFMM_REQUIRE(std::isfinite(amax) && (sizeof(T) == 8 || amax < 1e30),
               "fmm3_apply: translation entries out of range for this precision (lower p or raise k h)");
  P.A.upload(hA);
  // leaf recurrences: (a_n^m, b_n^m) for m <= n <= pl, then Q_m^m
  {
    const int pl_ = P.pl;
    std::vector<T> rec((size_t)(pl_ + 1) * (pl_ + 2) + pl_ + 1, T(0));
    for (int n = 0; n <= pl_; ++n)
      for (int m = 0; m <= n; ++m) {
        if (n > m) {
          rec[2 * tri(n, m)] = T(std::sqrt((4.0 * n * n - 1.0) / (double(n) * n - double(m) * m)));
          rec[2 * tri(n, m) + 1] =
              T(std::sqrt(std::max(0.0, ((n - 1.0) * (n - 1.0) - double(m) * m) / (4.0 * (n - 1.0) * (n - 1.0) - 1.0))));
        }
      }
    double qmm = 1.0 / std::sqrt(4.0 * kPi3);
    for (int m = 0; m <= pl_; ++m) {
      if (m > 0) qmm *= -std::sqrt((2.0 * m + 1.0) / (2.0 * m));
      rec[(size_t)(pl_ + 1) * (pl_ + 2) + m] = T(qmm);
    }
    P.rec.upload(rec);
  }
  {
    // the 189 interaction-list offsets of each parity class, d = target - source
    std::vector<int> offs;
    for (int par = 0; par < 8; ++par) {
      const int px = par & 1, py = (par >> 1) & 1, pz = (par >> 2) & 1;
      for (int dz = pz - 3; dz <= pz + 2; ++dz)
        for (int dy = py - 3; dy <= py + 2; ++dy)
          for (int dx = px - 3; dx <= px + 2; ++dx)
            if (std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz))) >= 2)
              offs.push_back((dx + 3) | ((dy + 3) << 4) | ((dz + 3) << 8));
    }
    if (offs.size() != 8 * 189) throw Error(HFMM_ERR_INTERNAL, "fmm3: interaction offsets are not 189 per class");
    P.offs.upload(offs);
  }
  {
    // partial sums of the translation launches split into groups
    size_t pmax = 0;
    for (int l = 2; l <= L; ++l) {
      const size_t outl = ((size_t)1 << (3 * l)) * P.Kp[l];
      const int h = 1 << (l - 1);
      size_t S = trans_groups<T>(h * h * h, P.Kp[l] / 16, 189 * (P.Kp[l] / 16), true);
      if (l < L) S = std::max<size_t>(S, trans_groups<T>(1 << (3 * l), P.Kp[l] / 16, P.Kp[l + 1] / 2, false));
      if (l > 2) S = std::max<size_t>(S, trans_groups<T>(1 << (3 * (l - 1)), 8 * P.Kp[l] / 16, P.Kp[l - 1] / 16, false));
      if (S > 1) pmax = std::max(pmax, S * outl);
    }
    if (pmax) P.part.alloc(pmax);
  }
  P.qs.alloc(t.n);
  P.near.alloc(t.n);
  for (auto& e : P.ev) HFMM_HIP(hipEventCreate(&e));
  Plan3<T>& ref = P;
  t.plans.emplace(key, std::move(pl));
  return ref;
}

}  // namespace

int tree3_depth(int64_t n, int leaf_size) {
  if (leaf_size <= 0) return 0;
  int L = 0;
  while ((double)leaf_size * std::pow(8.0, L) < (double)n) ++L;
  return std::max(2, L);
}

std::vector<int> fmm3_orders(const Tree3& t, double k, int p) {
  std::vector<int> o(t.L + 1);
  for (int l = 0; l <= t.L; ++l)
    o[l] = p + (int)std::floor(k * std::sqrt(3.0) * t.side_len / std::ldexp(1.0, l) / 2.0);
  return o;
}

std::unique_ptr<Tree3> build_tree3(const double* d_xyz, int64_t n, double x0, double y0, double z0, double side,
                                   int leaf_size, hipStream_t stream) {
  HFMM_REQUIRE(n >= 1, "build_tree3: n must be >= 1");
  HFMM_REQUIRE(n < (int64_t(1) << 30), "build_tree3: n must be below 2^30");
  HFMM_REQUIRE(std::isfinite(side) && side > 0, "build_tree3: side must be finite and > 0");
  HFMM_REQUIRE(std::isfinite(x0) && std::isfinite(y0) && std::isfinite(z0), "build_tree3: root corner must be finite");
  HFMM_REQUIRE(leaf_size >= 1, "build_tree3: leaf_size must be >= 1");
  HFMM_REQUIRE(d_xyz != nullptr, "build_tree3: d_xyz is NULL");
  auto t = std::make_unique<Tree3>();
  t->n = n;
  t->L = tree3_depth(n, leaf_size);
  HFMM_REQUIRE(t->L <= 7, "build_tree3: depth above 7 (raise leaf_size)");
  t->x0 = x0;
  t->y0 = y0;
  t->z0 = z0;
  t->side_len = side;
  t->leaf_size = leaf_size;
  t->nleaves = int64_t(1) << (3 * t->L);
  const int N = (int)n, blocks = (N + 255) / 256;
  DevBuf<uint32_t> keys(N);
  DevBuf<int32_t> vals(N);
  DevBuf<int> bad(1);
  HFMM_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), stream));
  k3_morton<<<blocks, 256, 0, stream>>>(d_xyz, N, x0, y0, z0, side, t->L, keys.p, vals.p, bad.p);
  HFMM_LAUNCH_CHECK();
  int hbad = 0;
  HFMM_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, stream));
  HFMM_HIP(hipStreamSynchronize(stream));
  HFMM_REQUIRE(hbad == 0, "build_tree3: a coordinate is non-finite or outside the root cube");
  radix_sort_pairs(keys, vals, N, 3 * t->L, stream);
  t->perm = std::move(vals);
  t->rel64.alloc(N);
  t->rel32.alloc(N);
  k3_finalize<<<blocks, 256, 0, stream>>>(d_xyz, keys.p, t->perm.p, N, x0, y0, z0, t->leaf_side(), t->rel64.p,
                                          t->rel32.p);
  HFMM_LAUNCH_CHECK();
  t->leaf_off.alloc(t->nleaves + 1);
  leaf_bounds(keys.p, N, t->nleaves, t->leaf_off.p, stream);
  std::vector<int32_t> off(t->nleaves + 1);
  HFMM_HIP(hipMemcpyAsync(off.data(), t->leaf_off.p, (t->nleaves + 1) * sizeof(int32_t), hipMemcpyDeviceToHost,
                          stream));
  HFMM_HIP(hipStreamSynchronize(stream));
  int mx = 0;
  for (int64_t b = 0; b < t->nleaves; ++b) mx = std::max(mx, off[b + 1] - off[b]);
  t->max_leaf = mx;
  if (off[t->nleaves] != N) throw Error(HFMM_ERR_INTERNAL, "build_tree3: leaf offsets do not sum to n");
  HFMM_HIP(hipStreamCreateWithFlags(&t->side, hipStreamNonBlocking));
  HFMM_HIP(hipEventCreateWithFlags(&t->fork, hipEventDisableTiming | hipEventDisableSystemFence));
  HFMM_HIP(hipEventCreateWithFlags(&t->join, hipEventDisableTiming | hipEventDisableSystemFence));
  return t;
}

Tree3::~Tree3() {
  if (side) {
    (void)hipStreamSynchronize(side);
    (void)hipStreamDestroy(side);
  }
  if (fork) (void)hipEventDestroy(fork);
  if (join) (void)hipEventDestroy(join);
}

template <class T>
void fmm3_apply(Tree3& t, double k, int p, const cplx<T>* d_q, cplx<T>* d_phi, hipStream_t stream,
                float* stage_ms) {
  HFMM_REQUIRE(t.L >= 2, "fmm3_apply: the tree needs depth >= 2");
  Plan3<T>& P = get_plan3<T>(t, k, p);
  const int L = t.L, N = (int)t.n;
  const int nleaves = (int)t.nleaves;
  Leaf3Args<T> la{};
  if constexpr (sizeof(T) == 8) la.rel = t.rel64.p;
  else la.rel = t.rel32.p;
  la.qs = P.qs.p;
  la.near = P.near.p;
  la.near_out = P.near.p;
  la.perm = t.perm.p;
  la.off = t.leaf_off.p;
  la.out = d_phi;
  la.rec = P.rec.p;
  la.p = P.pl;
  la.P2 = P.P2[L];
  la.Kp = P.Kp[L];
  la.nser = P.nser;
  la.L = L;
  la.k = T(k);
  la.h = T(t.leaf_side());
  {
    // the largest k r of a near pair: opposite corners of a 2 x 2 x 2 block of leaves
    const double krmax = k * 2.0 * std::sqrt(3.0) * t.leaf_side();
    la.ntay = 0;
    if (krmax <= 2.0)
      for (int nt : {7, 10, kTaylorMax3}) {
        // first omitted cosine term x^(2 nt) / (2 nt)!
        double term = 1.0;
        for (int i = 1; i <= 2 * nt; ++i) term *= krmax / i;
        if (term < 1e-17 || nt == kTaylorMax3) {
          la.ntay = nt;
          break;
        }
      }
    double f = 1.0;  // (2n)! then (2n+1)!
    for (int n = 0; n < 16; ++n) {
      const double sg = (n & 1) ? -1.0 : 1.0;
      if (n > 0) f *= (2.0 * n - 1.0) * (2.0 * n);
      la.tc[n] = n < la.ntay ? sg / f : 0.0;
      la.ts[n] = n < la.ntay ? sg / (f * (2.0 * n + 1.0)) : 0.0;
    }
  }
  if (stage_ms) HFMM_HIP(hipEventRecord(P.ev[0], stream));
  // upward pass
  k3_gather<T><<<(N + 255) / 256, 256, 0, stream>>>(d_q, t.perm.p, N, P.qs.p);
  HFMM_LAUNCH_CHECK();
  // the far-field chain on the side stream beside the P2P (serial when timed)
  const bool overlap = !stage_ms && t.side;
  hipStream_t fs = overlap ? t.side : stream;
  if (overlap) {
    HFMM_HIP(hipEventRecord(t.fork, stream));
    HFMM_HIP(hipStreamWaitEvent(fs, t.fork, 0));
  }
  la.E = P.M.p + P.eoff[L];
  {
    // P2M table: jh (p + 1 rows), jh Rh (pairs), w^m (2 (p + 1)), q (2), row stride cp + 1
    const int p_ = P.pl, rows = (p_ + 1) + (p_ + 1) * (p_ + 2) / 2 + 2 * (p_ + 1) + 2;
    size_t lds = 0;
    for (la.cp = 32; la.cp >= 4; la.cp /= 2) {
      lds = (2 * (size_t)P.P2[L] + (size_t)rows * (la.cp + 1)) * sizeof(T);
      if (lds <= 48 * 1024) break;
    }
    HFMM_REQUIRE(lds <= 48 * 1024, "fmm3: P2M table too large for LDS (lower p)");
    k3_p2m<T><<<nleaves, 64, lds, fs>>>(la);
  }
  HFMM_LAUNCH_CHECK();
  for (int l = L - 1; l >= 2; --l) {
    Tr3Args<T> a{};
    a.offs = P.offs.p;
    a.A = P.A.p + P.m2m_off[l];
    a.B = P.M.p + P.eoff[l + 1];
    a.C = P.M.p + P.eoff[l];
    a.RT = P.Kp[l] / 16;
    a.KS = 8 * P.Kp[l + 1] / 4;
    a.KSe = a.KS;  // the children's padding lies between them
    a.ncols = 1 << (3 * l);
    a.crows = P.Kp[l];
    a.accumulate = 0;
    a.ldb = 8 * P.Kp[l + 1];
    a.ldc = P.Kp[l];
    a.pstride = ((int64_t)1 << (3 * l)) * P.Kp[l];
    launch_trans<T>(a, P.part.p, P.part.n, fs);
  }
  if (stage_ms) HFMM_HIP(hipEventRecord(P.ev[1], stream));
  // M2L on every level
  for (int l = 2; l <= L; ++l) {
    Tr3Args<T> a{};
    a.offs = P.offs.p;
    a.A = P.A.p + P.m2l_off[l];
    a.B = P.M.p + P.eoff[l];
    a.C = P.Lc.p + P.eoff[l];
    a.RT = P.Kp[l] / 16;
    a.KS = P.Kp[l] / 4;
    a.KSe = (2 * P.P2[l] + 3) / 4;
    a.h = 1 << (l - 1);
    a.nb = 1 << l;
    a.ncols = a.h * a.h * a.h;
    a.crows = P.Kp[l];
    a.accumulate = 0;
    a.ldb = P.Kp[l];
    a.ldc = P.Kp[l];
    a.aslot = (int64_t)P.Kp[l] * P.Kp[l];
    a.m2l = 1;
    a.pstride = ((int64_t)1 << (3 * l)) * P.Kp[l];
    launch_trans<T>(a, P.part.p, P.part.n, fs);
  }
  if (stage_ms) HFMM_HIP(hipEventRecord(P.ev[2], stream));
  // downward pass
  for (int l = 3; l <= L; ++l) {
    Tr3Args<T> a{};
    a.offs = P.offs.p;
    a.A = P.A.p + P.l2l_off[l];
    a.B = P.Lc.p + P.eoff[l - 1];
    a.C = P.Lc.p + P.eoff[l];
    a.RT = 8 * P.Kp[l] / 16;
    a.KS = P.Kp[l - 1] / 4;
    a.KSe = (2 * P.P2[l - 1] + 3) / 4;
    a.ncols = 1 << (3 * (l - 1));
    a.crows = 8 * P.Kp[l];
    a.accumulate = 1;
    a.ldb = P.Kp[l - 1];
    a.ldc = 8 * P.Kp[l];
    a.pstride = ((int64_t)1 << (3 * l)) * P.Kp[l];
    launch_trans<T>(a, P.part.p, P.part.n, fs);
  }
  if (stage_ms) HFMM_HIP(hipEventRecord(P.ev[3], stream));
  if (overlap) HFMM_HIP(hipEventRecord(t.join, fs));
  if constexpr (sizeof(T) == 8) {
    switch (la.ntay) {
      case 7: k3_p2p<T, 7><<<nleaves, 64, 0, stream>>>(la); break;
      case 10: k3_p2p<T, 10><<<nleaves, 64, 0, stream>>>(la); break;
      case kTaylorMax3: k3_p2p<T, kTaylorMax3><<<nleaves, 64, 0, stream>>>(la); break;
      default: k3_p2p<T, 0><<<nleaves, 64, 0, stream>>>(la); break;
    }
  } else {
    k3_p2p<T, 0><<<nleaves, 64, 0, stream>>>(la);
  }
  HFMM_LAUNCH_CHECK();
  if (stage_ms) HFMM_HIP(hipEventRecord(P.ev[4], stream));
  if (overlap) HFMM_HIP(hipStreamWaitEvent(stream, t.join, 0));
  la.E = P.Lc.p + P.eoff[L];
  k3_l2p<T><<<nleaves, 64, 0, stream>>>(la);
  HFMM_LAUNCH_CHECK();
  if (stage_ms) {
    HFMM_HIP(hipEventRecord(P.ev[5], stream));
    HFMM_HIP(hipEventSynchronize(P.ev[5]));
    for (int s = 0; s < 5; ++s) HFMM_HIP(hipEventElapsedTime(&stage_ms[s], P.ev[s], P.ev[s + 1]));
    HFMM_HIP(hipEventElapsedTime(&stage_ms[5], P.ev[0], P.ev[5]));
  }
}

template void fmm3_apply<float>(Tree3&, double, int, const float2*, float2*, hipStream_t, float*);
template void fmm3_apply<double>(Tree3&, double, int, const double2*, double2*, hipStream_t, float*);

}  // namespace hfmm
