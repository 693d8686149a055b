// Level-to-level translations of the FMM on the matrix cores (MFMA): the
// M2L over the interaction lists of every level in one launch, and the M2M
// and L2L between adjacent levels (Sec. 5.1.2, the FMM calculation flow).
// Included once, by fmm.hip, inside its anonymous namespace; kept in a file
// of its own so that its source identifies the measured kernels.
#pragma once

#include "devutil.h"

// ------------------------------------------------------------------ L2L + M2L on MFMA
// Complex translations in real form: for an output coefficient m and input n,
//   [Re L_m]   [ Re T  -Im T ] [Re M_n]
//   [Im L_m] = [ Im T   Re T ] [Im M_n]
// so each translation is a (2P x 2P) real matrix A.  One wave owns a 4 x 4
// patch of target boxes = the 16 columns of a 16x16x4 MFMA; it walks the 40
// offset classes (a column whose box does not have the offset in its
// interaction list reads a zero) and the 4 L2L child positions (a column reads
// its parent's local expansion only for its own position).  A comes from
// tables already laid out per lane: frag[...][ks][lane] = A[16 rt + lane%16][4 ks + lane/16];
// B comes from the source multipoles staged in LDS for the block's window.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <class T> struct Acc4;
template <> struct Acc4<float> { typedef f32x4 type; };
template <> struct Acc4<double> { typedef f64x4 type; };
__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Row of the 16x16 accumulator held in register q of a lane in group kq =
// lane/16 (column = lane%16): 4 kq + q for the FP32 MFMA, 4 q + kq for FP64.
template <class T> __device__ __forceinline__ int out_row(int kq, int q);
template <> __device__ __forceinline__ int out_row<float>(int kq, int q) { return 4 * kq + q; }
template <> __device__ __forceinline__ int out_row<double>(int kq, int q) { return 4 * q + kq; }

constexpr int kMaxLev = 13;

// the 40 M2L offset classes, o = (ox + 3) * 7 + (oy + 3), in increasing o
__constant__ int kClassO[40] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 19, 20, 21, 22,
                                26, 27, 28, 29, 33, 34, 35, 36, 37, 38, 39, 40, 41, 42, 43, 44, 45, 46, 47, 48};

template <class T>
struct M2LLevel {
  const cplx<T>* M;
  cplx<T>* Lc;
  const T* Af;          // [49][RT][KSA][64]
  const uint8_t* fsrc;  // source flags of the level or NULL
  // KS = ceil(2 P / 4) k steps; KSA = KS rounded up to 4 (the table's
  // stride, zero beyond KS); KSL: k steps per LDS slice (all KS, or a
  // multiple of 4)
  int nb, P, RT, KS, KSA, KSL, tile, gx, block0;
  T oscale;  // output scale (a power of two: the FP16 rounding experiment scales the level's table down)
  // class groups: S > 1 splits the 40 offset classes over S blocks per
  // target tile and row tile; their partial sums go to `part`
  // ([nr][gx RT][S][NP][4][64]) and the last of the S blocks (counter
  // `cnt`, one per target tile and row tile, left at zero) adds them up
  int S;
  T* part;
  unsigned* cnt;
};

template <class T>
struct M2LAllArgs {
  M2LLevel<T> lv[kMaxLev];
  int nlev;
  const int* alive;
  int nrhs, r0, nr;
  int round;  // multipole operands rounded to FP16 (1) or BF16 (2) when staged; 0: none
};

// An M2L operand rounded to FP16 or BF16 (round to nearest even) and back:
// the products then see the inputs a matrix-core product with 16-bit
// operands would see, accumulated in FP32.
__device__ __forceinline__ float round_in(float v, int mode) {
  if (mode == 1) return (float)(_Float16)v;
  if (mode == 2) {
    uint32_t b = __float_as_uint(v);
    b += 0x7fffu + ((b >> 16) & 1u);
    return __uint_as_float(b & 0xffff0000u);
  }
  return v;
}
__device__ __forceinline__ double round_in(double v, int) { return v; }

// M2L of every level in one launch (the levels are independent; L2L runs
// afterwards, top down).  One block = a tile x tile patch of target boxes
// (4 or 1 patches of 4 x 4) and one row tile.  The block stages the source
// window (the targets' boxes plus a 2-box margin, clipped to the grid) in LDS
// as real columns [Re; Im; 0 pad] of stride KPs, followed by one all-zero box
// that stands in for sources outside the grid or not adjacent to the
// target's parent, so every operand read is unconditional.  The k steps are
// padded with zeros to whole chunks of 4.  Each of the 8 waves owns all
// patches of the block (one accumulator each, so one A fragment feeds up to 4
// MFMAs) and the offset classes whose index = wave (mod 8); the eight partial
// sums meet in LDS.  A level whose window does not fit is staged in slices
// of KSL k steps (the products of each slice accumulate).  The LDS stride of
// a box, 4 KSL + 2 = 2 m with m odd, puts the 16 columns of a patch times 2
// rows in distinct LDS banks (32 of 4 bytes) when the window is 12 boxes
// wide.
// 4 waves (one per SIMD), so that blocks fit in the registers the
// near-field blocks leave free on a CU and the chain runs beside them
constexpr int kM2LThreads = 256;

// With source flags (a pass whose sources sit in few boxes, such as the
// boundary pass of the preconditioner): true, uniformly over the block, when
// no box of the block's source window holds a source.
template <class T>
__device__ __forceinline__ bool m2l_window_empty(const M2LLevel<T>& a, int wx0, int wy0, int WW, int zb) {
  bool any = false;
  for (int b = threadIdx.x; b < zb && !any; b += kM2LThreads) {
    const int by = b / WW, bx = b - by * WW;
    any = a.fsrc[morton((uint32_t)(wx0 + bx), (uint32_t)(wy0 + by))] != 0;
  }
  return !__syncthreads_or(any);
}

// The block's local expansions when its window holds no source: zeros, in
// the rows and boxes the products would have written.
template <class T, int NP>
__device__ __forceinline__ void m2l_write_zero(const M2LAllArgs<T>& args, const M2LLevel<T>& a, int rt, int w,
                                               int lane, const uint32_t (&tbox)[NP]) {
  if (w >= NP) return;
  const int kq = lane >> 4, P = a.P;
  uint32_t tb = tbox[0];
#pragma unroll
  for (int p = 1; p < NP; ++p)
    if (w == p) tb = tbox[p];
  for (int r = 0; r < args.nr; ++r) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = rt * 16 + out_row<T>(kq, q);
      if (i < 2 * P) {
        T* dst = reinterpret_cast<T*>(a.Lc + ((size_t)tb * args.nrhs + args.r0 + r) * P + (i < P ? i : i - P));
        dst[i < P ? 0 : 1] = T(0);
      }
    }
  }
}

// Class groups: the block has stored its partial sums (agent-scope stores,
// written through to the device-coherent level); once they are complete the
// block counts itself in, and the last of the S blocks of its target tile
// and row tile adds the S partial sums in group order (agent-scope loads),
// writes the local expansions and resets the counter for the next launch.
// No device-scope fence: on this GPU one writes back and invalidates the
// whole L2 of the XCD, which costs the other blocks their cached tables.
template <class T>
__device__ __forceinline__ void part_store(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T part_load(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T, int NP>
__device__ __forceinline__ void m2l_groups_sum(const M2LAllArgs<T>& args, const M2LLevel<T>& a, int grp, int ngrp,
                                               int rt, int w, int lane, const uint32_t (&tbox)[NP], T* Ms) {
  int* last = reinterpret_cast<int*>(Ms);
  __builtin_amdgcn_s_waitcnt(0);  // this wave's partial-sum stores are complete
  __syncthreads();                // (and every wave is done with the LDS)
  if (threadIdx.x == 0)
    last[0] = __hip_atomic_fetch_add(a.cnt + grp, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
              (unsigned)(a.S - 1);
  __syncthreads();
  if (!last[0]) return;
  if (w < NP) {
    const int kq = lane >> 4, P = a.P;
    uint32_t tb = tbox[0];
#pragma unroll
    for (int p = 1; p < NP; ++p)
      if (w == p) tb = tbox[p];
    for (int r = 0; r < args.nr; ++r) {
      const T* src = a.part + ((size_t)r * ngrp + grp) * a.S * (NP * 256) + w * 256 + lane;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        T s = T(0);
        for (int g = 0; g < a.S; ++g) s += part_load(src + (size_t)g * (NP * 256) + q * 64);
        const int i = rt * 16 + out_row<T>(kq, q);
        if (i < 2 * P) {
          T* dst = reinterpret_cast<T*>(a.Lc + ((size_t)tb * args.nrhs + args.r0 + r) * P + (i < P ? i : i - P));
          dst[i < P ? 0 : 1] = s * a.oscale;
        }
      }
    }
  }
  if (threadIdx.x == 0) __hip_atomic_store(a.cnt + grp, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class T, int NP>
__device__ __forceinline__ void m2l_block(const M2LAllArgs<T>& args, const M2LLevel<T>& a, int lblock, T* Ms) {
  typedef typename Acc4<T>::type V4;
  T* red = Ms;  // the reduction reuses the window once the products are done
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nbt = a.nb / a.tile;
  const int ngrp = a.gx * a.RT, grp = lblock % ngrp, sg = lblock / ngrp;  // tile group, class group
  const int pb = grp % a.gx, rt = grp / a.gx;
  const int bx0 = (pb % nbt) * a.tile, by0 = (pb / nbt) * a.tile;
  const int wx0 = max(0, bx0 - 2), wy0 = max(0, by0 - 2);
  const int WW = min(a.nb, bx0 + a.tile + 2) - wx0, WH = min(a.nb, by0 + a.tile + 2) - wy0;
  const int zb = WW * WH;  // the zero box
  const int P = a.P, KS = a.KS, KSL = a.KSL;
  const int KPs = 4 * ((KSL + 3) & ~3) + 2;  // LDS stride of one box's slice (whole chunks)
  const int j = lane & 15, kq = lane >> 4;
  int tx[NP], ty[NP];
  uint32_t tbox[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    tx[p] = bx0 + (p & 1) * 4 + (j & 3);
    ty[p] = by0 + (p >> 1) * 4 + (j >> 2);
    tbox[p] = morton((uint32_t)tx[p], (uint32_t)ty[p]);
  }
  if (a.fsrc && m2l_window_empty<T>(a, wx0, wy0, WW, zb)) {  // the same for every class group
    if (sg == 0) m2l_write_zero<T, NP>(args, a, rt, w, lane, tbox);
    return;
  }
  const size_t cstride = (size_t)a.RT * a.KSA * 64;
  const T* Abase = a.Af + (size_t)rt * a.KSA * 64 + lane;
  // LDS position of the source box of class o for patch p (the zero box when
  // it is outside the grid or not adjacent to the target's parent)
  // (computed without branches: both positions, then a select)
  auto src_base = [&](int o, int p) {
    const int ox = o / 7 - 3, oy = o % 7 - 3;
    const int sx = tx[p] + ox, sy = ty[p] + oy;
    const bool v = ((unsigned)sx < (unsigned)a.nb) & ((unsigned)sy < (unsigned)a.nb) &
                   ((unsigned)((sx >> 1) - (tx[p] >> 1) + 1) <= 2u) & ((unsigned)((sy >> 1) - (ty[p] >> 1) + 1) <= 2u);
    const int in = __mul24(sy - wy0, WW) + (sx - wx0);
    return __mul24(v ? in : zb, KPs) + kq;
  };
  for (int r = 0; r < args.nr; ++r) {
    V4 acc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[p] = V4{0, 0, 0, 0};
    for (int k0 = 0; k0 < KS; k0 += KSL) {
      __syncthreads();
      // stage the slice [4 k0, 4 k0 + 4 KSL) of the real columns of the
      // window.  Lanes in groups of P take one complex coefficient each of
      // gpw boxes per wave step (lanes loop over coefficients when P > 64);
      // the loads of 4 steps are issued before their LDS stores.  The
      // columns past 2 P that the slice's whole MFMA chunks read are zeroed
      // apart.
      {
        const int gpw = P <= 64 ? 64 / P : 1;  // boxes per wave step
        const int g = P <= 64 ? lane / P : 0, m0 = P <= 64 ? lane - g * P : lane;
        const int lo = 4 * k0, hi = 4 * (k0 + KSL);  // real columns of the slice
        const uint32_t mW = 0xffffffffu / (uint32_t)WW + 1u;
        const bool on = g < gpw;
        const uint8_t* fl = a.fsrc;
        const size_t bstride = (size_t)args.nrhs * P;  // between boxes
        for (int m = m0; m < P; m += 64) {
          const cplx<T>* Mm = a.M + (size_t)(args.r0 + r) * P + m;
          for (int b0 = w * gpw; b0 < zb; b0 += 4 * 4 * gpw) {
            cplx<T> v[4];
            uint8_t f[4];
            int lb[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int box = b0 + u * 4 * gpw + g;
              lb[u] = on && box < zb ? box : -1;
              v[u] = mk<T>(0, 0);
              f[u] = 1;
              if (lb[u] >= 0) {
                const int by = (int)__umulhi((uint32_t)box, mW), bx = box - by * WW;
                const uint32_t gb = morton((uint32_t)(wx0 + bx), (uint32_t)(wy0 + by));
                v[u] = Mm[gb * bstride];
                if (fl) f[u] = fl[gb];
              }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (lb[u] >= 0) {
                T* row = Ms + (size_t)lb[u] * KPs - lo;
                const T re = f[u] ? round_in(v[u].x, args.round) : T(0);
                const T im = f[u] ? round_in(v[u].y, args.round) : T(0);
                if (m >= lo && m < hi) row[m] = re;
                if (m + P >= lo && m + P < hi) row[m + P] = im;
              }
          }
        }
        // zero padding: columns [2 P, 4 (k0 + min(KSL, KS - k0))) of every box
        const int z0 = max(2 * P, lo), z1 = 4 * (k0 + min(KSL, KS - k0));
        if (z1 > z0) {
          const int nz = z1 - z0;
          const uint32_t mZ = 0xffffffffu / (uint32_t)nz + 1u;
          for (int i = tid; i < zb * nz; i += kM2LThreads) {
            const int box = (int)__umulhi((uint32_t)i, mZ);
            Ms[(size_t)box * KPs + z0 - lo + (i - box * nz)] = T(0);
          }
        }
      }
      if (w == 0)
        for (int n = lane; n < KPs; n += 64) Ms[zb * KPs + n] = T(0);
      __syncthreads();
      const T* Ab = Abase + (size_t)k0 * 64;  // this slice's k steps
      // the wave's 10 / S offset classes (class index = wave mod 4, within
      // the block's class group) one after another; the A fragments of the
      // next chunk, also across classes, load one chunk ahead.  The last
      // chunk of a slice may have fewer than 4 k steps (ns).
      const int ncw = 10 / a.S;
      auto cls = [&](int i) {
        return a.S == 1 ? kClassO[8 * (i % 5) + w + 4 * (i / 5)] : kClassO[sg * 4 * ncw + w + 4 * i];
      };
      const int nst = min(KSL, KS - k0);
      const int nch = (nst + 3) >> 2;
      T an[4];
      {
        const T* A0 = Ab + (size_t)cls(0) * cstride;
#pragma unroll
        for (int u = 0; u < 4; ++u) an[u] = A0[u * 64];
      }
#pragma unroll 1
      for (int oi = 0; oi < ncw; ++oi) {
        const int o = cls(oi);
        int base[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) base[p] = src_base(o, p);
        const T* A = Ab + (size_t)o * cstride;
        const T* An = oi + 1 < ncw ? Ab + (size_t)cls(oi + 1) * cstride : A;
        for (int c = 0; c < nch; ++c) {
          T av[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) av[u] = an[u];
          // the next chunk's fragments: of this class, else of the next one
          // (after the last class, a harmless reload of this one)
          const T* nx = c + 1 < nch ? A + (c * 4 + 4) * 64 : An;
#pragma unroll
          for (int u = 0; u < 4; ++u) an[u] = nx[u * 64];
          T bv[NP][4];
#pragma unroll
          for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int u = 0; u < 4; ++u) bv[p][u] = Ms[base[p] + (c * 4 + u) * 4];  // in the box's stride
          const int ns = min(4, nst - 4 * c);
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (u < ns)
#pragma unroll
              for (int p = 0; p < NP; ++p) acc[p] = mfma16(av[u], bv[p][u], acc[p]);
        }
      }
    }
    // sum the 4 waves' partial products in LDS
    __syncthreads();
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) red[((w * NP + p) * 4 + q) * 64 + lane] = acc[p][q];
    __syncthreads();
    if (w < NP) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const T s = red[((0 * NP + w) * 4 + q) * 64 + lane] + red[((1 * NP + w) * 4 + q) * 64 + lane] +
                    red[((2 * NP + w) * 4 + q) * 64 + lane] + red[((3 * NP + w) * 4 + q) * 64 + lane];
        if (a.S > 1) {
          part_store(a.part + (((size_t)r * ngrp + grp) * a.S + sg) * (NP * 256) + (w * 4 + q) * 64 + lane, s);
          continue;
        }
        const int i = rt * 16 + out_row<T>(kq, q);
        if (i < 2 * P) {
          uint32_t tb = tbox[0];
#pragma unroll
          for (int p = 1; p < NP; ++p)
            if (w == p) tb = tbox[p];
          T* dst = reinterpret_cast<T*>(a.Lc + ((size_t)tb * args.nrhs + args.r0 + r) * P + (i < P ? i : i - P));
          dst[i < P ? 0 : 1] = s * a.oscale;
        }
      }
    }
  }
  if (a.S > 1) m2l_groups_sum<T, NP>(args, a, grp, ngrp, rt, w, lane, tbox, Ms);
}

// M2L offset classes, o = (ox + 3) * 7 + (oy + 3), by target parity: a
// target at even x has sources at ox in [-2, 3], at odd x in [-3, 2] (the
// children of its parent's neighbours), and likewise in y, less the 3 x 3
// near block: 27 classes per parity.  Grouped by the parities whose lists
// hold them: 16 classes with |ox|, |oy| <= 2 are in every list; the 5 with
// oy = +3 (|ox| <= 2) are in the lists of the two parities with even y, and
// likewise oy = -3 (odd y), ox = +3 (even x), ox = -3 (odd x); each parity
// adds one corner (ox, oy = +-3).  Wave w of a block takes 4 common classes,
// the pair group w (patches kPairA[w], kPairB[w]) and the corner of patch w:
// 27 MFMA k-step groups from 10 A fragments.
__constant__ int kCommonO[16] = {8, 9, 10, 11, 12, 15, 19, 22, 26, 29, 33, 36, 37, 38, 39, 40};
__constant__ int kPairO[4][5] = {{13, 20, 27, 34, 41}, {7, 14, 21, 28, 35}, {43, 44, 45, 46, 47}, {1, 2, 3, 4, 5}};
__constant__ int kPairA[4] = {0, 2, 0, 1};
__constant__ int kPairB[4] = {1, 3, 2, 3};
__constant__ int kCornerO[4] = {48, 6, 42, 0};

// The 8 x 8-target block with its four 4 x 4 patches grouped by target
// parity (patch p holds the targets of parity (p & 1, p >> 1), every other
// box of the tile), so each patch walks exactly its 27 interaction-list
// classes: 27 MFMA k-step groups per wave instead of 40 over all classes.
// The 8 x 8-target block with its four 4 x 4 patches grouped by target
// parity (patch p holds the targets of parity (p & 1, p >> 1), every other
// box of the tile), so each patch walks exactly its 27 interaction-list
// classes: 27 MFMA k-step groups per wave instead of 40 over all classes.
template <class T>
__device__ __forceinline__ void m2l_block_par(const M2LAllArgs<T>& args, const M2LLevel<T>& a, int lblock, T* Ms) {
  constexpr int NP = 4;
  typedef typename Acc4<T>::type V4;
  T* red = Ms;  // the reduction reuses the window once the products are done
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nbt = a.nb / a.tile;
  const int pb = lblock % a.gx, rt = lblock / a.gx;
  const int bx0 = (pb % nbt) * a.tile, by0 = (pb / nbt) * a.tile;
  const int wx0 = max(0, bx0 - 2), wy0 = max(0, by0 - 2);
  const int WW = min(a.nb, bx0 + a.tile + 2) - wx0, WH = min(a.nb, by0 + a.tile + 2) - wy0;
  const int zb = WW * WH;  // the zero box
  const int P = a.P, KS = a.KS, KSL = a.KSL;
  const int KPs = 4 * ((KSL + 3) & ~3) + 2;  // LDS stride of one box's slice (whole chunks)
  const int j = lane & 15, kq = lane >> 4;
  int tx[NP], ty[NP];
  uint32_t tbox[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {  // patch p = target parity (p & 1, p >> 1)
    tx[p] = bx0 + 2 * (j & 3) + (p & 1);
    ty[p] = by0 + 2 * (j >> 2) + (p >> 1);
    tbox[p] = morton((uint32_t)tx[p], (uint32_t)ty[p]);
  }
  if (a.fsrc && m2l_window_empty<T>(a, wx0, wy0, WW, zb)) {
    m2l_write_zero<T, NP>(args, a, rt, w, lane, tbox);
    return;
  }
  const size_t cstride = (size_t)a.RT * a.KSA * 64;
  const T* Abase = a.Af + (size_t)rt * a.KSA * 64 + lane;
  // LDS position of the source box of class o for patch p (the zero box when
  // it is outside the grid or not adjacent to the target's parent)
  // (the class lists below are exactly the interaction lists of each
  // parity, so only sources outside the grid read the zero box); p may be a
  // wave-uniform runtime value
  auto src_base = [&](int o, int p) {
    const int ox = o / 7 - 3, oy = o % 7 - 3;
    const int sx = bx0 + 2 * (j & 3) + (p & 1) + ox, sy = by0 + 2 * (j >> 2) + (p >> 1) + oy;
    const bool v = ((unsigned)sx < (unsigned)a.nb) & ((unsigned)sy < (unsigned)a.nb);
    const int in = __mul24(sy - wy0, WW) + (sx - wx0);
    return __mul24(v ? in : zb, KPs) + kq;
  };
  for (int r = 0; r < args.nr; ++r) {
    V4 acc[NP], accA = V4{0, 0, 0, 0}, accB = accA, accC = accA;
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[p] = V4{0, 0, 0, 0};
    for (int k0 = 0; k0 < KS; k0 += KSL) {
      __syncthreads();
      // stage the slice [4 k0, 4 k0 + 4 KSL) of the real columns of the
      // window.  Lanes in groups of P take one complex coefficient each of
      // gpw boxes per wave step (lanes loop over coefficients when P > 64);
      // the loads of 4 steps are issued before their LDS stores.  The
      // columns past 2 P that the slice's whole MFMA chunks read are zeroed
      // apart.
      {
        const int gpw = P <= 64 ? 64 / P : 1;  // boxes per wave step
        const int g = P <= 64 ? lane / P : 0, m0 = P <= 64 ? lane - g * P : lane;
        const int lo = 4 * k0, hi = 4 * (k0 + KSL);  // real columns of the slice
        const uint32_t mW = 0xffffffffu / (uint32_t)WW + 1u;
        const bool on = g < gpw;
        const uint8_t* fl = a.fsrc;
        const size_t bstride = (size_t)args.nrhs * P;  // between boxes
        for (int m = m0; m < P; m += 64) {
          const cplx<T>* Mm = a.M + (size_t)(args.r0 + r) * P + m;
          for (int b0 = w * gpw; b0 < zb; b0 += 4 * 4 * gpw) {
            cplx<T> v[4];
            uint8_t f[4];
            int lb[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int box = b0 + u * 4 * gpw + g;
              lb[u] = on && box < zb ? box : -1;
              v[u] = mk<T>(0, 0);
              f[u] = 1;
              if (lb[u] >= 0) {
                const int by = (int)__umulhi((uint32_t)box, mW), bx = box - by * WW;
                const uint32_t gb = morton((uint32_t)(wx0 + bx), (uint32_t)(wy0 + by));
                v[u] = Mm[gb * bstride];
                if (fl) f[u] = fl[gb];
              }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (lb[u] >= 0) {
                T* row = Ms + (size_t)lb[u] * KPs - lo;
                const T re = f[u] ? round_in(v[u].x, args.round) : T(0);
                const T im = f[u] ? round_in(v[u].y, args.round) : T(0);
                if (m >= lo && m < hi) row[m] = re;
                if (m + P >= lo && m + P < hi) row[m + P] = im;
              }
          }
        }
        // zero padding: columns [2 P, 4 (k0 + min(KSL, KS - k0))) of every box
        const int z0 = max(2 * P, lo), z1 = 4 * (k0 + min(KSL, KS - k0));
        if (z1 > z0) {
          const int nz = z1 - z0;
          const uint32_t mZ = 0xffffffffu / (uint32_t)nz + 1u;
          for (int i = tid; i < zb * nz; i += kM2LThreads) {
            const int box = (int)__umulhi((uint32_t)i, mZ);
            Ms[(size_t)box * KPs + z0 - lo + (i - box * nz)] = T(0);
          }
        }
      }
      if (w == 0)
        for (int n = lane; n < KPs; n += 64) Ms[zb * KPs + n] = T(0);
      __syncthreads();
      const T* Ab = Abase + (size_t)k0 * 64;  // this slice's k steps
      // the wave's 10 classes (4 common, 5 of its pair group, its corner);
      // the A fragments of the next chunk, also across classes, load one
      // chunk ahead.  The last chunk of a slice may have fewer than 4 k steps
      // (ns).
      const int pa = kPairA[w], pb = kPairB[w];
      auto cls = [&](int i) { return i < 4 ? kCommonO[w + 4 * i] : (i < 9 ? kPairO[w][i - 4] : kCornerO[w]); };
      const int nst = min(KSL, KS - k0);
      const int nch = (nst + 3) >> 2;
      T an[4];
      {
        const T* A0 = Ab + (size_t)cls(0) * cstride;
#pragma unroll
        for (int u = 0; u < 4; ++u) an[u] = A0[u * 64];
      }
      // one class: K = 0 common (the four patches), 1 pair (patches pa,
      // pb), 2 corner (patch w); the kind is a template constant so that the
      // chunk loop of each kind is straight-line code
      auto walk = [&](auto kc, int oi) {
        constexpr int K = decltype(kc)::value;
        constexpr int NB = K == 0 ? 4 : (K == 1 ? 2 : 1);
        const int o = cls(oi);
        int base[NB];
        if constexpr (K == 0) {
#pragma unroll
          for (int p = 0; p < 4; ++p) base[p] = src_base(o, p);
        } else if constexpr (K == 1) {
          base[0] = src_base(o, pa);
          base[1] = src_base(o, pb);
        } else {
          base[0] = src_base(o, w);
        }
        const T* A = Ab + (size_t)o * cstride;
        const T* An = oi + 1 < 10 ? Ab + (size_t)cls(oi + 1) * cstride : A;
        for (int c = 0; c < nch; ++c) {
          T av[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) av[u] = an[u];
          const T* nx = c + 1 < nch ? A + (c * 4 + 4) * 64 : An;
#pragma unroll
          for (int u = 0; u < 4; ++u) an[u] = nx[u * 64];
          T bv[NB][4];
#pragma unroll
          for (int h = 0; h < NB; ++h)
#pragma unroll
            for (int u = 0; u < 4; ++u) bv[h][u] = Ms[base[h] + (c * 4 + u) * 4];
          const int ns = min(4, nst - 4 * c);
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (u < ns) {
              if constexpr (K == 0) {
#pragma unroll
                for (int p = 0; p < 4; ++p) acc[p] = mfma16(av[u], bv[p][u], acc[p]);
              } else if constexpr (K == 1) {
                accA = mfma16(av[u], bv[0][u], accA);
                accB = mfma16(av[u], bv[1][u], accB);
              } else {
                accC = mfma16(av[u], bv[0][u], accC);
              }
            }
          }
        }
      };
#pragma unroll 1
      for (int oi = 0; oi < 4; ++oi) walk(std::integral_constant<int, 0>{}, oi);
#pragma unroll 1
      for (int oi = 4; oi < 9; ++oi) walk(std::integral_constant<int, 1>{}, oi);
      walk(std::integral_constant<int, 2>{}, 9);
    }
    {
      const int pa = kPairA[w], pb = kPairB[w];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        if (p == pa) acc[p] += accA;
        if (p == pb) acc[p] += accB;
        if (p == w) acc[p] += accC;
      }
    }
    // sum the 4 waves' partial products in LDS
    __syncthreads();
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) red[((w * NP + p) * 4 + q) * 64 + lane] = acc[p][q];
    __syncthreads();
    if (w < NP) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const T s = red[((0 * NP + w) * 4 + q) * 64 + lane] + red[((1 * NP + w) * 4 + q) * 64 + lane] +
                    red[((2 * NP + w) * 4 + q) * 64 + lane] + red[((3 * NP + w) * 4 + q) * 64 + lane];
        const int i = rt * 16 + out_row<T>(kq, q);
        if (i < 2 * P) {
          uint32_t tb = tbox[0];
#pragma unroll
          for (int p = 1; p < NP; ++p)
            if (w == p) tb = tbox[p];
          T* dst = reinterpret_cast<T*>(a.Lc + ((size_t)tb * args.nrhs + args.r0 + r) * P + (i < P ? i : i - P));
          dst[i < P ? 0 : 1] = s * a.oscale;
        }
      }
    }
  }
}

// FP32: at most 96 registers per lane (91 used), so that a block fits
// beside four near-field blocks on a CU
template <class T> struct M2LWaves { static constexpr int value = sizeof(T) == 4 ? 5 : 1; };

template <class T>
__global__ __launch_bounds__(kM2LThreads) __attribute__((amdgpu_waves_per_eu(M2LWaves<T>::value)))
void k_m2l_mfma(M2LAllArgs<T> args) {
  extern __shared__ unsigned char smem_raw[];
  chain_priority();
  T* Ms = reinterpret_cast<T*>(smem_raw);
  if (args.alive && !args.alive[0]) return;
  // the block's level, selected by constant indices (a runtime index into
  // the argument array would copy the array to registers)
  M2LLevel<T> a = args.lv[0];
#pragma unroll
  for (int i = 1; i < kMaxLev; ++i)
    if (i < args.nlev && (int)blockIdx.x >= args.lv[i].block0) a = args.lv[i];
  const int lblock = (int)blockIdx.x - a.block0;
  if (a.tile == 8 && a.S == 1)
    m2l_block_par<T>(args, a, lblock, Ms);
  else if (a.tile == 8)
    m2l_block<T, 4>(args, a, lblock, Ms);
  else
    m2l_block<T, 1>(args, a, lblock, Ms);
}

// Level-to-level translation on MFMA.  A block of 4 waves covers 16 boxes of
// the output level (columns) and one 16-row tile (blockIdx.y):
//   L2L (mode 0): child boxes 4 b + c of 16 consecutive parents b; wave c
//                 takes child position c; out += A_c * L_parent.
//   M2M (mode 1): 16 consecutive parents; wave c forms A_c * M_child(4 b + c)
//                 and the 4 partial products are summed in LDS.
// Input columns read the real form [Re; Im] of the source coefficients.  The
// k steps run in chunks of 16 whose loads are all issued before the chunk's
// MFMAs, so a wave waits for memory once per chunk, not once per step.
template <class T>
struct TTArgs {
  const cplx<T>* in;
  cplx<T>* out;
  const T* Wf;               // [4][RT][KS][64]
  const uint8_t* fin;        // flags of the input level (M2M) or NULL
  const uint8_t* fout;       // flags of the output level (M2M) or NULL
  const int* alive;
  int mode, nparents, Pin, Pout, RT, KS, nrhs, r0, nr;
};

constexpr int kTTChunk = 16;
// LDS budget of one M2L block (the launch takes the largest over its
// levels): small enough that a block fits beside the four near-field blocks
// a CU holds, so that the far-field chain progresses while the near field runs
constexpr size_t kM2LLds = 32 * 1024;
// Class groups: a level of fewer than kM2LSplitBlocks blocks whose waves
// would each walk more than kM2LChain dependent MFMA chunks is split
constexpr int kM2LSplitBlocks = 128;
constexpr int kM2LChain = 20;

template <class T>
__global__ __launch_bounds__(256) void k_tt_mfma(TTArgs<T> a) {
  typedef typename Acc4<T>::type V4;
  __shared__ T red[3][4][64];
  chain_priority();
  if (a.alive && !a.alive[0]) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, j = lane & 15, kq = lane >> 4;
  const int g = blockIdx.x, rt = blockIdx.y;
  const int parent = g * 16 + j;
  const bool colv = parent < a.nparents;
  if (a.mode == 1 && a.fout) {
    // block-uniform: every wave sees the same 16 parents
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    if (wave == 0 && colv && a.fout[parent]) any = 1;
    __syncthreads();
    if (!any) return;
  }
  const int c = wave;
  const int src = a.mode == 0 ? parent : 4 * parent + c;
  const bool bvalid = colv && (a.mode == 0 || !a.fin || a.fin[src]);
  const T* Wf = a.Wf + ((size_t)(c * a.RT + rt) * a.KS) * 64 + lane;
  for (int r = 0; r < a.nr; ++r) {
    V4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    const cplx<T>* col = a.in + ((size_t)(bvalid ? src : 0) * a.nrhs + a.r0 + r) * a.Pin;
    for (int k0 = 0; k0 < a.KS; k0 += kTTChunk) {
      T av[kTTChunk], bv[kTTChunk];
      // every load is issued (clamped to a valid element) before any is
      // used, so a chunk waits for memory once
#pragma unroll
      for (int u = 0; u < kTTChunk; ++u) {
        const int ks = min(k0 + u, a.KS - 1);
        av[u] = Wf[ks * 64];
        const int kk = ks * 4 + kq, kc = min(kk, 2 * a.Pin - 1);
        const cplx<T> pv = col[kc < a.Pin ? kc : kc - a.Pin];
        bv[u] = bvalid && k0 + u < a.KS && kk < 2 * a.Pin ? (kk < a.Pin ? pv.x : pv.y) : T(0);
      }
#pragma unroll
      for (int u = 0; u < kTTChunk; ++u)
        if (k0 + u < a.KS) {
          if (u & 1)
            acc1 = mfma16(av[u], bv[u], acc1);
          else
            acc0 = mfma16(av[u], bv[u], acc0);
        }
    }
    T s[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) s[q] = acc0[q] + acc1[q];
    if (a.mode == 1) {
      if (wave > 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) red[wave - 1][q][lane] = s[q];
      }
      __syncthreads();
      if (wave == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) s[q] += red[0][q][lane] + red[1][q][lane] + red[2][q][lane];
      }
      __syncthreads();
      if (wave > 0) continue;
    }
    if (!colv) continue;
    const int obox = a.mode == 0 ? 4 * parent + c : parent;
    if (a.mode == 1 && a.fout && !a.fout[obox]) continue;
    // L2L adds to the M2L part already there: the 4 old values load together
    T* dst[4];
    T old[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = min(rt * 16 + out_row<T>(kq, q), 2 * a.Pout - 1);
      dst[q] = reinterpret_cast<T*>(a.out + ((size_t)obox * a.nrhs + a.r0 + r) * a.Pout + (i < a.Pout ? i : i - a.Pout)) +
               (i < a.Pout ? 0 : 1);
      old[q] = a.mode == 0 ? *dst[q] : T(0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (rt * 16 + out_row<T>(kq, q) < 2 * a.Pout) *dst[q] = old[q] + s[q];
  }
}
