// Arguments of the near-field (P2P) and leaf far-field (L2P) kernels, and
// the near-field launcher, whose kernels are compiled in near.hip (one
// object per precision and column-group width).
#pragma once

#include "common.h"

namespace hfmm {

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
  // dipole sources (the double-layer term): when dn is set, column r of the
  // sources carries a density q and a unit normal dn[j] (sorted order), and
  // the pair kernel is dG/dn_y = (i k / 4) H1(k r) (x - y).n / r instead of G
  const cplx<T>* dn;
  // FP64 log2 table: 128 entries (1/c_i, log2 c_i), c_i = 1/2 + (i + 1/2)/256
  const double2* l2tab;
};

// Near field of one column group [r0, r0 + NR) on a tree of depth L with
// nleaves leaves: `fast` selects the fitted H0 polynomial with `deg`
// coefficients (else the full-range routine); G lanes share a target.
template <class T, int NR>
void launch_p2p(int L, int64_t nleaves, bool fast, int deg, const P2PArgs<T>& a, int G, hipStream_t st);

// Double-layer near field (dipole sources, a.dn set): the full-range FP64
// H1 routine per pair; one launch per column group.
template <class T, int NR>
void launch_p2p_dipole(int L, int64_t nleaves, const P2PArgs<T>& a, hipStream_t st);

}  // namespace hfmm
