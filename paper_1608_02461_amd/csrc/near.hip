// Near-field launchers (the P2P step of the FMM calculation flow, Sec. 5.1.2).
// This file is compiled once per precision and column-group width, with
// NEAR_T (float or double) and NEAR_NR (1, 2 or 4) defined on the command
// line, so that the many kernel instances build in parallel.
#include "devutil.h"
#include "p2p.h"
#include "special.h"

#ifndef NEAR_T
#define NEAR_T float
#endif
#ifndef NEAR_NR
#define NEAR_NR 1
#endif

namespace hfmm {

namespace {
#include "near.h"

template <class T, int NR, int D, bool FAST>
void launch_p2p4(int G, int grid, const P2PArgs<T>& a, hipStream_t st) {
  switch (G) {
    case 1: k_p2p4<T, NR, D, FAST, 1><<<grid, 256, 0, st>>>(a); break;
    case 2: k_p2p4<T, NR, D, FAST, 2><<<grid, 256, 0, st>>>(a); break;
    default: k_p2p4<T, NR, D, FAST, 4><<<grid, 256, 0, st>>>(a); break;
  }
}
}  // namespace

// The 4-sibling kernel for trees of depth >= 2, the per-leaf kernel for a
// single leaf.  The coefficient counts match the candidate lists of the plan.
template <class T, int NR>
void launch_p2p(int L, int64_t nleaves, bool fast, int deg, const P2PArgs<T>& a, int G, hipStream_t st) {
  if (L < 2) {
    const int grid = (int)nleaves;
    if (!fast) {
      k_p2p<T, NR, 1, false><<<grid, 64, 0, st>>>(a);
    } else if constexpr (std::is_same<T, float>::value) {
      switch (deg) {
        case 5: k_p2p<T, NR, 5, true><<<grid, 64, 0, st>>>(a); break;
        case 7: k_p2p<T, NR, 7, true><<<grid, 64, 0, st>>>(a); break;
        case 9: k_p2p<T, NR, 9, true><<<grid, 64, 0, st>>>(a); break;
        case 12: k_p2p<T, NR, 12, true><<<grid, 64, 0, st>>>(a); break;
        default: k_p2p<T, NR, 16, true><<<grid, 64, 0, st>>>(a); break;
      }
    } else {
      switch (deg) {
        case 8: k_p2p<T, NR, 8, true><<<grid, 64, 0, st>>>(a); break;
        case 10: k_p2p<T, NR, 10, true><<<grid, 64, 0, st>>>(a); break;
        case 12: k_p2p<T, NR, 12, true><<<grid, 64, 0, st>>>(a); break;
        case 16: k_p2p<T, NR, 16, true><<<grid, 64, 0, st>>>(a); break;
        default: k_p2p<T, NR, 24, true><<<grid, 64, 0, st>>>(a); break;
      }
    }
    HFMM_LAUNCH_CHECK();
    return;
  }
  const int grid = (int)(nleaves / 4);
  if (!fast) {
    launch_p2p4<T, NR, 1, false>(G, grid, a, st);
  } else if constexpr (std::is_same<T, float>::value) {
    switch (deg) {
      case 5: launch_p2p4<T, NR, 5, true>(G, grid, a, st); break;
      case 7: launch_p2p4<T, NR, 7, true>(G, grid, a, st); break;
      case 9: launch_p2p4<T, NR, 9, true>(G, grid, a, st); break;
      case 12: launch_p2p4<T, NR, 12, true>(G, grid, a, st); break;
      default: launch_p2p4<T, NR, 16, true>(G, grid, a, st); break;
    }
  } else {
    switch (deg) {
      case 8: launch_p2p4<T, NR, 8, true>(G, grid, a, st); break;
      case 10: launch_p2p4<T, NR, 10, true>(G, grid, a, st); break;
      case 12: launch_p2p4<T, NR, 12, true>(G, grid, a, st); break;
      case 16: launch_p2p4<T, NR, 16, true>(G, grid, a, st); break;
      default: launch_p2p4<T, NR, 24, true>(G, grid, a, st); break;
    }
  }
  HFMM_LAUNCH_CHECK();
}

template <class T, int NR>
void launch_p2p_dipole(int L, int64_t nleaves, const P2PArgs<T>& a, hipStream_t st) {
  (void)L;
  k_p2p_dipole<T, NR><<<(int)nleaves, 64, 0, st>>>(a);
  HFMM_LAUNCH_CHECK();
}

template void launch_p2p<NEAR_T, NEAR_NR>(int, int64_t, bool, int, const P2PArgs<NEAR_T>&, int, hipStream_t);
template void launch_p2p_dipole<NEAR_T, NEAR_NR>(int, int64_t, const P2PArgs<NEAR_T>&, hipStream_t);

}  // namespace hfmm
