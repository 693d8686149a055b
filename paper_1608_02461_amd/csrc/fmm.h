// FMM translation plan and the sorted-order FMM driver (Sec. 5.1.2:
// P2M, M2M, M2L, L2L, L2P and P2P on the uniform quad-tree).
//
// Expansions are partial-wave (Graf) expansions about box centres with
// in_v(z) = J_v(k|z|) e^{iv arg z}, out_v(z) = H_v(k|z|) e^{iv arg z}:
//   P2M  M_n  = sum_j q_j J_n(k rho_j) e^{-i n phi_j}
//   M2M  M'_l = sum_n M_n in_{n-l}(c_parent - c_child)
//   M2L  L_m  = sum_n M_n out_{n-m}(c_target - c_source)
//   L2L  L'_l = sum_m L_m in_{m-l}(c_child - c_parent)
//   L2P  phi  = (i/4) sum_m L_m in_m(x - c)
// Level l keeps n = -p_l..p_l with p_l = p + floor(k d_l / 2).  Stored
// coefficients are scaled for FP32 range: Mt_n = M_n / s_l^|n| and
// Lt_m = L_m s_l^|m| with s_l = min(1, k side_l); the tables carry the
// matching factors, so the same code runs in FP32 and FP64.
#pragma once

#include "special.h"
#include "tree.h"

#include <string>

namespace hfmm {

struct LevelInfo {
  int p = 0;           // order p_l
  int P = 0;           // 2 p_l + 1 coefficients
  double s = 1;        // scale s_l
  int64_t coef = 0;    // offset of the level in coefficient units (per column)
  int64_t box0 = 0;    // offset of the level in the per-box flag array
};

// Launch shape of the MFMA downward pass at one level.
struct MfmaLevel {
  bool on = false;
  int RT = 0, KS = 0, KSA = 0, KSp = 0, KSc = 0, tile = 0, gx = 0, gy = 0;
  int KSL = 0, KSL4 = 0;           // M2L k steps per LDS slice (8 x 8 and 4 x 4 tiles)
  int64_t af = 0, wf = 0, mm = 0;  // offsets into the M2L / L2L / M2M fragment tables
  size_t lds = 0, lds4 = 0;        // LDS of the default tile and of the 4 x 4 tile
  bool fit4 = false;
};

template <class T>
struct FmmPlan : PlanBase {
  double k = 0;
  int p = 0, L = 0;
  std::vector<LevelInfo> lv;
  int64_t coef_total = 0;   // sum over levels 2..L of 4^l P_l
  int64_t flag_total = 0;   // sum over levels 0..L of 4^l
  DevBuf<cplx<T>> m2m, l2l, m2l;
  std::vector<int64_t> m2m_off, l2l_off, m2l_off;
  std::vector<MfmaLevel> mf;   // per level
  DevBuf<T> afrag, wfrag, mfrag;  // per-lane MFMA fragments of the M2L / L2L / M2M matrices
  // M2L levels split into class groups: partial sums (for 4 columns) and the
  // per-tile counters of their last-block reduction (zero between launches)
  DevBuf<T> m2l_part;
  DevBuf<unsigned> m2l_cnt;
  int K = 0;
  // near field
  bool near_fast = false;
  NearPoly poly;
  // lanes per target in P2P, per column-group width (1, 2, 4 columns);
  // tuned[g] once the autotuner (or its cache) has chosen G[g]
  int G[3] = {1, 1, 1};
  bool tuned[3] = {false, false, false};
  bool use_mfma = true;     // MFMA downward pass where the level's tables exist
  int m2l_round = 0;        // M2L operands rounded to FP16 (1) or BF16 (2) (FP32 plans)
  std::vector<double> m2l_oscale;  // per level: power-of-two output scale of the M2L table (1 unless FP16)
  bool m2l_small = false;   // M2L on 4 x 4 target tiles (autotuned)
  bool m2l_split = true;    // coarse M2L levels split into class groups (autotuned)
  // P2P with G = 1, 2, 4 (one column); M2L 8x8, 4x4 tiles; M2L without, with class groups
  float tune_ms[7] = {0, 0, 0, 0, 0, 0, 0};
  int tune_source = 0;      // 0 defaults, 1 timed on this device, 2 from the tuning cache
  std::string tune_key;     // the cache key of this plan (without the column-group width)
  // work storage
  DevBuf<cplx<T>> M, Lc;
  int nrhs_cap = 0;
  DevBuf<cplx<T>> qs, phis;  // sorted scratch for the public apply
  DevBuf<cplx<T>> far;        // far field of a pass, in the output's point order
  DevBuf<cplx<T>> dns;        // sorted unit normals of a double-layer apply
  DevBuf<double2> l2tab;      // FP64 near field: log2 table (1/c_i, log2 c_i), 128 entries
  double max_table = 0;

  int64_t npts = 0;  // points of the tree
  void ensure_work(int nrhs) {
    if (nrhs > nrhs_cap) {
      M.alloc((size_t)coef_total * nrhs);
      Lc.alloc((size_t)coef_total * nrhs);
      far.ensure((size_t)npts * nrhs);  // far field of a pass
      nrhs_cap = nrhs;
    }
  }
};

// Work arrays of one FMM pass: multipole and local expansions of every
// level (coef_total x nrhs each) and the far field at the points (N x nrhs).
template <class T>
struct FmmWork {
  cplx<T>* M = nullptr;
  cplx<T>* Lc = nullptr;
  cplx<T>* far = nullptr;
};

// Column-group index of a group width (1, 2, 4 columns -> 0, 1, 2).
inline int nr_group(int nr) { return nr >= 4 ? 2 : (nr >= 2 ? 1 : 0); }

template <class T>
FmmPlan<T>& get_plan(Tree& t, double k, int p);
// The cached plan of (k, p) or NULL (creates nothing).
template <class T>
FmmPlan<T>* find_plan(Tree& t, double k, int p);
// Chooses the near-field lanes per target for the column-group widths that
// nrhs columns use (timed on the tree, or taken from the tuning cache).
// Not callable under stream capture.
template <class T>
void ensure_tuned(Tree& t, FmmPlan<T>& pl, int nrhs);

// Process-wide tuning cache: launch shapes chosen by the autotuner, keyed by
// the device architecture, the precision, the tree's depth and mean leaf
// occupancy, the level orders, the near-field polynomial and the column-group
// width.  Saved to / loaded from a text file so that later processes reuse it.
void tune_cache_save(const std::string& path);
int tune_cache_load(const std::string& path);
int tune_cache_size();
void tune_cache_clear();

// Optional stage timing: hipEvents recorded on the launch stream at stage
// boundaries; stage ids 0 gather, 1 upward (P2M+M2M), 2 downward (M2L+L2L),
// 3 L2P, 4 P2P, 5 scatter.
struct StageTimer {
  std::vector<hipEvent_t> ev;
  std::vector<int> stage, from;
  ~StageTimer();
  // records an event on st that closes stage s; the stage is timed from the
  // event with index `from_ev` (default: the previous one).  Returns the
  // index of the new event.
  int mark(int s, hipStream_t st, int from_ev = -1);
  void collect(float* ms, int nstage);
};

// phi (+)= FMM(q) on sorted arrays (column-major N x nrhs).  `flags` (or
// NULL for "every box") is a per-level array of 4^l bytes per level
// (concatenated from level 0) marking boxes that hold sources; `accumulate`
// adds into phi instead of overwriting.  `alive` (device int or NULL):
// when it holds 0 every kernel of the call returns at once.  With `perm`
// (the tree's sorted -> caller permutation; depth >= 2, no flags) q and phi
// are in caller order instead and `qs` (N x nrhs) receives the sorted charges.
//
// `w` (or NULL for the plan's own arrays, grown as needed) supplies the work
// arrays.  `dn` (sorted order, or NULL) turns the sources into dipoles with
// unit normals dn: the pass then sums q_j dG/dn_j (the double-layer kernel
// of Sec. 5.2) instead of q_j G.
template <class T>
void fmm_sorted(const Tree& t, FmmPlan<T>& pl, const cplx<T>* q, cplx<T>* phi, int nrhs, const uint8_t* flags,
                bool accumulate, hipStream_t st, const int* alive = nullptr, StageTimer* tm = nullptr,
                const int32_t* perm = nullptr, cplx<T>* qs = nullptr, const FmmWork<T>* w = nullptr,
                const cplx<T>* dn = nullptr);

// Per-level source flags for the points whose caller index lies in [lo, hi).
void source_flags(const Tree& t, int64_t lo, int64_t hi, uint8_t* d_flags, hipStream_t st);

// Public apply in caller order.
template <class T>
void fmm_apply(Tree& t, double k, int p, const cplx<T>* q, cplx<T>* phi, int nrhs, hipStream_t st,
               StageTimer* tm = nullptr);

// Double-layer apply in caller order: phi_i = sum_j q_j dG/dn_j(x_i, x_j)
// with unit normals `normals` (n x 2 FP64, caller order).
template <class T>
void fmm_apply_dipole(Tree& t, double k, int p, const cplx<T>* q, const double* normals, cplx<T>* phi, int nrhs,
                      hipStream_t st);

// The public apply on caller-provided work memory (`scratch`, `bytes`): no
// device allocation.  The plan of (k, p) must exist and be tuned for nrhs.
// Returns the bytes needed when they exceed `bytes` (nothing is launched
// then), else 0.
template <class T>
size_t fmm_apply_scratch(Tree& t, double k, int p, const cplx<T>* q, cplx<T>* phi, int nrhs, void* scratch,
                         size_t bytes, hipStream_t st);

}  // namespace hfmm
