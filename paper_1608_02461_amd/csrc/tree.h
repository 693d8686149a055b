// Uniform quad-tree over a square root box (hierarchical decomposition of
// Sec. 5.1.1), stored as a Morton-sorted point set with leaf offsets.
#pragma once

#include <map>
#include <memory>
#include <tuple>

#include "common.h"

namespace hfmm {

struct PlanBase {
  virtual ~PlanBase() = default;
};

struct Tree {
  int64_t n = 0;          // points
  int L = 0;              // depth; 4^L leaves
  double x0 = 0, y0 = 0, side_len = 1;  // root box corner and side
  int leaf_size = 0;
  int64_t nleaves = 1;
  int max_leaf = 0;
  DevBuf<int32_t> perm;       // sorted slot -> caller index
  DevBuf<int32_t> iperm;      // caller index -> sorted slot
  DevBuf<int32_t> leaf_off;   // nleaves + 1, Morton order
  DevBuf<double2> rel64;      // sorted point minus its leaf centre
  DevBuf<float2> rel32;       // the same in FP32
  std::vector<int32_t> leaf_off_h;
  // translation plans, keyed by (k, p, precision)
  std::map<std::tuple<double, int, int>, std::unique_ptr<PlanBase>> plans;
  // a second stream (default priority, non-blocking) on which the far-field
  // chain runs beside the near field, and the events that fork and join it;
  // created with the tree (depth >= 2) so that no call under graph capture
  // creates them
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  // options of the plans made from now on (hfmm_tree_set_options): the VALU
  // downward kernels instead of MFMA (reference and ablation), and whether
  // the autotuner times launch shapes (else defaults; the cache still applies)
  bool m2l_valu = false;
  bool autotune = true;
  // accuracy experiment: the M2L's operands rounded to FP16 (1) or BF16 (2)
  // before the FP32 matrix-core products (FP32 plans only; 0: none)
  int m2l_round = 0;

  Tree() = default;
  Tree(const Tree&) = delete;
  Tree& operator=(const Tree&) = delete;
  ~Tree();
  double leaf_side() const { return side_len / double(1u << L); }
};

// Depth rule: 0 for leaf_size <= 0, else max(2, smallest L with leaf*4^L >= n).
int tree_depth(int64_t n, int leaf_size);

// Stable LSD radix sort (8-bit digits) of (key, value) pairs on the low
// `nbits` bits of the keys; the sorted pairs are left in ka, va.  Synchronises
// `stream`.
void radix_sort_pairs(DevBuf<uint32_t>& ka, DevBuf<int32_t>& va, int n, int nbits, hipStream_t stream);

// Leaf offsets (nleaves + 1 entries) from sorted leaf keys: off[b] is the
// first slot whose key is >= b.
void leaf_bounds(const uint32_t* sorted_keys, int n, int64_t nleaves, int32_t* off, hipStream_t stream);

// Builds the tree on `stream` (synchronises it).  Throws Error on bad input.
std::unique_ptr<Tree> build_tree(const double* d_xy, int64_t n, double x0, double y0, double side,
                                 int leaf_size, hipStream_t stream);

}  // namespace hfmm
