// 3-D Helmholtz FMM on a uniform oct-tree (the 3-D decomposition of
// Sec. 5.1.1 and the kernel exp(i k r) / (4 pi r) of Sec. 5.2), with the
// calculation flow of Sec. 5.1.2.
#pragma once

#include <map>
#include <memory>
#include <tuple>
#include <vector>

#include "common.h"

namespace hfmm {

struct Plan3Base {
  virtual ~Plan3Base() = default;
};

// Morton keys of the oct-tree: bit 3b of a key is bit b of the x box index,
// bit 3b+1 of y, bit 3b+2 of z (10 bits per axis).
__host__ __device__ __forceinline__ uint32_t spread3(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}
__host__ __device__ __forceinline__ uint32_t compact3(uint32_t v) {
  v &= 0x09249249u;
  v = (v | (v >> 2)) & 0x030c30c3u;
  v = (v | (v >> 4)) & 0x0300f00fu;
  v = (v | (v >> 8)) & 0x030000ffu;
  v = (v | (v >> 16)) & 0x3ffu;
  return v;
}
__host__ __device__ __forceinline__ uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

struct Tree3 {
  int64_t n = 0;
  int L = 0;  // depth; 8^L leaves
  double x0 = 0, y0 = 0, z0 = 0, side_len = 1;
  int leaf_size = 0;
  int64_t nleaves = 1;
  int max_leaf = 0;
  DevBuf<int32_t> perm;      // sorted slot -> caller index
  DevBuf<int32_t> leaf_off;  // nleaves + 1, Morton order
  DevBuf<double4> rel64;     // sorted point minus its leaf centre (w = 0)
  DevBuf<float4> rel32;      // the same in FP32
  // translation plans, keyed by (k, p, precision)
  std::map<std::tuple<double, int, int>, std::unique_ptr<Plan3Base>> plans;
  // a second stream (default priority, non-blocking) on which the far-field
  // chain runs beside the near field, and the events that fork and join it
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  Tree3() = default;
  Tree3(const Tree3&) = delete;
  Tree3& operator=(const Tree3&) = delete;
  ~Tree3();
  double leaf_side() const { return side_len / double(1u << L); }
};

// Depth rule: 0 for leaf_size <= 0, else max(2, smallest L with leaf*8^L >= n).
int tree3_depth(int64_t n, int leaf_size);

// Builds the oct-tree on `stream` (synchronises it).  Throws Error on bad input.
std::unique_ptr<Tree3> build_tree3(const double* d_xyz, int64_t n, double x0, double y0, double z0, double side,
                                   int leaf_size, hipStream_t stream);

// Expansion order of each level 0..L: p_l = p + floor(k d_l / 2), d_l the box
// diameter sqrt(3) side / 2^l.
std::vector<int> fmm3_orders(const Tree3& t, double k, int p);

// phi_i = sum_{j, r_ij != 0} exp(i k r_ij) / (4 pi r_ij) q_j, caller order.
// The far-field chain (P2M, M2M, M2L, L2L) runs on the tree's second stream
// beside the P2P; the L2P waits for both.  stage_ms (or NULL): the stages
// one after another on `stream` (upward: gather, P2M, M2M; M2L; L2L; P2P;
// L2P; total), each timed with hipEvents.
template <class T>
void fmm3_apply(Tree3& t, double k, int p, const cplx<T>* d_q, cplx<T>* d_phi, hipStream_t stream,
                float* stage_ms);

}  // namespace hfmm
