// Tree build: Morton keys, a stable LSD radix sort (8-bit digits, per-tile
// histograms, one scan, wave-ballot ranking), leaf offsets and leaf-relative
// coordinates.  HBM-bound; runs once per geometry.
#include <algorithm>
#include <cmath>

#include "tree.h"

namespace hfmm {

namespace {

constexpr int kThreads = 256;
constexpr int kTile = 1024;  // 4 rounds of 256 elements per block

__global__ void k_morton(const double* __restrict__ xy, int n, double x0, double y0, double side, int L,
                         uint32_t* __restrict__ keys, int32_t* __restrict__ vals, int* __restrict__ bad) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x = xy[2 * i], y = xy[2 * i + 1];
  bool ok = isfinite(x) && isfinite(y) && x >= x0 && x <= x0 + side && y >= y0 && y <= y0 + side;
  if (!ok) bad[0] = 1;
  int nb = 1 << L;
  int ix = 0, iy = 0;
  if (ok) {
    ix = (int)floor((x - x0) / side * nb);
    iy = (int)floor((y - y0) / side * nb);
    ix = ix < 0 ? 0 : (ix >= nb ? nb - 1 : ix);
    iy = iy < 0 ? 0 : (iy >= nb ? nb - 1 : iy);
  }
  keys[i] = morton((uint32_t)ix, (uint32_t)iy);
  vals[i] = i;
}

__global__ __launch_bounds__(kThreads) void k_digit_hist(const uint32_t* __restrict__ keys, int n, int shift,
                                                         uint32_t* __restrict__ hist, int ntiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  int base = blockIdx.x * kTile;
  for (int r = 0; r < kTile / kThreads; ++r) {
    int e = base + r * kThreads + threadIdx.x;
    if (e < n) atomicAdd(&h[(keys[e] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Exclusive prefix sum in three phases: per-block sums of 1024-element
// chunks, a one-block scan of those sums, then a per-block scan with the
// block's offset added.
__device__ __forceinline__ uint32_t block_excl_scan_1024(uint32_t v, uint32_t* s, uint32_t& total) {
  const int t = threadIdx.x;
  s[t] = v;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t u = t >= off ? s[t - off] : 0u;
    __syncthreads();
    s[t] += u;
    __syncthreads();
  }
  total = s[1023];
  const uint32_t r = s[t] - v;
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(1024) void k_scan_sums(const uint32_t* __restrict__ a, int64_t m,
                                                    uint32_t* __restrict__ sums) {
  __shared__ uint32_t s[1024];
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  uint32_t tot;
  block_excl_scan_1024(i < m ? a[i] : 0u, s, tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// exclusive scan of nb <= 1024 * per block sums, one block
__global__ __launch_bounds__(1024) void k_scan_top(uint32_t* __restrict__ sums, int nb) {
  __shared__ uint32_t s[1024];
  const int per = (nb + 1023) / 1024;
  const int lo = threadIdx.x * per, hi = min(lo + per, nb);
  uint32_t loc = 0;
  for (int i = lo; i < hi; ++i) loc += sums[i];
  uint32_t tot;
  uint32_t run = block_excl_scan_1024(loc, s, tot);
  for (int i = lo; i < hi; ++i) {
    const uint32_t v = sums[i];
    sums[i] = run;
    run += v;
  }
}

__global__ __launch_bounds__(1024) void k_scan_apply(uint32_t* __restrict__ a, int64_t m,
                                                     const uint32_t* __restrict__ sums) {
  __shared__ uint32_t s[1024];
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  uint32_t tot;
  const uint32_t r = block_excl_scan_1024(i < m ? a[i] : 0u, s, tot);
  if (i < m) a[i] = r + sums[blockIdx.x];
}

// Leaf offsets from the sorted keys: slot i opens every leaf in (key[i-1], key[i]].
__global__ void k_leaf_bounds(const uint32_t* __restrict__ skeys, int n, int64_t nleaves,
                              int32_t* __restrict__ off) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t k = skeys[i];
  const int64_t prev = i > 0 ? (int64_t)skeys[i - 1] : -1;
  for (int64_t b = prev + 1; b <= k; ++b) off[b] = i;
  if (i == n - 1)
    for (int64_t b = k + 1; b <= nleaves; ++b) off[b] = n;
}

__global__ __launch_bounds__(kThreads) void k_digit_scatter(const uint32_t* __restrict__ kin,
                                                            const int32_t* __restrict__ vin,
                                                            uint32_t* __restrict__ kout, int32_t* __restrict__ vout,
                                                            int n, int shift, const uint32_t* __restrict__ offs,
                                                            int ntiles) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[kThreads / 64][256];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  run[tid] = offs[(size_t)tid * ntiles + blockIdx.x];
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  int base = blockIdx.x * kTile;
  for (int r = 0; r < kTile / kThreads; ++r) {
    for (int j = 0; j < kThreads / 64; ++j) wcnt[j][tid] = 0;
    __syncthreads();
    int e = base + r * kThreads + tid;
    bool valid = e < n;
    uint32_t key = valid ? kin[e] : 0u;
    int32_t val = valid ? vin[e] : 0;
    uint32_t d = (key >> shift) & 255u;
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      int bit = (d >> b) & 1u;
      uint64_t bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    uint32_t rank = (uint32_t)__popcll(m & lt);
    if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(m);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[d] + rank;
      for (int j = 0; j < w; ++j) pos += wcnt[j][d];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int j = 0; j < kThreads / 64; ++j) add += wcnt[j][tid];
    run[tid] += add;
    __syncthreads();
  }
}

__global__ void k_finalize(const double* __restrict__ xy, const uint32_t* __restrict__ skeys,
                           const int32_t* __restrict__ perm, int n, double x0, double y0, double lside,
                           int32_t* __restrict__ iperm, double2* __restrict__ rel64, float2* __restrict__ rel32) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int o = perm[i];
  iperm[o] = i;
  int ix, iy;
  demorton(skeys[i], ix, iy);
  double cx = x0 + (ix + 0.5) * lside, cy = y0 + (iy + 0.5) * lside;
  double2 r;
  r.x = xy[2 * o] - cx;
  r.y = xy[2 * o + 1] - cy;
  rel64[i] = r;
  rel32[i] = make_float2((float)r.x, (float)r.y);
}

void scan_excl(uint32_t* a, int64_t m, DevBuf<uint32_t>& sums, hipStream_t st) {
  const int nb = (int)((m + 1023) / 1024);
  HFMM_REQUIRE(nb <= 1024 * 1024, "scan: too many elements");
  sums.ensure(nb);
  k_scan_sums<<<nb, 1024, 0, st>>>(a, m, sums.p);
  k_scan_top<<<1, 1024, 0, st>>>(sums.p, nb);
  k_scan_apply<<<nb, 1024, 0, st>>>(a, m, sums.p);
  HFMM_LAUNCH_CHECK();
}

}  // namespace

void radix_sort_pairs(DevBuf<uint32_t>& ka, DevBuf<int32_t>& va, int n, int nbits, hipStream_t stream) {
  HFMM_REQUIRE(n >= 1 && n < (1 << 31) - kTile, "radix_sort_pairs: bad n");
  HFMM_REQUIRE(ka.n >= (size_t)n && va.n >= (size_t)n, "radix_sort_pairs: buffers too small");
  DevBuf<uint32_t> kb(n);
  DevBuf<int32_t> vb(n);
  const int ntiles = (n + kTile - 1) / kTile;
  DevBuf<uint32_t> hist((size_t)256 * ntiles), sums;
  for (int shift = 0; shift < nbits; shift += 8) {
    k_digit_hist<<<ntiles, kThreads, 0, stream>>>(ka.p, n, shift, hist.p, ntiles);
    HFMM_LAUNCH_CHECK();
    scan_excl(hist.p, (int64_t)256 * ntiles, sums, stream);
    k_digit_scatter<<<ntiles, kThreads, 0, stream>>>(ka.p, va.p, kb.p, vb.p, n, shift, hist.p, ntiles);
    HFMM_LAUNCH_CHECK();
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  // the buffers swapped back and forth: the sorted pairs are in ka, va, and
  // the scratch pair (freed here) is the other one.  Freeing synchronises
  // nothing, so wait for the passes before the scratch goes.
  HFMM_HIP(hipStreamSynchronize(stream));
}

void leaf_bounds(const uint32_t* sorted_keys, int n, int64_t nleaves, int32_t* off, hipStream_t stream) {
  k_leaf_bounds<<<(n + 255) / 256, 256, 0, stream>>>(sorted_keys, n, nleaves, off);
  HFMM_LAUNCH_CHECK();
}

int tree_depth(int64_t n, int leaf_size) {
  if (leaf_size <= 0) return 0;
  int L = 0;
  while ((double)leaf_size * std::pow(4.0, L) < (double)n) ++L;
  return std::max(2, L);
}

std::unique_ptr<Tree> build_tree(const double* d_xy, int64_t n, double x0, double y0, double side,
                                 int leaf_size, hipStream_t stream) {
  HFMM_REQUIRE(n >= 1, "build_tree: n must be >= 1");
  HFMM_REQUIRE(n < (int64_t(1) << 31) - kTile, "build_tree: n must fit in int32");
  HFMM_REQUIRE(std::isfinite(side) && side > 0, "build_tree: side must be finite and > 0");
  HFMM_REQUIRE(std::isfinite(x0) && std::isfinite(y0), "build_tree: root corner must be finite");
  HFMM_REQUIRE(leaf_size >= 0, "build_tree: leaf_size must be >= 0");
  HFMM_REQUIRE(d_xy != nullptr, "build_tree: d_xy is NULL");
  auto t = std::make_unique<Tree>();
  t->n = n;
  t->L = tree_depth(n, leaf_size);
  HFMM_REQUIRE(t->L <= 12, "build_tree: depth above 12 (raise leaf_size)");
  t->x0 = x0;
  t->y0 = y0;
  t->side_len = side;
  t->leaf_size = leaf_size;
  t->nleaves = int64_t(1) << (2 * t->L);
  const int N = (int)n;
  const int blocks = (N + 255) / 256;

  DevBuf<uint32_t> ka(N), kb(N);
  DevBuf<int32_t> va(N), vb(N);
  DevBuf<int> bad(1);
  HFMM_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), stream));
  k_morton<<<blocks, 256, 0, stream>>>(d_xy, N, x0, y0, side, t->L, ka.p, va.p, bad.p);
  HFMM_LAUNCH_CHECK();
  int hbad = 0;
  HFMM_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, stream));
  HFMM_HIP(hipStreamSynchronize(stream));
  HFMM_REQUIRE(hbad == 0, "build_tree: a coordinate is non-finite or outside the root box");

  // stable LSD radix sort of (key, index) over the 2L key bits
  const int ntiles = (N + kTile - 1) / kTile;
  DevBuf<uint32_t> hist((size_t)256 * ntiles), sums;
  for (int shift = 0; shift < 2 * t->L; shift += 8) {
    k_digit_hist<<<ntiles, kThreads, 0, stream>>>(ka.p, N, shift, hist.p, ntiles);
    HFMM_LAUNCH_CHECK();
    scan_excl(hist.p, (int64_t)256 * ntiles, sums, stream);
    k_digit_scatter<<<ntiles, kThreads, 0, stream>>>(ka.p, va.p, kb.p, vb.p, N, shift, hist.p, ntiles);
    HFMM_LAUNCH_CHECK();
    std::swap(ka, kb);
    std::swap(va, vb);
  }

  t->perm = std::move(va);
  t->iperm.alloc(N);
  t->rel64.alloc(N);
  t->rel32.alloc(N);
  k_finalize<<<blocks, 256, 0, stream>>>(d_xy, ka.p, t->perm.p, N, x0, y0, t->leaf_side(), t->iperm.p,
                                         t->rel64.p, t->rel32.p);
  HFMM_LAUNCH_CHECK();
  t->leaf_off.alloc(t->nleaves + 1);
  k_leaf_bounds<<<blocks, 256, 0, stream>>>(ka.p, N, t->nleaves, t->leaf_off.p);
  HFMM_LAUNCH_CHECK();
  t->leaf_off_h.resize(t->nleaves + 1);
  HFMM_HIP(hipMemcpyAsync(t->leaf_off_h.data(), t->leaf_off.p, (t->nleaves + 1) * sizeof(int32_t),
                          hipMemcpyDeviceToHost, stream));
  HFMM_HIP(hipStreamSynchronize(stream));
  int mx = 0;
  for (int64_t b = 0; b < t->nleaves; ++b) mx = std::max(mx, t->leaf_off_h[b + 1] - t->leaf_off_h[b]);
  t->max_leaf = mx;
  if (t->leaf_off_h[t->nleaves] != N) throw Error(HFMM_ERR_INTERNAL, "build_tree: leaf offsets do not sum to n");
  if (t->L >= 2) {
    HFMM_HIP(hipStreamCreateWithFlags(&t->side, hipStreamNonBlocking));
    HFMM_HIP(hipEventCreateWithFlags(&t->fork, hipEventDisableTiming | hipEventDisableSystemFence));
    HFMM_HIP(hipEventCreateWithFlags(&t->join, hipEventDisableTiming | hipEventDisableSystemFence));
  }
  return t;
}

Tree::~Tree() {
  if (side) {
    (void)hipStreamSynchronize(side);
    (void)hipStreamDestroy(side);
  }
  if (fork) (void)hipEventDestroy(fork);
  if (join) (void)hipEventDestroy(join);
}

}  // namespace hfmm
