// Internal declarations shared by the libhfmm translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "hfmm.h"

namespace hfmm {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  hfmm_status code;
  Error(hfmm_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

#define HFMM_HIP(expr)                                                                        \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      throw ::hfmm::Error(e_ == hipErrorOutOfMemory ? HFMM_ERR_OOM : HFMM_ERR_HIP,            \
                          std::string(#expr) + ": " + hipGetErrorString(e_));                 \
  } while (0)

#define HFMM_REQUIRE(cond, msg)                              \
  do {                                                       \
    if (!(cond)) throw ::hfmm::Error(HFMM_ERR_ARG, (msg));   \
  } while (0)

#define HFMM_LAUNCH_CHECK() HFMM_HIP(hipGetLastError())

// ---------------------------------------------------------------- device buffer
// Owning device allocation (setup paths only).
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t count) {
    release();
    if (count) {
      const hipError_t e = hipMalloc(&p, count * sizeof(T));
      if (e != hipSuccess) {
        p = nullptr;
        throw Error(e == hipErrorOutOfMemory ? HFMM_ERR_OOM : HFMM_ERR_HIP,
                    "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes: " + hipGetErrorString(e));
      }
    }
    n = count;
  }
  void ensure(size_t count) { if (count > n) alloc(count); }
  void release() { if (p) (void)hipFree(p); p = nullptr; n = 0; }
  void upload(const T* h, size_t count) {
    ensure(count);
    if (count) HFMM_HIP(hipMemcpy(p, h, count * sizeof(T), hipMemcpyHostToDevice));
  }
  void upload(const std::vector<T>& h) { upload(h.data(), h.size()); }
};

// ---------------------------------------------------------------- complex helpers
template <class T> struct c2 { using type = void; };
template <> struct c2<float> { using type = float2; };
template <> struct c2<double> { using type = double2; };
template <class T> using cplx = typename c2<T>::type;

template <class T>
__host__ __device__ __forceinline__ cplx<T> mk(T re, T im) { cplx<T> r; r.x = re; r.y = im; return r; }

// ---------------------------------------------------------------- Morton keys
// bit 2b of a key is bit b of the x box index, bit 2b+1 is bit b of y.
__host__ __device__ __forceinline__ uint32_t spread_bits(uint32_t v) {
  v &= 0x0000ffffu;
  v = (v | (v << 8)) & 0x00ff00ffu;
  v = (v | (v << 4)) & 0x0f0f0f0fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}
__host__ __device__ __forceinline__ uint32_t compact_bits(uint32_t v) {
  v &= 0x55555555u;
  v = (v | (v >> 1)) & 0x33333333u;
  v = (v | (v >> 2)) & 0x0f0f0f0fu;
  v = (v | (v >> 4)) & 0x00ff00ffu;
  v = (v | (v >> 8)) & 0x0000ffffu;
  return v;
}
__host__ __device__ __forceinline__ uint32_t morton(uint32_t ix, uint32_t iy) {
  return spread_bits(ix) | (spread_bits(iy) << 1);
}
__host__ __device__ __forceinline__ void demorton(uint32_t key, int& ix, int& iy) {
  ix = (int)compact_bits(key);
  iy = (int)compact_bits(key >> 1);
}

}  // namespace hfmm
