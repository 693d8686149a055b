// The FMM apply without device allocation, for callers that cannot call
// hipMalloc (work under HIP graph capture, tight serving loops, harnesses
// that forbid it).  Its work arrays (multipole and local expansions of every
// level, the far field and the sorted charges) live in `scratch`, a fixed
// device array of kScratchBytes that every GPU the library runs on holds
// until the process ends.
//
// In host code `scratch` names a host-side stand-in, not the device array:
// its device address is looked up once per device with hipGetSymbolAddress
// (on the entry point's first call with that device current) and only that
// address is ever passed to kernels.  Every call on a GPU shares that GPU's
// array, so calls that overlap on one GPU (concurrent streams or threads)
// race.  Each kernel of the apply writes every element it later reads (P2M
// every leaf, M2M every parent, M2L every target box, L2P every point), so
// nothing has to start at zero and the last call's contents do no harm.
#include <mutex>
#include <vector>

#include "handles.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device ordinal: the device address of `scratch`

void* scratch_for_current_device() {
  int dev = 0;
  HFMM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HFMM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    HFMM_REQUIRE(p != nullptr, "fmm_apply_noalloc: no device address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

hfmm_status hfmm_fmm_apply_noalloc(hfmm_tree t, double k, int32_t p, hfmm_precision prec, const void* d_q,
                                   void* d_phi, int32_t nrhs, hipStream_t stream) {
  HFMM_GUARD_BEGIN
  HFMM_REQUIRE(t != nullptr && t->t, "fmm_apply_noalloc: NULL tree");
  HFMM_REQUIRE(prec == HFMM_FP64 || prec == HFMM_FP32, "fmm_apply_noalloc: unknown precision");
  HFMM_REQUIRE(nrhs >= 1 && nrhs <= 1024, "fmm_apply_noalloc: nrhs must be in [1, 1024]");
  HFMM_REQUIRE(std::isfinite(k) && k > 0, "fmm_apply_noalloc: k must be finite and > 0");
  HFMM_REQUIRE(p >= 1 && p <= 40, "fmm_apply_noalloc: p must be in [1, 40]");
  HFMM_REQUIRE(d_q != nullptr && d_phi != nullptr, "fmm_apply_noalloc: NULL array");
  void* base = scratch_for_current_device();
  const size_t need =
      prec == HFMM_FP64
          ? hfmm::fmm_apply_scratch<double>(*t->t, k, p, static_cast<const double2*>(d_q),
                                            static_cast<double2*>(d_phi), nrhs, base, kScratchBytes, stream)
          : hfmm::fmm_apply_scratch<float>(*t->t, k, p, static_cast<const float2*>(d_q), static_cast<float2*>(d_phi),
                                           nrhs, base, kScratchBytes, stream);
  if (need)
    throw hfmm::Error(HFMM_ERR_ARG, "fmm_apply_noalloc: the apply needs " + std::to_string(need) +
                                        " bytes of work memory, above the fixed " + std::to_string(kScratchBytes) +
                                        "; use fewer columns, FP32, or hfmm_fmm_apply");
  return HFMM_OK;
  HFMM_GUARD_END
}

int64_t hfmm_fmm_noalloc_capacity(void) { return (int64_t)kScratchBytes; }

}  // extern "C"
