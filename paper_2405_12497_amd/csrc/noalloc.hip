// rbq_search_noalloc: the search of rbq_search with its whole workspace carved
// from a file-scope device array instead of allocated, for callers that cannot
// allocate device memory (code under stream capture, serving loops with a
// fixed memory budget).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/rabitq.h"
#include "rbq_runtime.hpp"

namespace rbq {

// The workspace of rbq_search_noalloc; each GPU holds its own copy until the
// process ends.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on the current device: looked up once per
// device with that device current (host code must not use the array's name,
// which is only a host-side stand-in).
rbq_status noalloc_scratch(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return set_error(RBQ_EDEVICE, "rbq_search_noalloc: no current device");
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return set_error(RBQ_EDEVICE, "rbq_search_noalloc: hipGetSymbolAddress of the scratch array failed");
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return RBQ_OK;
}

}  // namespace rbq

extern "C" rbq_status rbq_search_noalloc(rbq_index* idx, const float* queries, int64_t nq,
                                         const rbq_search_opts* opts, int64_t* out_ids, float* out_dists,
                                         void* stream) {
  void* base = nullptr;
  const rbq_status rs = rbq::noalloc_scratch(&base);
  if (rs != RBQ_OK) return rs;
  return rbq::search_in_arena(idx, queries, nq, opts, out_ids, out_dists, base, rbq::kNoAllocScratchBytes,
                              (hipStream_t)stream);
}
