// hc_count_values_noalloc: the multi-value count pass for callers that cannot
// allocate device memory (code being captured into a HIP graph, serving loops that
// forbid allocation).  Its scratch memory -- the scan's tile sums and the long-query
// list -- lives in a fixed device array of this translation unit, one per GPU, held
// until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hc.h"
#include "hc_launch.hpp"

namespace hc {

constexpr uint64_t NOALLOC_SCRATCH_BYTES = 16ull << 20;
constexpr uint64_t NOALLOC_MAX_QUERIES = 1ull << 28;

// Device memory of the no-allocation entry point.  In host code this name is only a
// symbol: kernels get the device address from hipGetSymbolAddress (per device).
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static void* g_scratch[64];
static std::mutex g_scratch_mu;

// The device address of `scratch` on device `dev` (the current device), looked up once.
static hc_err scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= 64) return fail(HC_E_DEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the scratch array");
    if (p == nullptr) return fail(HC_E_DEVICE, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return HC_OK;
}

}  // namespace hc

extern "C" {

hc_err hc_count_values_noalloc(hc_table t, const uint32_t* d_keys, uint64_t n, uint32_t* d_counts,
                               uint64_t* d_offsets, uint64_t* h_total, uint32_t group, void* stream) {
  using namespace hc;
  if (t == nullptr) return fail(HC_E_ARG, "table handle is NULL");
  if (n > NOALLOC_MAX_QUERIES)
    return fail(HC_E_ARG, "hc_count_values_noalloc takes at most %llu queries (%llu given)",
                (unsigned long long)NOALLOC_MAX_QUERIES, (unsigned long long)n);
  // the table's device is made current before the symbol lookup and the launches
  int dev = -1;
  if (hc_err r = table_device(t, &dev); r != HC_OK) return r;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(HC_E_DEVICE, "hipGetDevice failed");
  if (cur != dev) {
    const hipError_t e = hipSetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  }
  void* ws = nullptr;
  if (hc_err r = scratch_address(dev, &ws); r != HC_OK) return r;
  return count_values_into(t, d_keys, n, d_counts, d_offsets, h_total, group, ws, NOALLOC_SCRATCH_BYTES, stream);
}

}  // extern "C"
