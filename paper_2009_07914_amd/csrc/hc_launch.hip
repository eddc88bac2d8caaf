// Host side of kernel launches: error recording, device geometry, occupancy, and
// the per-device ring of per-launch work counters.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <string>
#include <unordered_map>

#include "hc_launch.hpp"

namespace hc {

static thread_local std::string g_last_error;

const char* last_error_text() { return g_last_error.c_str(); }

hc_err fail(hc_err e, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return e;
}

hc_err hip_fail(hipError_t e, const char* what) {
  return fail(HC_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

hc_err check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, what);
  return HC_OK;
}

int device_cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) cu = 256;
    cached[dev] = cu;
  }
  return cached[dev];
}

int blocks_per_cu_threads(const void* kernel, int threads) {
  static std::mutex mu;
  static std::unordered_map<const void*, int> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(kernel);
  if (it != cache.end()) return it->second;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess || nb <= 0) nb = 1;
  cache.emplace(kernel, nb);
  return nb;
}

int blocks_per_cu(const void* kernel) { return blocks_per_cu_threads(kernel, BLOCK); }

// Launch slots: per device, LAUNCH_SLOTS pairs of work counters.  A launch's last
// wavefront resets its pair, and the launches of one stream run one after another,
// so every stream gets a pair of its own (the first LAUNCH_SLOTS streams that launch
// on the device; the per-thread default stream counts once per thread): launches of
// different streams never share a pair, however many of them are in flight.  Beyond
// that many streams, pairs are handed out round-robin over the whole ring.
constexpr uint32_t LAUNCH_SLOTS = 1024;
constexpr uint32_t SLOT_WORDS = 16;  // 128 bytes per pair: no two pairs share a cache line

struct DeviceRing {
  unsigned long long* d_ring = nullptr;
  std::mutex mu;
  std::unordered_map<uint64_t, uint32_t> of_stream;  // stream key -> pair
  uint32_t next = 0;                                 // round-robin once every pair is taken
};
static DeviceRing g_rings[64];
static std::mutex g_ring_mu;

hc_err ensure_ring(int dev) {
  if (dev < 0 || dev >= 64) return fail(HC_E_DEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_ring_mu);
  if (g_rings[dev].d_ring) return HC_OK;
  unsigned long long* p = nullptr;
  hipError_t e = hipMalloc((void**)&p, (size_t)LAUNCH_SLOTS * SLOT_WORDS * sizeof(unsigned long long));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(HC_E_NOMEM, "hipMalloc of the launch-slot ring failed");
  }
  e = hipMemset(p, 0, (size_t)LAUNCH_SLOTS * SLOT_WORDS * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    (void)hipFree(p);
    return hip_fail(e, "launch-slot ring init");
  }
  g_rings[dev].d_ring = p;
  return HC_OK;
}

// Workspace pools, one per device, created on first use.
static hipMemPool_t g_pools[64];
static std::mutex g_pool_mu;

hc_err ws_alloc(void** out, uint64_t bytes, hipStream_t s) {
  *out = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return fail(HC_E_DEVICE, "hipGetDevice failed");
  hipMemPool_t pool = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_pool_mu);
    if (g_pools[dev] == nullptr) {
      hipMemPoolProps props = {};
      props.allocType = hipMemAllocationTypePinned;
      props.handleTypes = hipMemHandleTypeNone;
      props.location.type = hipMemLocationTypeDevice;
      props.location.id = dev;
      hipError_t e = hipMemPoolCreate(&pool, &props);
      if (e != hipSuccess) return hip_fail(e, "workspace pool: hipMemPoolCreate");
      uint64_t keep = ~0ull;  // keep freed blocks for the next call
      e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
      if (e != hipSuccess) {
        (void)hipMemPoolDestroy(pool);
        return hip_fail(e, "workspace pool: release threshold");
      }
      g_pools[dev] = pool;
    }
    pool = g_pools[dev];
  }
  if (bytes == 0) bytes = 256;
  const hipError_t e = hipMallocFromPoolAsync(out, bytes, pool, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *out = nullptr;
    return fail(HC_E_NOMEM, "workspace of %llu bytes: %s", (unsigned long long)bytes, hipGetErrorString(e));
  }
  return HC_OK;
}

void ws_release(void* p, hipStream_t s) {
  if (p != nullptr && hipFreeAsync(p, s) != hipSuccess) (void)hipGetLastError();
}

// A key per stream: the handle, or for the per-thread default stream the calling thread
// (each thread has its own such stream).
static uint64_t stream_key(hipStream_t s) {
  if (s != hipStreamPerThread) return (uint64_t)(uintptr_t)s;
  static std::atomic<uint64_t> threads{0};
  thread_local const uint64_t mine = (1ull << 63) | threads.fetch_add(1);
  return mine;
}

WorkCtl work_for(uint64_t n, int G, unsigned grid, hipStream_t s) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  DeviceRing& r = g_rings[dev];
  uint32_t slot;
  {
    std::lock_guard<std::mutex> lock(r.mu);
    const uint64_t key = stream_key(s);
    auto it = r.of_stream.find(key);
    if (it != r.of_stream.end()) {
      slot = it->second;
    } else if (r.of_stream.size() < LAUNCH_SLOTS) {
      slot = (uint32_t)r.of_stream.size();
      r.of_stream.emplace(key, slot);
    } else {
      slot = r.next++ % LAUNCH_SLOTS;
    }
  }
  WorkCtl c;
  c.counters = r.d_ring + (size_t)slot * SLOT_WORDS;
  const uint64_t gpw = 64 / G;  // groups per wavefront
  const uint64_t waves = (uint64_t)grid * (BLOCK / 64);
  uint64_t ch = (n + 2 * waves - 1) / (2 * waves);
  if (ch < gpw) ch = gpw;
  if (ch > 64 * gpw) ch = 64 * gpw;
  c.chunk = (uint32_t)ch;
  return c;
}


}  // namespace hc
