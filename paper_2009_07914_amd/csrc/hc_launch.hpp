// Host-side launch helpers shared by the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "hc.h"
#include "hc_device.hpp"

namespace hc {

// Record a message for hc_last_error() (thread-local) and return `e`.
hc_err fail(hc_err e, const char* fmt, ...);
hc_err hip_fail(hipError_t e, const char* what);  // HC_E_DEVICE with the HIP error text
const char* last_error_text();
// Allocate the device's launch-slot ring (once per device; synchronises the first time).
hc_err ensure_ring(int dev);

// Per-call device workspace.  Each call that needs scratch memory takes its own
// block from a library-owned memory pool of the current device, ordered on the
// call's stream, and gives it back on the same stream when its last kernel is
// enqueued; calls on different streams therefore never share a workspace, and
// no call synchronises the device to grow or release one.  The pool keeps freed
// blocks for reuse instead of returning them to the system.
hc_err ws_alloc(void** out, uint64_t bytes, hipStream_t s);
void ws_release(void* p, hipStream_t s);

// A workspace held for the duration of one call (released on every return path).
struct CallWs {
  void* p = nullptr;
  hipStream_t s = nullptr;
  explicit CallWs(hipStream_t stream) : s(stream) {}
  CallWs(const CallWs&) = delete;
  CallWs& operator=(const CallWs&) = delete;
  hc_err get(uint64_t bytes) { return ws_alloc(&p, bytes, s); }
  ~CallWs() {
    if (p) ws_release(p, s);
  }
};

// The device a table lives on.
hc_err table_device(hc_table t, int* dev);

// hc_count_values in a caller-given workspace (256-byte aligned, ws_bytes long): the scan's
// tile sums, then a long-query list of as many entries as fit (at most n/16 + 1024).
// HC_E_ARG if the tile sums or a single list entry do not fit.
hc_err count_values_into(hc_table t, const uint32_t* d_keys, uint64_t n, uint32_t* d_counts, uint64_t* d_offsets,
                         uint64_t* h_total, uint32_t group, void* ws, uint64_t ws_bytes, void* stream);

// Number of compute units of the current device (cached per device).
int device_cu_count();

// Resident blocks per CU of a kernel (occupancy calculator, cached per kernel).
int blocks_per_cu(const void* kernel);
int blocks_per_cu_threads(const void* kernel, int threads);

// Grid for a bulk kernel: the device's resident capacity, or fewer blocks when
// the batch is small (at most one element per group).
template <typename Kernel>
inline unsigned grid_for(Kernel kernel, uint64_t n, int G) {
  const uint64_t gpb = BLOCK / G;
  const uint64_t need = (n + gpb - 1) / gpb;
  const uint64_t cap = (uint64_t)device_cu_count() * (uint64_t)blocks_per_cu(reinterpret_cast<const void*>(kernel));
  const uint64_t g = need < cap ? need : cap;
  return (unsigned)(g == 0 ? 1 : g);
}

// Work control of one launch on stream s: the stream's counter pair from the device's
// launch slots and a chunk size giving every wavefront about two chunks, between one
// element per group and 64 elements per group.
WorkCtl work_for(uint64_t n, int G, unsigned grid, hipStream_t s);

hc_err check_launch(const char* what);

template <int V>
using ic = std::integral_constant<int, V>;

// Call f(ic<G>, ic<W>) for runtime G in {1..64} and W in {8,16,32,64}.
template <int W, typename F>
inline hc_err dispatch_g(uint32_t G, F&& f) {
  switch (G) {
    case 1: return f(ic<1>{}, ic<W>{});
    case 2: return f(ic<2>{}, ic<W>{});
    case 4: return f(ic<4>{}, ic<W>{});
    case 8: return f(ic<8>{}, ic<W>{});
    case 16: return f(ic<16>{}, ic<W>{});
    case 32: return f(ic<32>{}, ic<W>{});
    case 64: return f(ic<64>{}, ic<W>{});
    default: return fail(HC_E_ARG, "group size %u is not a power of two in [1, 64]", G);
  }
}

template <typename F>
inline hc_err dispatch_gw(uint32_t G, uint32_t W, F&& f) {
  switch (W) {
    case 8: return dispatch_g<8>(G, f);
    case 16: return dispatch_g<16>(G, f);
    case 32: return dispatch_g<32>(G, f);
    case 64: return dispatch_g<64>(G, f);
    default: return fail(HC_E_ARG, "window %u is not one of 8, 16, 32, 64", W);
  }
}

// Launchers, one translation unit each.
hc_err launch_insert(const TableView& t, int kind, uint32_t G, uint32_t W, const uint32_t* keys,
                     const uint32_t* values, uint64_t n, uint8_t* status, hipStream_t stream);
// Counting insert with the equal keys of each tile combined in LDS first (hc_k_count.hip).
hc_err launch_count_insert(const TableView& t, uint32_t G, uint32_t W, const uint32_t* keys, uint64_t n,
                           uint8_t* status, hipStream_t stream);
hc_err launch_retrieve(const TableView& t, uint32_t G, uint32_t W, const uint32_t* keys, uint64_t n,
                       uint32_t* values_out, uint8_t* found_out, hipStream_t stream);
hc_err launch_erase(const TableView& t, int kind, uint32_t G, uint32_t W, const uint32_t* keys, uint64_t n,
                    uint8_t* status, hipStream_t stream);
// budget: windows a group scans before handing the query to the long-query kernel
// (appending it to long_list, which holds long_cap entries; once it is full, groups
// walk on by themselves); 0xFFFFFFFF: never.
hc_err launch_count_multi(const TableView& t, uint32_t G, uint32_t W, const uint32_t* keys, uint64_t n,
                          uint32_t* counts, uint64_t* offsets, uint8_t* found_out, uint32_t budget,
                          uint64_t* long_list, unsigned long long* long_n, uint64_t long_cap, hipStream_t stream);
hc_err launch_write_multi(const TableView& t, uint32_t G, uint32_t W, const uint32_t* keys, uint64_t n,
                          const uint64_t* offsets, uint32_t* out, uint32_t budget, uint64_t* long_list,
                          unsigned long long* long_n, uint64_t long_cap, hipStream_t stream);

}  // namespace hc
