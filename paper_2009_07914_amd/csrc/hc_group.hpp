// Grouped multi-value insert and long-query continuation (see hc_group.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hc.h"
#include "hc_device.hpp"

namespace hc {

constexpr uint64_t HEAVY_RUN = 2048;   // runs at least this long are claimed by a whole block
constexpr uint32_t LONG_BUDGET = 64;   // windows a group scans before handing a query over

uint64_t grouped_workspace_bytes(uint64_t n);
// kind: KIND_MULTI (pairs) or KIND_COUNT (keys; values unused); G: group of the counting insert.
hc_err launch_grouped_insert(const TableView& t, int kind, uint32_t G, uint32_t W, const uint32_t* keys,
                             const uint32_t* values, uint64_t n, void* ws, hipStream_t s);
hc_err launch_zero_u64(unsigned long long* p, uint32_t count, hipStream_t s);

struct BucketView;
// Grouped insert into a bucket list table (one ticket per run of equal keys).
uint64_t bl_grouped_workspace_bytes(uint64_t n);
hc_err launch_bl_grouped(const TableView& t, const BucketView& b, uint32_t G, uint32_t W, const uint32_t* keys,
                         const uint32_t* values, uint64_t n, void* work, hipStream_t s);

// Queries handed over by the count (mode 0) or write (mode 1) pass after `budget`
// windows, and the state of the rounds that finish them, all in one workspace.
struct LongState {
  uint64_t cap;                     // entries the workspace holds
  const unsigned long long* nlong;  // hand-over attempts (word 0 of the workspace; entries: min(*nlong, cap))
  unsigned long long* nopen;        // open entries at the start of each round
  uint64_t* entries;                // mode 0: query index; mode 1: (query index, values written)
  uint64_t* base;                   // next window of the entry's sequence
  uint32_t* flag;                   // 1 once the entry is finished
  uint32_t* done;                   // segments of the current round finished
  uint32_t* lists[2];               // open entries of the current and the next round
};
// Entries of the hand-over list for n queries: long queries are rare; past this many,
// groups walk on by themselves.
uint64_t long_capacity(uint64_t n);
uint64_t long_workspace_bytes(uint64_t cap, int mode);
LongState long_layout(void* ws, uint64_t cap, int mode);
hc_err launch_long_queries(const TableView& t, uint32_t W, int mode, const uint32_t* keys, const LongState& ls,
                           uint64_t n, uint32_t budget, uint64_t* offsets, uint32_t* counts, uint32_t* out,
                           hipStream_t s);

}  // namespace hc
