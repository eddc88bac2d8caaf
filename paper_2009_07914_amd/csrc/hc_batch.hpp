// Device descriptor of one operation of a batched launch.
#pragma once

#include <vector>

#include "hc.h"
#include "hc_device.hpp"

namespace hc {

// Operation kinds of batched launches (BATCH_COUNT: insert into a counting table).
enum : uint32_t { BATCH_INSERT = 0, BATCH_RETRIEVE = 1, BATCH_ERASE = 2, BATCH_COUNT = 3 };

struct BatchDesc {
  TableView t;
  const uint32_t* keys;
  const uint32_t* values;   // insert into a single-value table
  uint32_t* values_out;     // retrieve (optional)
  uint8_t* flags;           // status (insert / erase) or found (retrieve); optional
  uint64_t n;
  uint32_t chunk;           // elements per chunk
  uint32_t op;              // BATCH_*
  uint32_t variant;         // index of (G, W) in the mixed-launch set, or MIXED_NONE
  uint32_t reserved;
};

// (group size, window) pairs that one mixed launch can run side by side: the
// windows 8, 16 and 32 with at most 8 slots per lane (a wavefront takes each
// chunk with the chunk's own pair).  Pairs outside it get launches of their own.
constexpr uint32_t MIXED_NONE = 0xFFFFFFFFu;
constexpr uint32_t MIXED_COUNT = 11;
uint32_t mixed_variant(uint32_t G, uint32_t W);

// One persistent launch over descs[0..ndesc) (device arrays, all of operation
// kind `op`, group size G and window W) on `stream`.  counters: the launch's pair of
// work counters (zero at the start, reset by the launch's last wavefront), or NULL
// for a pair from the device's launch-slot ring.
hc_err launch_batch(uint32_t op, uint32_t G, uint32_t W, const BatchDesc* d_descs, const uint64_t* d_chunk_start,
                    uint32_t ndesc, uint64_t total_chunks, unsigned long long* counters, hipStream_t stream);
// The same over descriptors of several (G, W) pairs of the mixed-launch set.
hc_err launch_batch_mixed(uint32_t op, const BatchDesc* d_descs, const uint64_t* d_chunk_start, uint32_t ndesc,
                          uint64_t total_chunks, unsigned long long* counters, hipStream_t stream);

// Words between the counter pairs of consecutive launches of a plan (one 128-byte line each).
constexpr uint32_t PLAN_COUNTER_STRIDE = 16;

struct PlanLaunch {
  uint32_t op, G, W;           // G = W = 0: a mixed launch (each descriptor's own pair)
  uint32_t first_desc, ndesc;  // descriptors [first_desc, first_desc + ndesc)
  uint64_t cs_offset;          // this launch's chunk starts
  uint64_t total_chunks;
};

// Host side of a plan: descriptors, per-launch chunk starts, launches in phase order.
struct PlanHost {
  std::vector<BatchDesc> descs;
  std::vector<uint64_t> cs;
  std::vector<PlanLaunch> launches;
  uint32_t phases = 0;
};

// Validate and lay out `ops` (tables on device `dev`); no device work.
hc_err build_plan(const hc_batch_op* ops, uint32_t count, int dev, PlanHost* out);

// Enqueue a plan whose descriptors and chunk starts are in device memory.  counters:
// PLAN_COUNTER_STRIDE words per launch owned by the plan (zeroed once), or NULL for
// pairs from the launch-slot ring.
hc_err launch_plan(const std::vector<PlanLaunch>& launches, const BatchDesc* d_descs, const uint64_t* d_cs,
                   unsigned long long* counters, hipStream_t stream);

}  // namespace hc
