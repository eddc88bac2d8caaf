// Device descriptor of one operation of a batched launch.
#pragma once

#include <vector>

#include "hc.h"
#include "hc_device.hpp"

namespace hc {

// Operation kinds of batched launches (BATCH_COUNT: insert into a counting table).
// BATCH_ALL marks a launch whose descriptors carry kinds of their own (one-launch plans).
enum : uint32_t { BATCH_INSERT = 0, BATCH_RETRIEVE = 1, BATCH_ERASE = 2, BATCH_COUNT = 3, BATCH_ALL = 4 };

// No completion counter (BatchDesc::gate_post / gate_wait).
constexpr uint32_t NO_GATE = 0xFFFFFFFFu;

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
  // one-launch plans: a chunk first waits until completion counter gate_wait reaches
  // gate_need (every chunk of the table's previous phase done), and afterwards adds 1 to
  // counter gate_post (read by the table's next phase); NO_GATE: neither
  uint32_t gate_post;
  uint32_t gate_wait;
  uint32_t pad;
  uint64_t gate_need;
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

// One launch over the descriptors of every phase (all with group size G and window W,
// any kinds, ordered by phase): chunks of a table's later phase wait on the device for
// the completion counters of its previous phase.  gates: ngates counters (zero at the
// start, reset by the launch's last wavefront); abandoned: incremented by every wait given
// up after wait_ticks ticks of the device's constant-rate clock.
hc_err launch_batch_one(uint32_t G, uint32_t W, const BatchDesc* d_descs, const uint64_t* d_chunk_start,
                        uint32_t ndesc, uint64_t total_chunks, unsigned long long* counters,
                        unsigned long long* gates, uint32_t ngates, unsigned long long* abandoned,
                        uint64_t wait_ticks, hipStream_t stream);

// Words between the counter pairs of consecutive launches of a plan (one 128-byte line each).
constexpr uint32_t PLAN_COUNTER_STRIDE = 16;

struct PlanLaunch {
  uint32_t op, G, W;           // G = W = 0: a mixed launch (each descriptor's own pair)
  uint32_t first_desc, ndesc;  // descriptors [first_desc, first_desc + ndesc)
  uint64_t cs_offset;          // this launch's chunk starts
  uint64_t total_chunks;
};

// Host side of a plan: descriptors, per-launch chunk starts, launches in phase order.
// A one-launch plan has a single launch of kind BATCH_ALL and `gates` completion counters.
struct PlanHost {
  std::vector<BatchDesc> descs;
  std::vector<uint64_t> cs;
  std::vector<PlanLaunch> launches;
  uint32_t phases = 0;
  uint32_t gates = 0;
};

// Validate and lay out `ops` (tables on device `dev`); no device work.  one_launch: every
// phase in one gated launch (every operation must have the same group size and window).
hc_err build_plan(const hc_batch_op* ops, uint32_t count, int dev, PlanHost* out, bool one_launch = false);

// Words of a plan's counter block: the launches' counter pairs, then (one-launch plans, with
// or without completion counters) a line holding the abandoned-wait count, then the
// completion counters.
inline uint64_t plan_counter_words(const PlanHost& p) {
  bool one = false;
  for (const PlanLaunch& L : p.launches) one |= L.op == BATCH_ALL;
  return (uint64_t)p.launches.size() * PLAN_COUNTER_STRIDE + (one ? PLAN_COUNTER_STRIDE + p.gates : 0);
}

// Enqueue a plan whose descriptors and chunk starts are in device memory.  counters:
// plan_counter_words() words owned by the plan (zeroed once), or NULL for pairs from the
// launch-slot ring (plans without gates only).  wait_ticks: see launch_batch_one.
hc_err launch_plan(const std::vector<PlanLaunch>& launches, const BatchDesc* d_descs, const uint64_t* d_cs,
                   unsigned long long* counters, hipStream_t stream, uint32_t gates = 0, uint64_t wait_ticks = 0);

}  // namespace hc
