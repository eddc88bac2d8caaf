// Batched launches over many tables (one persistent kernel per phase).
//
// A phase is a list of operations that may run concurrently: operations on
// different tables are independent, and operations of one kind on one table may
// overlap (Sec. IV-D).  Every wavefront takes (operation, chunk) items from a
// global counter in list order and processes the chunk with the operation's own
// kind, group size and window, so tables of very different sizes and tunings
// share one launch.  Operations on a table whose kind changes go to a later
// phase, i.e. a later launch on the same stream; the kernel boundary orders them
// and makes the earlier phase's writes visible on every XCD.
#include "hc_batch.hpp"
#include "hc_kernels.hpp"
#include "hc_launch.hpp"

namespace hc {

// Per-wavefront LDS ring of the batched retrieve's outputs (see drive_range_staged).
using BatchRing = OutRing<128, uint32_t>;

template <uint32_t OP, int G, int W>
__device__ __forceinline__ void run_chunk(const BatchDesc& d, uint64_t begin, uint64_t end, BatchRing* ring) {
  if constexpr (OP == BATCH_INSERT) {
    InsertUnique<G, W, KIND_SINGLE> op;
    op.t = d.t;
    op.keys = d.keys;
    op.values = d.values;
    op.status = d.flags;
    drive_range<G>(begin, end, op);
  } else if constexpr (OP == BATCH_COUNT) {
    InsertUnique<G, W, KIND_COUNT> op;
    op.t = d.t;
    op.keys = d.keys;
    op.values = nullptr;
    op.status = d.flags;
    drive_range<G>(begin, end, op);
  } else if constexpr (OP == BATCH_RETRIEVE) {
    Retrieve<G, W> op;
    op.t = d.t;
    op.keys = d.keys;
    op.values_out = d.values_out;
    op.found_out = d.flags;
    drive_range_staged<G, Retrieve<G, W>::RING>(begin, end, op, *ring);
  } else {
    Erase<G, W, KIND_SINGLE> op;
    op.t = d.t;
    op.keys = d.keys;
    op.status = d.flags;
    drive_range<G>(begin, end, op);
  }
}

// Every wavefront takes (descriptor, chunk) items from the launch's counter until
// none is left and runs body(descriptor, first element, end) on each; the last
// wavefront to leave resets the counters for the launch slot's next use (and the
// nreset words at `reset`).
// chunk_start[d] = first global chunk of descriptor d; chunk_start[ndesc] = total.
template <typename Body>
__device__ __forceinline__ void take_chunks(const BatchDesc* __restrict__ descs,
                                            const uint64_t* __restrict__ chunk_start, uint32_t ndesc, WorkCtl ctl,
                                            Body&& body, unsigned long long* reset = nullptr,
                                            uint32_t nreset = 0) {
  const uint32_t lane = __lane_id();
  const uint64_t total = chunk_start[ndesc];
  for (;;) {
    unsigned long long c = 0;
    if (lane == 0) c = atomicAdd(ctl.counters, 1ull);
    c = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(c >> 32)) << 32) |
        __builtin_amdgcn_readfirstlane((uint32_t)c);
    if (c >= total) break;
    uint32_t lo = 0, hi = ndesc;  // the last d with chunk_start[d] <= c
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) / 2;
      if (chunk_start[mid] <= c) lo = mid;
      else hi = mid;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const BatchDesc d = descs[lo];
    const uint64_t begin = (c - chunk_start[lo]) * d.chunk;
    const uint64_t end = begin + d.chunk < d.n ? begin + d.chunk : d.n;
    body(d, begin, end);
  }
  uint32_t last = 0;
  if (lane == 0) {
    const unsigned long long waves = (unsigned long long)gridDim.x * (BLOCK / 64);
    if (atomicAdd(ctl.counters + 1, 1ull) == waves - 1) {
      atomicExch(ctl.counters, 0ull);
      atomicExch(ctl.counters + 1, 0ull);
      last = 1;
    }
  }
  if (nreset != 0 && __builtin_amdgcn_readfirstlane(last) != 0)
    for (uint32_t j = lane; j < nreset; j += 64) atomicExch(reset + j, 0ull);
}

// One kernel per (operation kind, group size, window): every descriptor of a
// launch has them, so the kernel keeps the register budget of a single-table
// kernel.
template <uint32_t OP, int G, int W>
__global__ __launch_bounds__(BLOCK) void k_batch(const BatchDesc* __restrict__ descs,
                                                 const uint64_t* __restrict__ chunk_start, uint32_t ndesc,
                                                 WorkCtl ctl) {
  __shared__ BatchRing rings[OP == BATCH_RETRIEVE ? BLOCK / 64 : 1];
  BatchRing* ring = &rings[OP == BATCH_RETRIEVE ? (threadIdx.x >> 6) : 0];
  take_chunks(descs, chunk_start, ndesc, ctl,
              [ring](const BatchDesc& d, uint64_t begin, uint64_t end) { run_chunk<OP, G, W>(d, begin, end, ring); });
}

// Mixed launch: each chunk runs with its descriptor's (G, W) pair, so tables
// tuned to different pairs still share one launch per operation kind (the
// descriptor is wavefront-uniform, so is the branch).  The register budget is
// that of the largest pair of the set.
template <uint32_t OP>
__global__ __launch_bounds__(BLOCK) void k_batch_mixed(const BatchDesc* __restrict__ descs,
                                                       const uint64_t* __restrict__ chunk_start, uint32_t ndesc,
                                                       WorkCtl ctl) {
  __shared__ BatchRing rings[OP == BATCH_RETRIEVE ? BLOCK / 64 : 1];
  BatchRing* ring = &rings[OP == BATCH_RETRIEVE ? (threadIdx.x >> 6) : 0];
  take_chunks(descs, chunk_start, ndesc, ctl, [ring](const BatchDesc& d, uint64_t begin, uint64_t end) {
    switch (d.variant) {
      case 0: run_chunk<OP, 1, 8>(d, begin, end, ring); break;
      case 1: run_chunk<OP, 2, 8>(d, begin, end, ring); break;
      case 2: run_chunk<OP, 4, 8>(d, begin, end, ring); break;
      case 3: run_chunk<OP, 8, 8>(d, begin, end, ring); break;
      case 4: run_chunk<OP, 2, 16>(d, begin, end, ring); break;
      case 5: run_chunk<OP, 4, 16>(d, begin, end, ring); break;
      case 6: run_chunk<OP, 8, 16>(d, begin, end, ring); break;
      case 7: run_chunk<OP, 16, 16>(d, begin, end, ring); break;
      case 8: run_chunk<OP, 4, 32>(d, begin, end, ring); break;
      case 9: run_chunk<OP, 8, 32>(d, begin, end, ring); break;
      case 10: run_chunk<OP, 16, 32>(d, begin, end, ring); break;
      default: break;  // the planner puts no other pair into a mixed launch
    }
  });
}

// ---- one launch over every phase -------------------------------------------------------
//
// A plan's phases exist because a table's operations of different kinds must not
// overlap.  Here the chunks of all phases are handed out from one counter in phase
// order, and a chunk of a table's later phase first waits for the table's previous
// phase: each finished chunk adds 1 to its (table, phase) completion counter after a
// device-scope release, and the waiting wavefront spins on that counter and then
// acquires.  Waiting cannot deadlock: every chunk waited for was taken earlier from the
// same counter by a wavefront that is running and only waits, if at all, on chunks taken
// earlier still, down to the first phase, which never waits.  Each wait is still bounded
// by the device clock (a plan bug then shows as a counted abandoned wait, never a hang).

__device__ __forceinline__ void gate_wait(unsigned long long* gate, uint64_t need, unsigned long long* abandoned,
                                          uint64_t ticks) {
  if (__lane_id() == 0) {
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(gate, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
      if (wall_clock64() - t0 > ticks) {
        atomicAdd(abandoned, 1ull);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the previous phase's writes, from every XCD
}

__device__ __forceinline__ void gate_post(unsigned long long* gate) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // this chunk's writes before it counts as done
  if (__lane_id() == 0) atomicAdd(gate, 1ull);
}

template <int G, int W>
__global__ __launch_bounds__(BLOCK) void k_batch_one(const BatchDesc* __restrict__ descs,
                                                     const uint64_t* __restrict__ chunk_start, uint32_t ndesc,
                                                     WorkCtl ctl, unsigned long long* gates, uint32_t ngates,
                                                     unsigned long long* abandoned, uint64_t ticks) {
  __shared__ BatchRing rings[BLOCK / 64];
  BatchRing* ring = &rings[threadIdx.x >> 6];
  // the last counter this wavefront saw complete: a later chunk waiting for it needs no
  // second wait or acquire (no write of that phase remains to be seen)
  uint32_t passed = NO_GATE;
  take_chunks(
      descs, chunk_start, ndesc, ctl,
      [&](const BatchDesc& d, uint64_t begin, uint64_t end) {
        if (d.gate_wait != NO_GATE && d.gate_wait != passed) {
          gate_wait(gates + d.gate_wait, d.gate_need, abandoned, ticks);
          passed = d.gate_wait;
        }
        switch (d.op) {
          case BATCH_INSERT: run_chunk<BATCH_INSERT, G, W>(d, begin, end, ring); break;
          case BATCH_COUNT: run_chunk<BATCH_COUNT, G, W>(d, begin, end, ring); break;
          case BATCH_RETRIEVE: run_chunk<BATCH_RETRIEVE, G, W>(d, begin, end, ring); break;
          default: run_chunk<BATCH_ERASE, G, W>(d, begin, end, ring); break;
        }
        if (d.gate_post != NO_GATE) gate_post(gates + d.gate_post);
      },
      gates, ngates);
}

uint32_t mixed_variant(uint32_t G, uint32_t W) {
  switch (W) {
    case 8: return G == 1 ? 0 : G == 2 ? 1 : G == 4 ? 2 : G == 8 ? 3 : MIXED_NONE;
    case 16: return G == 2 ? 4 : G == 4 ? 5 : G == 8 ? 6 : G == 16 ? 7 : MIXED_NONE;
    case 32: return G == 4 ? 8 : G == 8 ? 9 : G == 16 ? 10 : MIXED_NONE;
    default: return MIXED_NONE;
  }
}

template <typename K, typename... Extra>
static hc_err launch_persistent(K k, const BatchDesc* d_descs, const uint64_t* d_chunk_start, uint32_t ndesc,
                                uint64_t total_chunks, unsigned long long* counters, hipStream_t stream,
                                Extra... extra) {
  const uint64_t cap = (uint64_t)device_cu_count() * (uint64_t)blocks_per_cu(reinterpret_cast<const void*>(k));
  const uint64_t need = (total_chunks + (BLOCK / 64) - 1) / (BLOCK / 64);
  const unsigned grid = (unsigned)(need < cap ? need : cap);
  WorkCtl ctl = work_for(0, 64, grid, stream);
  if (counters != nullptr) ctl.counters = counters;
  hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, stream, d_descs, d_chunk_start, ndesc, ctl, extra...);
  return check_launch("batch");
}

hc_err launch_batch_one(uint32_t G, uint32_t W, const BatchDesc* d_descs, const uint64_t* d_chunk_start,
                        uint32_t ndesc, uint64_t total_chunks, unsigned long long* counters,
                        unsigned long long* gates, uint32_t ngates, unsigned long long* abandoned,
                        uint64_t wait_ticks, hipStream_t stream) {
  if (ndesc == 0 || total_chunks == 0) return HC_OK;
  if (counters == nullptr || (ngates != 0 && gates == nullptr) || abandoned == nullptr)
    return fail(HC_E_ARG, "a one-launch plan needs its own counters");
  return dispatch_gw(G, W, [&](auto g, auto w) -> hc_err {
    constexpr int GG = decltype(g)::value, WW = decltype(w)::value;
    return launch_persistent(k_batch_one<GG, WW>, d_descs, d_chunk_start, ndesc, total_chunks, counters, stream,
                             gates, ngates, abandoned, wait_ticks);
  });
}

template <uint32_t OP>
static hc_err launch_batch_op(uint32_t G, uint32_t W, const BatchDesc* d_descs, const uint64_t* d_chunk_start,
                              uint32_t ndesc, uint64_t total_chunks, unsigned long long* counters,
                              hipStream_t stream) {
  return dispatch_gw(G, W, [&](auto g, auto w) -> hc_err {
    constexpr int GG = decltype(g)::value, WW = decltype(w)::value;
    return launch_persistent(k_batch<OP, GG, WW>, d_descs, d_chunk_start, ndesc, total_chunks, counters, stream);
  });
}

hc_err launch_batch(uint32_t op, uint32_t G, uint32_t W, const BatchDesc* d_descs, const uint64_t* d_chunk_start,
                    uint32_t ndesc, uint64_t total_chunks, unsigned long long* counters, hipStream_t stream) {
  if (ndesc == 0 || total_chunks == 0) return HC_OK;
  switch (op) {
    case BATCH_INSERT:
      return launch_batch_op<BATCH_INSERT>(G, W, d_descs, d_chunk_start, ndesc, total_chunks, counters, stream);
    case BATCH_COUNT:
      return launch_batch_op<BATCH_COUNT>(G, W, d_descs, d_chunk_start, ndesc, total_chunks, counters, stream);
    case BATCH_RETRIEVE:
      return launch_batch_op<BATCH_RETRIEVE>(G, W, d_descs, d_chunk_start, ndesc, total_chunks, counters, stream);
    case BATCH_ERASE:
      return launch_batch_op<BATCH_ERASE>(G, W, d_descs, d_chunk_start, ndesc, total_chunks, counters, stream);
  }
  return fail(HC_E_ARG, "unknown batched operation %u", op);
}

hc_err launch_batch_mixed(uint32_t op, const BatchDesc* d_descs, const uint64_t* d_chunk_start, uint32_t ndesc,
                          uint64_t total_chunks, unsigned long long* counters, hipStream_t stream) {
  if (ndesc == 0 || total_chunks == 0) return HC_OK;
  switch (op) {
    case BATCH_INSERT:
      return launch_persistent(k_batch_mixed<BATCH_INSERT>, d_descs, d_chunk_start, ndesc, total_chunks, counters,
                               stream);
    case BATCH_COUNT:
      return launch_persistent(k_batch_mixed<BATCH_COUNT>, d_descs, d_chunk_start, ndesc, total_chunks, counters,
                               stream);
    case BATCH_RETRIEVE:
      return launch_persistent(k_batch_mixed<BATCH_RETRIEVE>, d_descs, d_chunk_start, ndesc, total_chunks, counters,
                               stream);
    case BATCH_ERASE:
      return launch_persistent(k_batch_mixed<BATCH_ERASE>, d_descs, d_chunk_start, ndesc, total_chunks, counters,
                               stream);
  }
  return fail(HC_E_ARG, "unknown batched operation %u", op);
}

}  // namespace hc
