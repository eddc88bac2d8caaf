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

template <uint32_t OP, int G, int W>
__device__ __forceinline__ void run_chunk(const BatchDesc& d, uint64_t begin, uint64_t end) {
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
    drive_range<G>(begin, end, op);
  } else {
    Erase<G, W, KIND_SINGLE> op;
    op.t = d.t;
    op.keys = d.keys;
    op.status = d.flags;
    drive_range<G>(begin, end, op);
  }
}

// One kernel per (operation kind, group size, window): every descriptor of a
// launch has them, so the kernel keeps the register budget of a single-table
// kernel.  chunk_start[d] = first global chunk of descriptor d;
// chunk_start[ndesc] = total chunks.
template <uint32_t OP, int G, int W>
__global__ __launch_bounds__(BLOCK) void k_batch(const BatchDesc* __restrict__ descs,
                                                 const uint64_t* __restrict__ chunk_start, uint32_t ndesc,
                                                 WorkCtl ctl) {
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
    run_chunk<OP, G, W>(d, begin, end);
  }
  if (lane == 0) {
    const unsigned long long waves = (unsigned long long)gridDim.x * (BLOCK / 64);
    if (atomicAdd(ctl.counters + 1, 1ull) == waves - 1) {
      atomicExch(ctl.counters, 0ull);
      atomicExch(ctl.counters + 1, 0ull);
    }
  }
}

template <uint32_t OP>
static hc_err launch_batch_op(uint32_t G, uint32_t W, const BatchDesc* d_descs, const uint64_t* d_chunk_start,
                              uint32_t ndesc, uint64_t total_chunks, hipStream_t stream) {
  return dispatch_gw(G, W, [&](auto g, auto w) -> hc_err {
    constexpr int GG = decltype(g)::value, WW = decltype(w)::value;
    auto k = k_batch<OP, GG, WW>;
    const uint64_t cap = (uint64_t)device_cu_count() * (uint64_t)blocks_per_cu(reinterpret_cast<const void*>(k));
    const uint64_t need = (total_chunks + (BLOCK / 64) - 1) / (BLOCK / 64);
    const unsigned grid = (unsigned)(need < cap ? need : cap);
    WorkCtl ctl = work_for(0, 64, grid);
    hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, stream, d_descs, d_chunk_start, ndesc, ctl);
    return check_launch("batch");
  });
}

hc_err launch_batch(uint32_t op, uint32_t G, uint32_t W, const BatchDesc* d_descs, const uint64_t* d_chunk_start,
                    uint32_t ndesc, uint64_t total_chunks, hipStream_t stream) {
  if (ndesc == 0 || total_chunks == 0) return HC_OK;
  switch (op) {
    case BATCH_INSERT:
      return launch_batch_op<BATCH_INSERT>(G, W, d_descs, d_chunk_start, ndesc, total_chunks, stream);
    case BATCH_COUNT:
      return launch_batch_op<BATCH_COUNT>(G, W, d_descs, d_chunk_start, ndesc, total_chunks, stream);
    case BATCH_RETRIEVE:
      return launch_batch_op<BATCH_RETRIEVE>(G, W, d_descs, d_chunk_start, ndesc, total_chunks, stream);
    case BATCH_ERASE:
      return launch_batch_op<BATCH_ERASE>(G, W, d_descs, d_chunk_start, ndesc, total_chunks, stream);
  }
  return fail(HC_E_ARG, "unknown batched operation %u", op);
}

}  // namespace hc
