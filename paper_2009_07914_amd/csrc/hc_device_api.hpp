// Device-side API: the bulk operations' per-element state machines, callable one
// element at a time from user kernels (the paper's device-sided table operations,
// used to fuse table work into a producer kernel, Sec. IV-A and Sec. VI).
//
// A table's device view comes from hc_device_view() (C ABI).  Every function is
// called by a group: the G lanes of an aligned G-lane tile of the wavefront
// (lanes r*G .. r*G + G - 1) call it together with the same arguments; other
// groups of the same wavefront may call it with other arguments, or not at all.
// W is the table's window (hc_info().window).  Concurrency follows the bulk
// calls: operations of one kind may run concurrently; a kernel must not mix
// writes with other operations on the same table.
#pragma once

#include "hc_kernels.hpp"

namespace hc {
namespace dev {

// Single-value (KIND_SINGLE: insert or update to `value`) or counting
// (KIND_COUNT: count += 1) insert of `key`.  Returns the per-element status
// (ST_OK new key, ST_DUPLICATE present, ST_FULL, ST_INVALID_KEY).
template <int G, int W, int KIND = KIND_SINGLE>
__device__ __forceinline__ uint8_t insert(const TableView& t, uint32_t key, uint32_t value = 0) {
  static_assert(KIND == KIND_SINGLE || KIND == KIND_COUNT, "single-value or counting tables");
  InsertUnique<G, W, KIND> op;
  uint8_t st = ST_OK;
  op.t = t;
  op.keys = &key;
  op.values = (KIND == KIND_COUNT) ? nullptr : &value;
  op.status = &st;
  op.load(0);
  op.begin(0);
  while (!op.step()) {
  }
  if (op.added) atomicAdd(t.size + CTR_SIZE, (unsigned long long)op.added);
  if (op.fails) atomicAdd(t.size + CTR_CAS_FAILS, (unsigned long long)op.fails);
  return op.ln.g.bcast(st, 0);  // written by the group's first lane
}

// Value (single-value) or count (counting, multi-value: number of values) of
// `key`; returns whether the key is present.
template <int G, int W>
__device__ __forceinline__ bool retrieve(const TableView& t, uint32_t key, uint32_t& value) {
  Retrieve<G, W> op;
  uint32_t v = 0;
  uint8_t f = 0;
  op.t = t;
  op.keys = &key;
  op.values_out = &v;
  op.found_out = &f;
  op.load(0);
  op.begin(0);
  while (!op.step()) {
  }
  // exactly one lane of the group wrote the result, the others hold zeros
  value = op.ln.g.sum(v);
  return op.ln.g.sum(f) != 0;
}

// Erase `key` (single-value / counting: its slot; multi-value: all its pairs).
// Returns ST_OK, ST_NOT_FOUND or ST_INVALID_KEY.
template <int G, int W, int KIND = KIND_SINGLE>
__device__ __forceinline__ uint8_t erase(const TableView& t, uint32_t key) {
  Erase<G, W, KIND> op;
  uint8_t st = ST_OK;
  op.t = t;
  op.keys = &key;
  op.status = &st;
  op.load(0);
  op.begin(0);
  while (!op.step()) {
  }
  if (op.added) atomicAdd(t.size, (unsigned long long)op.added);
  return op.ln.g.bcast(st, 0);
}

// Calls f(key, value) once for every stored pair, one thread per slot (value is
// the count for counting tables).  Launch with any grid of any block size.
template <typename F>
__global__ void for_all(TableView t, uint32_t W, F f) {
  const uint64_t C = (uint64_t)t.P * W;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < C; i += stride) {
    const uint64_t w = t.slots[i];
    if (!reserved_key(slot_key(w))) f(slot_key(w), slot_value(w));
  }
}

}  // namespace dev
}  // namespace hc
