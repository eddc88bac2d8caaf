// Device-side API: the bulk operations' per-element state machines, callable one
// element at a time from user kernels (the paper's device-sided interface, Sec. IV-A;
// its use case fuses k-mer generation with multi-value inserts in one kernel, Sec. V-C).
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

// Insert of `key` into a single-value (KIND_SINGLE: insert, or update to `value`),
// counting (KIND_COUNT: count += 1) or multi-value table (KIND_MULTI: store (key, value)
// as one more pair at the first reusable position of its sequence, Sec. IV-B3).
// Returns the per-element status (ST_OK new key / stored pair, ST_DUPLICATE present,
// ST_FULL, ST_INVALID_KEY).
template <int G, int W, int KIND = KIND_SINGLE>
__device__ __forceinline__ uint8_t insert(const TableView& t, uint32_t key, uint32_t value = 0) {
  static_assert(KIND == KIND_SINGLE || KIND == KIND_COUNT || KIND == KIND_MULTI, "table kind");
  using Op = std::conditional_t<KIND == KIND_MULTI, InsertMulti<G, W>, InsertUnique<G, W, KIND>>;
  Op op;
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

// Calls f(value, j) once for each value stored under `key`, j = 0, 1, ..., count - 1 in
// the order of the key's slots along its window sequence (for a multi-value table every
// pair of the key, Sec. IV-B4; for single-value and counting tables the one value or
// count), the group's lanes calling f in parallel for the matches they hold.  Returns
// the number of values (the same in every lane of the group).  The walk ends at the
// first window holding an empty slot, as retrieval does: no copy of a key lies beyond
// it.  This is the one-pass alternative to hc_count_values + hc_retrieve_all for a
// caller that consumes the values in place (e.g. writes them at j past its own offset).
template <int G, int W, typename F>
__device__ __forceinline__ uint32_t for_each(const TableView& t, uint32_t key, F&& f) {
  using L = Lane<G, W>;
  constexpr int SPL = L::SPL;
  if (reserved_key(key)) return 0;
  L ln;
  Seq s{};
  uint32_t lbase = 0;
  ln.start(t, key, s, lbase);
  uint32_t n = 0;
  for (;;) {
    Window<SPL> win;
    load_step<G, W>(t, ln, s, lbase, key, win);
    const uint32_t c = popcount(win.match);
    uint32_t j = n + ln.g.exclusive_scan(c);
#pragma unroll
    for (int q = 0; q < SPL; ++q)
      if ((win.match >> q) & 1) f(slot_value(win.word[q]), j++);
    n += ln.g.sum(c);
    if (ln.g.bits(win.empty != 0) || ln.exhausted(t, lbase)) break;
    ln.advance(t, s, lbase);
  }
  return n;
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
