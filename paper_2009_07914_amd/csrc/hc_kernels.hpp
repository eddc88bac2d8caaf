// Bulk-operation kernels of the cooperative-probing tables.
//
// Launch shape: BLOCK threads per block, G lanes per operation (Sec. IV-B3: one
// group per input element).  The grid is sized to the resident capacity of the
// device and every group walks the batch with a stride, so a group that finishes
// its element picks up the next one in the same loop iteration; the groups of a
// wavefront therefore never wait for the slowest group of an earlier element.
// Each loop iteration is one probing step of every live group: load the step's
// window(s), vote (wavefront ballot), act.
//
// Concurrency (Sec. IV-D): within one launch, slots only move from reusable
// (empty or tombstone) to occupied, and an occupied slot keeps its key.  Plain
// loads may therefore show an older state of a slot, i.e. "reusable" where it has
// since been claimed, never the reverse.  Every claim is a 64-bit CAS whose
// returned word is acted on, which keeps the table exact:
//   * a key is stored at the first reusable position of its sequence, after the
//     scan has reached a window holding an empty slot without meeting the key
//     (Sec. IV-B4: a key sits at its lowest possible position, so retrieval may
//     stop at an empty slot);
//   * a CAS that fails on the same key turns into an update of that slot, one
//     that fails on another key moves to the next candidate position; a failed
//     claim of a tombstone remembered from an earlier window restarts the scan.
#pragma once

#include <type_traits>

#include "hc_device.hpp"

namespace hc {

// Per-lane slot masks: bit j refers to the lane's j-th slot (64 slots need 64 bits).
template <int SPL>
using MaskT = std::conditional_t<(SPL > 32), uint64_t, uint32_t>;

__device__ __forceinline__ int lowbit(uint32_t m) { return __ffs(m) - 1; }
__device__ __forceinline__ int lowbit(uint64_t m) { return __ffsll((unsigned long long)m) - 1; }
__device__ __forceinline__ uint32_t popcount(uint32_t m) { return (uint32_t)__popc(m); }
__device__ __forceinline__ uint32_t popcount(uint64_t m) { return (uint32_t)__popcll((unsigned long long)m); }

// Select word[j] for a runtime j without dynamic register indexing.
template <int SPL>
__device__ __forceinline__ uint64_t pick(const uint64_t (&w)[SPL], int j) {
  uint64_t r = w[0];
#pragma unroll
  for (int q = 1; q < SPL; ++q) r = (j == q) ? w[q] : r;
  return r;
}

template <int G, int W>
struct Lane {
  using S = Step<G, W>;
  static constexpr int SPL = S::SPL;
  static constexpr int WPS = S::WPS;
  GroupCtx<G> g;
  uint32_t sub;    // which window of a step this lane covers (G > W)
  uint32_t jbase;  // first slot of this lane inside its window
  __device__ __forceinline__ Lane() {
    sub = (G > W) ? (g.glane / W) : 0u;
    jbase = (G > W) ? (g.glane % W) : (g.glane * SPL);
  }
  __device__ __forceinline__ void start(const TableView& t, uint32_t k, Seq& s, uint32_t& lbase) const {
    seq_start(t, k, s);
    for (uint32_t r = 0; r < sub; ++r) seq_next(t, s);
    lbase = 0;
  }
  __device__ __forceinline__ void advance(const TableView& t, Seq& s, uint32_t& lbase) const {
#pragma unroll
    for (int q = 0; q < WPS; ++q) seq_next(t, s);
    lbase += WPS;
  }
  __device__ __forceinline__ bool valid(const TableView& t, uint32_t lbase) const {
    return (G > W) ? (lbase + sub < t.P) : true;
  }
  __device__ __forceinline__ bool exhausted(const TableView& t, uint32_t lbase) const {
    return lbase + WPS >= t.P;
  }
};

// Classify this lane's slots: bit j of each mask refers to word[j].
template <int SPL>
__device__ __forceinline__ void classify(const uint64_t (&w)[SPL], uint32_t k, bool valid, MaskT<SPL>& m_match,
                                         MaskT<SPL>& m_empty, MaskT<SPL>& m_tomb) {
  using M = MaskT<SPL>;
  m_match = m_empty = m_tomb = 0;
#pragma unroll
  for (int j = 0; j < SPL; ++j) {
    const uint32_t key = slot_key(w[j]);
    m_match |= (M)(key == k) << j;
    m_empty |= (M)(key == KEY_EMPTY) << j;
    m_tomb |= (M)(key == KEY_TOMB) << j;
  }
  if (!valid) m_match = m_empty = m_tomb = 0;
}

// ------------------------------------------------------------------------------
// Single-value and counting insert (Sec. IV-B2 steps 1-7; Sec. IV-B3).
// ------------------------------------------------------------------------------
template <int G, int W, int KIND>
__global__ __launch_bounds__(BLOCK) void k_insert_unique(TableView t, const uint32_t* __restrict__ keys,
                                                         const uint32_t* __restrict__ values, uint64_t n,
                                                         uint8_t* __restrict__ status) {
  using L = Lane<G, W>;
  constexpr int SPL = L::SPL;
  const L ln;
  const auto& g = ln.g;
  const uint64_t gpb = BLOCK / G;
  const uint64_t stride = (uint64_t)gridDim.x * gpb;
  uint64_t i = (uint64_t)blockIdx.x * gpb + threadIdx.x / G;

  bool active = i < n;
  uint32_t k = 0, v = 0, lbase = 0;
  Seq s{};
  bool cand = false;
  uint64_t cand_idx = 0;
  long long added = 0;

  auto begin = [&]() {
    k = keys[i];
    v = (KIND == KIND_COUNT) ? 1u : values[i];
    ln.start(t, k, s, lbase);
    cand = false;
  };
  auto finish = [&](uint8_t st) {
    if (status != nullptr && g.glane == 0) status[i] = st;
    i += stride;
    active = i < n;
    if (active) begin();
  };
  auto update = [&](uint64_t idx) {  // key present at idx
    if constexpr (KIND == KIND_COUNT) atomicAdd((unsigned long long*)&t.slots[idx], 1ull << 32);
    else atomicExch((unsigned long long*)&t.slots[idx], (unsigned long long)make_slot(k, v));
  };
  if (active) begin();

  while (__ballot(active) != 0) {
    if (!active) continue;
    if (reserved_key(k)) { finish(ST_INVALID_KEY); continue; }

    const bool lv = ln.valid(t, lbase);
    const uint64_t first = (uint64_t)s.w * W + ln.jbase;
    uint64_t word[SPL];
    if (lv) load_slots<SPL>(t.slots, first, word);
    else {
#pragma unroll
      for (int j = 0; j < SPL; ++j) word[j] = WORD_EMPTY;
    }
    MaskT<SPL> m_match, m_empty, m_tomb;
    classify<SPL>(word, k, lv, m_match, m_empty, m_tomb);
    const uint64_t b_match = g.bits(m_match != 0);

    if (b_match) {  // key present: update in place (Sec. IV-B3 duplicate warning)
      if (g.glane == (uint32_t)ffs64(b_match)) update(first + (lowbit(m_match)));
      finish(ST_DUPLICATE);
      continue;
    }
    const uint64_t b_empty = g.bits(m_empty != 0);
    MaskT<SPL> m_reuse = m_empty | m_tomb;
    uint64_t b_reuse = g.bits(m_reuse != 0);
    const bool last = ln.exhausted(t, lbase);

    if (b_empty || last) {  // the key is absent up to here: claim
      if (cand) {           // a tombstone from an earlier window comes first
        uint32_t outcome = 0;
        if (g.glane == 0) {
          const uint64_t r = atomicCAS((unsigned long long*)&t.slots[cand_idx], (unsigned long long)WORD_TOMB,
                                       (unsigned long long)make_slot(k, v));
          if (r == WORD_TOMB) { outcome = 1; ++added; }
          else if (slot_key(r) == k) { update(cand_idx); outcome = 2; }
          else outcome = 3;
        }
        outcome = g.bcast(outcome, 0);
        if (outcome == 1) { finish(ST_OK); continue; }
        if (outcome == 2) { finish(ST_DUPLICATE); continue; }
        ln.start(t, k, s, lbase);  // lost it to another key: scan again
        cand = false;
        continue;
      }
      uint32_t outcome = 0;
      while (b_reuse) {
        const uint32_t r = (uint32_t)ffs64(b_reuse);
        if (g.glane == r) {
          const int j = lowbit(m_reuse);
          const uint64_t obs = ((m_empty >> j) & 1) ? WORD_EMPTY : WORD_TOMB;
          m_reuse &= m_reuse - 1;
          const uint64_t idx = first + j;
          const uint64_t res = atomicCAS((unsigned long long*)&t.slots[idx], (unsigned long long)obs,
                                         (unsigned long long)make_slot(k, v));
          if (res == obs) { outcome = 1; ++added; }
          else if (slot_key(res) == k) { update(idx); outcome = 2; }
          else outcome = 3;
        }
        outcome = g.bcast(outcome, r);
        if (outcome != 3) break;
        outcome = 0;
        b_reuse = g.bits(m_reuse != 0);
      }
      if (outcome == 1) { finish(ST_OK); continue; }
      if (outcome == 2) { finish(ST_DUPLICATE); continue; }
      if (last) { finish(ST_FULL); continue; }
    } else if (!cand && b_reuse) {  // first tombstone on the way: remember it
      const uint32_t r = (uint32_t)ffs64(b_reuse);
      cand_idx = g.bcast64(first + (lowbit(m_reuse)), r);
      cand = true;
    }
    ln.advance(t, s, lbase);
  }
  wave_add_to(t.size, added);
}

// ------------------------------------------------------------------------------
// Multi-value insert: store one more pair at the first reusable position.
// ------------------------------------------------------------------------------
template <int G, int W>
__global__ __launch_bounds__(BLOCK) void k_insert_multi(TableView t, const uint32_t* __restrict__ keys,
                                                        const uint32_t* __restrict__ values, uint64_t n,
                                                        uint8_t* __restrict__ status) {
  using L = Lane<G, W>;
  constexpr int SPL = L::SPL;
  const L ln;
  const auto& g = ln.g;
  const uint64_t gpb = BLOCK / G;
  const uint64_t stride = (uint64_t)gridDim.x * gpb;
  uint64_t i = (uint64_t)blockIdx.x * gpb + threadIdx.x / G;

  bool active = i < n;
  uint32_t k = 0, v = 0, lbase = 0;
  Seq s{};
  long long added = 0;
  auto begin = [&]() {
    k = keys[i];
    v = values[i];
    ln.start(t, k, s, lbase);
  };
  auto finish = [&](uint8_t st) {
    if (status != nullptr && g.glane == 0) status[i] = st;
    i += stride;
    active = i < n;
    if (active) begin();
  };
  if (active) begin();

  while (__ballot(active) != 0) {
    if (!active) continue;
    if (reserved_key(k)) { finish(ST_INVALID_KEY); continue; }
    const bool lv = ln.valid(t, lbase);
    const uint64_t first = (uint64_t)s.w * W + ln.jbase;
    uint64_t word[SPL];
    if (lv) load_slots<SPL>(t.slots, first, word);
    else {
#pragma unroll
      for (int j = 0; j < SPL; ++j) word[j] = WORD_EMPTY;
    }
    MaskT<SPL> m_match, m_empty, m_tomb;
    classify<SPL>(word, k, lv, m_match, m_empty, m_tomb);
    MaskT<SPL> m_reuse = m_empty | m_tomb;
    uint64_t b_reuse = g.bits(m_reuse != 0);
    bool done = false;
    while (b_reuse) {
      const uint32_t r = (uint32_t)ffs64(b_reuse);
      uint32_t ok = 0;
      if (g.glane == r) {
        const int j = lowbit(m_reuse);
        const uint64_t obs = ((m_empty >> j) & 1) ? WORD_EMPTY : WORD_TOMB;
        m_reuse &= m_reuse - 1;
        const uint64_t res = atomicCAS((unsigned long long*)&t.slots[first + j], (unsigned long long)obs,
                                       (unsigned long long)make_slot(k, v));
        if (res == obs) { ok = 1; ++added; }
      }
      if (g.bcast(ok, r)) { done = true; break; }
      b_reuse = g.bits(m_reuse != 0);
    }
    if (done) { finish(ST_OK); continue; }
    if (ln.exhausted(t, lbase)) { finish(ST_FULL); continue; }
    ln.advance(t, s, lbase);
  }
  wave_add_to(t.size, added);
}

// ------------------------------------------------------------------------------
// Single-value / counting retrieval (Sec. IV-B4): stop at the key or at the first
// window holding an empty slot.
// ------------------------------------------------------------------------------
template <int G, int W>
__global__ __launch_bounds__(BLOCK) void k_retrieve(TableView t, const uint32_t* __restrict__ keys, uint64_t n,
                                                    uint32_t* __restrict__ values_out,
                                                    uint8_t* __restrict__ found_out) {
  using L = Lane<G, W>;
  constexpr int SPL = L::SPL;
  const L ln;
  const auto& g = ln.g;
  const uint64_t gpb = BLOCK / G;
  const uint64_t stride = (uint64_t)gridDim.x * gpb;
  uint64_t i = (uint64_t)blockIdx.x * gpb + threadIdx.x / G;

  bool active = i < n;
  uint32_t k = 0, lbase = 0;
  Seq s{};
  auto begin = [&]() {
    k = keys[i];
    ln.start(t, k, s, lbase);
  };
  auto next = [&]() {
    i += stride;
    active = i < n;
    if (active) begin();
  };
  auto miss = [&]() {
    if (g.glane == 0) {
      if (values_out != nullptr) values_out[i] = 0u;
      if (found_out != nullptr) found_out[i] = 0;
    }
    next();
  };
  if (active) begin();

  while (__ballot(active) != 0) {
    if (!active) continue;
    if (reserved_key(k)) { miss(); continue; }
    const bool lv = ln.valid(t, lbase);
    const uint64_t first = (uint64_t)s.w * W + ln.jbase;
    uint64_t word[SPL];
    if (lv) load_slots<SPL>(t.slots, first, word);
    else {
#pragma unroll
      for (int j = 0; j < SPL; ++j) word[j] = WORD_EMPTY;
    }
    MaskT<SPL> m_match, m_empty, m_tomb;
    classify<SPL>(word, k, lv, m_match, m_empty, m_tomb);
    const uint64_t b_match = g.bits(m_match != 0);
    if (b_match) {
      if (g.glane == (uint32_t)ffs64(b_match)) {
        const uint64_t w = pick<SPL>(word, lowbit(m_match));
        if (values_out != nullptr) values_out[i] = slot_value(w);
        if (found_out != nullptr) found_out[i] = 1;
      }
      next();
      continue;
    }
    if (g.bits(m_empty != 0) || ln.exhausted(t, lbase)) { miss(); continue; }
    ln.advance(t, s, lbase);
  }
}

// ------------------------------------------------------------------------------
// Deletion by tombstone (Sec. IV-B5).  Single-value / counting: the one slot of
// the key.  Multi-value: every slot of the key up to the first empty window.
// ------------------------------------------------------------------------------
template <int G, int W, int KIND>
__global__ __launch_bounds__(BLOCK) void k_erase(TableView t, const uint32_t* __restrict__ keys, uint64_t n,
                                                 uint8_t* __restrict__ status) {
  using L = Lane<G, W>;
  constexpr int SPL = L::SPL;
  const L ln;
  const auto& g = ln.g;
  const uint64_t gpb = BLOCK / G;
  const uint64_t stride = (uint64_t)gridDim.x * gpb;
  uint64_t i = (uint64_t)blockIdx.x * gpb + threadIdx.x / G;

  bool active = i < n;
  uint32_t k = 0, lbase = 0, removed = 0;
  Seq s{};
  long long added = 0;
  auto begin = [&]() {
    k = keys[i];
    ln.start(t, k, s, lbase);
    removed = 0;
  };
  auto finish = [&](uint8_t st) {
    if (status != nullptr && g.glane == 0) status[i] = st;
    i += stride;
    active = i < n;
    if (active) begin();
  };
  if (active) begin();

  while (__ballot(active) != 0) {
    if (!active) continue;
    if (reserved_key(k)) { finish(ST_INVALID_KEY); continue; }
    const bool lv = ln.valid(t, lbase);
    const uint64_t first = (uint64_t)s.w * W + ln.jbase;
    uint64_t word[SPL];
    if (lv) load_slots<SPL>(t.slots, first, word);
    else {
#pragma unroll
      for (int j = 0; j < SPL; ++j) word[j] = WORD_EMPTY;
    }
    MaskT<SPL> m_match, m_empty, m_tomb;
    classify<SPL>(word, k, lv, m_match, m_empty, m_tomb);
    const bool stop = g.bits(m_empty != 0) || ln.exhausted(t, lbase);

    if constexpr (KIND == KIND_MULTI) {
      uint32_t mine = 0;
#pragma unroll
      for (int j = 0; j < SPL; ++j) {
        if ((m_match >> j) & 1) {
          const uint64_t res = atomicCAS((unsigned long long*)&t.slots[first + j], (unsigned long long)word[j],
                                         (unsigned long long)WORD_TOMB);
          mine += (res == word[j]);
        }
      }
      added -= mine;
      removed += g.sum(mine);
      if (stop) { finish(removed ? ST_OK : ST_NOT_FOUND); continue; }
    } else {
      const uint64_t b_match = g.bits(m_match != 0);
      if (b_match) {
        const uint32_t r = (uint32_t)ffs64(b_match);
        uint32_t ok = 0;
        if (g.glane == r) {
          const uint64_t idx = first + (lowbit(m_match));
          uint64_t obs = pick<SPL>(word, lowbit(m_match));
          for (;;) {  // the value half may change under a concurrent update; the key cannot
            const uint64_t res = atomicCAS((unsigned long long*)&t.slots[idx], (unsigned long long)obs,
                                           (unsigned long long)WORD_TOMB);
            if (res == obs) { ok = 1; --added; break; }
            if (slot_key(res) != k) break;  // erased by another group meanwhile
            obs = res;
          }
        }
        finish(g.bcast(ok, r) ? ST_OK : ST_NOT_FOUND);
        continue;
      }
      if (stop) { finish(ST_NOT_FOUND); continue; }
    }
    ln.advance(t, s, lbase);
  }
  wave_add_to(t.size, added);
}

// ------------------------------------------------------------------------------
// Multi-value pass 1 (Sec. IV-B4): count the pairs of each query.  Writes the count
// into offsets[i] (to be scanned in place) and optionally into counts / found.
// ------------------------------------------------------------------------------
template <int G, int W>
__global__ __launch_bounds__(BLOCK) void k_count_multi(TableView t, const uint32_t* __restrict__ keys, uint64_t n,
                                                       uint32_t* __restrict__ counts, uint64_t* __restrict__ offsets,
                                                       uint8_t* __restrict__ found_out) {
  using L = Lane<G, W>;
  constexpr int SPL = L::SPL;
  const L ln;
  const auto& g = ln.g;
  const uint64_t gpb = BLOCK / G;
  const uint64_t stride = (uint64_t)gridDim.x * gpb;
  uint64_t i = (uint64_t)blockIdx.x * gpb + threadIdx.x / G;

  bool active = i < n;
  uint32_t k = 0, lbase = 0, cnt = 0;
  Seq s{};
  auto begin = [&]() {
    k = keys[i];
    ln.start(t, k, s, lbase);
    cnt = 0;
  };
  auto finish = [&]() {
    if (g.glane == 0) {
      if (counts != nullptr) counts[i] = cnt;
      if (offsets != nullptr) offsets[i] = cnt;
      if (found_out != nullptr) found_out[i] = cnt != 0;
    }
    i += stride;
    active = i < n;
    if (active) begin();
  };
  if (active) begin();

  while (__ballot(active) != 0) {
    if (!active) continue;
    if (reserved_key(k)) { finish(); continue; }
    const bool lv = ln.valid(t, lbase);
    const uint64_t first = (uint64_t)s.w * W + ln.jbase;
    uint64_t word[SPL];
    if (lv) load_slots<SPL>(t.slots, first, word);
    else {
#pragma unroll
      for (int j = 0; j < SPL; ++j) word[j] = WORD_EMPTY;
    }
    MaskT<SPL> m_match, m_empty, m_tomb;
    classify<SPL>(word, k, lv, m_match, m_empty, m_tomb);
    cnt += g.sum(popcount(m_match));
    if (g.bits(m_empty != 0) || ln.exhausted(t, lbase)) { finish(); continue; }
    ln.advance(t, s, lbase);
  }
}

// ------------------------------------------------------------------------------
// Multi-value pass 2 (Sec. IV-B4): probe again and write each query's values into
// its segment [offsets[i], offsets[i+1]).
// ------------------------------------------------------------------------------
template <int G, int W>
__global__ __launch_bounds__(BLOCK) void k_write_multi(TableView t, const uint32_t* __restrict__ keys, uint64_t n,
                                                       const uint64_t* __restrict__ offsets,
                                                       uint32_t* __restrict__ out) {
  using L = Lane<G, W>;
  constexpr int SPL = L::SPL;
  const L ln;
  const auto& g = ln.g;
  const uint64_t gpb = BLOCK / G;
  const uint64_t stride = (uint64_t)gridDim.x * gpb;
  uint64_t i = (uint64_t)blockIdx.x * gpb + threadIdx.x / G;

  bool active = i < n;
  uint32_t k = 0, lbase = 0;
  uint64_t base = 0, limit = 0, written = 0;
  Seq s{};
  auto begin = [&]() {
    k = keys[i];
    ln.start(t, k, s, lbase);
    base = offsets[i];
    limit = offsets[i + 1] - base;
    written = 0;
  };
  auto next = [&]() {
    i += stride;
    active = i < n;
    if (active) begin();
  };
  if (active) begin();

  while (__ballot(active) != 0) {
    if (!active) continue;
    if (reserved_key(k) || limit == 0) { next(); continue; }
    const bool lv = ln.valid(t, lbase);
    const uint64_t first = (uint64_t)s.w * W + ln.jbase;
    uint64_t word[SPL];
    if (lv) load_slots<SPL>(t.slots, first, word);
    else {
#pragma unroll
      for (int j = 0; j < SPL; ++j) word[j] = WORD_EMPTY;
    }
    MaskT<SPL> m_match, m_empty, m_tomb;
    classify<SPL>(word, k, lv, m_match, m_empty, m_tomb);
    const uint32_t c = popcount(m_match);
    const uint32_t before = g.exclusive_scan(c);
    const uint32_t total = g.sum(c);
    uint64_t rank = written + before;
#pragma unroll
    for (int j = 0; j < SPL; ++j) {
      if ((m_match >> j) & 1) {
        if (rank < limit) out[base + rank] = slot_value(word[j]);
        ++rank;
      }
    }
    written += total;
    if (written >= limit || g.bits(m_empty != 0) || ln.exhausted(t, lbase)) { next(); continue; }
    ln.advance(t, s, lbase);
  }
}

}  // namespace hc
