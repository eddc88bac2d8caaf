// Bulk-operation kernels of the cooperative-probing tables.
//
// Launch shape: BLOCK threads per block, G lanes per operation (Sec. IV-B3: one
// group per input element).  The grid is sized to the resident capacity of the
// device; see drive() for how elements reach groups.  Each loop iteration is one
// probing step of every live group: load the step's window(s), vote (wavefront
// ballot), act.
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

// The word of the lowest set bit of m (0 if none), selected by mask bits rather
// than by an index, so the slots stay in registers.
template <int SPL, typename M>
__device__ __forceinline__ uint64_t pick_lowest(const uint64_t (&w)[SPL], M m) {
  uint64_t r = 0;
#pragma unroll
  for (int q = SPL - 1; q >= 0; --q) r = ((m >> q) & 1) ? w[q] : r;
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

// One probing step of one lane: its slots of the step's window(s) and their classes.
template <int SPL>
struct Window {
  uint64_t word[SPL];
  MaskT<SPL> match, empty, tomb;
  uint64_t first;  // slot index of word[0]
};

template <int G, int W>
__device__ __forceinline__ void load_step(const TableView& t, const Lane<G, W>& ln, const Seq& s, uint32_t lbase,
                                          uint32_t k, Window<Lane<G, W>::SPL>& win) {
  constexpr int SPL = Lane<G, W>::SPL;
  const bool lv = ln.valid(t, lbase);
  win.first = (uint64_t)s.w * W + ln.jbase;
  if (lv) {
    load_slots<SPL>(t.slots, win.first, win.word);
  } else {
#pragma unroll
    for (int j = 0; j < SPL; ++j) win.word[j] = WORD_EMPTY;
  }
  classify<SPL>(win.word, k, lv, win.match, win.empty, win.tomb);
}

// ------------------------------------------------------------------------------
// Work distribution.  Every wavefront takes chunks of `ctl.chunk` consecutive
// elements from a global counter (one atomic per chunk) and hands each chunk's
// elements to its groups strictly in order.  The elements in flight in a
// wavefront therefore stay within a window of about two elements per group, so
// the 128-byte lines of every output array are completed while they are still
// in the L2 cache and the inputs are read as streams; and a block that starts
// late, or a wavefront that meets long probe sequences, simply takes fewer
// chunks, so no part of the grid waits for another.  Each group holds its
// current element and the reserved next one, whose inputs are already being
// loaded (Op::load), so starting an element costs no round trip.  Each loop
// iteration is one probing step of every group holding an element; a group that
// completes one starts the next in the same iteration.  The last wavefront to
// finish resets the launch's counters for the next launch that uses them.
// ------------------------------------------------------------------------------
template <int G, typename Op>
__device__ __forceinline__ void drive(uint64_t n, const WorkCtl& ctl, Op& op) {
  const GroupCtx<G>& g = op.ln.g;
  const uint32_t chunk = ctl.chunk;
  uint64_t cur = 0;       // chunk held by this wavefront (wavefront-uniform)
  uint32_t used = chunk;  // elements of it already handed out (wavefront-uniform)
  // The wavefront's next element index for every group with `want_group` set.
  // Called by every lane of the wavefront.
  auto reserve = [&](bool want_group) -> uint64_t {
    const uint64_t want = __ballot(want_group && g.glane == 0);
    if (want == 0) return ~0ull;
    const uint32_t cnt = (uint32_t)__popcll(want);
    const uint32_t rank = (uint32_t)__popcll(want & ((1ull << g.lane) - 1ull));
    const uint32_t room = chunk - used;
    uint64_t nxt = cur;
    if (cnt > room) {  // cnt <= groups per wavefront <= chunk: at most one new chunk
      unsigned long long c = 0;
      if (g.lane == 0) c = atomicAdd(ctl.counters, 1ull);
      nxt = ((uint64_t)__shfl((uint32_t)(c >> 32), 0, 64) << 32) | __shfl((uint32_t)c, 0, 64);
    }
    const uint64_t idx = (rank < room) ? cur * chunk + used + rank : nxt * chunk + (rank - room);
    if (cnt > room) {
      cur = nxt;
      used = cnt - room;
    } else {
      used += cnt;
    }
    return g.bcast64(idx, 0);
  };
  uint64_t i_next = reserve(true);
  bool has_next = i_next < n;
  if (has_next) op.load(i_next);
  bool active = false;
  for (;;) {
    const bool start = !active && has_next;
    if (start) {
      op.begin(i_next);
      active = true;
    }
    const uint64_t r = reserve(start);
    if (start) {
      i_next = r;
      has_next = r < n;
      if (has_next) op.load(r);
    }
    if (__ballot(active) == 0) break;
    if (active && op.step()) active = false;
  }
  op.end();
  if (g.lane == 0) {
    const unsigned long long waves = (unsigned long long)gridDim.x * (BLOCK / 64);
    if (atomicAdd(ctl.counters + 1, 1ull) == waves - 1) {  // every chunk has been taken
      atomicExch(ctl.counters, 0ull);
      atomicExch(ctl.counters + 1, 0ull);
    }
  }
}

// The same loop over the elements [begin, end) of one chunk that this wavefront
// already holds (batched launches): elements are handed to the groups in order,
// and the call returns when every element of the chunk is done.
template <int G, typename Op>
__device__ __forceinline__ void drive_range(uint64_t begin, uint64_t end, Op& op) {
  const GroupCtx<G>& g = op.ln.g;
  uint64_t pos = begin;  // wavefront-uniform
  auto reserve = [&](bool want_group) -> uint64_t {
    const uint64_t want = __ballot(want_group && g.glane == 0);
    if (want == 0) return ~0ull;
    const uint32_t rank = (uint32_t)__popcll(want & ((1ull << g.lane) - 1ull));
    const uint64_t idx = pos + rank;
    pos += (uint32_t)__popcll(want);
    return g.bcast64(idx, 0);
  };
  uint64_t i_next = reserve(true);
  bool has_next = i_next < end;
  if (has_next) op.load(i_next);
  bool active = false;
  for (;;) {
    const bool start = !active && has_next;
    if (start) {
      op.begin(i_next);
      active = true;
    }
    const uint64_t r = reserve(start);
    if (start) {
      i_next = r;
      has_next = r < end;
      if (has_next) op.load(r);
    }
    if (__ballot(active) == 0) break;
    if (active && op.step()) active = false;
  }
  op.end();
}

// ------------------------------------------------------------------------------
// drive() with the outputs staged per wavefront.  The elements a wavefront hands
// out are numbered in hand-out order (seq); a group finishing element `seq`
// puts its result into the wavefront's LDS ring at seq % RB.  Whenever the 64
// oldest ring entries are all finished, the wavefront writes them back together,
// 64 lanes to 64 output elements: the elements of one chunk are consecutive, so
// these are whole cache lines, written once, instead of lines completed piecemeal
// over many iterations (and evicted half-written in between).  Before handing out
// an element that would overrun the ring, the oldest 64 entries are written back
// as they are; a result that arrives after its entry was written back (seq below
// the flush mark) goes straight to memory.
// ------------------------------------------------------------------------------
template <int RB, typename V = uint32_t>
struct OutRing {
  uint64_t idx[RB];   // element index of each entry
  V val[RB];
  uint8_t found[RB];
  uint8_t done[RB];   // 0 pending, 1 finished, 2 no element
};

template <int G, int RB, typename Op, typename V>
__device__ __forceinline__ void drive_staged(uint64_t n, const WorkCtl& ctl, Op& op, OutRing<RB, V>& ring) {
  static_assert(RB % 64 == 0 && RB >= 128, "ring of whole 64-entry blocks, at least two");
  const GroupCtx<G>& g = op.ln.g;
  const uint32_t chunk = ctl.chunk;
  uint64_t cur = 0;
  uint32_t used = chunk;
  uint64_t hcount = 0;  // elements handed out (wavefront-uniform)
  uint64_t flushed = 0; // ring entries below this are written back (wavefront-uniform, multiple of 64)
#pragma unroll
  for (int j = 0; j < RB / 64; ++j) ring.done[j * 64 + g.lane] = 0;
  auto write_back = [&](bool only_full) -> bool {  // the block [flushed, flushed + 64)
    const uint64_t e = flushed + g.lane;
    const uint32_t r = (uint32_t)(e % RB);
    const bool handed = e < hcount;
    const uint8_t st = handed ? ring.done[r] : (uint8_t)0;
    if (only_full && (flushed + 64 > hcount || __ballot(st != 0) != ~0ull)) return false;
    if (st == 1) op.write_out(ring.idx[r], ring.val[r], ring.found[r]);
    if (handed) ring.done[r] = 0;
    flushed += 64;
    op.flushed = flushed;
    return true;
  };
  auto reserve = [&](bool want_group, uint64_t& seq_out) -> uint64_t {
    const uint64_t want = __ballot(want_group && g.glane == 0);
    if (want == 0) return ~0ull;
    const uint32_t cnt = (uint32_t)__popcll(want);
    const uint32_t rank = (uint32_t)__popcll(want & ((1ull << g.lane) - 1ull));
    while (hcount + cnt > flushed + RB) write_back(false);  // make room: at most once (cnt <= 64)
    const uint32_t room = chunk - used;
    uint64_t nxt = cur;
    if (cnt > room) {
      unsigned long long c = 0;
      if (g.lane == 0) c = atomicAdd(ctl.counters, 1ull);
      nxt = ((uint64_t)__shfl((uint32_t)(c >> 32), 0, 64) << 32) | __shfl((uint32_t)c, 0, 64);
    }
    const uint64_t idx = (rank < room) ? cur * chunk + used + rank : nxt * chunk + (rank - room);
    if (cnt > room) {
      cur = nxt;
      used = cnt - room;
    } else {
      used += cnt;
    }
    if ((want >> g.lane) & 1ull) {
      const uint32_t r = (uint32_t)((hcount + rank) % RB);
      ring.idx[r] = idx;
      ring.done[r] = idx < n ? 0 : 2;
    }
    seq_out = g.bcast64(hcount + rank, 0);
    hcount += cnt;
    return g.bcast64(idx, 0);
  };
  op.ring_val = ring.val;
  op.ring_found = ring.found;
  op.ring_done = ring.done;
  op.flushed = 0;
  uint64_t seq_next = 0;
  uint64_t i_next = reserve(true, seq_next);
  bool has_next = i_next < n;
  if (has_next) op.load(i_next);
  bool active = false;
  for (;;) {
    const bool start = !active && has_next;
    if (start) {
      op.seq = seq_next;
      op.begin(i_next);
      active = true;
    }
    uint64_t sq = 0;
    const uint64_t r = reserve(start, sq);
    if (start) {
      i_next = r;
      seq_next = sq;
      has_next = r < n;
      if (has_next) op.load(r);
    }
    if (__ballot(active) == 0) break;
    if (active && op.step()) active = false;
    while (write_back(true)) {
    }
  }
  while (flushed < hcount) write_back(false);
  op.end();
  if (g.lane == 0) {
    const unsigned long long waves = (unsigned long long)gridDim.x * (BLOCK / 64);
    if (atomicAdd(ctl.counters + 1, 1ull) == waves - 1) {
      atomicExch(ctl.counters, 0ull);
      atomicExch(ctl.counters + 1, 0ull);
    }
  }
}

// drive_range() with the outputs staged as in drive_staged(): the elements of the
// chunk [begin, end) are numbered in hand-out order from 0, results go to the
// wavefront's LDS ring, and every 64 consecutive finished results leave as whole
// lines; the ring is empty again when the call returns.
template <int G, int RB, typename Op, typename V>
__device__ __forceinline__ void drive_range_staged(uint64_t begin, uint64_t end, Op& op, OutRing<RB, V>& ring) {
  static_assert(RB % 64 == 0 && RB >= 128, "ring of whole 64-entry blocks, at least two");
  const GroupCtx<G>& g = op.ln.g;
  uint64_t pos = begin;  // next element to hand out (wavefront-uniform)
  uint64_t hcount = 0;   // elements handed out
  uint64_t flushed = 0;  // ring entries below this are written back (multiple of 64)
#pragma unroll
  for (int j = 0; j < RB / 64; ++j) ring.done[j * 64 + g.lane] = 0;
  auto write_back = [&](bool only_full) -> bool {
    const uint64_t e = flushed + g.lane;
    const uint32_t r = (uint32_t)(e % RB);
    const bool handed = e < hcount;
    const uint8_t st = handed ? ring.done[r] : (uint8_t)0;
    if (only_full && (flushed + 64 > hcount || __ballot(st != 0) != ~0ull)) return false;
    if (st == 1) op.write_out(ring.idx[r], ring.val[r], ring.found[r]);
    if (handed) ring.done[r] = 0;
    flushed += 64;
    op.flushed = flushed;
    return true;
  };
  auto reserve = [&](bool want_group, uint64_t& seq_out) -> uint64_t {
    const uint64_t want = __ballot(want_group && g.glane == 0);
    if (want == 0) return ~0ull;
    const uint32_t cnt = (uint32_t)__popcll(want);
    const uint32_t rank = (uint32_t)__popcll(want & ((1ull << g.lane) - 1ull));
    while (hcount + cnt > flushed + RB) write_back(false);
    const uint64_t idx = pos + rank;
    pos += cnt;
    if ((want >> g.lane) & 1ull) {
      const uint32_t r = (uint32_t)((hcount + rank) % RB);
      ring.idx[r] = idx;
      ring.done[r] = idx < end ? 0 : 2;
    }
    seq_out = g.bcast64(hcount + rank, 0);
    hcount += cnt;
    return g.bcast64(idx, 0);
  };
  op.ring_val = ring.val;
  op.ring_found = ring.found;
  op.ring_done = ring.done;
  op.flushed = 0;
  uint64_t seq_next = 0;
  uint64_t i_next = reserve(true, seq_next);
  bool has_next = i_next < end;
  if (has_next) op.load(i_next);
  bool active = false;
  for (;;) {
    const bool start = !active && has_next;
    if (start) {
      op.seq = seq_next;
      op.begin(i_next);
      active = true;
    }
    uint64_t sq = 0;
    const uint64_t r = reserve(start, sq);
    if (start) {
      i_next = r;
      seq_next = sq;
      has_next = r < end;
      if (has_next) op.load(r);
    }
    if (__ballot(active) == 0) break;
    if (active && op.step()) active = false;
    while (write_back(true)) {
    }
  }
  while (flushed < hcount) write_back(false);
  op.end();
}

// ------------------------------------------------------------------------------
// Single-value and counting insert (Sec. IV-B2 steps 1-7; Sec. IV-B3).
// ------------------------------------------------------------------------------
template <int G, int W, int KIND>
struct InsertUnique {
  using L = Lane<G, W>;
  static constexpr int SPL = L::SPL;
  L ln;
  TableView t;
  const uint32_t* __restrict__ keys;
  const uint32_t* __restrict__ values;
  uint8_t* __restrict__ status;
  uint64_t i = 0, cand_idx = 0;
  uint32_t k = 0, v = 0, lbase = 0;
  uint32_t k_nx = 0, v_nx = 0;
  Seq s{};
  bool cand = false;
  long long added = 0;
  uint32_t fails = 0;  // failed claim CASes (Sec. IV-B2: the collisions an insert pays for)

  __device__ __forceinline__ void load(uint64_t op) {
    k_nx = keys[op];
    v_nx = (KIND == KIND_COUNT && values == nullptr) ? 1u : values[op];  // counting: increment
  }
  __device__ __forceinline__ void begin(uint64_t op) {
    i = op;
    k = k_nx;
    v = v_nx;
    ln.start(t, k, s, lbase);
    cand = false;
  }
  __device__ __forceinline__ bool done(uint8_t st) {
    if (status != nullptr && ln.g.glane == 0) status[i] = st;
    return true;
  }
  // The key is present at idx, whose word was seen as `seen`.  An upsert whose value is the one
  // seen leaves the line clean: the result is that of this write ordered before any other write
  // of the call to the key (any order of one call's writes is valid), and a hot key rewritten
  // with its own value costs no atomics.
  __device__ __forceinline__ void update(uint64_t idx, uint64_t seen) {
    if constexpr (KIND == KIND_COUNT) atomicAdd((unsigned long long*)&t.slots[idx], (unsigned long long)v << 32);
    else if (slot_value(seen) != v) atomicExch((unsigned long long*)&t.slots[idx], (unsigned long long)make_slot(k, v));
  }
  // CAS a reusable slot: 1 claimed, 2 found the key there (updated), 3 lost to another key.
  __device__ __forceinline__ uint32_t claim(uint64_t idx, uint64_t expect) {
    const uint64_t r = atomicCAS((unsigned long long*)&t.slots[idx], (unsigned long long)expect,
                                 (unsigned long long)make_slot(k, v));
    if (r == expect) { ++added; return 1; }
    ++fails;
    if (slot_key(r) == k) { update(idx, r); return 2; }
    return 3;
  }
  __device__ __forceinline__ bool step() {
    const auto& g = ln.g;
    if (reserved_key(k)) return done(ST_INVALID_KEY);
    Window<SPL> win;
    load_step<G, W>(t, ln, s, lbase, k, win);
    const uint64_t b_match = g.bits(win.match != 0);
    if (b_match) {  // key present: update in place (Sec. IV-B3 duplicate warning)
      if (g.glane == (uint32_t)ffs64(b_match))
        update(win.first + lowbit(win.match), pick_lowest<SPL>(win.word, win.match));
      return done(ST_DUPLICATE);
    }
    const bool any_empty = g.bits(win.empty != 0) != 0;
    MaskT<SPL> reuse = win.empty | win.tomb;
    uint64_t b_reuse = g.bits(reuse != 0);
    const bool last = ln.exhausted(t, lbase);
    if (any_empty || last) {  // the key is absent up to here: claim
      if (cand) {             // a tombstone from an earlier window comes first
        uint32_t outcome = 0;
        if (g.glane == 0) outcome = claim(cand_idx, WORD_TOMB);
        outcome = g.bcast(outcome, 0);
        if (outcome == 1) return done(ST_OK);
        if (outcome == 2) return done(ST_DUPLICATE);
        ln.start(t, k, s, lbase);  // lost it to another key: scan again
        cand = false;
        return false;
      }
      while (b_reuse) {  // reusable slots of this step in position order
        const uint32_t r = (uint32_t)ffs64(b_reuse);
        uint32_t outcome = 0;
        if (g.glane == r) {
          const int j = lowbit(reuse);
          const uint64_t expect = ((win.empty >> j) & 1) ? WORD_EMPTY : WORD_TOMB;
          reuse &= reuse - 1;
          outcome = claim(win.first + j, expect);
        }
        outcome = g.bcast(outcome, r);
        if (outcome == 1) return done(ST_OK);
        if (outcome == 2) return done(ST_DUPLICATE);
        b_reuse = g.bits(reuse != 0);
      }
      if (last) return done(ST_FULL);
    } else if (!cand && b_reuse) {  // first tombstone on the way: remember it
      const uint32_t r = (uint32_t)ffs64(b_reuse);
      cand_idx = g.bcast64(win.first + lowbit(reuse), r);
      cand = true;
    }
    ln.advance(t, s, lbase);
    return false;
  }
  __device__ __forceinline__ void end() {
    wave_add_to(t.size + CTR_SIZE, added);
    wave_add_to(t.size + CTR_CAS_FAILS, fails);
  }
};

template <int G, int W, int KIND>
__global__ __launch_bounds__(BLOCK) void k_insert_unique(TableView t, WorkCtl ctl, const uint32_t* __restrict__ keys,
                                                         const uint32_t* __restrict__ values, uint64_t n,
                                                         uint8_t* __restrict__ status) {
  InsertUnique<G, W, KIND> op;
  op.t = t;
  op.keys = keys;
  op.values = values;
  op.status = status;
  drive<G>(n, ctl, op);
}

// ------------------------------------------------------------------------------
// Multi-value insert: store one more pair at the first reusable position.
// ------------------------------------------------------------------------------
template <int G, int W>
struct InsertMulti {
  using L = Lane<G, W>;
  static constexpr int SPL = L::SPL;
  L ln;
  TableView t;
  const uint32_t* __restrict__ keys;
  const uint32_t* __restrict__ values;
  uint8_t* __restrict__ status;
  uint64_t i = 0;
  uint32_t k = 0, v = 0, lbase = 0, k_nx = 0, v_nx = 0;
  Seq s{};
  long long added = 0;
  uint32_t fails = 0;  // failed claim CASes

  __device__ __forceinline__ void load(uint64_t op) {
    k_nx = keys[op];
    v_nx = values[op];
  }
  __device__ __forceinline__ void begin(uint64_t op) {
    i = op;
    k = k_nx;
    v = v_nx;
    ln.start(t, k, s, lbase);
  }
  __device__ __forceinline__ bool done(uint8_t st) {
    if (status != nullptr && ln.g.glane == 0) status[i] = st;
    return true;
  }
  __device__ __forceinline__ bool step() {
    const auto& g = ln.g;
    if (reserved_key(k)) return done(ST_INVALID_KEY);
    Window<SPL> win;
    load_step<G, W>(t, ln, s, lbase, k, win);
    MaskT<SPL> reuse = win.empty | win.tomb;
    uint64_t b_reuse = g.bits(reuse != 0);
    while (b_reuse) {
      const uint32_t r = (uint32_t)ffs64(b_reuse);
      uint32_t ok = 0;
      if (g.glane == r) {
        const int j = lowbit(reuse);
        const uint64_t expect = ((win.empty >> j) & 1) ? WORD_EMPTY : WORD_TOMB;
        reuse &= reuse - 1;
        const uint64_t res = atomicCAS((unsigned long long*)&t.slots[win.first + j], (unsigned long long)expect,
                                       (unsigned long long)make_slot(k, v));
        if (res == expect) { ok = 1; ++added; } else { ++fails; }
      }
      if (g.bcast(ok, r)) return done(ST_OK);
      b_reuse = g.bits(reuse != 0);
    }
    if (ln.exhausted(t, lbase)) return done(ST_FULL);
    ln.advance(t, s, lbase);
    return false;
  }
  __device__ __forceinline__ void end() {
    wave_add_to(t.size + CTR_SIZE, added);
    wave_add_to(t.size + CTR_CAS_FAILS, fails);
  }
};

template <int G, int W>
__global__ __launch_bounds__(BLOCK) void k_insert_multi(TableView t, WorkCtl ctl, const uint32_t* __restrict__ keys,
                                                        const uint32_t* __restrict__ values, uint64_t n,
                                                        uint8_t* __restrict__ status) {
  InsertMulti<G, W> op;
  op.t = t;
  op.keys = keys;
  op.values = values;
  op.status = status;
  drive<G>(n, ctl, op);
}

// ------------------------------------------------------------------------------
// Single-value / counting retrieval (Sec. IV-B4): stop at the key or at the first
// window holding an empty slot.
// ------------------------------------------------------------------------------
template <int G, int W>
struct Retrieve {
  using L = Lane<G, W>;
  static constexpr int SPL = L::SPL;
  L ln;
  TableView t;
  const uint32_t* __restrict__ keys;
  uint32_t* __restrict__ values_out;
  uint8_t* __restrict__ found_out;
  uint64_t i = 0;
  uint32_t k = 0, lbase = 0, k_nx = 0;
  Seq s{};
  // output staging (drive_staged); ring_val == nullptr: results go straight to memory
  uint32_t* ring_val = nullptr;
  uint8_t* ring_found = nullptr;
  uint8_t* ring_done = nullptr;
  uint64_t seq = 0, flushed = 0;
  static constexpr uint32_t RING = 128;

  __device__ __forceinline__ void load(uint64_t op) { k_nx = keys[op]; }
  __device__ __forceinline__ void begin(uint64_t op) {
    i = op;
    k = k_nx;
    ln.start(t, k, s, lbase);
  }
  __device__ __forceinline__ void write_out(uint64_t e, uint32_t v, uint8_t f) {
    if (values_out != nullptr) values_out[e] = v;
    if (found_out != nullptr) found_out[e] = f;
  }
  __device__ __forceinline__ void emit(uint32_t v, uint8_t f) {
    if (ring_val != nullptr && seq >= flushed) {
      const uint32_t r = (uint32_t)(seq % RING);
      ring_val[r] = v;
      ring_found[r] = f;
      ring_done[r] = 1;
    } else {
      write_out(i, v, f);
    }
  }
  __device__ __forceinline__ bool miss() {
    if (ln.g.glane == 0) emit(0u, 0);
    return true;
  }
  __device__ __forceinline__ bool step() {
    const auto& g = ln.g;
    if (reserved_key(k)) return miss();
    Window<SPL> win;
    load_step<G, W>(t, ln, s, lbase, k, win);
    const uint64_t b_match = g.bits(win.match != 0);
    if (b_match) {
      if (g.glane == (uint32_t)ffs64(b_match)) emit(slot_value(pick_lowest<SPL>(win.word, win.match)), 1);
      return true;
    }
    if (g.bits(win.empty != 0) || ln.exhausted(t, lbase)) return miss();
    ln.advance(t, s, lbase);
    return false;
  }
  __device__ __forceinline__ void end() {}
};

template <int G, int W>
__global__ __launch_bounds__(BLOCK) void k_retrieve(TableView t, WorkCtl ctl, const uint32_t* __restrict__ keys, uint64_t n,
                                                    uint32_t* __restrict__ values_out,
                                                    uint8_t* __restrict__ found_out) {
  using R = Retrieve<G, W>;
  __shared__ OutRing<R::RING> rings[BLOCK / 64];
  R op;
  op.t = t;
  op.keys = keys;
  op.values_out = values_out;
  op.found_out = found_out;
  drive_staged<G, R::RING>(n, ctl, op, rings[threadIdx.x >> 6]);
}

// ------------------------------------------------------------------------------
// Deletion by tombstone (Sec. IV-B5).  Single-value / counting: the one slot of
// the key.  Multi-value: every slot of the key up to the first empty window.
// ------------------------------------------------------------------------------
template <int G, int W, int KIND>
struct Erase {
  using L = Lane<G, W>;
  static constexpr int SPL = L::SPL;
  L ln;
  TableView t;
  const uint32_t* __restrict__ keys;
  uint8_t* __restrict__ status;
  uint64_t i = 0;
  uint32_t k = 0, lbase = 0, removed = 0, k_nx = 0;
  Seq s{};
  long long added = 0;

  __device__ __forceinline__ void load(uint64_t op) { k_nx = keys[op]; }
  __device__ __forceinline__ void begin(uint64_t op) {
    i = op;
    k = k_nx;
    ln.start(t, k, s, lbase);
    removed = 0;
  }
  __device__ __forceinline__ bool done(uint8_t st) {
    if (status != nullptr && ln.g.glane == 0) status[i] = st;
    return true;
  }
  __device__ __forceinline__ bool step() {
    const auto& g = ln.g;
    if (reserved_key(k)) return done(ST_INVALID_KEY);
    Window<SPL> win;
    load_step<G, W>(t, ln, s, lbase, k, win);
    const bool stop = g.bits(win.empty != 0) || ln.exhausted(t, lbase);
    if constexpr (KIND == KIND_MULTI) {
      uint32_t mine = 0;
#pragma unroll
      for (int j = 0; j < SPL; ++j) {
        if ((win.match >> j) & 1) {
          const uint64_t res = atomicCAS((unsigned long long*)&t.slots[win.first + j],
                                         (unsigned long long)win.word[j], (unsigned long long)WORD_TOMB);
          mine += (res == win.word[j]);
        }
      }
      added -= mine;
      removed += g.sum(mine);
      if (stop) return done(removed ? ST_OK : ST_NOT_FOUND);
    } else {
      const uint64_t b_match = g.bits(win.match != 0);
      if (b_match) {
        const uint32_t r = (uint32_t)ffs64(b_match);
        uint32_t ok = 0;
        if (g.glane == r) {
          const uint64_t idx = win.first + lowbit(win.match);
          uint64_t expect = pick_lowest<SPL>(win.word, win.match);
          for (;;) {  // the value half may change under a concurrent update; the key cannot
            const uint64_t res = atomicCAS((unsigned long long*)&t.slots[idx], (unsigned long long)expect,
                                           (unsigned long long)WORD_TOMB);
            if (res == expect) { ok = 1; --added; break; }
            if (slot_key(res) != k) break;  // erased by another group meanwhile
            expect = res;
          }
        }
        return done(g.bcast(ok, r) ? ST_OK : ST_NOT_FOUND);
      }
      if (stop) return done(ST_NOT_FOUND);
    }
    ln.advance(t, s, lbase);
    return false;
  }
  __device__ __forceinline__ void end() { wave_add_to(t.size, added); }
};

template <int G, int W, int KIND>
__global__ __launch_bounds__(BLOCK) void k_erase(TableView t, WorkCtl ctl, const uint32_t* __restrict__ keys, uint64_t n,
                                                 uint8_t* __restrict__ status) {
  Erase<G, W, KIND> op;
  op.t = t;
  op.keys = keys;
  op.status = status;
  drive<G>(n, ctl, op);
}

// ------------------------------------------------------------------------------
// Multi-value pass 1 (Sec. IV-B4): count the pairs of each query.  Writes the count
// into offsets[i] (to be scanned in place) and optionally into counts / found.
// ------------------------------------------------------------------------------
template <int G, int W>
struct CountMulti {
  using L = Lane<G, W>;
  static constexpr int SPL = L::SPL;
  L ln;
  TableView t;
  const uint32_t* __restrict__ keys;
  uint32_t* __restrict__ counts;
  uint64_t* __restrict__ offsets;
  uint8_t* __restrict__ found_out;
  uint32_t budget = 0xFFFFFFFFu;              // windows before handing the query over
  uint64_t* __restrict__ long_list = nullptr;  // handed-over queries
  unsigned long long* long_n = nullptr;
  uint64_t long_cap = 0;                       // entries the list holds; past them groups walk on
  uint64_t i = 0;
  uint32_t k = 0, lbase = 0, cnt = 0, k_nx = 0;
  Seq s{};
  // output staging (drive_staged): the count goes through the ring; a query handed over to the
  // long rounds writes its partial count directly (its ring entry stays pending and is skipped)
  uint32_t* ring_val = nullptr;
  uint8_t* ring_found = nullptr;
  uint8_t* ring_done = nullptr;
  uint64_t seq = 0, flushed = 0;
  static constexpr uint32_t RING = 128;

  __device__ __forceinline__ void load(uint64_t op) { k_nx = keys[op]; }
  __device__ __forceinline__ void begin(uint64_t op) {
    i = op;
    k = k_nx;
    ln.start(t, k, s, lbase);
    cnt = 0;
  }
  __device__ __forceinline__ void write_out(uint64_t e, uint32_t c, uint8_t) {
    if (counts != nullptr) counts[e] = c;
    if (offsets != nullptr) offsets[e] = c;
    if (found_out != nullptr) found_out[e] = c != 0;
  }
  __device__ __forceinline__ bool done() {
    if (ln.g.glane == 0) {
      if (ring_val != nullptr && seq >= flushed) {
        const uint32_t r = (uint32_t)(seq % RING);
        ring_val[r] = cnt;
        ring_found[r] = 0;
        ring_done[r] = 1;
      } else {
        write_out(i, cnt, 0);
      }
    }
    return true;
  }
  __device__ __forceinline__ bool step() {
    const auto& g = ln.g;
    if (reserved_key(k)) return done();
    Window<SPL> win;
    load_step<G, W>(t, ln, s, lbase, k, win);
    cnt += g.sum(popcount(win.match));
    if (g.bits(win.empty != 0) || ln.exhausted(t, lbase)) return done();
    if (lbase + L::WPS >= budget) {  // long: continued by the block-wide kernel from window `budget`
      unsigned long long j = 0;
      if (g.glane == 0) j = atomicAdd(long_n, 1ull);
      j = g.bcast64(j, 0);
      if (j < long_cap) {
        if (g.glane == 0) {
          long_list[j] = i;
          offsets[i] = cnt;
        }
        return true;
      }
      budget = 0xFFFFFFFFu;  // the list is full: this group walks on by itself
    }
    ln.advance(t, s, lbase);
    return false;
  }
  __device__ __forceinline__ void end() {}
};

template <int G, int W>
__global__ __launch_bounds__(BLOCK) void k_count_multi(TableView t, WorkCtl ctl, const uint32_t* __restrict__ keys, uint64_t n,
                                                       uint32_t* __restrict__ counts, uint64_t* __restrict__ offsets,
                                                       uint8_t* __restrict__ found_out, uint32_t budget,
                                                       uint64_t* __restrict__ long_list, unsigned long long* long_n,
                                                       uint64_t long_cap) {
  using C = CountMulti<G, W>;
  __shared__ OutRing<C::RING> rings[BLOCK / 64];
  C op;
  op.t = t;
  op.keys = keys;
  op.counts = counts;
  op.offsets = offsets;
  op.found_out = found_out;
  op.budget = budget;
  op.long_list = long_list;
  op.long_n = long_n;
  op.long_cap = long_cap;
  drive_staged<G, C::RING>(n, ctl, op, rings[threadIdx.x >> 6]);
}

// ------------------------------------------------------------------------------
// Multi-value pass 2 (Sec. IV-B4): probe again and write each query's values into
// its segment [offsets[i], offsets[i+1]).
// ------------------------------------------------------------------------------
template <int G, int W>
struct WriteMulti {
  using L = Lane<G, W>;
  static constexpr int SPL = L::SPL;
  L ln;
  TableView t;
  const uint32_t* __restrict__ keys;
  const uint64_t* __restrict__ offsets;
  uint32_t* __restrict__ out;
  uint32_t budget = 0xFFFFFFFFu;
  uint64_t* __restrict__ long_list = nullptr;  // (query, values written) pairs
  unsigned long long* long_n = nullptr;
  uint64_t long_cap = 0;                       // entries the list holds; past them groups walk on
  uint64_t i = 0, base = 0, limit = 0, written = 0, base_nx = 0, end_nx = 0;
  uint32_t k = 0, lbase = 0, k_nx = 0;
  Seq s{};

  __device__ __forceinline__ void load(uint64_t op) {
    k_nx = keys[op];
    base_nx = offsets[op];
    end_nx = offsets[op + 1];
  }
  __device__ __forceinline__ void begin(uint64_t op) {
    i = op;
    k = k_nx;
    ln.start(t, k, s, lbase);
    base = base_nx;
    limit = end_nx - base_nx;
    written = 0;
  }
  __device__ __forceinline__ bool step() {
    const auto& g = ln.g;
    if (reserved_key(k) || limit == 0) return true;
    Window<SPL> win;
    load_step<G, W>(t, ln, s, lbase, k, win);
    const uint32_t c = popcount(win.match);
    const uint32_t before = g.exclusive_scan(c);
    const uint32_t total = g.sum(c);
    uint64_t rank = written + before;
#pragma unroll
    for (int j = 0; j < SPL; ++j) {
      if ((win.match >> j) & 1) {
        if (rank < limit) out[base + rank] = slot_value(win.word[j]);
        ++rank;
      }
    }
    written += total;
    if (written >= limit || g.bits(win.empty != 0) || ln.exhausted(t, lbase)) return true;
    if (lbase + L::WPS >= budget) {
      unsigned long long j = 0;
      if (g.glane == 0) j = atomicAdd(long_n, 1ull);
      j = g.bcast64(j, 0);
      if (j < long_cap) {
        if (g.glane == 0) {
          long_list[2 * j] = i;
          long_list[2 * j + 1] = written;
        }
        return true;
      }
      budget = 0xFFFFFFFFu;  // the list is full: this group walks on by itself
    }
    ln.advance(t, s, lbase);
    return false;
  }
  __device__ __forceinline__ void end() {}
};

template <int G, int W>
__global__ __launch_bounds__(BLOCK) void k_write_multi(TableView t, WorkCtl ctl, const uint32_t* __restrict__ keys, uint64_t n,
                                                       const uint64_t* __restrict__ offsets,
                                                       uint32_t* __restrict__ out, uint32_t budget,
                                                       uint64_t* __restrict__ long_list, unsigned long long* long_n,
                                                       uint64_t long_cap) {
  WriteMulti<G, W> op;
  op.t = t;
  op.keys = keys;
  op.offsets = offsets;
  op.out = out;
  op.budget = budget;
  op.long_list = long_list;
  op.long_n = long_n;
  op.long_cap = long_cap;
  drive<G>(n, ctl, op);
}

}  // namespace hc
