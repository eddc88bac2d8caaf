// HashSet: a set of 32-bit keys (one of the structures built on the same
// principles as the hash tables, Sec. IV): slots of 4 bytes holding only the
// key, so a window of W = 16 slots is one 64-byte line, half the bytes of the
// single-value table's window.  The empty key is 0 and the tombstone
// 0xFFFFFFFF, both reserved as for the 32-bit tables.
//
// Probing is the tables' cooperative scheme (Sec. IV-B2) with their window
// sequence and hash (h1, h2 of the key), so a set and a single-value table of
// the same geometry put a key into the same window: a group of G <= W lanes
// loads a window (W/G keys per lane, vector loads), votes with a ballot and
// claims the first reusable slot, once the window shows the key absent up to an
// empty slot, with a 32-bit CAS.  Contains stops at the key or at a window with
// an empty slot; erase turns the key's slot into a tombstone.
#include "hc_kernels.hpp"
#include "hc_launch.hpp"
#include "hc_set.hpp"

namespace hc {

// One group's view of a window: SPL keys per lane.
template <int G, int W>
struct SetLane {
  static_assert(G <= W, "sets take groups no larger than the window");
  static constexpr int SPL = W / G;
  using M = MaskT<SPL>;
  GroupCtx<G> g;
  Seq s{};
  M match, empty, tomb;
  uint64_t first = 0;  // slot index of this lane's first slot

  __device__ __forceinline__ void start(const TableView& t, uint32_t k) { seq_start(t, k, s); }
  __device__ __forceinline__ bool exhausted(const TableView& t) const { return s.l + 1 >= t.P; }
  __device__ __forceinline__ void advance(const TableView& t) { seq_next(t, s); }
  __device__ __forceinline__ void load(const uint32_t* keys, uint32_t k) {
    first = (uint64_t)s.w * W + (uint64_t)g.glane * SPL;
    uint32_t w[SPL];
    if constexpr (SPL % 4 == 0) {
      const uint4* p = reinterpret_cast<const uint4*>(keys + first);
#pragma unroll
      for (int j = 0; j < SPL / 4; ++j) {
        const uint4 q = p[j];
        w[4 * j] = q.x;
        w[4 * j + 1] = q.y;
        w[4 * j + 2] = q.z;
        w[4 * j + 3] = q.w;
      }
    } else if constexpr (SPL == 2) {
      const uint2 q = *reinterpret_cast<const uint2*>(keys + first);
      w[0] = q.x;
      w[1] = q.y;
    } else {
      w[0] = keys[first];
    }
    match = empty = tomb = 0;
#pragma unroll
    for (int j = 0; j < SPL; ++j) {
      match |= (M)(w[j] == k) << j;
      empty |= (M)(w[j] == KEY_EMPTY) << j;
      tomb |= (M)(w[j] == KEY_TOMB) << j;
    }
  }
};

template <int G, int W>
struct SetInsert {
  SetLane<G, W> ln;
  TableView t;
  uint32_t* slots;
  const uint32_t* __restrict__ keys;
  uint8_t* __restrict__ status;
  uint64_t i = 0, cand_idx = 0;
  uint32_t k = 0, k_nx = 0;
  bool cand = false;
  long long added = 0;

  __device__ __forceinline__ void load(uint64_t op) { k_nx = keys[op]; }
  __device__ __forceinline__ void begin(uint64_t op) {
    i = op;
    k = k_nx;
    ln.start(t, k);
    cand = false;
  }
  __device__ __forceinline__ bool done(uint8_t st) {
    if (status != nullptr && ln.g.glane == 0) status[i] = st;
    return true;
  }
  // CAS a reusable slot: 1 claimed, 2 the key is there (a concurrent insert), 3 lost to another key.
  __device__ __forceinline__ uint32_t claim(uint64_t idx, uint32_t expect) {
    const uint32_t r = atomicCAS(slots + idx, expect, k);
    if (r == expect) {
      ++added;
      return 1;
    }
    return r == k ? 2 : 3;
  }
  __device__ __forceinline__ bool step() {
    const auto& g = ln.g;
    if (reserved_key(k)) return done(ST_INVALID_KEY);
    ln.load(slots, k);
    if (g.bits(ln.match != 0)) return done(ST_DUPLICATE);
    const bool any_empty = g.bits(ln.empty != 0) != 0;
    typename SetLane<G, W>::M reuse = ln.empty | ln.tomb;
    uint64_t b_reuse = g.bits(reuse != 0);
    const bool last = ln.exhausted(t);
    if (any_empty || last) {
      if (cand) {  // a tombstone in an earlier window comes first
        uint32_t outcome = 0;
        if (g.glane == 0) outcome = claim(cand_idx, KEY_TOMB);
        outcome = g.bcast(outcome, 0);
        if (outcome == 1) return done(ST_OK);
        if (outcome == 2) return done(ST_DUPLICATE);
        ln.start(t, k);  // lost it to another key: scan again from the first window
        cand = false;
        return false;
      }
      while (b_reuse) {
        const uint32_t r = (uint32_t)ffs64(b_reuse);
        uint32_t outcome = 0;
        if (g.glane == r) {
          const int j = lowbit(reuse);
          const uint32_t expect = ((ln.empty >> j) & 1) ? KEY_EMPTY : KEY_TOMB;
          reuse &= reuse - 1;
          outcome = claim(ln.first + j, expect);
        }
        outcome = g.bcast(outcome, r);
        if (outcome == 1) return done(ST_OK);
        if (outcome == 2) return done(ST_DUPLICATE);
        b_reuse = g.bits(reuse != 0);
      }
      if (last) return done(ST_FULL);
    } else if (!cand && b_reuse) {
      const uint32_t r = (uint32_t)ffs64(b_reuse);
      cand_idx = g.bcast64(ln.first + lowbit(reuse), r);
      cand = true;
    }
    ln.advance(t);
    return false;
  }
  __device__ __forceinline__ void end() { wave_add_to(t.size, added); }
};

template <int G, int W>
struct SetContains {
  SetLane<G, W> ln;
  TableView t;
  const uint32_t* slots;
  const uint32_t* __restrict__ keys;
  uint8_t* __restrict__ found_out;
  uint64_t i = 0;
  uint32_t k = 0, k_nx = 0;
  // output staging (drive_staged), as for the tables' queries
  uint32_t* ring_val = nullptr;
  uint8_t* ring_found = nullptr;
  uint8_t* ring_done = nullptr;
  uint64_t seq = 0, flushed = 0;
  static constexpr uint32_t RING = 128;

  __device__ __forceinline__ void load(uint64_t op) { k_nx = keys[op]; }
  __device__ __forceinline__ void begin(uint64_t op) {
    i = op;
    k = k_nx;
    ln.start(t, k);
  }
  __device__ __forceinline__ void write_out(uint64_t e, uint32_t, uint8_t f) { found_out[e] = f; }
  __device__ __forceinline__ bool out(uint8_t f) {
    if (ln.g.glane == 0) {
      if (ring_val != nullptr && seq >= flushed) {
        const uint32_t r = (uint32_t)(seq % RING);
        ring_found[r] = f;
        ring_done[r] = 1;
      } else {
        write_out(i, 0, f);
      }
    }
    return true;
  }
  __device__ __forceinline__ bool step() {
    const auto& g = ln.g;
    if (reserved_key(k)) return out(0);
    ln.load(slots, k);
    if (g.bits(ln.match != 0)) return out(1);
    if (g.bits(ln.empty != 0) || ln.exhausted(t)) return out(0);
    ln.advance(t);
    return false;
  }
  __device__ __forceinline__ void end() {}
};

template <int G, int W>
struct SetErase {
  SetLane<G, W> ln;
  TableView t;
  uint32_t* slots;
  const uint32_t* __restrict__ keys;
  uint8_t* __restrict__ status;
  uint64_t i = 0;
  uint32_t k = 0, k_nx = 0;
  long long added = 0;

  __device__ __forceinline__ void load(uint64_t op) { k_nx = keys[op]; }
  __device__ __forceinline__ void begin(uint64_t op) {
    i = op;
    k = k_nx;
    ln.start(t, k);
  }
  __device__ __forceinline__ bool done(uint8_t st) {
    if (status != nullptr && ln.g.glane == 0) status[i] = st;
    return true;
  }
  __device__ __forceinline__ bool step() {
    const auto& g = ln.g;
    if (reserved_key(k)) return done(ST_INVALID_KEY);
    ln.load(slots, k);
    const uint64_t b_match = g.bits(ln.match != 0);
    if (b_match) {
      const uint32_t r = (uint32_t)ffs64(b_match);
      uint32_t ok = 0;
      if (g.glane == r && atomicCAS(slots + ln.first + lowbit(ln.match), k, KEY_TOMB) == k) {
        ok = 1;
        --added;
      }
      return done(g.bcast(ok, r) ? ST_OK : ST_NOT_FOUND);
    }
    if (g.bits(ln.empty != 0) || ln.exhausted(t)) return done(ST_NOT_FOUND);
    ln.advance(t);
    return false;
  }
  __device__ __forceinline__ void end() { wave_add_to(t.size, added); }
};

template <int G, int W>
__global__ __launch_bounds__(BLOCK) void k_set_insert(TableView t, WorkCtl ctl, const uint32_t* __restrict__ keys,
                                                      uint64_t n, uint8_t* __restrict__ status) {
  SetInsert<G, W> op;
  op.t = t;
  op.slots = reinterpret_cast<uint32_t*>(t.slots);
  op.keys = keys;
  op.status = status;
  drive<G>(n, ctl, op);
}

template <int G, int W>
__global__ __launch_bounds__(BLOCK) void k_set_contains(TableView t, WorkCtl ctl, const uint32_t* __restrict__ keys,
                                                        uint64_t n, uint8_t* __restrict__ found_out) {
  using C = SetContains<G, W>;
  __shared__ OutRing<C::RING> rings[BLOCK / 64];
  C op;
  op.t = t;
  op.slots = reinterpret_cast<const uint32_t*>(t.slots);
  op.keys = keys;
  op.found_out = found_out;
  drive_staged<G, C::RING>(n, ctl, op, rings[threadIdx.x >> 6]);
}

template <int G, int W>
__global__ __launch_bounds__(BLOCK) void k_set_erase(TableView t, WorkCtl ctl, const uint32_t* __restrict__ keys,
                                                     uint64_t n, uint8_t* __restrict__ status) {
  SetErase<G, W> op;
  op.t = t;
  op.slots = reinterpret_cast<uint32_t*>(t.slots);
  op.keys = keys;
  op.status = status;
  drive<G>(n, ctl, op);
}

hc_err launch_set(int op, const TableView& t, uint32_t G, uint32_t W, const uint32_t* keys, uint64_t n,
                  uint8_t* flags, hipStream_t s) {
  if (G > W) return fail(HC_E_ARG, "sets need group <= window (group %u, window %u)", G, W);
  return dispatch_gw(G, W, [&](auto g, auto w) -> hc_err {
    constexpr int GG = decltype(g)::value, WW = decltype(w)::value;
    if constexpr (GG > WW) {
      return fail(HC_E_ARG, "group %d over window %d", GG, WW);
    } else {
      if (op == SET_INSERT) {
        auto k = k_set_insert<GG, WW>;
        const unsigned grid = grid_for(k, n, GG);
        hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, s, t, work_for(n, GG, grid, s), keys, n, flags);
      } else if (op == SET_CONTAINS) {
        auto k = k_set_contains<GG, WW>;
        const unsigned grid = grid_for(k, n, GG);
        hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, s, t, work_for(n, GG, grid, s), keys, n, flags);
      } else {
        auto k = k_set_erase<GG, WW>;
        const unsigned grid = grid_for(k, n, GG);
        hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, s, t, work_for(n, GG, grid, s), keys, n, flags);
      }
      return check_launch("hash set");
    }
  });
}

}  // namespace hc
