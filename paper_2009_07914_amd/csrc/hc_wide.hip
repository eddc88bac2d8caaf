// Single-value table with 64-bit keys and 64-bit values (the wider types of
// Sec. IV-B1), in either layout the paper names:
//  * array of structures (AoS): a slot is 16 bytes, key word then value word;
//    a window of W = 8 slots is one 128-byte line;
//  * structure of arrays (SoA): C key words, then C value words, in one
//    allocation; a window's keys (W = 16: one 128-byte line) are probed without
//    touching values, and a hit reads one value word.
// The empty key is 0 and the tombstone key 2^64 - 1 (value 0).
//
// The probe is the cooperative scheme of the 32-bit tables (Sec. IV-B2): a group
// of G <= W lanes loads a whole window (W/G slots per lane, 16-byte loads),
// votes with a ballot and claims the first reusable slot once the window shows
// the key absent up to an empty slot.  A claim is a 64-bit CAS of the key word
// only; the value word is then written with a relaxed atomic store, so a
// reader in a later launch sees a whole pair.  Within one
// launch a reader may find a freshly claimed key before its value store lands
// (the torn-read hazard of a key-only CAS): inserts and queries of one table
// belong in different launches, as for every table here.  An update of a
// present key rewrites its value word (which of a repeated key's values
// survives is unspecified, as for the 32-bit table).  Hash: h1 and h2 are the
// low and high halves of fmix64(k ^ seed), MurmurHash3's 64-bit finaliser.
#include "hc_kernels.hpp"
#include "hc_launch.hpp"
#include "hc_wide.hpp"

namespace hc {

constexpr uint64_t KEY64_EMPTY = 0ull;
constexpr uint64_t KEY64_TOMB = ~0ull;

__device__ __forceinline__ uint64_t fmix64(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return x;
}

__device__ __forceinline__ void seq_start64(const TableView& t, uint64_t k, Seq& s) {
  const uint64_t x = fmix64(k ^ (((uint64_t)t.seed_hi << 32) | t.seed_lo));
  const uint32_t h1 = (uint32_t)x, h2 = (uint32_t)(x >> 32);
  s.w = reduce_window(t, h1);
  s.l = 0;
  s.step = 1;
  if (t.scheme == SCHEME_DOUBLE) s.step = t.pow2 ? ((h2 & t.pmask) | 1u) : (1u + __umulhi(h2, t.P - 1u));
}

__device__ __forceinline__ bool reserved64(uint64_t k) { return k == KEY64_EMPTY || k == KEY64_TOMB; }

// Key and value words of slot idx (C = P * W slots).
template <bool SOA>
__device__ __forceinline__ unsigned long long* key_word(const TableView& t, uint64_t idx) {
  return (unsigned long long*)(SOA ? t.slots + idx : t.slots + 2 * idx);
}
template <bool SOA, int W>
__device__ __forceinline__ unsigned long long* value_word(const TableView& t, uint64_t idx) {
  return (unsigned long long*)(SOA ? t.slots + (uint64_t)t.P * W + idx : t.slots + 2 * idx + 1);
}
// The value word after a claim or for an update: a relaxed atomic store (a
// whole 8-byte word, no return: not a second read-modify-write of the line).
template <bool SOA, int W>
__device__ __forceinline__ void store_value(const TableView& t, uint64_t idx, uint64_t v) {
  __hip_atomic_store(value_word<SOA, W>(t, idx), (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One group's view of a window: SPL slots per lane, keys (and values, AoS).
template <int G, int W, bool SOA>
struct Wide {
  static_assert(G <= W, "64-bit tables take groups no larger than the window");
  static constexpr int SPL = W / G;
  GroupCtx<G> g;
  Seq s{};
  uint64_t key[SPL], val[SPL];
  MaskT<SPL> match, empty, tomb;
  uint64_t first = 0;  // slot index of this lane's first slot

  __device__ __forceinline__ void start(const TableView& t, uint64_t k) { seq_start64(t, k, s); }
  __device__ __forceinline__ bool exhausted(const TableView& t) const { return s.l + 1 >= t.P; }
  __device__ __forceinline__ void advance(const TableView& t) { seq_next(t, s); }
  __device__ __forceinline__ void load(const TableView& t, uint64_t k) {
    first = (uint64_t)s.w * W + (uint64_t)g.glane * SPL;
    if constexpr (SOA) {
      if constexpr (SPL % 2 == 0) {
        const ulonglong2* p = reinterpret_cast<const ulonglong2*>(t.slots + first);
#pragma unroll
        for (int j = 0; j < SPL / 2; ++j) {
          const ulonglong2 q = p[j];
          key[2 * j] = q.x;
          key[2 * j + 1] = q.y;
        }
      } else {
        key[0] = t.slots[first];
      }
    } else {
      const ulonglong2* p = reinterpret_cast<const ulonglong2*>(t.slots) + first;
#pragma unroll
      for (int j = 0; j < SPL; ++j) {
        const ulonglong2 q = p[j];
        key[j] = q.x;
        val[j] = q.y;
      }
    }
    match = empty = tomb = 0;
#pragma unroll
    for (int j = 0; j < SPL; ++j) {
      match |= (MaskT<SPL>)(key[j] == k) << j;
      empty |= (MaskT<SPL>)(key[j] == KEY64_EMPTY) << j;
      tomb |= (MaskT<SPL>)(key[j] == KEY64_TOMB) << j;
    }
  }
  // Value of this lane's lowest matching slot (AoS: already loaded; SoA: one load).
  __device__ __forceinline__ uint64_t matched_value(const TableView& t) const {
    if constexpr (SOA) return *value_word<true, W>(t, first + lowbit(match));
    else return pick_lowest<SPL>(val, match);
  }
};

template <int G, int W, bool SOA>
struct WideInsert {
  Wide<G, W, SOA> ln;
  TableView t;
  const uint64_t* __restrict__ keys;
  const uint64_t* __restrict__ values;
  uint8_t* __restrict__ status;
  uint64_t i = 0, k = 0, v = 0, k_nx = 0, v_nx = 0, cand_idx = 0;
  bool cand = false;
  long long added = 0;

  __device__ __forceinline__ void load(uint64_t op) {
    k_nx = keys[op];
    v_nx = values[op];
  }
  __device__ __forceinline__ void begin(uint64_t op) {
    i = op;
    k = k_nx;
    v = v_nx;
    ln.start(t, k);
    cand = false;
  }
  __device__ __forceinline__ bool done(uint8_t st) {
    if (status != nullptr && ln.g.glane == 0) status[i] = st;
    return true;
  }
  // CAS the key word of a reusable slot: 1 claimed, 2 found the key there (updated), 3 lost to another key.
  __device__ __forceinline__ uint32_t claim(uint64_t idx, uint64_t expect) {
    const uint64_t r = atomicCAS(key_word<SOA>(t, idx), (unsigned long long)expect, (unsigned long long)k);
    if (r == expect) {
      store_value<SOA, W>(t, idx, v);
      ++added;
      return 1;
    }
    if (r == k) {
      store_value<SOA, W>(t, idx, v);
      return 2;
    }
    return 3;
  }
  __device__ __forceinline__ bool step() {
    const auto& g = ln.g;
    if (reserved64(k)) return done(ST_INVALID_KEY);
    ln.load(t, k);
    const uint64_t b_match = g.bits(ln.match != 0);
    if (b_match) {  // present: replace the value
      if (g.glane == (uint32_t)ffs64(b_match)) store_value<SOA, W>(t, ln.first + lowbit(ln.match), v);
      return done(ST_DUPLICATE);
    }
    const bool any_empty = g.bits(ln.empty != 0) != 0;
    MaskT<Wide<G, W, SOA>::SPL> reuse = ln.empty | ln.tomb;
    uint64_t b_reuse = g.bits(reuse != 0);
    const bool last = ln.exhausted(t);
    if (any_empty || last) {
      if (cand) {  // a tombstone from an earlier window comes first
        uint32_t outcome = 0;
        if (g.glane == 0) outcome = claim(cand_idx, KEY64_TOMB);
        outcome = g.bcast(outcome, 0);
        if (outcome == 1) return done(ST_OK);
        if (outcome == 2) return done(ST_DUPLICATE);
        ln.start(t, k);  // lost it to another key: scan again
        cand = false;
        return false;
      }
      while (b_reuse) {
        const uint32_t r = (uint32_t)ffs64(b_reuse);
        uint32_t outcome = 0;
        if (g.glane == r) {
          const int j = lowbit(reuse);
          const uint64_t expect = ((ln.empty >> j) & 1) ? KEY64_EMPTY : KEY64_TOMB;
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

template <int G, int W, bool SOA>
struct WideRetrieve {
  Wide<G, W, SOA> ln;
  TableView t;
  const uint64_t* __restrict__ keys;
  uint64_t* __restrict__ values_out;
  uint8_t* __restrict__ found_out;
  uint64_t i = 0, k = 0, k_nx = 0;
  // output staging (drive_staged), as for the 32-bit retrieve
  uint64_t* ring_val = nullptr;
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
  __device__ __forceinline__ void write_out(uint64_t e, uint64_t v, uint8_t f) {
    if (values_out != nullptr) values_out[e] = v;
    if (found_out != nullptr) found_out[e] = f;
  }
  __device__ __forceinline__ void emit(uint64_t v, uint8_t f) {
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
    if (ln.g.glane == 0) emit(0, 0);
    return true;
  }
  __device__ __forceinline__ bool step() {
    const auto& g = ln.g;
    if (reserved64(k)) return miss();
    ln.load(t, k);
    const uint64_t b_match = g.bits(ln.match != 0);
    if (b_match) {
      if (g.glane == (uint32_t)ffs64(b_match)) emit(ln.matched_value(t), 1);
      return true;
    }
    if (g.bits(ln.empty != 0) || ln.exhausted(t)) return miss();
    ln.advance(t);
    return false;
  }
  __device__ __forceinline__ void end() {}
};

template <int G, int W, bool SOA>
struct WideErase {
  Wide<G, W, SOA> ln;
  TableView t;
  const uint64_t* __restrict__ keys;
  uint8_t* __restrict__ status;
  uint64_t i = 0, k = 0, k_nx = 0;
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
    if (reserved64(k)) return done(ST_INVALID_KEY);
    ln.load(t, k);
    const uint64_t b_match = g.bits(ln.match != 0);
    if (b_match) {
      const uint32_t r = (uint32_t)ffs64(b_match);
      uint32_t ok = 0;
      if (g.glane == r) {
        const uint64_t idx = ln.first + lowbit(ln.match);
        if (atomicCAS(key_word<SOA>(t, idx), (unsigned long long)k, (unsigned long long)KEY64_TOMB) == k) {
          store_value<SOA, W>(t, idx, 0);
          ok = 1;
          --added;
        }
      }
      return done(g.bcast(ok, r) ? ST_OK : ST_NOT_FOUND);
    }
    if (g.bits(ln.empty != 0) || ln.exhausted(t)) return done(ST_NOT_FOUND);
    ln.advance(t);
    return false;
  }
  __device__ __forceinline__ void end() { wave_add_to(t.size, added); }
};

template <int G, int W, bool SOA>
__global__ __launch_bounds__(BLOCK) void k_wide_insert(TableView t, WorkCtl ctl, const uint64_t* __restrict__ keys,
                                                       const uint64_t* __restrict__ values, uint64_t n,
                                                       uint8_t* __restrict__ status) {
  WideInsert<G, W, SOA> op;
  op.t = t;
  op.keys = keys;
  op.values = values;
  op.status = status;
  drive<G>(n, ctl, op);
}

template <int G, int W, bool SOA>
__global__ __launch_bounds__(BLOCK) void k_wide_retrieve(TableView t, WorkCtl ctl, const uint64_t* __restrict__ keys,
                                                         uint64_t n, uint64_t* __restrict__ values_out,
                                                         uint8_t* __restrict__ found_out) {
  using R = WideRetrieve<G, W, SOA>;
  __shared__ OutRing<R::RING, uint64_t> rings[BLOCK / 64];
  R op;
  op.t = t;
  op.keys = keys;
  op.values_out = values_out;
  op.found_out = found_out;
  drive_staged<G, R::RING>(n, ctl, op, rings[threadIdx.x >> 6]);
}

template <int G, int W, bool SOA>
__global__ __launch_bounds__(BLOCK) void k_wide_erase(TableView t, WorkCtl ctl, const uint64_t* __restrict__ keys,
                                                      uint64_t n, uint8_t* __restrict__ status) {
  WideErase<G, W, SOA> op;
  op.t = t;
  op.keys = keys;
  op.status = status;
  drive<G>(n, ctl, op);
}

// (G, W) pairs with G <= W; others are rejected by the caller.
template <typename F>
static hc_err dispatch_wide(uint32_t G, uint32_t W, F&& f) {
  if (G > W) return fail(HC_E_ARG, "64-bit tables need group <= window (group %u, window %u)", G, W);
  return dispatch_gw(G, W, [&](auto g, auto w) -> hc_err {
    constexpr int GG = decltype(g)::value, WW = decltype(w)::value;
    if constexpr (GG > WW) {
      return fail(HC_E_ARG, "group %d over window %d", GG, WW);
    } else {
      return f(g, w);
    }
  });
}

template <bool SOA>
static hc_err launch_wide_layout(int op, const TableView& t, uint32_t G, uint32_t W, const uint64_t* keys,
                                 const uint64_t* values, uint64_t n, uint64_t* values_out, uint8_t* flags,
                                 hipStream_t s) {
  return dispatch_wide(G, W, [&](auto g, auto w) -> hc_err {
    constexpr int GG = decltype(g)::value, WW = decltype(w)::value;
    if (op == WIDE_INSERT) {
      auto k = k_wide_insert<GG, WW, SOA>;
      const unsigned grid = grid_for(k, n, GG);
      hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, s, t, work_for(n, GG, grid, s), keys, values, n, flags);
    } else if (op == WIDE_RETRIEVE) {
      auto k = k_wide_retrieve<GG, WW, SOA>;
      const unsigned grid = grid_for(k, n, GG);
      hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, s, t, work_for(n, GG, grid, s), keys, n, values_out, flags);
    } else {
      auto k = k_wide_erase<GG, WW, SOA>;
      const unsigned grid = grid_for(k, n, GG);
      hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, s, t, work_for(n, GG, grid, s), keys, n, flags);
    }
    return check_launch("64-bit table");
  });
}

hc_err launch_wide(int op, bool soa, const TableView& t, uint32_t G, uint32_t W, const uint64_t* keys,
                   const uint64_t* values, uint64_t n, uint64_t* values_out, uint8_t* flags, hipStream_t s) {
  return soa ? launch_wide_layout<true>(op, t, G, W, keys, values, n, values_out, flags, s)
             : launch_wide_layout<false>(op, t, G, W, keys, values, n, values_out, flags, s);
}

}  // namespace hc
