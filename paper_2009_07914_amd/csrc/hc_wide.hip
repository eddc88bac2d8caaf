// Single-value table with 64-bit keys and 64-bit values (the wider types of
// Sec. IV-B1, array-of-structures layout): a slot is 16 bytes, key word then
// value word; the empty key is 0 and the tombstone key 2^64 - 1 (value 0).
// A window of W = 8 slots is one 128-byte line.
//
// The probe is the cooperative scheme of the 32-bit tables (Sec. IV-B2): a group
// of G <= W lanes loads a whole window (W/G slots per lane, 16-byte loads),
// votes with a ballot and claims the first reusable slot once the window shows
// the key absent up to an empty slot.  A claim is a 64-bit CAS of the key word
// only; the value word is then written with an atomic exchange, so a reader in
// a later launch sees a whole pair.  Within one launch an update of a present
// key is an exchange of its value word (which of a repeated key's values
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

// One group's view of a window: SPL slots per lane, keys and values.
template <int G, int W>
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
    const ulonglong2* p = reinterpret_cast<const ulonglong2*>(t.slots) + first;
    match = empty = tomb = 0;
#pragma unroll
    for (int j = 0; j < SPL; ++j) {
      const ulonglong2 q = p[j];
      key[j] = q.x;
      val[j] = q.y;
      match |= (MaskT<SPL>)(q.x == k) << j;
      empty |= (MaskT<SPL>)(q.x == KEY64_EMPTY) << j;
      tomb |= (MaskT<SPL>)(q.x == KEY64_TOMB) << j;
    }
  }
};

__device__ __forceinline__ unsigned long long* key_word(const TableView& t, uint64_t idx) {
  return (unsigned long long*)(t.slots + 2 * idx);
}
__device__ __forceinline__ unsigned long long* value_word(const TableView& t, uint64_t idx) {
  return (unsigned long long*)(t.slots + 2 * idx + 1);
}

template <int G, int W>
struct WideInsert {
  Wide<G, W> ln;
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
    const uint64_t r = atomicCAS(key_word(t, idx), (unsigned long long)expect, (unsigned long long)k);
    if (r == expect) {
      atomicExch(value_word(t, idx), (unsigned long long)v);
      ++added;
      return 1;
    }
    if (r == k) {
      atomicExch(value_word(t, idx), (unsigned long long)v);
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
      if (g.glane == (uint32_t)ffs64(b_match)) atomicExch(value_word(t, ln.first + lowbit(ln.match)), (unsigned long long)v);
      return done(ST_DUPLICATE);
    }
    const bool any_empty = g.bits(ln.empty != 0) != 0;
    MaskT<Wide<G, W>::SPL> reuse = ln.empty | ln.tomb;
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

template <int G, int W>
struct WideRetrieve {
  Wide<G, W> ln;
  TableView t;
  const uint64_t* __restrict__ keys;
  uint64_t* __restrict__ values_out;
  uint8_t* __restrict__ found_out;
  uint64_t i = 0, k = 0, k_nx = 0;

  __device__ __forceinline__ void load(uint64_t op) { k_nx = keys[op]; }
  __device__ __forceinline__ void begin(uint64_t op) {
    i = op;
    k = k_nx;
    ln.start(t, k);
  }
  __device__ __forceinline__ bool out(uint64_t v, uint8_t f) {
    if (values_out != nullptr) values_out[i] = v;
    if (found_out != nullptr) found_out[i] = f;
    return true;
  }
  __device__ __forceinline__ bool step() {
    const auto& g = ln.g;
    if (reserved64(k)) return g.glane == 0 ? out(0, 0) : true;
    ln.load(t, k);
    const uint64_t b_match = g.bits(ln.match != 0);
    if (b_match) {
      if (g.glane == (uint32_t)ffs64(b_match)) out(pick_lowest<Wide<G, W>::SPL>(ln.val, ln.match), 1);
      return true;
    }
    if (g.bits(ln.empty != 0) || ln.exhausted(t)) return g.glane == 0 ? out(0, 0) : true;
    ln.advance(t);
    return false;
  }
  __device__ __forceinline__ void end() {}
};

template <int G, int W>
struct WideErase {
  Wide<G, W> ln;
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
        if (atomicCAS(key_word(t, idx), (unsigned long long)k, (unsigned long long)KEY64_TOMB) == k) {
          atomicExch(value_word(t, idx), 0ull);
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

template <int G, int W>
__global__ __launch_bounds__(BLOCK) void k_wide_insert(TableView t, WorkCtl ctl, const uint64_t* __restrict__ keys,
                                                       const uint64_t* __restrict__ values, uint64_t n,
                                                       uint8_t* __restrict__ status) {
  WideInsert<G, W> op;
  op.t = t;
  op.keys = keys;
  op.values = values;
  op.status = status;
  drive<G>(n, ctl, op);
}

template <int G, int W>
__global__ __launch_bounds__(BLOCK) void k_wide_retrieve(TableView t, WorkCtl ctl, const uint64_t* __restrict__ keys,
                                                         uint64_t n, uint64_t* __restrict__ values_out,
                                                         uint8_t* __restrict__ found_out) {
  WideRetrieve<G, W> op;
  op.t = t;
  op.keys = keys;
  op.values_out = values_out;
  op.found_out = found_out;
  drive<G>(n, ctl, op);
}

template <int G, int W>
__global__ __launch_bounds__(BLOCK) void k_wide_erase(TableView t, WorkCtl ctl, const uint64_t* __restrict__ keys,
                                                      uint64_t n, uint8_t* __restrict__ status) {
  WideErase<G, W> op;
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

hc_err launch_wide(int op, const TableView& t, uint32_t G, uint32_t W, const uint64_t* keys, const uint64_t* values,
                   uint64_t n, uint64_t* values_out, uint8_t* flags, hipStream_t s) {
  return dispatch_wide(G, W, [&](auto g, auto w) -> hc_err {
    constexpr int GG = decltype(g)::value, WW = decltype(w)::value;
    if (op == WIDE_INSERT) {
      auto k = k_wide_insert<GG, WW>;
      const unsigned grid = grid_for(k, n, GG);
      hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, s, t, work_for(n, GG, grid), keys, values, n, flags);
    } else if (op == WIDE_RETRIEVE) {
      auto k = k_wide_retrieve<GG, WW>;
      const unsigned grid = grid_for(k, n, GG);
      hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, s, t, work_for(n, GG, grid), keys, n, values_out, flags);
    } else {
      auto k = k_wide_erase<GG, WW>;
      const unsigned grid = grid_for(k, n, GG);
      hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, s, t, work_for(n, GG, grid), keys, n, flags);
    }
    return check_launch("64-bit table");
  });
}

}  // namespace hc
