// Bucket list hash table (Sec. IV-C).
//
// Each distinct key occupies one slot of a cooperative-probing table; the
// slot's value half counts the key's values, and a per-slot record holds the pool
// offset of the key's last bucket.  Bucket i holds s_i values, s_0 given,
// s_i = ceil(growth * s_{i-1}) up to a cap; every bucket but the first starts
// with the pool offset of the bucket before it, so a list is walked from its
// last bucket back to the first.  The pool is one preallocated array handed out
// by an atomic counter.
//
// The paper appends under a per-key handle lock taken with CAS, with busy waiting
// while another thread holds it.  A bulk insert here needs no lock and no
// waiting, and leaves the same lists:
//   1. every pair probes for its key (claiming a slot with count 1 if absent,
//      else adding 1 to the count with one 64-bit atomic): the count before the
//      add is the pair's ticket, its rank among all values of the key;
//   2. the pair holding the key's last ticket of the batch (its ticket is the
//      count after the batch minus one, read from the slot) takes the buckets the
//      batch's tickets need from the pool in one allocation (one pool atomic per
//      block), links them (previous-bucket offsets) and updates the slot's 16-byte
//      record: buckets held, buckets held before the batch, last bucket and first
//      new bucket.  If the pool is exhausted the record says so, and the key keeps
//      what its existing buckets hold;
//   3. every pair writes its value where its ticket falls: ticket t lies in the
//      bucket i with S(i) <= t < S(i+1), S(i) = s_0 + ... + s_{i-1}; the record
//      of its slot gives the bucket's offset.
// Values of a key therefore appear in its list in ticket order.  A record says
// "no buckets yet" after hc_clear and after the key in its slot is erased, so a
// key that claims a slot finds it so without writing it.
//
// Bucket 0 of the key in slot p is never allocated: it is the s_0 pool words at
// p * s_0 (the first C * s_0 words of the pool are reserved for them; later buckets
// come from the rest of the pool), and the record is only read for keys with more
// than one bucket.  So a pair of the per-pair insert that claims a new slot for its
// key -- it holds ticket 0 -- stores its value right away and skips phases 2 and 3:
// for keys seen once per batch (the common case at low multiplicity) the insert is
// one probe, one claim and one store.
#include <cmath>

#include "hc_bucket.hpp"
#include "hc_kernels.hpp"
#include "hc_launch.hpp"

namespace hc {

// ---- bucket geometry ----------------------------------------------------------------

__device__ __forceinline__ uint64_t bl_S(const BucketView& b, uint64_t i) {  // values in buckets 0..i-1
  return (i <= b.m) ? b.cum[i] : b.cum[b.m] + (i - b.m) * (uint64_t)b.smax;
}

__device__ __forceinline__ uint64_t bl_bucket_of(const BucketView& b, uint64_t t) {  // S(i) <= t < S(i+1)
  const uint64_t ramp = b.cum[b.m];
  if (t >= ramp) return b.m + (t - ramp) / b.smax;
  uint32_t lo = 0, hi = b.m - 1;  // cum[0] = 0 <= t < cum[m]
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) / 2;
    if (b.cum[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ uint64_t bl_buckets(const BucketView& b, uint64_t c) {  // buckets holding c values
  return c == 0 ? 0 : bl_bucket_of(b, c - 1) + 1;
}

// Pool words of buckets [b0, b1): their values plus one link word for each i >= 1.
__device__ __forceinline__ uint64_t bl_words(const BucketView& b, uint64_t b0, uint64_t b1) {
  if (b1 <= b0) return 0;
  const uint64_t links = b1 - (b0 > 1 ? b0 : 1);
  return bl_S(b, b1) - bl_S(b, b0) + (b1 >= 1 ? links : 0);
}

// ---- phase 1: key probe, tickets ------------------------------------------------------

template <int G, int W>
struct BlTicket {
  using L = Lane<G, W>;
  static constexpr int SPL = L::SPL;
  L ln;
  TableView t;
  BucketView b;
  const uint32_t* __restrict__ keys;
  const uint32_t* __restrict__ incr;  // values per element (runs of a grouped insert); NULL: 1
  const uint32_t* __restrict__ values = nullptr;  // per-pair insert: the values (fast path); NULL: none
  uint64_t* __restrict__ pos;     // per pair: slot of its key
  uint32_t* __restrict__ ticket;  // per pair: rank among the key's values
  uint8_t* __restrict__ st;       // per pair: ST_OK provisional, BL_PLACED, or the final failure
  uint64_t i = 0, cand_idx = 0;
  uint32_t k = 0, lbase = 0, k_nx = 0, inc = 1, inc_nx = 1, v = 0, v_nx = 0;
  Seq s{};
  bool cand = false;
  long long added = 0;
  long long placed = 0;  // values stored by claims (phase 1)

  __device__ __forceinline__ void load(uint64_t op) {
    k_nx = keys[op];
    inc_nx = incr != nullptr ? incr[op] : 1u;
    if (values != nullptr) v_nx = values[op];
  }
  __device__ __forceinline__ void begin(uint64_t op) {
    i = op;
    k = k_nx;
    inc = inc_nx;
    v = v_nx;
    ln.start(t, k, s, lbase);
    cand = false;
  }
  __device__ __forceinline__ bool fail(uint8_t code) {
    if (ln.g.glane == 0) st[i] = code;
    return true;
  }
  // One lane: the pair now holds ticket tk at slot idx.
  __device__ __forceinline__ void record(uint64_t idx, uint32_t tk) {
    pos[i] = idx;
    ticket[i] = tk;
    st[i] = ST_OK;
  }
  __device__ __forceinline__ void add_one(uint64_t idx) {  // `inc` more values (tickets old .. old + inc - 1)
    const uint64_t old = atomicAdd((unsigned long long*)&t.slots[idx], (unsigned long long)inc << 32);
    record(idx, slot_value(old));
  }
  // CAS a reusable slot: 1 claimed (ticket 0), 2 the key was there (ticket taken), 3 lost to another key.
  // A claim by a per-pair insert stores its value at once (claimed()).
  __device__ __forceinline__ uint32_t claim(uint64_t idx, uint64_t expect) {
    const uint64_t r = atomicCAS((unsigned long long*)&t.slots[idx], (unsigned long long)expect,
                                 (unsigned long long)make_slot(k, inc));
    if (r == expect) {
      ++added;
      if (values == nullptr) record(idx, 0u);
      return 1;
    }
    if (slot_key(r) == k) {
      add_one(idx);
      return 2;
    }
    return 3;
  }
  // A claim succeeded at slot idx (known to group rank r): a per-pair insert holds ticket 0, the
  // first word of the slot's bucket 0.
  __device__ __forceinline__ bool claimed(uint64_t idx, uint32_t r) {
    if (values == nullptr) return true;
    const uint64_t p = ln.g.bcast64(idx, r);
    if (ln.g.glane == 0) {
      b.pool[p * b.s0] = v;  // a key with one bucket has it at p * s0: no record to update
      st[i] = BL_PLACED;
      ++placed;
    }
    return true;
  }
  __device__ __forceinline__ bool step() {
    const auto& g = ln.g;
    if (reserved_key(k)) return fail(ST_INVALID_KEY);
    Window<SPL> win;
    load_step<G, W>(t, ln, s, lbase, k, win);
    const uint64_t b_match = g.bits(win.match != 0);
    if (b_match) {
      if (g.glane == (uint32_t)ffs64(b_match)) add_one(win.first + lowbit(win.match));
      return true;
    }
    const bool any_empty = g.bits(win.empty != 0) != 0;
    MaskT<SPL> reuse = win.empty | win.tomb;
    uint64_t b_reuse = g.bits(reuse != 0);
    const bool lastw = ln.exhausted(t, lbase);
    if (any_empty || lastw) {
      if (cand) {  // a tombstone from an earlier window comes first
        uint32_t outcome = 0;
        if (g.glane == 0) outcome = claim(cand_idx, WORD_TOMB);
        outcome = g.bcast(outcome, 0);
        if (outcome == 1) return claimed(cand_idx, 0);
        if (outcome != 3) return true;
        ln.start(t, k, s, lbase);
        cand = false;
        return false;
      }
      while (b_reuse) {
        const uint32_t r = (uint32_t)ffs64(b_reuse);
        uint32_t outcome = 0;
        uint64_t at = 0;
        if (g.glane == r) {
          const int j = lowbit(reuse);
          const uint64_t expect = ((win.empty >> j) & 1) ? WORD_EMPTY : WORD_TOMB;
          reuse &= reuse - 1;
          at = win.first + j;
          outcome = claim(at, expect);
        }
        outcome = g.bcast(outcome, r);
        if (outcome == 1) return claimed(at, r);
        if (outcome != 3) return true;
        b_reuse = g.bits(reuse != 0);
      }
      if (lastw) return fail(ST_FULL);
    } else if (!cand && b_reuse) {
      const uint32_t r = (uint32_t)ffs64(b_reuse);
      cand_idx = g.bcast64(win.first + lowbit(reuse), r);
      cand = true;
    }
    ln.advance(t, s, lbase);
    return false;
  }
  __device__ __forceinline__ void end() { wave_add_to(t.size, placed); }  // the others count in phase 3
};

// n_dev non-NULL: the element count is *n_dev (runs counted on the device).
template <int G, int W>
__global__ __launch_bounds__(BLOCK) void k_bl_ticket(TableView t, WorkCtl ctl, BucketView b,
                                                     const uint32_t* __restrict__ keys,
                                                     const uint32_t* __restrict__ incr,
                                                     const uint32_t* __restrict__ values, uint64_t n,
                                                     const uint64_t* __restrict__ n_dev,
                                                     uint64_t* __restrict__ pos, uint32_t* __restrict__ ticket,
                                                     uint8_t* __restrict__ st) {
  BlTicket<G, W> op;
  op.t = t;
  op.b = b;
  op.keys = keys;
  op.incr = incr;
  op.values = values;
  op.pos = pos;
  op.ticket = ticket;
  op.st = st;
  drive<G>(n_dev != nullptr ? *n_dev : n, ctl, op);
}

// Pair j of a sorted batch takes the ticket of its run plus its rank in the run; the
// pairs before the last of a run only place their values (BL_FOLLOW), so the allocation
// pass reads the key's slot once, for the pair holding its last ticket.
// scan: exclusive scan of the run-start flags (scan[j + 1] - 1 = run of j).
__global__ __launch_bounds__(256) void k_bl_expand(const uint64_t* __restrict__ scan,
                                                   const uint64_t* __restrict__ starts, uint64_t n,
                                                   const uint64_t* __restrict__ rpos,
                                                   const uint32_t* __restrict__ rticket,
                                                   const uint8_t* __restrict__ rst, uint64_t* __restrict__ pos,
                                                   uint32_t* __restrict__ ticket, uint8_t* __restrict__ st) {
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t j = (uint64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += stride) {
    const uint64_t r = scan[j + 1] - 1;
    const uint8_t c = rst[r];
    st[j] = (c == ST_OK && j + 1 != starts[r + 1]) ? BL_FOLLOW : c;
    pos[j] = rpos[r];
    ticket[j] = rticket[r] + (uint32_t)(j - starts[r]);
  }
}

// ---- phase 2: buckets per key -----------------------------------------------------------

// Run by every pair; the pair holding its key's last ticket of the batch (ticket + 1
// equals the slot's count after phase 1) allocates.  Pool words are taken with one atomic per block of 1024 pairs (a
// scan over the block's wavefronts in LDS): every pool atomic hits the same
// word, so their number, not their bytes, bounds this kernel.
constexpr int ALLOC_BLOCK = 1024;

__global__ __launch_bounds__(ALLOC_BLOCK) void k_bl_alloc(TableView t, BucketView b, uint64_t n,
                                                          const uint64_t* __restrict__ pos,
                                                          const uint32_t* __restrict__ ticket,
                                                          uint8_t* __restrict__ st) {
  constexpr int NW = ALLOC_BLOCK / 64;
  __shared__ unsigned long long wave_off[NW];
  __shared__ unsigned long long block_base;
  const uint64_t stride = (uint64_t)gridDim.x * ALLOC_BLOCK;
  const uint32_t lane = __lane_id(), wv = threadIdx.x / 64;
  // the trip count depends only on blockIdx, so every thread of a block reaches each barrier
  for (uint64_t i0 = (uint64_t)blockIdx.x * ALLOC_BLOCK; i0 < n; i0 += stride) {
    const uint64_t i = i0 + threadIdx.x;
    uint64_t p = 0, b1 = 0, bp = 1, words = 0;
    uint32_t old_last = 0;
    bool mine = false;
    if (i < n && st[i] == ST_OK) {
      p = pos[i];
      // the count after phase 1 (nothing changes it before phase 3): its last ticket allocates,
      // unless bucket 0 still holds every value (then the record is neither read nor written)
      const uint64_t c1 = slot_value(t.slots[p]);
      mine = (uint64_t)ticket[i] + 1 == c1 && c1 > b.s0;  // more than bucket 0 (s_0 values) holds
      if (mine) {
        b1 = bl_buckets(b, c1);
        const ulonglong2 rec = b.meta[p];
        const uint32_t held = (uint32_t)rec.x;  // buckets before this batch (0 or 1: bucket 0 only)
        bp = held > 1 ? held : 1;                // bucket 0 is the slot's own, never allocated
        old_last = held > 1 ? (uint32_t)rec.y : (uint32_t)(p * b.s0);
        words = b1 > bp ? bl_words(b, bp, b1) : 0;
      }
    }
    // inclusive scan of the words over the wavefront, then over the block's wavefronts
    uint64_t incl = words;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t lo = __shfl_up((uint32_t)incl, d, 64), hi = __shfl_up((uint32_t)(incl >> 32), d, 64);
      if (lane >= (uint32_t)d) incl += (uint64_t)lo | ((uint64_t)hi << 32);
    }
    if (lane == 63) wave_off[wv] = incl;
    __syncthreads();
    if (wv == 0) {
      const uint64_t tot = lane < (uint32_t)NW ? wave_off[lane] : 0;
      uint64_t x = tot;
#pragma unroll
      for (int d = 1; d < NW; d <<= 1) {
        const uint32_t lo = __shfl_up((uint32_t)x, d, 64), hi = __shfl_up((uint32_t)(x >> 32), d, 64);
        if (lane >= (uint32_t)d) x += (uint64_t)lo | ((uint64_t)hi << 32);
      }
      if (lane < (uint32_t)NW) wave_off[lane] = x - tot;  // exclusive offset of each wavefront
      if (lane == NW - 1) block_base = x ? atomicAdd(b.pool_next, (unsigned long long)x) : 0ull;
    }
    __syncthreads();
    if (mine) {
      uint32_t first_new = BL_NONE, new_last = old_last, held = (uint32_t)bp;
      if (b1 > bp) {
        const uint64_t base = b.bump + block_base + wave_off[wv] + incl - words;
        if (base + words > b.pool_cap || base + words > 0xFFFFFFFFull) {
          first_new = BL_CUT;  // pool exhausted: the key keeps what its bp buckets hold (phase 3)
        } else {
          uint64_t o = base, prev = old_last;
          for (uint64_t j = bp; j < b1; ++j) {  // every allocated bucket starts with its link
            b.pool[o] = (uint32_t)prev;
            prev = o;
            o += bl_S(b, j + 1) - bl_S(b, j) + 1;
          }
          new_last = (uint32_t)prev;
          first_new = (uint32_t)base;
          held = (uint32_t)b1;
        }
      }
      b.meta[p] = make_ulonglong2((uint64_t)held | (bp << 32), (uint64_t)new_last | ((uint64_t)first_new << 32));
      st[i] = BL_ALLOC;
    }
    __syncthreads();  // wave_off and block_base are rewritten by the next round
  }
}

// ---- phase 3: values -----------------------------------------------------------------

__global__ __launch_bounds__(256) void k_bl_place(TableView t, BucketView b, const uint32_t* __restrict__ values,
                                                  uint64_t n, const uint64_t* __restrict__ pos,
                                                  const uint32_t* __restrict__ ticket, uint8_t* __restrict__ st,
                                                  uint8_t* __restrict__ status) {
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  long long stored = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    uint8_t code = st[i];
    if (code == BL_PLACED) {  // stored in phase 1 (and counted there)
      code = ST_OK;
    } else if (code == ST_OK || code == BL_FOLLOW || code == BL_ALLOC) {
      const bool allocator = code == BL_ALLOC;
      code = ST_OK;
      const uint64_t p = pos[i], tk = ticket[i];
      // bucket 0 is the slot's own; a later bucket's offset comes from the slot's record: one the
      // batch allocated lies at a known distance from the first new one, the key's last bucket
      // before the batch is the one the first new bucket links to (or the record's last bucket)
      const uint64_t bi = bl_bucket_of(b, tk);
      uint64_t o = p * b.s0;
      if (bi >= 1) {
        const ulonglong2 rec = b.meta[p];
        const uint32_t held = (uint32_t)rec.x, bp = (uint32_t)(rec.x >> 32), fn = (uint32_t)(rec.y >> 32);
        if (fn == BL_CUT) {  // the pool ran out: the key keeps the values its held buckets take
          const uint64_t keep = bl_S(b, held);
          if (allocator) {
            const uint64_t w = t.slots[p];
            atomicExch((unsigned long long*)&t.slots[p], (unsigned long long)make_slot(slot_key(w), (uint32_t)keep));
          }
          if (tk >= keep) code = ST_FULL;
        }
        if (code == ST_OK)
          o = bi >= bp ? fn + bl_words(b, bp, bi) : (fn < BL_CUT ? b.pool[fn] : (uint32_t)rec.y);
      }
      if (code == ST_OK) {
        b.pool[o + (bi >= 1 ? 1 : 0) + (tk - bl_S(b, bi))] = values[i];
        ++stored;
      }
    }
    if (status != nullptr) status[i] = code;
  }
  wave_add_to(t.size, stored);
}

// ---- retrieval -------------------------------------------------------------------------

// Probe for the key (as a single-value lookup); count mode writes the key's
// count, write mode walks its list back from the last bucket, the group's lanes
// copying each bucket's values.
template <int G, int W, bool WRITE>
struct BlProbe {
  using L = Lane<G, W>;
  static constexpr int SPL = L::SPL;
  L ln;
  TableView t;
  BucketView b;
  const uint32_t* __restrict__ keys;
  uint32_t* __restrict__ counts;
  uint64_t* __restrict__ offsets;
  uint32_t* __restrict__ out;
  unsigned long long* long_n = nullptr;  // lists longer than BL_LONG_LIST values: (query, slot, count)
  uint64_t* long_list = nullptr;
  uint64_t i = 0, base_nx = 0, end_nx = 0, base = 0, limit = 0;
  uint32_t k = 0, lbase = 0, k_nx = 0;
  Seq s{};
  // output staging of the count pass (drive_staged), as for the tables' queries
  uint32_t* ring_val = nullptr;
  uint8_t* ring_found = nullptr;
  uint8_t* ring_done = nullptr;
  uint64_t seq = 0, flushed = 0;
  static constexpr uint32_t RING = 128;

  __device__ __forceinline__ void write_out(uint64_t e, uint32_t c, uint8_t) {
    offsets[e] = c;
    if (counts != nullptr) counts[e] = c;
  }
  __device__ __forceinline__ void load(uint64_t op) {
    k_nx = keys[op];
    if constexpr (WRITE) {
      base_nx = offsets[op];
      end_nx = offsets[op + 1];
    }
  }
  __device__ __forceinline__ void begin(uint64_t op) {
    i = op;
    k = k_nx;
    ln.start(t, k, s, lbase);
    base = base_nx;
    limit = end_nx - base_nx;
  }
  __device__ __forceinline__ bool found(uint64_t c, uint64_t p) {  // every lane of the group
    if constexpr (!WRITE) {
      if (ln.g.glane == 0) {
        if (ring_val != nullptr && seq >= flushed) {
          const uint32_t r = (uint32_t)(seq % RING);
          ring_val[r] = (uint32_t)c;
          ring_found[r] = 0;
          ring_done[r] = 1;
        } else {
          write_out(i, (uint32_t)c, 0);
        }
      }
    } else {
      if (c == 0 || limit == 0) return true;
      if (c > BL_LONG_LIST) {  // copied by a whole block
        if (ln.g.glane == 0) {
          const unsigned long long e = atomicAdd(long_n, 1ull);
          long_list[3 * e] = i;
          long_list[3 * e + 1] = p;
          long_list[3 * e + 2] = c;
        }
        return true;
      }
      uint64_t bi = bl_bucket_of(b, c - 1);
      uint64_t o = bi == 0 ? p * b.s0 : (uint32_t)b.meta[p].y;  // one bucket: at p * s0
      for (;;) {
        const uint64_t lo = bl_S(b, bi), hi = bl_S(b, bi + 1) < c ? bl_S(b, bi + 1) : c;
        const uint64_t v0 = o + (bi >= 1 ? 1 : 0);
        for (uint64_t j = ln.g.glane; j < hi - lo; j += G)
          if (lo + j < limit) out[base + lo + j] = b.pool[v0 + j];  // never leave the segment
        if (bi == 0) break;
        o = b.pool[o];
        --bi;
      }
    }
    return true;
  }
  __device__ __forceinline__ bool step() {
    const auto& g = ln.g;
    if (reserved_key(k)) return found(0, 0);
    Window<SPL> win;
    load_step<G, W>(t, ln, s, lbase, k, win);
    const uint64_t b_match = g.bits(win.match != 0);
    if (b_match) {
      const uint32_t r = (uint32_t)ffs64(b_match);
      uint64_t c = 0, p = 0;
      if (g.glane == r) {
        c = slot_value(pick_lowest<SPL>(win.word, win.match));
        p = win.first + lowbit(win.match);
      }
      return found(g.bcast64(c, r), g.bcast64(p, r));
    }
    if (g.bits(win.empty != 0) || ln.exhausted(t, lbase)) return found(0, 0);
    ln.advance(t, s, lbase);
    return false;
  }
  __device__ __forceinline__ void end() {}
};

template <int G, int W, bool WRITE>
__global__ __launch_bounds__(BLOCK) void k_bl_probe(TableView t, WorkCtl ctl, BucketView b,
                                                    const uint32_t* __restrict__ keys, uint64_t n,
                                                    uint32_t* __restrict__ counts, uint64_t* __restrict__ offsets,
                                                    uint32_t* __restrict__ out, unsigned long long* long_n,
                                                    uint64_t* long_list) {
  using P = BlProbe<G, W, WRITE>;
  P op;
  op.t = t;
  op.b = b;
  op.keys = keys;
  op.counts = counts;
  op.offsets = offsets;
  op.out = out;
  op.long_n = long_n;
  op.long_list = long_list;
  if constexpr (WRITE) {
    drive<G>(n, ctl, op);
  } else {
    __shared__ OutRing<P::RING> rings[BLOCK / 64];
    drive_staged<G, P::RING>(n, ctl, op, rings[threadIdx.x >> 6]);
  }
}

// Long lists: one block per list walks it back from the last bucket, all its
// threads copying each bucket's values.
__global__ __launch_bounds__(1024) void k_bl_write_long(BucketView b, const uint64_t* __restrict__ offsets,
                                                        uint32_t* __restrict__ out, WorkCtl ctl,
                                                        const unsigned long long* __restrict__ long_n,
                                                        const uint64_t* __restrict__ long_list) {
  __shared__ unsigned long long s_item;
  const uint64_t L = *long_n;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(ctl.counters, 1ull);
    __syncthreads();
    const uint64_t e = s_item;
    __syncthreads();
    if (e >= L) break;
    const uint64_t i = long_list[3 * e], p = long_list[3 * e + 1], c = long_list[3 * e + 2];
    const uint64_t base = offsets[i], limit = offsets[i + 1] - base;
    uint64_t bi = bl_bucket_of(b, c - 1);
    uint64_t o = bi == 0 ? p * b.s0 : (uint32_t)b.meta[p].y;  // one bucket: at p * s0
    for (;;) {
      const uint64_t lo = bl_S(b, bi), hi = bl_S(b, bi + 1) < c ? bl_S(b, bi + 1) : c;
      const uint64_t v0 = o + (bi >= 1 ? 1 : 0);
      for (uint64_t j = threadIdx.x; j < hi - lo; j += 1024)
        if (lo + j < limit) out[base + lo + j] = b.pool[v0 + j];  // never leave the segment
      if (bi == 0) break;
      o = b.pool[o];
      --bi;
    }
  }
  if (threadIdx.x == 0) {
    if (atomicAdd(ctl.counters + 1, 1ull) == (unsigned long long)gridDim.x - 1) {
      atomicExch(ctl.counters, 0ull);
      atomicExch(ctl.counters + 1, 0ull);
    }
  }
}

// ---- erase: the key's slot becomes a tombstone, its values leave the count ------------

template <int G, int W>
struct BlErase {
  using L = Lane<G, W>;
  static constexpr int SPL = L::SPL;
  L ln;
  TableView t;
  ulonglong2* meta;
  const uint32_t* __restrict__ keys;
  uint8_t* __restrict__ status;
  uint64_t i = 0;
  uint32_t k = 0, lbase = 0, k_nx = 0;
  Seq s{};
  long long added = 0;

  __device__ __forceinline__ void load(uint64_t op) { k_nx = keys[op]; }
  __device__ __forceinline__ void begin(uint64_t op) {
    i = op;
    k = k_nx;
    ln.start(t, k, s, lbase);
  }
  __device__ __forceinline__ bool done(uint8_t code) {
    if (status != nullptr && ln.g.glane == 0) status[i] = code;
    return true;
  }
  __device__ __forceinline__ bool step() {
    const auto& g = ln.g;
    if (reserved_key(k)) return done(ST_INVALID_KEY);
    Window<SPL> win;
    load_step<G, W>(t, ln, s, lbase, k, win);
    const uint64_t b_match = g.bits(win.match != 0);
    if (b_match) {
      const uint32_t r = (uint32_t)ffs64(b_match);
      uint32_t ok = 0;
      if (g.glane == r) {
        const uint64_t idx = win.first + lowbit(win.match);
        const uint64_t res = atomicExch((unsigned long long*)&t.slots[idx], (unsigned long long)WORD_TOMB);
        if (slot_key(res) == k) {  // else erased by another group of this launch
          ok = 1;
          added -= (long long)slot_value(res);
          meta[idx].x = 0ull;  // no buckets recorded: a key that claims this slot later starts afresh
        }
      }
      return done(g.bcast(ok, r) ? ST_OK : ST_NOT_FOUND);
    }
    if (g.bits(win.empty != 0) || ln.exhausted(t, lbase)) return done(ST_NOT_FOUND);
    ln.advance(t, s, lbase);
    return false;
  }
  __device__ __forceinline__ void end() { wave_add_to(t.size, added); }
};

template <int G, int W>
__global__ __launch_bounds__(BLOCK) void k_bl_erase(TableView t, WorkCtl ctl, ulonglong2* meta,
                                                    const uint32_t* __restrict__ keys, uint64_t n,
                                                    uint8_t* __restrict__ status) {
  BlErase<G, W> op;
  op.t = t;
  op.meta = meta;
  op.keys = keys;
  op.status = status;
  drive<G>(n, ctl, op);
}

__global__ __launch_bounds__(64) void k_bl_zero1(unsigned long long* p) {
  if (threadIdx.x == 0) *p = 0ull;
}

__global__ __launch_bounds__(256) void k_bl_reset(ulonglong2* meta, uint64_t C) {
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < C; i += stride) meta[i].x = 0ull;
}

__global__ __launch_bounds__(256) void k_bl_dump_last(const ulonglong2* __restrict__ meta, uint64_t C,
                                                      uint32_t* __restrict__ dst) {
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < C; i += stride) dst[i] = (uint32_t)meta[i].y;
}

// ---- host side ----------------------------------------------------------------------------

bool bucket_ramp(uint32_t s0, double growth, uint32_t smax, uint64_t* cum, uint32_t* m) {
  uint64_t s = s0, total = 0;
  uint32_t i = 0;
  cum[0] = 0;
  while (s < smax) {
    if (i >= BL_MAX_RAMP) return false;
    total += s;
    cum[++i] = total;
    const double next = std::ceil(growth * (double)s);
    s = next >= (double)smax ? smax : (uint64_t)next;
  }
  *m = i;
  return true;
}

static uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

uint64_t bl_insert_workspace(uint64_t n) { return align256(8 * n) + align256(4 * n) + align256(n); }

static unsigned stream_grid(uint64_t n) {
  uint64_t g = (n + 255) / 256;
  const uint64_t cap = (uint64_t)device_cu_count() * 8;
  if (g > cap) g = cap;
  return (unsigned)(g ? g : 1);
}

hc_err launch_bl_insert(const TableView& t, const BucketView& b, uint32_t G, uint32_t W, const uint32_t* keys,
                        const uint32_t* values, uint64_t n, uint8_t* status, void* ws, hipStream_t s) {
  char* p = (char*)ws;
  uint64_t* pos = (uint64_t*)p; p += align256(8 * n);
  uint32_t* ticket = (uint32_t*)p; p += align256(4 * n);
  uint8_t* st = (uint8_t*)p;
  hc_err r = launch_bl_tickets(t, b, G, W, keys, nullptr, values, n, nullptr, pos, ticket, st, s);
  if (r != HC_OK) return r;
  return launch_bl_finish(t, b, values, n, pos, ticket, st, status, s);
}

hc_err launch_bl_tickets(const TableView& t, const BucketView& b, uint32_t G, uint32_t W, const uint32_t* keys,
                         const uint32_t* incr, const uint32_t* values, uint64_t n, const uint64_t* n_dev,
                         uint64_t* pos, uint32_t* ticket, uint8_t* st, hipStream_t s) {
  return dispatch_gw(G, W, [&](auto g, auto w) -> hc_err {
    constexpr int GG = decltype(g)::value, WW = decltype(w)::value;
    auto k = k_bl_ticket<GG, WW>;
    const unsigned grid = grid_for(k, n, GG);
    hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, s, t, work_for(n_dev ? n / 8 : n, GG, grid, s), b, keys, incr,
                       values, n, n_dev, pos, ticket, st);
    return check_launch("bucket list tickets");
  });
}

hc_err launch_bl_expand(const uint64_t* scan, const uint64_t* starts, uint64_t n, const uint64_t* rpos,
                        const uint32_t* rticket, const uint8_t* rst, uint64_t* pos, uint32_t* ticket, uint8_t* st,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_bl_expand, dim3(stream_grid(n)), dim3(256), 0, s, scan, starts, n, rpos, rticket, rst, pos,
                     ticket, st);
  return check_launch("bucket list tickets of pairs");
}

hc_err launch_bl_finish(const TableView& t, const BucketView& b, const uint32_t* values, uint64_t n,
                        const uint64_t* pos, const uint32_t* ticket, const uint8_t* st, uint8_t* status,
                        hipStream_t s) {
  uint64_t ga = (n + ALLOC_BLOCK - 1) / ALLOC_BLOCK;
  const uint64_t cap = (uint64_t)device_cu_count() * 2;
  if (ga > cap) ga = cap;
  hipLaunchKernelGGL(k_bl_alloc, dim3((unsigned)(ga ? ga : 1)), dim3(ALLOC_BLOCK), 0, s, t, b, n, pos, ticket,
                     const_cast<uint8_t*>(st));
  if (hc_err r = check_launch("bucket list allocation"); r != HC_OK) return r;
  hipLaunchKernelGGL(k_bl_place, dim3(stream_grid(n)), dim3(256), 0, s, t, b, values, n, pos, ticket,
                     const_cast<uint8_t*>(st), status);
  return check_launch("bucket list values");
}

hc_err launch_bl_count(const TableView& t, uint32_t G, uint32_t W, const uint32_t* keys, uint64_t n, uint32_t* counts,
                       uint64_t* offsets, hipStream_t s) {
  return dispatch_gw(G, W, [&](auto g, auto w) -> hc_err {
    constexpr int GG = decltype(g)::value, WW = decltype(w)::value;
    auto k = k_bl_probe<GG, WW, false>;
    const unsigned grid = grid_for(k, n, GG);
    hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, s, t, work_for(n, GG, grid, s), BucketView{}, keys, n, counts,
                       offsets, nullptr, nullptr, nullptr);
    return check_launch("bucket list count");
  });
}

uint64_t bl_write_workspace(uint64_t n) { return 256 + 24 * n; }

hc_err launch_bl_write(const TableView& t, const BucketView& b, uint32_t G, uint32_t W, const uint32_t* keys,
                       uint64_t n, const uint64_t* offsets, uint32_t* out, void* ws, hipStream_t s) {
  unsigned long long* long_n = (unsigned long long*)ws;
  uint64_t* long_list = (uint64_t*)((char*)ws + 256);
  hipLaunchKernelGGL(k_bl_zero1, dim3(1), dim3(64), 0, s, long_n);
  hc_err r = check_launch("bucket list write");
  if (r != HC_OK) return r;
  r = dispatch_gw(G, W, [&](auto g, auto w) -> hc_err {
    constexpr int GG = decltype(g)::value, WW = decltype(w)::value;
    auto k = k_bl_probe<GG, WW, true>;
    const unsigned grid = grid_for(k, n, GG);
    hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, s, t, work_for(n, GG, grid, s), b, keys, n, nullptr,
                       const_cast<uint64_t*>(offsets), out, long_n, long_list);  // the write pass only reads offsets
    return check_launch("bucket list write");
  });
  if (r != HC_OK) return r;
  const uint64_t cap = (uint64_t)device_cu_count() * (uint64_t)blocks_per_cu_threads(
                           reinterpret_cast<const void*>(k_bl_write_long), 1024);
  const unsigned grid = (unsigned)(cap < n ? cap : (n ? n : 1));
  hipLaunchKernelGGL(k_bl_write_long, dim3(grid), dim3(1024), 0, s, b, offsets, out, work_for(0, 64, grid * 4, s), long_n,
                     long_list);
  return check_launch("bucket list long write");
}

hc_err launch_bl_erase(const TableView& t, const BucketView& b, uint32_t G, uint32_t W, const uint32_t* keys,
                       uint64_t n, uint8_t* status, hipStream_t s) {
  return dispatch_gw(G, W, [&](auto g, auto w) -> hc_err {
    constexpr int GG = decltype(g)::value, WW = decltype(w)::value;
    auto k = k_bl_erase<GG, WW>;
    const unsigned grid = grid_for(k, n, GG);
    hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, s, t, work_for(n, GG, grid, s), b.meta, keys, n, status);
    return check_launch("bucket list erase");
  });
}

hc_err launch_bl_reset(const BucketView& b, uint64_t C, hipStream_t s) {
  hipLaunchKernelGGL(k_bl_reset, dim3(stream_grid(C)), dim3(256), 0, s, b.meta, C);
  return check_launch("bucket list reset");
}

hc_err launch_bl_dump_last(const BucketView& b, uint64_t C, uint32_t* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_bl_dump_last, dim3(stream_grid(C)), dim3(256), 0, s, b.meta, C, dst);
  return check_launch("bucket list dump");
}

}  // namespace hc
