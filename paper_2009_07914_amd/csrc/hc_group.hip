// Multi-value tables under heavy key skew.
//
// The paper's multi-value insert stores every pair at the first reusable
// position of its key's window sequence (Sec. IV-B3), so the i-th copy of a key
// scans past the i-1 earlier ones: a key with m copies costs about m^2/(2W)
// window visits, and retrieving it scans about m/W windows (Sec. V-B: throughput
// degrades with the number of values per key).  Two additions keep the same
// stored multiset and the same layout invariant (no empty position before any
// stored position of a key) while removing the quadratic term:
//   * grouped insert: pairs are sorted by key; each run of one key claims its m
//     slots in one pass along the sequence: a group of the bulk driver per short
//     run (16 runs in flight per wavefront at g = 4), a wavefront per run of
//     SMALL_RUN or more pairs.  A run of at
//     least HEAVY_RUN pairs is first spread over the whole grid in claim rounds:
//     a round hands out, in segments of one block step, exactly as many further
//     windows of the key's sequence as the values still to be placed could fill
//     (remaining / W), so every reusable slot in them is certainly needed and is
//     claimed, whatever block gets there first; what is left after the rounds is
//     claimed by one block walking on from where they ended.  Claims CAS the
//     reusable word to a placeholder (k, 0); the block then writes values, taken
//     from the run by a per-run counter, with atomic exchanges;
//   * long queries: count and write passes give up after `budget` windows and
//     hand the query to rounds in which blocks scan segments of its sequence in
//     parallel (4^r segments per open query in round r).  Speculative segments
//     past the end of a key's copies find no match, since no copy of a key lies
//     after a window holding an empty slot, so counts add up exactly; a query whose
//     segments all missed an empty window goes on to the next round.  There are
//     enough rounds for their segments to cover a whole sequence.
//   * counting tables: the sorted keys are reduced to (key, run length) and each
//     distinct key is inserted once with its run length as the increment, so a
//     key that makes up a large part of a batch costs one atomic, not millions on
//     the same slot.
#include "hc_group.hpp"
#include "hc_bucket.hpp"
#include "hc_kernels.hpp"
#include "hc_launch.hpp"
#include "hc_sort.hpp"

namespace hc {

// A slot claimed with the placeholder (key, 0) takes its value: no other claim
// can target it (it is neither empty nor a tombstone) and no query runs in the
// same launch, so a relaxed atomic store suffices (an exchange would be a
// second read-modify-write of the line).
__device__ __forceinline__ void fill_claimed(unsigned long long* slot, unsigned long long word) {
  __hip_atomic_store(slot, word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}


constexpr int GB = 1024;              // threads per block of the run / long-query kernels
constexpr int GB_WAVES = GB / 64;
constexpr int GB_SPL = 4;             // slots per lane in block mode
constexpr uint32_t RUN_GRAB = 4;      // medium runs taken per wavefront atomic
constexpr uint64_t SMALL_RUN = 128;   // shorter runs are claimed by one group of the bulk driver
constexpr int IROUNDS = 10;           // claim rounds of heavy runs
constexpr uint64_t ROUND_MIN = 4ull * GB * GB_SPL;  // heavy runs with fewer values left finish in one block
constexpr int QROUNDS_MAX = 16;       // long-query rounds; round r gives each open query 4^r segments
// Slots per lane of a long-query segment: a segment item costs a chain of dependent
// loads and atomics (item, entry, query, key; completion) whatever its size, so
// segments are made twice the block-mode width (512 windows of 16 slots per item).
constexpr int LQ_SPL = 8;

struct KeySeq {
  uint32_t w0, step;
};

__device__ __forceinline__ KeySeq key_seq(const TableView& t, uint32_t k) {
  Seq s;
  seq_start(t, k, s);
  return {s.w, s.step};
}

// Window of sequence index l: the closed forms of seq_next.
__device__ __forceinline__ uint32_t window_at(const TableView& t, const KeySeq& q, uint64_t l) {
  uint64_t off;
  if (t.scheme == SCHEME_LINEAR) off = l;
  else if (t.scheme == SCHEME_QUADRATIC) off = l * (l + 1) / 2;
  else off = l * (uint64_t)q.step;
  if (t.pow2) return (uint32_t)((q.w0 + off) & t.pmask);
  return (uint32_t)((q.w0 + off) % t.P);
}

// Block-wide exclusive scan (GB threads); *total gets the sum.  lds: GB_WAVES words.
__device__ __forceinline__ uint32_t block_scan(uint32_t x, uint32_t* total, uint32_t* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t incl = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) lds[wave] = incl;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < GB_WAVES; ++w) {
    const uint32_t v = lds[w];
    before += (w < wave) ? v : 0u;
    all += v;
  }
  __syncthreads();
  *total = all;
  return before + incl - x;
}

// ---- grouped insert -------------------------------------------------------------

// Claim m slots for key k with a whole block, walking its sequence from window l0
// (every reusable slot before l0 is already taken); the values are vals[0..m).
template <int W>
__device__ __forceinline__ void claim_run_block(const TableView& t, uint32_t k, const uint32_t* __restrict__ vals, uint64_t m,
                                uint64_t l0, uint64_t& added, uint32_t* lds) {
  constexpr uint32_t WPS_B = GB * GB_SPL / W;  // sequence windows per step
  const KeySeq q = key_seq(t, k);
  const uint32_t widx = (threadIdx.x * GB_SPL) / W, j0 = (threadIdx.x * GB_SPL) % W;
  uint64_t claimed = 0;
  for (uint64_t lbase = l0; claimed < m && lbase < t.P; lbase += WPS_B) {
    const uint64_t l = lbase + widx;
    uint64_t first = 0, word[GB_SPL];
    uint32_t reuse = 0, emptym = 0;
    if (l < t.P) {
      first = (uint64_t)window_at(t, q, l) * W + j0;
      load_slots<GB_SPL>(t.slots, first, word);
#pragma unroll
      for (int j = 0; j < GB_SPL; ++j) {
        const uint32_t key = slot_key(word[j]);
        emptym |= (uint32_t)(key == KEY_EMPTY) << j;
        reuse |= (uint32_t)(key == KEY_EMPTY || key == KEY_TOMB) << j;
      }
    }
    for (;;) {  // attempted slots leave `reuse`, so every round shrinks it
      uint32_t tot;
      const uint32_t ex = block_scan((uint32_t)__popc(reuse), &tot, lds);
      if (tot == 0) break;
      const uint64_t need = m - claimed;
      uint32_t succ = 0, tried = 0, rank = ex;
#pragma unroll
      for (int j = 0; j < GB_SPL; ++j) {
        if ((reuse >> j) & 1u) {
          if (rank < need) {
            const uint64_t expect = ((emptym >> j) & 1u) ? WORD_EMPTY : WORD_TOMB;
            const uint64_t r = atomicCAS((unsigned long long*)&t.slots[first + j], (unsigned long long)expect,
                                         (unsigned long long)make_slot(k, 0u));
            succ |= (uint32_t)(r == expect) << j;
            tried |= 1u << j;
          }
          ++rank;
        }
      }
      reuse &= ~tried;
      uint32_t stot;
      const uint32_t sex = block_scan((uint32_t)__popc(succ), &stot, lds);
      uint32_t rr = 0;
#pragma unroll
      for (int j = 0; j < GB_SPL; ++j) {
        if ((succ >> j) & 1u) {
          fill_claimed((unsigned long long*)&t.slots[first + j],
                     (unsigned long long)make_slot(k, vals[claimed + sex + rr]));
          ++rr;
        }
      }
      claimed += stot;
      if (claimed >= m) break;
    }
  }
  if (threadIdx.x == 0) added += claimed;
}

// Runs still short of their pairs after LONG_BUDGET windows (their sequence runs
// through a long stretch of full windows): the walk is handed over to find
// rounds, which look for the first window with a reusable slot in parallel.
struct WalkState {
  unsigned long long* nwalk;  // entries handed over
  unsigned long long* nopen;  // open entries at the start of each find round
  uint64_t* entry;            // run index (low 32 bits) and pairs placed (high 32 bits)
  uint64_t* base;             // next window of the sequence to look at
  unsigned long long* found;  // first window with a reusable slot (~0: none yet)
  uint32_t* done;             // segments of the current round finished
  uint32_t* lists[2];
  uint64_t cap;               // list capacity (nwalk may count past it)
};

// Where the claim kernels append hand-overs.
struct WalkOut {
  unsigned long long* nwalk;
  uint64_t* entry;
  uint64_t* base;
  uint64_t cap;
};

// Returns false when the list is full: the caller then walks on itself.
__device__ __forceinline__ bool walk_hand_over(const WalkOut& wo, uint64_t r, uint64_t claimed, uint64_t next_l) {
  const unsigned long long e = atomicAdd(wo.nwalk, 1ull);
  if (e >= wo.cap) return false;
  wo.entry[e] = r | (claimed << 32);
  wo.base[e] = next_l;
  return true;
}

// Claim m slots for key k (run r) with one wavefront (one slot per lane).
template <int W>
__device__ __forceinline__ void claim_run_wave(const TableView& t, uint32_t k, const uint32_t* __restrict__ vals, uint64_t m,
                               uint64_t r, const WalkOut& ws, uint64_t& added) {
  constexpr uint32_t WPS_W = 64 / W;  // W <= 64
  const uint32_t lane = __lane_id();
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const KeySeq q = key_seq(t, k);
  const uint32_t widx = lane / W, j = lane % W;
  uint64_t claimed = 0;
  for (uint64_t lbase = 0; claimed < m && lbase < t.P; lbase += WPS_W) {
    if (lbase == LONG_BUDGET) {  // hand the rest of the walk over (once)
      uint32_t ok = 0;
      if (lane == 0) ok = walk_hand_over(ws, r, claimed, lbase);
      if (__shfl(ok, 0, 64)) break;
    }
    const uint64_t l = lbase + widx;
    uint64_t idx = 0, word = 0;
    bool reuse = false;
    if (l < t.P) {
      idx = (uint64_t)window_at(t, q, l) * W + j;
      word = t.slots[idx];
      const uint32_t key = slot_key(word);
      reuse = key == KEY_EMPTY || key == KEY_TOMB;
    }
    for (;;) {
      const uint64_t bal = __ballot(reuse);
      if (bal == 0) break;
      const uint64_t need = m - claimed;
      const uint32_t rank = (uint32_t)__popcll(bal & below);
      bool ok = false;
      if (reuse && rank < need) {
        const uint64_t expect = (slot_key(word) == KEY_EMPTY) ? WORD_EMPTY : WORD_TOMB;
        const uint64_t r = atomicCAS((unsigned long long*)&t.slots[idx], (unsigned long long)expect,
                                     (unsigned long long)make_slot(k, 0u));
        ok = r == expect;
        reuse = false;
      }
      const uint64_t sb = __ballot(ok);
      if (ok)
        fill_claimed((unsigned long long*)&t.slots[idx],
                   (unsigned long long)make_slot(k, vals[claimed + __popcll(sb & below)]));
      claimed += (uint64_t)__popcll(sb);
      if (claimed >= m) break;
    }
  }
  if (lane == 0) added += claimed;
}

__global__ __launch_bounds__(256) void k_run_flags(const uint32_t* __restrict__ keys, uint64_t n,
                                                   uint64_t* __restrict__ flags, unsigned long long* nlists) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i == 0) {  // heavy list, medium list and hand-over list lengths
    nlists[0] = 0ull;
    nlists[1] = 0ull;
    nlists[2] = 0ull;
  }
  if (i < n) flags[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1ull : 0ull;
}

// scan[i] = runs before element i (exclusive scan of the flags), scan[n] = runs.
__global__ __launch_bounds__(256) void k_run_starts(const uint64_t* __restrict__ scan, uint64_t n,
                                                    uint64_t* __restrict__ starts) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n && scan[i + 1] != scan[i]) starts[scan[i]] = i;
  if (i == n) starts[scan[n]] = n;
}

// Lists of heavy runs (>= HEAVY_RUN pairs) and medium runs (SMALL_RUN .. HEAVY_RUN - 1).
__global__ __launch_bounds__(256) void k_run_lists(const uint64_t* __restrict__ starts,
                                                   const uint64_t* __restrict__ nruns, uint64_t max_runs,
                                                   uint32_t* __restrict__ heavy, unsigned long long* nheavy,
                                                   uint32_t* __restrict__ medium, unsigned long long* nmedium) {
  const uint64_t r = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (r < max_runs && r < *nruns) {
    const uint64_t m = starts[r + 1] - starts[r];
    if (m >= HEAVY_RUN) heavy[atomicAdd(nheavy, 1ull)] = (uint32_t)r;
    else if (m >= SMALL_RUN) medium[atomicAdd(nmedium, 1ull)] = (uint32_t)r;
  }
}

// Short runs: one group per run in the bulk driver.  Each step claims, in
// position order, the first (pairs still to place) reusable slots of the step's
// window(s); claims lost to other keys are replaced by later reusable slots of
// the same window before the sequence moves on, so no empty slot is left before
// a stored pair.
template <int G, int W>
struct ClaimRun {
  using L = Lane<G, W>;
  static constexpr int SPL = L::SPL;
  L ln;
  TableView t;
  const uint32_t* __restrict__ keys;
  const uint32_t* __restrict__ vals;
  const uint64_t* __restrict__ starts;
  WalkOut ws;
  uint64_t st = 0, m = 0, claimed = 0, st_nx = 0, en_nx = 0, run = 0;
  uint32_t k = 0, lbase = 0, k_nx = 0;
  Seq s{};
  long long added = 0;

  __device__ __forceinline__ void load(uint64_t r) {
    st_nx = starts[r];
    en_nx = starts[r + 1];
    k_nx = keys[st_nx];
  }
  __device__ __forceinline__ void begin(uint64_t r) {
    run = r;
    st = st_nx;
    m = en_nx - st_nx;
    k = k_nx;
    claimed = 0;
    ln.start(t, k, s, lbase);
  }
  __device__ __forceinline__ bool step() {
    const auto& g = ln.g;
    if (m >= SMALL_RUN || reserved_key(k)) return true;
    Window<SPL> win;
    load_step<G, W>(t, ln, s, lbase, k, win);
    MaskT<SPL> reuse = win.empty | win.tomb;
    for (;;) {  // attempted slots leave `reuse`, so every round shrinks it
      const uint32_t c = popcount(reuse);
      if (g.sum(c) == 0) break;
      const uint64_t need = m - claimed;
      uint32_t rank = g.exclusive_scan(c);
      MaskT<SPL> tried = 0, succ = 0;
#pragma unroll
      for (int j = 0; j < SPL; ++j) {
        if ((reuse >> j) & 1) {
          if (rank < need) {
            const uint64_t expect = ((win.empty >> j) & 1) ? WORD_EMPTY : WORD_TOMB;
            const uint64_t r = atomicCAS((unsigned long long*)&t.slots[win.first + j], (unsigned long long)expect,
                                         (unsigned long long)make_slot(k, 0u));
            tried |= (MaskT<SPL>)1 << j;
            if (r == expect) succ |= (MaskT<SPL>)1 << j;
          }
          ++rank;
        }
      }
      reuse &= ~tried;
      const uint32_t sc = popcount(succ);
      uint32_t vr = g.exclusive_scan(sc);
      const uint32_t stot = g.sum(sc);
#pragma unroll
      for (int j = 0; j < SPL; ++j) {
        if ((succ >> j) & 1) {
          fill_claimed((unsigned long long*)&t.slots[win.first + j],
                     (unsigned long long)make_slot(k, vals[st + claimed + vr]));
          ++vr;
        }
      }
      claimed += stot;
      if (g.glane == 0) added += stot;
      if (claimed >= m) return true;
    }
    if (ln.exhausted(t, lbase)) return true;  // table full: the rest of the run is dropped
    if (lbase + L::WPS == LONG_BUDGET) {      // a long walk: handed over to the find rounds (once)
      uint32_t ok = 0;
      if (g.glane == 0) ok = walk_hand_over(ws, run, claimed, lbase + L::WPS);
      if (g.bcast(ok, 0)) return true;
    }
    ln.advance(t, s, lbase);
    return false;
  }
  __device__ __forceinline__ void end() { wave_add_to(t.size, added); }
};

template <int G, int W>
__global__ __launch_bounds__(BLOCK) void k_claim_small(TableView t, WorkCtl ctl, const uint32_t* __restrict__ keys,
                                                       const uint32_t* __restrict__ vals,
                                                       const uint64_t* __restrict__ starts,
                                                       const uint64_t* __restrict__ nruns, WalkOut ws) {
  ClaimRun<G, W> op;
  op.t = t;
  op.keys = keys;
  op.vals = vals;
  op.starts = starts;
  op.ws = ws;
  drive<G>(*nruns, ctl, op);
}

// One find round: every open entry gets 4^round segments of SEGW windows from its
// next window on; found[e] becomes the first window of the segments holding a
// reusable slot.  Windows found full stay full (claims only fill slots), so the
// claim can start there.
template <int W>
__global__ __launch_bounds__(GB) void k_walk_round(TableView t, WorkCtl ctl, const uint32_t* __restrict__ keys,
                                                   const uint64_t* __restrict__ starts, WalkState ws,
                                                   uint32_t round) {
  constexpr uint64_t SEGW = GB * GB_SPL / W;
  __shared__ unsigned long long s_item, s_min;
  const uint64_t S = 1ull << (2 * round);
  const uint32_t* lin = ws.lists[round & 1];
  uint32_t* lout = ws.lists[(round + 1) & 1];
  const uint64_t N = ws.nopen[round] * S;
  if (N == 0) return;  // no open walk: no item is taken and the work counters stay at zero
  const uint32_t widx = (threadIdx.x * GB_SPL) / W, j0 = (threadIdx.x * GB_SPL) % W;
  for (;;) {
    if (threadIdx.x == 0) {
      s_item = atomicAdd(ctl.counters, 1ull);
      s_min = ~0ull;
    }
    __syncthreads();
    const uint64_t item = s_item;
    if (item >= N) break;
    const uint32_t e = lin[item / S];
    const uint64_t seg = item % S;
    const uint32_t r = (uint32_t)ws.entry[e];
    const uint32_t k = keys[starts[r]];
    const KeySeq q = key_seq(t, k);
    const uint64_t l = ws.base[e] + seg * SEGW + widx;
    if (l < t.P && l < ws.base[e] + (seg + 1) * SEGW) {
      uint64_t word[GB_SPL];
      load_slots<GB_SPL>(t.slots, (uint64_t)window_at(t, q, l) * W + j0, word);
      bool reusable = false;
#pragma unroll
      for (int jj = 0; jj < GB_SPL; ++jj) {
        const uint32_t kk = slot_key(word[jj]);
        reusable |= kk == KEY_EMPTY || kk == KEY_TOMB;
      }
      if (reusable) atomicMin(&s_min, (unsigned long long)l);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      if (s_min != ~0ull) atomicMin(ws.found + e, s_min);
      if (atomicAdd(ws.done + e, 1u) == (uint32_t)(S - 1)) {  // every segment of this round is done
        const uint64_t nb = ws.base[e] + S * SEGW;
        if (atomicMin(ws.found + e, ~0ull) == ~0ull && nb < t.P) {
          atomicExch((unsigned long long*)(ws.base + e), (unsigned long long)nb);
          atomicExch(ws.done + e, 0u);
          lout[atomicAdd(ws.nopen + round + 1, 1ull)] = e;
        }
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (atomicAdd(ctl.counters + 1, 1ull) == (unsigned long long)gridDim.x - 1) {
      atomicExch(ctl.counters, 0ull);
      atomicExch(ctl.counters + 1, 0ull);
    }
  }
}

// Round state of every handed-over walk; round 0 lists all of them.
__global__ __launch_bounds__(256) void k_walk_init(WalkState ws) {
  const uint64_t L = *ws.nwalk < ws.cap ? *ws.nwalk : ws.cap;
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x; e < L; e += stride) {
    ws.found[e] = ~0ull;
    ws.done[e] = 0u;
    ws.lists[0][e] = (uint32_t)e;
  }
  if (blockIdx.x == 0 && threadIdx.x <= QROUNDS_MAX) ws.nopen[threadIdx.x] = threadIdx.x == 0 ? L : 0ull;
}

// The handed-over runs: one block each claims the rest from the window found.
template <int W>
__global__ __launch_bounds__(GB) void k_walk_claim(TableView t, WorkCtl ctl, const uint32_t* __restrict__ keys,
                                                   const uint32_t* __restrict__ vals,
                                                   const uint64_t* __restrict__ starts, WalkState ws) {
  __shared__ uint32_t lds[GB_WAVES];
  __shared__ unsigned long long s_item;
  const uint64_t L = *ws.nwalk < ws.cap ? *ws.nwalk : ws.cap;
  if (L == 0) return;  // no handed-over run: no item is taken and the work counters stay at zero
  uint64_t added = 0;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(ctl.counters, 1ull);
    __syncthreads();
    const uint64_t e = s_item;
    __syncthreads();
    if (e >= L) break;
    const uint64_t r = (uint32_t)ws.entry[e], claimed = ws.entry[e] >> 32;
    const uint64_t st = starts[r], m = starts[r + 1] - st, f = ws.found[e];
    if (f != ~0ull)  // else no reusable slot left anywhere on the sequence: the rest is dropped
      claim_run_block<W>(t, keys[st], vals + st + claimed, m - claimed, f, added, lds);
  }
  __syncthreads();
  wave_add_to(t.size, (long long)added);
  if (threadIdx.x == 0) {
    if (atomicAdd(ctl.counters + 1, 1ull) == (unsigned long long)gridDim.x - 1) {
      atomicExch(ctl.counters, 0ull);
      atomicExch(ctl.counters + 1, 0ull);
    }
  }
}

// Per heavy run: next sequence window of the current round, windows in it, values placed.
struct HeavyState {
  uint64_t* pos;
  uint64_t* nw;
  unsigned long long* used;
  uint64_t* seg;  // exclusive prefix of the round's segments per heavy run; seg[H] = total
};

// Plan one claim round (one block): advance every heavy run past the previous
// round's windows and give it remaining / W more, in segments of one block step.
template <int W>
__global__ __launch_bounds__(GB) void k_heavy_plan(TableView t, const uint32_t* __restrict__ keys,
                                                   const uint64_t* __restrict__ starts,
                                                   const uint32_t* __restrict__ heavy,
                                                   const unsigned long long* __restrict__ nheavy, HeavyState hs,
                                                   int first) {
  constexpr uint64_t SEGW = GB * GB_SPL / W;
  __shared__ uint32_t lds[GB_WAVES];
  const uint64_t H = *nheavy;
  uint64_t carry = 0;
  for (uint64_t b = 0; b < H; b += GB) {
    const uint64_t h = b + threadIdx.x;
    uint32_t segs = 0;
    if (h < H) {
      const uint64_t r = heavy[h], st = starts[r], m = starts[r + 1] - st;
      uint64_t pos = 0, used = 0;
      if (!first) {
        pos = hs.pos[h] + hs.nw[h];
        used = hs.used[h];
      } else {
        hs.used[h] = 0;
      }
      const uint64_t rem = m - used;
      uint64_t nw = 0;
      if (!reserved_key(keys[st]) && rem >= ROUND_MIN && pos < t.P) {
        nw = rem / W;
        if (nw > t.P - pos) nw = t.P - pos;
      }
      hs.pos[h] = pos;
      hs.nw[h] = nw;
      segs = (uint32_t)((nw + SEGW - 1) / SEGW);
    }
    uint32_t tot;
    const uint32_t ex = block_scan(segs, &tot, lds);
    if (h < H) hs.seg[h] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) hs.seg[H] = carry;
}

// One claim round: blocks take segments of any heavy run; each claims every
// reusable slot of its segment and takes that many of the run's values.
template <int W>
__global__ __launch_bounds__(GB) void k_heavy_round(TableView t, WorkCtl ctl, const uint32_t* __restrict__ keys,
                                                    const uint32_t* __restrict__ vals,
                                                    const uint64_t* __restrict__ starts,
                                                    const uint32_t* __restrict__ heavy,
                                                    const unsigned long long* __restrict__ nheavy, HeavyState hs) {
  constexpr uint64_t SEGW = GB * GB_SPL / W;
  __shared__ uint32_t lds[GB_WAVES];
  __shared__ unsigned long long s_item, s_base;
  __shared__ uint32_t s_h;
  const uint64_t H = *nheavy, T = hs.seg[H];
  if (T == 0) return;  // no segment this round: no item is taken and the work counters stay at zero
  const uint32_t widx = (threadIdx.x * GB_SPL) / W, j0 = (threadIdx.x * GB_SPL) % W;
  uint64_t added = 0;
  for (;;) {
    if (threadIdx.x == 0) {
      const unsigned long long it = atomicAdd(ctl.counters, 1ull);
      s_item = it;
      if (it < T) {  // the heavy run owning segment `it`: last h with seg[h] <= it
        uint64_t lo = 0, hi = H - 1;
        while (lo < hi) {
          const uint64_t mid = (lo + hi + 1) / 2;
          if (hs.seg[mid] <= it) lo = mid;
          else hi = mid - 1;
        }
        s_h = (uint32_t)lo;
      }
    }
    __syncthreads();
    const uint64_t it = s_item;
    const uint32_t h = s_h;
    __syncthreads();
    if (it >= T) break;
    const uint64_t r = heavy[h], st = starts[r], m = starts[r + 1] - st;
    const uint32_t k = keys[st];
    const KeySeq q = key_seq(t, k);
    const uint64_t lend = hs.pos[h] + hs.nw[h];
    const uint64_t l = hs.pos[h] + (it - hs.seg[h]) * SEGW + widx;
    uint64_t first = 0;
    uint32_t succ = 0;
    if (l < lend) {
      uint64_t word[GB_SPL];
      first = (uint64_t)window_at(t, q, l) * W + j0;
      load_slots<GB_SPL>(t.slots, first, word);
#pragma unroll
      for (int j = 0; j < GB_SPL; ++j) {
        const uint32_t key = slot_key(word[j]);
        if (key == KEY_EMPTY || key == KEY_TOMB) {
          const uint64_t expect = key == KEY_EMPTY ? WORD_EMPTY : WORD_TOMB;
          const uint64_t rw = atomicCAS((unsigned long long*)&t.slots[first + j], (unsigned long long)expect,
                                        (unsigned long long)make_slot(k, 0u));
          succ |= (uint32_t)(rw == expect) << j;
        }
      }
    }
    uint32_t stot;
    const uint32_t sex = block_scan((uint32_t)__popc(succ), &stot, lds);
    if (threadIdx.x == 0) {
      s_base = stot ? atomicAdd(hs.used + h, (unsigned long long)stot) : 0ull;
      added += stot;
    }
    __syncthreads();
    // the round gave out at most (values left) slots, so base + stot <= m
    uint64_t rank = s_base + sex;
#pragma unroll
    for (int j = 0; j < GB_SPL; ++j) {
      if ((succ >> j) & 1u) {
        if (rank < m)
          fill_claimed((unsigned long long*)&t.slots[first + j], (unsigned long long)make_slot(k, vals[st + rank]));
        ++rank;
      }
    }
    __syncthreads();
  }
  wave_add_to(t.size, (long long)added);
  if (threadIdx.x == 0) {
    if (atomicAdd(ctl.counters + 1, 1ull) == (unsigned long long)gridDim.x - 1) {
      atomicExch(ctl.counters, 0ull);
      atomicExch(ctl.counters + 1, 0ull);
    }
  }
}

template <int W>
__global__ __launch_bounds__(GB) void k_claim_runs(TableView t, WorkCtl ctl, const uint32_t* __restrict__ keys,
                                                   const uint32_t* __restrict__ vals,
                                                   const uint64_t* __restrict__ starts,
                                                   const uint64_t* __restrict__ nruns,
                                                   const uint32_t* __restrict__ heavy,
                                                   const unsigned long long* __restrict__ nheavy, HeavyState hs,
                                                   const uint32_t* __restrict__ medium,
                                                   const unsigned long long* __restrict__ nmedium, WalkOut ws) {
  __shared__ uint32_t lds[GB_WAVES];
  __shared__ unsigned long long s_item;
  const uint64_t M = *nmedium, H = *nheavy;
  uint64_t added = 0;
  for (;;) {  // what the rounds left of each heavy run, one block each
    if (threadIdx.x == 0) s_item = atomicAdd(ctl.counters, 1ull);
    __syncthreads();
    const uint64_t h = s_item;
    __syncthreads();
    if (h >= H) break;
    const uint64_t r = heavy[h], st = starts[r], m = starts[r + 1] - st;
    const uint64_t used = hs.used[h];
    const uint32_t k = keys[st];
    if (!reserved_key(k) && used < m)
      claim_run_block<W>(t, k, vals + st + used, m - used, hs.pos[h] + hs.nw[h], added, lds);
  }
  const uint32_t lane = __lane_id();
  for (;;) {  // medium runs, one wavefront each, RUN_GRAB runs per atomic
    unsigned long long c = 0;
    if (lane == 0) c = atomicAdd(ctl.counters + 2, 1ull);
    c = __builtin_amdgcn_readfirstlane((uint32_t)c);
    const uint64_t i0 = (uint64_t)c * RUN_GRAB;
    if (i0 >= M) break;
    for (uint64_t i = i0; i < i0 + RUN_GRAB && i < M; ++i) {
      const uint64_t r = medium[i], st = starts[r], m = starts[r + 1] - st;
      const uint32_t k = keys[st];
      if (!reserved_key(k)) claim_run_wave<W>(t, k, vals + st, m, r, ws, added);
    }
  }
  __syncthreads();
  wave_add_to(t.size, (long long)added);
  if (threadIdx.x == 0) {
    if (atomicAdd(ctl.counters + 1, 1ull) == (unsigned long long)gridDim.x - 1) {
      atomicExch(ctl.counters, 0ull);
      atomicExch(ctl.counters + 1, 0ull);
      atomicExch(ctl.counters + 2, 0ull);
    }
  }
}

// ---- counting tables: one insert per distinct key ------------------------------------

// (key, run length) of every run.
__global__ __launch_bounds__(256) void k_run_lengths(const uint32_t* __restrict__ keys,
                                                     const uint64_t* __restrict__ starts,
                                                     const uint64_t* __restrict__ nruns, uint64_t max_runs,
                                                     uint32_t* __restrict__ ukeys, uint32_t* __restrict__ ucount) {
  const uint64_t r = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (r < max_runs && r < *nruns) {
    ukeys[r] = keys[starts[r]];
    ucount[r] = (uint32_t)(starts[r + 1] - starts[r]);
  }
}

template <int G, int W>
__global__ __launch_bounds__(BLOCK) void k_insert_counts(TableView t, WorkCtl ctl, const uint32_t* __restrict__ ukeys,
                                                         const uint32_t* __restrict__ ucount,
                                                         const uint64_t* __restrict__ nruns) {
  InsertUnique<G, W, KIND_COUNT> op;
  op.t = t;
  op.keys = ukeys;
  op.values = ucount;
  op.status = nullptr;
  drive<G>(*nruns, ctl, op);
}

// ---- long queries -----------------------------------------------------------------

__global__ __launch_bounds__(256) void k_zero_u64(unsigned long long* p, uint32_t count) {
  if (threadIdx.x < count) p[threadIdx.x] = 0ull;
}

// Scan windows [l, l + 1 window of this thread) ... of one segment: the thread's
// LQ_SPL slots of window l (if l < lend), its match mask and whether the window
// part holds an empty slot.
template <int W>
__device__ __forceinline__ uint32_t seg_slots(const TableView& t, const KeySeq& q, uint32_t k, uint64_t l,
                                              uint64_t lend, uint32_t j0, uint64_t (&word)[LQ_SPL], bool& empty) {
  uint32_t mm = 0;
  empty = false;
  if (l < lend) {
    load_slots<LQ_SPL>(t.slots, (uint64_t)window_at(t, q, l) * W + j0, word);
#pragma unroll
    for (int j = 0; j < LQ_SPL; ++j) {
      mm |= (uint32_t)(slot_key(word[j]) == k) << j;
      empty |= slot_key(word[j]) == KEY_EMPTY;
    }
  }
  return mm;
}

// The matches of one segment, added to the count or written through the
// query's cursor.  Returns (all threads) whether the query is finished: the
// segment met a window with an empty slot, reached the end of the sequence, or
// (write) the query's values are all written.
template <int W, int MODE>
__device__ __forceinline__ bool seg_visit(const TableView& t, const KeySeq& q, uint32_t k, uint64_t l0, uint64_t lend,
                                          uint64_t i, unsigned long long* cursor, uint64_t* __restrict__ offsets,
                                          uint32_t* __restrict__ out, uint64_t base, uint64_t limit, uint32_t* lds,
                                          unsigned long long* s_base) {
  const uint32_t widx = (threadIdx.x * LQ_SPL) / W, j0 = (threadIdx.x * LQ_SPL) % W;
  uint64_t word[LQ_SPL];
  bool empty;
  const uint32_t mm = seg_slots<W>(t, q, k, l0 + widx, lend, j0, word, empty);
  // matches (at most GB * LQ_SPL = 2^13 per block) in the low 16 bits, windows with an empty slot above
  uint32_t tot;
  const uint32_t ex = block_scan((uint32_t)__popc(mm) | ((uint32_t)empty << 16), &tot, lds) & 0xFFFFu;
  const uint32_t nm = tot & 0xFFFFu;
  bool fin = (tot >> 16) != 0 || lend >= t.P;
  if constexpr (MODE == 0) {
    if (threadIdx.x == 0 && nm) atomicAdd((unsigned long long*)&offsets[i], (unsigned long long)nm);
  } else {
    if (threadIdx.x == 0) *s_base = nm ? atomicAdd(cursor, (unsigned long long)nm) : atomicAdd(cursor, 0ull);
    __syncthreads();
    const uint64_t b = *s_base;
    uint64_t rank = b + ex;
#pragma unroll
    for (int j = 0; j < LQ_SPL; ++j) {
      if ((mm >> j) & 1u) {
        if (rank < limit) out[base + rank] = slot_value(word[j]);
        ++rank;
      }
    }
    fin = fin || b + nm >= limit;
    __syncthreads();
  }
  return fin;
}

// One round: every open entry gets S segments of SEGW windows from its next
// window on.  The last segment of an entry to finish decides whether it goes on.
// Items are latency chains (see LQ_SPL), so the kernel is held to the registers of
// two blocks per CU (8 wavefronts per SIMD).
template <int W, int MODE>
__global__ __launch_bounds__(GB, 8) void k_long_round(TableView t, WorkCtl ctl, const uint32_t* __restrict__ keys,
                                                      LongState ls, uint32_t round, uint64_t* __restrict__ offsets,
                                                      uint32_t* __restrict__ out) {
  constexpr uint64_t SEGW = GB * LQ_SPL / W;
  __shared__ uint32_t lds[GB_WAVES];
  __shared__ unsigned long long s_item, s_base;
  const uint64_t S = 1ull << (2 * round);
  const uint32_t* lin = ls.lists[round & 1];
  uint32_t* lout = ls.lists[(round + 1) & 1];
  const uint64_t N = ls.nopen[round] * S;
  // no open entry (every later round of a pass with no long query): no block takes an
  // item, so the work counters stay at zero and nothing is left to reset
  if (N == 0) return;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(ctl.counters, 1ull);
    __syncthreads();
    const uint64_t item = s_item;
    __syncthreads();
    if (item >= N) break;
    const uint32_t e = lin[item / S];
    const uint64_t seg = item % S;
    const uint64_t i = MODE == 0 ? ls.entries[e] : ls.entries[2 * e];
    const uint32_t k = keys[i];
    const KeySeq q = key_seq(t, k);
    const uint64_t l0 = ls.base[e] + seg * SEGW;
    uint64_t lend = l0 + SEGW;
    if (lend > t.P) lend = t.P;
    uint64_t obase = 0, limit = 0;
    if constexpr (MODE == 1) {
      obase = offsets[i];
      limit = offsets[i + 1] - obase;
    }
    const bool fin = l0 < t.P && seg_visit<W, MODE>(t, q, k, l0, lend, i,
                                                     (unsigned long long*)(ls.entries + 2 * e + 1), offsets, out,
                                                     obase, limit, lds, &s_base);
    if (threadIdx.x == 0) {
      if (fin || l0 >= t.P) atomicOr(ls.flag + e, 1u);
      if (atomicAdd(ls.done + e, 1u) == (uint32_t)(S - 1)) {  // every segment of this round is done
        const uint64_t nb = ls.base[e] + S * SEGW;
        if (atomicOr(ls.flag + e, 0u) == 0u && nb < t.P) {
          atomicExch((unsigned long long*)(ls.base + e), (unsigned long long)nb);
          atomicExch(ls.done + e, 0u);
          lout[atomicAdd(ls.nopen + round + 1, 1ull)] = e;
        }
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (atomicAdd(ctl.counters + 1, 1ull) == (unsigned long long)gridDim.x - 1) {
      atomicExch(ctl.counters, 0ull);
      atomicExch(ctl.counters + 1, 0ull);
    }
  }
}

// Round state of every handed-over entry; round 0 lists all of them.
__global__ __launch_bounds__(256) void k_long_init(LongState ls, uint32_t budget) {
  const uint64_t L = *ls.nlong < ls.cap ? *ls.nlong : ls.cap;
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x; e < L; e += stride) {
    ls.base[e] = budget;
    ls.flag[e] = 0u;
    ls.done[e] = 0u;
    ls.lists[0][e] = (uint32_t)e;
  }
  if (blockIdx.x == 0 && threadIdx.x <= QROUNDS_MAX) ls.nopen[threadIdx.x] = threadIdx.x == 0 ? L : 0ull;
}

// counts[i] of the handed-over queries, once their offsets hold the full counts.
__global__ __launch_bounds__(256) void k_long_counts_out(LongState ls, const uint64_t* __restrict__ offsets,
                                                         uint32_t* __restrict__ counts) {
  const uint64_t L = *ls.nlong < ls.cap ? *ls.nlong : ls.cap;
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x; e < L; e += stride) {
    const uint64_t i = ls.entries[e];
    counts[i] = (uint32_t)offsets[i];
  }
}

// ---- host side ----------------------------------------------------------------------

template <typename F>
static hc_err dispatch_w(uint32_t W, F&& f) {
  switch (W) {
    case 8: return f(ic<8>{});
    case 16: return f(ic<16>{});
    case 32: return f(ic<32>{});
    case 64: return f(ic<64>{});
  }
  return fail(HC_E_ARG, "window %u is not one of 8, 16, 32, 64", W);
}

static unsigned block_grid(const void* kernel, uint64_t items) {
  const uint64_t cap = (uint64_t)device_cu_count() * (uint64_t)blocks_per_cu_threads(kernel, GB);
  const uint64_t g = items < cap ? items : cap;
  return (unsigned)(g == 0 ? 1 : g);
}

static uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

// Entries of the hand-over list: runs whose walk outlasts LONG_BUDGET windows are
// rare; past this many, groups walk on themselves.
static uint64_t walk_capacity(uint64_t n) { return n / 16 + 1024; }

// Windows covered by rounds 0..R-1 of 4^r segments: enough rounds for a whole sequence.
static uint32_t rounds_to_cover(uint64_t P, uint64_t segw) {
  const uint64_t need = (P + segw - 1) / segw;
  uint32_t rounds = 1;
  for (uint64_t cover = 1; cover < need; cover = 4 * cover + 1) ++rounds;
  return rounds;
}

uint64_t grouped_workspace_bytes(uint64_t n) {
  const uint64_t hist = sort_pairs_workspace(n);
  const uint64_t scan_n = (hist > n + 1 ? hist : n + 1);
  const uint64_t hmax = n / HEAVY_RUN + 1;
  const uint64_t mmax = n / SMALL_RUN + 1, wmax = walk_capacity(n);
  return 4 * align256(4 * n) + align256(8 * hist) + align256(8 * scan_tiles_needed(scan_n)) + align256(8 * (n + 1)) +
         align256(8 * (n + 2)) + align256(4 * hmax) + align256(4 * mmax) + 256 + 3 * align256(8 * hmax) +
         align256(8 * (hmax + 1)) + 3 * align256(8 * wmax) + 3 * align256(4 * wmax) + 256;
}

hc_err launch_grouped_insert(const TableView& t, int kind, uint32_t G, uint32_t W, const uint32_t* keys,
                             const uint32_t* values, uint64_t n, void* work, hipStream_t s) {
  if (n == 0) return HC_OK;
  const bool counting = kind == KIND_COUNT;
  char* p = (char*)work;
  uint32_t* kc = (uint32_t*)p; p += align256(4 * n);
  uint32_t* vc = (uint32_t*)p; p += align256(4 * n);
  uint32_t* kt = (uint32_t*)p; p += align256(4 * n);
  uint32_t* vt = (uint32_t*)p; p += align256(4 * n);
  const uint64_t hist_n = sort_pairs_workspace(n);
  uint64_t* hist = (uint64_t*)p; p += align256(8 * hist_n);
  const uint64_t scan_n = (hist_n > n + 1 ? hist_n : n + 1);
  uint64_t* tiles = (uint64_t*)p; p += align256(8 * scan_tiles_needed(scan_n));
  uint64_t* flags = (uint64_t*)p; p += align256(8 * (n + 1));
  uint64_t* starts = (uint64_t*)p; p += align256(8 * (n + 2));
  const uint64_t hmax = n / HEAVY_RUN + 1;
  uint32_t* heavy = (uint32_t*)p; p += align256(4 * hmax);
  uint32_t* medium = (uint32_t*)p; p += align256(4 * (n / SMALL_RUN + 1));
  unsigned long long* nheavy = (unsigned long long*)p;  // nheavy, nmedium, nwalk, nopen[QROUNDS_MAX + 1]
  unsigned long long* nmedium = nheavy + 1;
  p += 256;
  WalkState wk;
  wk.nwalk = nheavy + 2;
  wk.nopen = nheavy + 3;
  wk.cap = walk_capacity(n);
  wk.entry = (uint64_t*)p; p += align256(8 * wk.cap);
  wk.base = (uint64_t*)p; p += align256(8 * wk.cap);
  wk.found = (unsigned long long*)p; p += align256(8 * wk.cap);
  wk.done = (uint32_t*)p; p += align256(4 * wk.cap);
  wk.lists[0] = (uint32_t*)p; p += align256(4 * wk.cap);
  wk.lists[1] = (uint32_t*)p; p += align256(4 * wk.cap);
  const WalkOut wo{wk.nwalk, wk.entry, wk.base, wk.cap};
  HeavyState hs;
  hs.pos = (uint64_t*)p; p += align256(8 * hmax);
  hs.nw = (uint64_t*)p; p += align256(8 * hmax);
  hs.used = (unsigned long long*)p; p += align256(8 * hmax);
  hs.seg = (uint64_t*)p;
  hipError_t e = hipMemcpyAsync(kc, keys, 4 * n, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && !counting) e = hipMemcpyAsync(vc, values, 4 * n, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return fail(HC_E_DEVICE, "grouped insert copy: %s", hipGetErrorString(e));
  if (hc_err r = sort_pairs(kc, counting ? nullptr : vc, kt, counting ? nullptr : vt, n, hist, tiles, s); r != HC_OK)
    return r;
  const unsigned g256 = (unsigned)((n + 256) / 256);
  hipLaunchKernelGGL(k_run_flags, dim3(g256), dim3(256), 0, s, kc, n, flags, nheavy);
  if (hc_err r = check_launch("run flags"); r != HC_OK) return r;
  if (hc_err r = exclusive_scan_inplace(flags, n, tiles, s); r != HC_OK) return r;
  hipLaunchKernelGGL(k_run_starts, dim3(g256), dim3(256), 0, s, flags, n, starts);
  if (hc_err r = check_launch("run starts"); r != HC_OK) return r;
  if (counting) {
    // kt / vt: distinct keys and their run lengths; flags + n: the number of runs
    hipLaunchKernelGGL(k_run_lengths, dim3(g256), dim3(256), 0, s, kc, starts, flags + n, n, kt, vt);
    if (hc_err r = check_launch("run lengths"); r != HC_OK) return r;
    return dispatch_gw(G, W, [&](auto g, auto w) -> hc_err {
      constexpr int GG = decltype(g)::value, WW = decltype(w)::value;
      auto k = k_insert_counts<GG, WW>;
      const unsigned grid = grid_for(k, n, GG);
      hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, s, t, work_for(n / 8, GG, grid, s), kt, vt, flags + n);
      return check_launch("insert counts");
    });
  }
  hipLaunchKernelGGL(k_run_lists, dim3(g256), dim3(256), 0, s, starts, flags + n, n, heavy, nheavy, medium, nmedium);
  if (hc_err r = check_launch("run lists"); r != HC_OK) return r;
  hc_err r = dispatch_w(W, [&](auto w) -> hc_err {
    constexpr int WW = decltype(w)::value;
    auto kr = k_heavy_round<WW>;
    const unsigned rgrid = block_grid(reinterpret_cast<const void*>(kr), ~0ull);
    for (int round = 0; round < IROUNDS; ++round) {
      hipLaunchKernelGGL(k_heavy_plan<WW>, dim3(1), dim3(GB), 0, s, t, kc, starts, heavy, nheavy, hs, round == 0);
      if (hc_err r = check_launch("heavy plan"); r != HC_OK) return r;
      WorkCtl ctl = work_for(0, 64, rgrid * (GB / 256), s);
      hipLaunchKernelGGL(kr, dim3(rgrid), dim3(GB), 0, s, t, ctl, kc, vc, starts, heavy, nheavy, hs);
      if (hc_err r = check_launch("heavy round"); r != HC_OK) return r;
    }
    auto k = k_claim_runs<WW>;
    const unsigned grid = block_grid(reinterpret_cast<const void*>(k), ~0ull);
    WorkCtl ctl = work_for(0, 64, grid * (GB / 256), s);  // a launch slot (counters 0..2 reset by the kernel)
    hipLaunchKernelGGL(k, dim3(grid), dim3(GB), 0, s, t, ctl, kc, vc, starts, flags + n, heavy, nheavy, hs, medium,
                       nmedium, wo);
    return check_launch("claim runs");
  });
  if (r != HC_OK) return r;
  r = dispatch_gw(G, W, [&](auto g, auto w) -> hc_err {
    constexpr int GG = decltype(g)::value, WW = decltype(w)::value;
    auto k = k_claim_small<GG, WW>;
    const unsigned grid = grid_for(k, n, GG);
    hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, s, t, work_for(n / 8, GG, grid, s), kc, vc, starts, flags + n, wo);
    return check_launch("claim short runs");
  });
  if (r != HC_OK) return r;
  // long walks: find rounds, then one block per run from the first window with room
  const unsigned ig = (unsigned)((wk.cap + 255) / 256 < 1024 ? (wk.cap + 255) / 256 : 1024);
  hipLaunchKernelGGL(k_walk_init, dim3(ig), dim3(256), 0, s, wk);
  if (hc_err e2 = check_launch("walk init"); e2 != HC_OK) return e2;
  return dispatch_w(W, [&](auto w) -> hc_err {
    constexpr int WW = decltype(w)::value;
    auto kr = k_walk_round<WW>;
    const unsigned grid = block_grid(reinterpret_cast<const void*>(kr), ~0ull);
    const uint32_t rounds = rounds_to_cover(t.P, GB * GB_SPL / WW);
    if (rounds > (uint32_t)QROUNDS_MAX) return fail(HC_E_ARG, "sequence too long for the find rounds");
    for (uint32_t round = 0; round < rounds; ++round) {
      WorkCtl ctl = work_for(0, 64, grid * (GB / 256), s);
      hipLaunchKernelGGL(kr, dim3(grid), dim3(GB), 0, s, t, ctl, kc, starts, wk, round);
      if (hc_err e2 = check_launch("walk round"); e2 != HC_OK) return e2;
    }
    auto kc2 = k_walk_claim<WW>;
    const unsigned cgrid = block_grid(reinterpret_cast<const void*>(kc2), ~0ull);
    WorkCtl ctl = work_for(0, 64, cgrid * (GB / 256), s);
    hipLaunchKernelGGL(kc2, dim3(cgrid), dim3(GB), 0, s, t, ctl, kc, vc, starts, wk);
    return check_launch("walk claim");
  });
}

// Bucket list table, grouped: sort, one ticket per run (the run's length added to the
// key's count with one atomic), pair tickets by rank in the run, then the bucket
// allocation and placement of a plain bulk insert.
uint64_t bl_grouped_workspace_bytes(uint64_t n) {
  return 4 * align256(4 * n) + align256(8 * sort_pairs_workspace(n)) +
         align256(8 * scan_tiles_needed(sort_pairs_workspace(n) > n + 1 ? sort_pairs_workspace(n) : n + 1)) +
         align256(8 * (n + 1)) + align256(8 * (n + 2)) + 256 + 2 * (align256(8 * n) + align256(4 * n) + align256(n));
}

hc_err launch_bl_grouped(const TableView& t, const BucketView& b, uint32_t G, uint32_t W, const uint32_t* keys,
                         const uint32_t* values, uint64_t n, void* work, hipStream_t s) {
  if (n == 0) return HC_OK;
  char* p = (char*)work;
  uint32_t* kc = (uint32_t*)p; p += align256(4 * n);
  uint32_t* vc = (uint32_t*)p; p += align256(4 * n);
  uint32_t* kt = (uint32_t*)p; p += align256(4 * n);
  uint32_t* vt = (uint32_t*)p; p += align256(4 * n);
  const uint64_t hist_n = sort_pairs_workspace(n);
  uint64_t* hist = (uint64_t*)p; p += align256(8 * hist_n);
  uint64_t* tiles = (uint64_t*)p; p += align256(8 * scan_tiles_needed(hist_n > n + 1 ? hist_n : n + 1));
  uint64_t* flags = (uint64_t*)p; p += align256(8 * (n + 1));
  uint64_t* starts = (uint64_t*)p; p += align256(8 * (n + 2));
  unsigned long long* nlists = (unsigned long long*)p; p += 256;
  uint64_t* rpos = (uint64_t*)p; p += align256(8 * n);
  uint32_t* rticket = (uint32_t*)p; p += align256(4 * n);
  uint8_t* rst = (uint8_t*)p; p += align256(n);
  uint64_t* pos = (uint64_t*)p; p += align256(8 * n);
  uint32_t* ticket = (uint32_t*)p; p += align256(4 * n);
  uint8_t* st = (uint8_t*)p;
  hipError_t e = hipMemcpyAsync(kc, keys, 4 * n, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(vc, values, 4 * n, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return fail(HC_E_DEVICE, "grouped insert copy: %s", hipGetErrorString(e));
  if (hc_err r = sort_pairs(kc, vc, kt, vt, n, hist, tiles, s); r != HC_OK) return r;
  const unsigned g256 = (unsigned)((n + 256) / 256);
  hipLaunchKernelGGL(k_run_flags, dim3(g256), dim3(256), 0, s, kc, n, flags, nlists);
  if (hc_err r = check_launch("run flags"); r != HC_OK) return r;
  if (hc_err r = exclusive_scan_inplace(flags, n, tiles, s); r != HC_OK) return r;
  hipLaunchKernelGGL(k_run_starts, dim3(g256), dim3(256), 0, s, flags, n, starts);
  if (hc_err r = check_launch("run starts"); r != HC_OK) return r;
  hipLaunchKernelGGL(k_run_lengths, dim3(g256), dim3(256), 0, s, kc, starts, flags + n, n, kt, vt);
  if (hc_err r = check_launch("run lengths"); r != HC_OK) return r;
  if (hc_err r = launch_bl_tickets(t, b, G, W, kt, vt, nullptr, n, flags + n, rpos, rticket, rst, s); r != HC_OK)
    return r;
  if (hc_err r = launch_bl_expand(flags, starts, n, rpos, rticket, rst, pos, ticket, st, s); r != HC_OK) return r;
  return launch_bl_finish(t, b, vc, n, pos, ticket, st, nullptr, s);
}

hc_err launch_zero_u64(unsigned long long* p, uint32_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(256), 0, s, p, count);
  return check_launch("zero");
}

uint64_t long_capacity(uint64_t n) { return n < walk_capacity(n) ? n : walk_capacity(n); }

uint64_t long_workspace_bytes(uint64_t n, int mode) {
  return 256 + align256((mode == 0 ? 8 : 16) * n) + align256(8 * n) + 4 * align256(4 * n) + 256;
}

LongState long_layout(void* ws, uint64_t n, int mode) {
  char* p = (char*)ws;
  LongState ls;
  ls.cap = n;
  ls.nlong = (const unsigned long long*)p;
  ls.nopen = (unsigned long long*)p + 1;  // QROUNDS_MAX + 1 words after the entry count
  p += 256;
  ls.entries = (uint64_t*)p; p += align256((mode == 0 ? 8 : 16) * n);
  ls.base = (uint64_t*)p; p += align256(8 * n);
  ls.flag = (uint32_t*)p; p += align256(4 * n);
  ls.done = (uint32_t*)p; p += align256(4 * n);
  ls.lists[0] = (uint32_t*)p; p += align256(4 * n);
  ls.lists[1] = (uint32_t*)p;
  return ls;
}

hc_err launch_long_queries(const TableView& t, uint32_t W, int mode, const uint32_t* keys, const LongState& ls,
                           uint64_t n, uint32_t budget, uint64_t* offsets, uint32_t* counts, uint32_t* out,
                           hipStream_t s) {
  const unsigned ig = (unsigned)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
  hipLaunchKernelGGL(k_long_init, dim3(ig ? ig : 1), dim3(256), 0, s, ls, budget);
  if (hc_err r = check_launch("long init"); r != HC_OK) return r;
  hc_err r = dispatch_w(W, [&](auto w) -> hc_err {
    constexpr int WW = decltype(w)::value;
    auto body = [&](auto mc) -> hc_err {
      constexpr int MODE = decltype(mc)::value;
      auto kr = k_long_round<WW, MODE>;
      const unsigned grid = block_grid(reinterpret_cast<const void*>(kr), ~0ull);
      // rounds 0..R-1 give an entry (4^R - 1) / 3 segments in all: enough for the whole sequence
      const uint32_t rounds = rounds_to_cover(t.P, GB * LQ_SPL / WW);
      if (rounds > (uint32_t)QROUNDS_MAX) return fail(HC_E_ARG, "sequence too long for the long-query rounds");
      for (uint32_t round = 0; round < rounds; ++round) {
        WorkCtl ctl = work_for(0, 64, grid * (GB / 256), s);
        hipLaunchKernelGGL(kr, dim3(grid), dim3(GB), 0, s, t, ctl, keys, ls, round, offsets, out);
        if (hc_err e = check_launch("long round"); e != HC_OK) return e;
      }
      return HC_OK;
    };
    return mode == 0 ? body(ic<0>{}) : body(ic<1>{});
  });
  if (r != HC_OK) return r;
  if (mode == 0 && counts != nullptr) {
    hipLaunchKernelGGL(k_long_counts_out, dim3(ig ? ig : 1), dim3(256), 0, s, ls, offsets, counts);
    return check_launch("long counts");
  }
  return HC_OK;
}

}  // namespace hc
