// Device building blocks of the cooperative-probing tables (gfx950, wave64).
//
// Slot codec (Sec. IV-B1, packed AoS): one 64-bit word per slot, key in bits 0-31,
// value (or count) in bits 32-63.  The empty word is 0 (empty indicator k_e = 0);
// the tombstone word is 0x00000000FFFFFFFF (k_t = 2^32 - 1, Sec. IV-B5).
//
// Window sequence (Sec. II schemes applied to windows, Sec. IV-B2): the table is
// P windows of W consecutive slots; window w covers slots [w*W, w*W + W).  Step l
// of a key's sequence is window w_l:
//   linear     w_l = (h1 + l) mod P
//   quadratic  w_l = (h1 + l(l+1)/2) mod P            (P a power of two)
//   double     w_l = (h1 + l*s) mod P, s = (h2 mod P) | 1 for a power-of-two P,
//              s = 1 + floor(h2 (P-1) / 2^32) for a prime P
// with h1 = fmix32(k ^ seed_lo), h2 = fmix32((k ^ seed_hi) + 0x9E3779B9), reduced
// to [0, P) by a mask (power of two) or by multiply-high.  fmix32 is the MurmurHash3
// finaliser (Appleby, public domain).  Every scheme visits each window exactly once
// in P steps, so a probe never exceeds the capacity.
//
// Groups (Sec. IV-B2, sub-warp tiles): G lanes of one 64-lane wavefront share an
// operation.  For G <= W the group covers one window per step and each lane holds
// SPL = W/G consecutive slots; for G > W the group covers G/W consecutive sequence
// windows per step, one slot per lane.  Either way the position order inside a step
// is lane-major, so "lowest lane, then lowest slot" is the lowest candidate
// position in sequence order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hc {

constexpr uint32_t KEY_EMPTY = 0u;
constexpr uint32_t KEY_TOMB = 0xFFFFFFFFu;
constexpr uint64_t WORD_EMPTY = 0ull;
constexpr uint64_t WORD_TOMB = 0x00000000FFFFFFFFull;

enum : uint8_t { ST_OK = 0, ST_DUPLICATE = 1, ST_FULL = 2, ST_INVALID_KEY = 3, ST_NOT_FOUND = 4 };
enum : uint32_t { SCHEME_LINEAR = 0, SCHEME_QUADRATIC = 1, SCHEME_DOUBLE = 2 };
enum : int { KIND_SINGLE = 0, KIND_MULTI = 1, KIND_COUNT = 2 };

constexpr int BLOCK = 256;  // threads per block: 4 wavefronts

__host__ __device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

__device__ __forceinline__ uint32_t slot_key(uint64_t w) { return (uint32_t)w; }
__device__ __forceinline__ uint32_t slot_value(uint64_t w) { return (uint32_t)(w >> 32); }
__device__ __forceinline__ uint64_t make_slot(uint32_t k, uint32_t v) {
  return (uint64_t)k | ((uint64_t)v << 32);
}
__device__ __forceinline__ bool reserved_key(uint32_t k) { return k == KEY_EMPTY || k == KEY_TOMB; }

// Words of the table's counter block (TableView::size points at word 0).
constexpr int CTR_SIZE = 0;        // live entries (wrapping add of +/- deltas)
constexpr int CTR_POOL = 1;        // bucket list tables: pool words handed out
constexpr int CTR_CAS_FAILS = 2;   // claim CASes of inserts that found the slot changed

// Kernel-side view of a table (passed by value).
struct TableView {
  uint64_t* slots;
  unsigned long long* size;  // the counter block: size[CTR_SIZE], size[CTR_POOL], size[CTR_CAS_FAILS]
  uint32_t P;                // windows, 1 <= P <= 2^31
  uint32_t pmask;            // P - 1 when P is a power of two, else 0
  uint32_t pow2;             // 1 if P is a power of two
  uint32_t scheme;
  uint32_t seed_lo, seed_hi;
};

// Per-launch work counters: counters[0] hands out chunks, counters[1] counts
// finished wavefronts; both are zero when a launch starts.
struct WorkCtl {
  unsigned long long* counters;
  uint32_t chunk;  // elements per chunk, 64 <= chunk
};

// Position in a key's window sequence.
struct Seq {
  uint32_t w;     // current window
  uint32_t step;  // double-hashing stride (1 for linear)
  uint32_t l;     // sequence index of w
};

__device__ __forceinline__ uint32_t reduce_window(const TableView& t, uint32_t x) {
  return t.pow2 ? (x & t.pmask) : __umulhi(x, t.P);
}

__device__ __forceinline__ void seq_start(const TableView& t, uint32_t k, Seq& s) {
  s.w = reduce_window(t, fmix32(k ^ t.seed_lo));
  s.l = 0;
  s.step = 1;
  if (t.scheme == SCHEME_DOUBLE) {
    const uint32_t h2 = fmix32((k ^ t.seed_hi) + 0x9E3779B9u);
    s.step = t.pow2 ? ((h2 & t.pmask) | 1u) : (1u + __umulhi(h2, t.P - 1u));
  }
}

__device__ __forceinline__ void seq_next(const TableView& t, Seq& s) {
  s.l += 1;
  if (t.scheme == SCHEME_QUADRATIC) {
    s.w = (s.w + s.l) & t.pmask;  // T(l) - T(l-1) = l
  } else {
    s.w += s.step;                // step < P <= 2^31: no overflow
    if (s.w >= t.P) s.w -= t.P;
  }
}

// ---- group helpers ------------------------------------------------------------

template <int G>
struct GroupCtx {
  static constexpr uint64_t MASK = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
  uint32_t lane;   // lane in wavefront
  uint32_t glane;  // rank in group
  uint32_t gbase;  // first lane of the group
  __device__ __forceinline__ GroupCtx() {
    lane = __lane_id();
    glane = lane & (G - 1);
    gbase = lane & ~(uint32_t)(G - 1);
  }
  // The group's bits of a wavefront ballot, as a G-bit mask (bit r = group rank r).
  __device__ __forceinline__ uint64_t bits(bool pred) const {
    const uint64_t b = __ballot(pred);
    if constexpr (G == 64) return b;
    return (b >> gbase) & MASK;
  }
  template <typename T>
  __device__ __forceinline__ T bcast(T v, uint32_t rank) const {
    return __shfl(v, (int)(gbase + rank), 64);
  }
  __device__ __forceinline__ uint64_t bcast64(uint64_t v, uint32_t rank) const {
    const uint32_t lo = __shfl((uint32_t)v, (int)(gbase + rank), 64);
    const uint32_t hi = __shfl((uint32_t)(v >> 32), (int)(gbase + rank), 64);
    return (uint64_t)lo | ((uint64_t)hi << 32);
  }
  // Sum over the group (all lanes get the result).
  __device__ __forceinline__ uint32_t sum(uint32_t x) const {
#pragma unroll
    for (int d = 1; d < G; d <<= 1) x += __shfl_xor(x, d, 64);
    return x;
  }
  // Exclusive prefix sum over the group ranks.
  __device__ __forceinline__ uint32_t exclusive_scan(uint32_t x) const {
    uint32_t incl = x;
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
      const uint32_t y = __shfl_up(incl, d, G);
      if (glane >= (uint32_t)d) incl += y;
    }
    return incl - x;
  }
};

__device__ __forceinline__ int ffs64(uint64_t x) { return __ffsll((unsigned long long)x) - 1; }

// Geometry of one probing step for group size G and window W.
template <int G, int W>
struct Step {
  static_assert(G >= 1 && G <= 64 && (G & (G - 1)) == 0, "group size must be a power of two <= 64");
  static_assert(W >= 1 && W <= 64 && (W & (W - 1)) == 0, "window must be a power of two <= 64");
  static constexpr int SPL = (G <= W) ? (W / G) : 1;  // slots per lane
  static constexpr int WPS = (G <= W) ? 1 : (G / W);  // sequence windows per step
};

// Load the SPL consecutive slots starting at slot index `first` (SPL * 8-byte aligned).
template <int SPL>
__device__ __forceinline__ void load_slots(const uint64_t* __restrict__ slots, uint64_t first, uint64_t (&w)[SPL]) {
  if constexpr (SPL == 1) {
    w[0] = slots[first];
  } else {
    const ulonglong2* p = reinterpret_cast<const ulonglong2*>(slots + first);
#pragma unroll
    for (int j = 0; j < SPL / 2; ++j) {
      const ulonglong2 q = p[j];
      w[2 * j] = q.x;
      w[2 * j + 1] = q.y;
    }
  }
}

// Wavefront-wide sum, then one atomic per wavefront (lanes must be converged).
__device__ __forceinline__ void wave_add_to(unsigned long long* counter, long long x) {
  unsigned long long v = (unsigned long long)x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t lo = __shfl_xor((uint32_t)v, d, 64);
    const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), d, 64);
    v += (unsigned long long)lo | ((unsigned long long)hi << 32);
  }
  if (__lane_id() == 0 && v != 0) atomicAdd(counter, v);
}

}  // namespace hc
