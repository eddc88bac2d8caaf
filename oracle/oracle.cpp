/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  The product path (the HIP library and its binding)
 * never imports, links or calls it, and it shares no code, header, table or
 * constant generator with that path.
 *
 * What it computes (WarpCore, arXiv 2009.07914):
 *
 *  (1) The observable semantics of the three table kinds, applied op by op in
 *      batch index order on one thread, over a plain associative container
 *      (std::unordered_map) plus an explicit capacity:
 *        - single-value table: a finite map K -> V of bounded capacity
 *          (Sec. II; Sec. IV, SingleValueHashTable; Sec. IV-B1: the array size
 *          fixes the capacity).  Re-inserting a present key is reported as a
 *          duplicate (Sec. IV-B3) and overwrites the value (upsert reading).
 *        - multi-value table: a finite multimap; every insert stores one pair
 *          (Sec. IV, MultiValueHashTable); retrieval of all values of a batch
 *          of queries is a per-query count, an exclusive prefix sum into n+1
 *          offsets, then the values of query i in segment i (Sec. IV-B4).
 *        - counting table: a map K -> number of occurrences (Sec. IV,
 *          CountingHashTable), counts wrapping modulo 2^32.
 *      Deletion removes the key (Sec. IV-B5); for the multimap it removes
 *      every pair of the key.  Keys 0 (empty indicator k_e) and 2^32-1
 *      (tombstone k_t) are reserved (Sec. IV-B1, IV-B5) and are rejected.
 *      An insert of a new key into a table holding `capacity` live entries
 *      fails (the probing abort criterion of Sec. II: every slot visited).
 *
 *  (2) A layout checker for a dumped slot array of the GPU table.  It
 *      re-derives, independently, each key's window sequence (Sec. II
 *      probing schemes; Sec. IV-B2 cooperative probing with an inner linear
 *      window) and verifies the invariants retrieval relies on (Sec. IV-B4:
 *      a key sits at its lowest possible position, so no earlier position of
 *      its sequence is empty), key uniqueness for single-value and counting
 *      tables, slot encodings, and the live count.
 *
 *  (3) A sequential scalar model of the same probing (one key at a time,
 *      first reusable position in sequence order), used to produce valid
 *      layouts for the checker's own tests and to measure windows per
 *      operation on actual key sets.
 *
 *  (4) The Bloom filter (Sec. IV lists a BloomFilter answering set membership
 *      queries; the paper gives no design), in the blocked form read for it:
 *      the bit array is B blocks of `words` 32-bit words; key x picks block
 *      reduce(h1(x), B) and sets one bit in every word of it, bit
 *      fmix32(h2(x) + i * 0x9E3779B9) >> 27 of word i (a split-block filter:
 *      k = words bits per key, one per word).  A query answers yes iff all
 *      of them are set.
 *
 * Where the paper is silent the readings are: hash h1(k) = fmix32(k ^ seed_lo),
 * h2(k) = fmix32((k ^ seed_hi) + 0x9E3779B9) (MurmurHash3's finaliser,
 * Appleby, public domain); window index reduction by mask (power-of-two P)
 * or multiply-high (other P); quadratic probing by triangular numbers over a
 * power-of-two window count; double hashing with an odd step (power-of-two P)
 * or a step in [1, P-1] (prime P).
 */
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <unordered_map>
#include <unordered_set>
#include <vector>

namespace {

enum Kind { KIND_SINGLE = 0, KIND_MULTI = 1, KIND_COUNT = 2 };
enum Scheme { SCHEME_LINEAR = 0, SCHEME_QUADRATIC = 1, SCHEME_DOUBLE = 2 };
enum Status : uint8_t { ST_OK = 0, ST_DUPLICATE = 1, ST_FULL = 2, ST_INVALID_KEY = 3, ST_NOT_FOUND = 4 };

const uint32_t KEY_EMPTY = 0u;
const uint32_t KEY_TOMB = 0xFFFFFFFFu;

bool reserved(uint32_t k) { return k == KEY_EMPTY || k == KEY_TOMB; }

struct Table {
  int kind;
  uint64_t capacity;
  std::unordered_map<uint32_t, uint32_t> single;               // SV value, CT count
  std::unordered_map<uint32_t, std::vector<uint32_t>> multi;   // MV value lists
  uint64_t pairs = 0;                                          // MV live pairs
};

uint64_t live(const Table* t) { return t->kind == KIND_MULTI ? t->pairs : t->single.size(); }

}  // namespace

extern "C" {

void* orc_create(int kind, uint64_t capacity) {
  if (kind < 0 || kind > 2) return nullptr;
  Table* t = new Table();
  t->kind = kind;
  t->capacity = capacity;
  return t;
}

void orc_destroy(void* h) { delete static_cast<Table*>(h); }

void orc_clear(void* h) {
  Table* t = static_cast<Table*>(h);
  t->single.clear();
  t->multi.clear();
  t->pairs = 0;
}

uint64_t orc_size(void* h) { return live(static_cast<Table*>(h)); }

uint64_t orc_num_keys(void* h) {
  Table* t = static_cast<Table*>(h);
  return t->kind == KIND_MULTI ? t->multi.size() : t->single.size();
}

/* Insert a batch op by op.  values may be NULL for counting tables; status may be NULL. */
void orc_insert(void* h, const uint32_t* keys, const uint32_t* values, uint64_t n, uint8_t* status) {
  Table* t = static_cast<Table*>(h);
  for (uint64_t i = 0; i < n; ++i) {
    const uint32_t k = keys[i];
    uint8_t st;
    if (reserved(k)) {
      st = ST_INVALID_KEY;
    } else if (t->kind == KIND_SINGLE) {
      auto it = t->single.find(k);
      if (it != t->single.end()) { it->second = values[i]; st = ST_DUPLICATE; }
      else if (t->single.size() < t->capacity) { t->single.emplace(k, values[i]); st = ST_OK; }
      else st = ST_FULL;
    } else if (t->kind == KIND_COUNT) {
      auto it = t->single.find(k);
      if (it != t->single.end()) { it->second += 1u; st = ST_DUPLICATE; }
      else if (t->single.size() < t->capacity) { t->single.emplace(k, 1u); st = ST_OK; }
      else st = ST_FULL;
    } else {
      if (t->pairs < t->capacity) { t->multi[k].push_back(values[i]); t->pairs += 1; st = ST_OK; }
      else st = ST_FULL;
    }
    if (status) status[i] = st;
  }
}

/* Single-value: value / found.  Counting: count / found.  Multi-value: first is
 * not defined, so values_out gets the number of stored pairs (count) and found = count > 0. */
void orc_retrieve(void* h, const uint32_t* keys, uint64_t n, uint32_t* values_out, uint8_t* found_out) {
  Table* t = static_cast<Table*>(h);
  for (uint64_t i = 0; i < n; ++i) {
    const uint32_t k = keys[i];
    uint32_t v = 0;
    uint8_t f = 0;
    if (!reserved(k)) {
      if (t->kind == KIND_MULTI) {
        auto it = t->multi.find(k);
        if (it != t->multi.end()) { v = (uint32_t)it->second.size(); f = 1; }
      } else {
        auto it = t->single.find(k);
        if (it != t->single.end()) { v = it->second; f = 1; }
      }
    }
    if (values_out) values_out[i] = v;
    if (found_out) found_out[i] = f;
  }
}

void orc_erase(void* h, const uint32_t* keys, uint64_t n, uint8_t* status) {
  Table* t = static_cast<Table*>(h);
  for (uint64_t i = 0; i < n; ++i) {
    const uint32_t k = keys[i];
    uint8_t st;
    if (reserved(k)) {
      st = ST_INVALID_KEY;
    } else if (t->kind == KIND_MULTI) {
      auto it = t->multi.find(k);
      if (it != t->multi.end()) { t->pairs -= it->second.size(); t->multi.erase(it); st = ST_OK; }
      else st = ST_NOT_FOUND;
    } else {
      st = t->single.erase(k) ? ST_OK : ST_NOT_FOUND;
    }
    if (status) status[i] = st;
  }
}

/* Multi-value pass 1: counts[i] = number of pairs with key q_i; offsets = exclusive
 * prefix sum with n+1 entries (offsets[n] = total). counts may be NULL. */
void orc_count_values(void* h, const uint32_t* keys, uint64_t n, uint32_t* counts, uint64_t* offsets) {
  Table* t = static_cast<Table*>(h);
  uint64_t acc = 0;
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t c = 0;
    if (!reserved(keys[i])) {
      if (t->kind == KIND_MULTI) {
        auto it = t->multi.find(keys[i]);
        if (it != t->multi.end()) c = it->second.size();
      } else {
        c = t->single.count(keys[i]);
      }
    }
    if (counts) counts[i] = (uint32_t)c;
    if (offsets) offsets[i] = acc;
    acc += c;
  }
  if (offsets) offsets[n] = acc;
}

/* Multi-value pass 2: segment i = the values of q_i, in ascending order (the
 * order inside a segment is not specified by the method). */
void orc_retrieve_all(void* h, const uint32_t* keys, uint64_t n, const uint64_t* offsets, uint32_t* values_out) {
  Table* t = static_cast<Table*>(h);
  for (uint64_t i = 0; i < n; ++i) {
    if (reserved(keys[i])) continue;
    std::vector<uint32_t> seg;
    if (t->kind == KIND_MULTI) {
      auto it = t->multi.find(keys[i]);
      if (it != t->multi.end()) seg = it->second;
    } else {
      auto it = t->single.find(keys[i]);
      if (it != t->single.end()) seg.push_back(it->second);
    }
    std::sort(seg.begin(), seg.end());
    const uint64_t want = offsets[i + 1] - offsets[i];
    for (uint64_t j = 0; j < seg.size() && j < want; ++j) values_out[offsets[i] + j] = seg[j];
  }
}

/* Export the content: for SV/CT one (key, value) per live key, for MV every pair;
 * sorted by (key, value).  Returns the number of entries written (max_out bounds it). */
uint64_t orc_dump(void* h, uint32_t* keys_out, uint32_t* values_out, uint64_t max_out) {
  Table* t = static_cast<Table*>(h);
  std::vector<std::pair<uint32_t, uint32_t>> all;
  if (t->kind == KIND_MULTI) {
    for (auto& kv : t->multi) for (uint32_t v : kv.second) all.emplace_back(kv.first, v);
  } else {
    for (auto& kv : t->single) all.emplace_back(kv.first, kv.second);
  }
  std::sort(all.begin(), all.end());
  uint64_t m = std::min<uint64_t>(all.size(), max_out);
  for (uint64_t i = 0; i < m; ++i) { keys_out[i] = all[i].first; values_out[i] = all[i].second; }
  return m;
}

/* ------------------------------------------------------------------------- *
 * Probe geometry, re-derived from the paper's definitions (Sec. II probing
 * schemes; Sec. IV-B2 window = W consecutive slots scanned by the group).
 * ------------------------------------------------------------------------- */

uint32_t orc_fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

static bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }

static bool is_prime(uint64_t x) {
  if (x < 2) return false;
  for (uint64_t d = 2; d * d <= x; ++d) if (x % d == 0) return false;
  return true;
}

/* Window count actually used for a requested capacity: P = ceil(C / W), then
 * quadratic probing needs a power of two and double hashing a power of two or a prime. */
uint64_t orc_round_windows(uint64_t capacity, uint32_t window, int scheme) {
  uint64_t P = (capacity + window - 1) / window;
  if (P == 0) P = 1;
  if (scheme == SCHEME_QUADRATIC) {
    uint64_t q = 1;
    while (q < P) q <<= 1;
    P = q;
  } else if (scheme == SCHEME_DOUBLE && !is_pow2(P)) {
    while (!is_prime(P)) ++P;
  }
  return P;
}

static uint32_t reduce(uint32_t x, uint64_t P) {
  if (is_pow2(P)) return (uint32_t)(x & (P - 1));
  return (uint32_t)(((uint64_t)x * P) >> 32);
}

/* Window index of sequence step l for key k (written as the closed forms). */
uint64_t orc_window_at(uint32_t k, uint64_t l, uint64_t P, int scheme, uint64_t seed) {
  const uint32_t seed_lo = (uint32_t)seed, seed_hi = (uint32_t)(seed >> 32);
  const uint64_t w0 = reduce(orc_fmix32(k ^ seed_lo), P);
  if (scheme == SCHEME_LINEAR) return (w0 + l) % P;
  if (scheme == SCHEME_QUADRATIC) {
    /* T(l) = l (l + 1) / 2 taken mod P (P a power of two); 128-bit to avoid overflow */
    unsigned __int128 tri = (unsigned __int128)l * (l + 1) / 2;
    return (uint64_t)((w0 + tri) % P);
  }
  const uint32_t h2 = orc_fmix32((k ^ seed_hi) + 0x9E3779B9u);
  uint64_t step;
  if (is_pow2(P)) step = (h2 & (P - 1)) | 1u;
  else step = 1 + (((uint64_t)h2 * (P - 1)) >> 32);
  unsigned __int128 s = (unsigned __int128)l * step;
  return (uint64_t)((w0 + s) % P);
}

/* Fill out[0..count) with the window sequence of k. */
void orc_window_sequence(uint32_t k, uint64_t count, uint64_t P, int scheme, uint64_t seed, uint64_t* out) {
  for (uint64_t l = 0; l < count; ++l) out[l] = orc_window_at(k, l, P, scheme, seed);
}

/*
 * Layout check of a dumped slot array (P * W packed words: key in bits 0-31,
 * value in bits 32-63; empty word 0; tombstone word 0x00000000FFFFFFFF).
 * Returns 0 if every invariant holds, else an error code:
 *   1 bad empty/tombstone encoding, 2 a key stored past an empty position of its
 *   own sequence, 3 a key stored twice (single-value / counting),
 *   4 a key stored where its sequence never reaches (sequence does not cover).
 * stats[0] = live slots, stats[1] = tombstones, stats[2] = max windows to reach a
 * stored key, stats[3] = sum of windows over stored keys, stats[4] = index of the
 * first offending slot (or ~0).
 */
int orc_check_layout(const uint64_t* slots, uint64_t P, uint32_t W, int scheme, uint64_t seed, int kind,
                     uint64_t* stats) {
  // The offending slot reported is the lowest-indexed one; at one slot the
  // encoding is checked first, then uniqueness, then the position.
  uint64_t bad = ~0ull;
  int code = 0;
  auto note = [&](uint64_t i, int c) {
    if (i < bad || (i == bad && c < code)) { bad = i; code = c; }
  };
  uint64_t live_n = 0, tombs = 0, maxw = 0, sumw = 0;
  std::unordered_map<uint32_t, std::vector<uint64_t>> copies;  // slots of each stored key
  const uint64_t C = P * W;
  for (uint64_t i = 0; i < C; ++i) {
    const uint32_t k = (uint32_t)slots[i];
    const uint32_t v = (uint32_t)(slots[i] >> 32);
    if (k == KEY_EMPTY) { if (v != 0) note(i, 1); continue; }
    if (k == KEY_TOMB) { if (v != 0) note(i, 1); ++tombs; continue; }
    ++live_n;
    std::vector<uint64_t>& c = copies[k];
    if (kind != KIND_MULTI && !c.empty()) { note(i, 3); continue; }
    c.push_back(i);
  }
  // Each key's sequence is walked once, up to its last stored slot.  A stored
  // slot is out of place if an empty slot comes before it in the sequence
  // (windows in sequence order, slots in index order inside a window), or if
  // the sequence never reaches its window.
  for (auto& kv : copies) {
    const uint32_t k = kv.first;
    std::unordered_map<uint64_t, std::vector<uint64_t>> in_window;
    for (uint64_t i : kv.second) in_window[i / W].push_back(i);
    uint64_t remaining = kv.second.size();
    bool empty_before = false;  // an empty slot in an earlier window of the sequence
    for (uint64_t l = 0; l < P && remaining > 0; ++l) {
      const uint64_t w = orc_window_at(k, l, P, scheme, seed);
      auto it = in_window.find(w);
      if (it != in_window.end()) {
        for (uint64_t i : it->second) {
          bool behind_empty = empty_before;
          for (uint64_t j = w * W; j < i && !behind_empty; ++j) behind_empty = slots[j] == 0;
          if (behind_empty) note(i, 2);
          maxw = std::max<uint64_t>(maxw, l + 1);
          sumw += l + 1;
          --remaining;
        }
        in_window.erase(it);
      }
      for (uint64_t j = 0; j < W && !empty_before; ++j) empty_before = slots[w * W + j] == 0;
    }
    for (auto& rest : in_window)
      for (uint64_t i : rest.second) note(i, 4);
  }
  stats[0] = live_n;
  stats[1] = tombs;
  stats[2] = maxw;
  stats[3] = sumw;
  stats[4] = bad;
  return code;
}

/*
 * Sequential scalar model of cooperative probing: keys are inserted one at a
 * time at the first reusable (empty or tombstone) position of their sequence,
 * after the sequence up to the first window with an empty slot shows the key
 * absent.  Distinct keys only (a present key is skipped).  `windows` (optional)
 * receives the number of windows each insert visited.  Returns the number of
 * keys that found no slot.
 */
uint64_t orc_model_insert(uint64_t* slots, uint64_t P, uint32_t W, int scheme, uint64_t seed, const uint32_t* keys,
                          const uint32_t* values, uint64_t n, uint32_t* windows) {
  uint64_t failed = 0;
  for (uint64_t i = 0; i < n; ++i) {
    const uint32_t k = keys[i];
    int64_t cand = -1;
    uint64_t l = 0, visited = 0;
    bool present = false;
    for (; l < P; ++l) {
      const uint64_t w = orc_window_at(k, l, P, scheme, seed);
      ++visited;
      bool has_empty = false;
      for (uint32_t j = 0; j < W; ++j) {
        const uint64_t s = slots[w * W + j];
        const uint32_t sk = (uint32_t)s;
        if (sk == k) present = true;
        if (sk == KEY_EMPTY) has_empty = true;
        if ((sk == KEY_EMPTY || sk == KEY_TOMB) && cand < 0) cand = (int64_t)(w * W + j);
      }
      if (present || has_empty) break;
    }
    if (windows) windows[i] = (uint32_t)visited;
    if (present) continue;
    if (cand < 0) { ++failed; continue; }
    slots[cand] = (uint64_t)k | ((uint64_t)values[i] << 32);
  }
  return failed;
}

/* Windows a lookup of each key visits in the scalar model (to the match, or to the
 * first window holding an empty slot, or P). */
void orc_model_lookup_windows(const uint64_t* slots, uint64_t P, uint32_t W, int scheme, uint64_t seed,
                              const uint32_t* keys, uint64_t n, uint32_t* windows) {
  for (uint64_t i = 0; i < n; ++i) {
    const uint32_t k = keys[i];
    uint64_t visited = 0;
    for (uint64_t l = 0; l < P; ++l) {
      const uint64_t w = orc_window_at(k, l, P, scheme, seed);
      ++visited;
      bool stop = false;
      for (uint32_t j = 0; j < W; ++j) {
        const uint32_t sk = (uint32_t)slots[w * W + j];
        if (sk == k || sk == KEY_EMPTY) stop = true;
      }
      if (stop) break;
    }
    windows[i] = (uint32_t)visited;
  }
}

/* ------------------------------------------------------------------------- *
 * Single-value table with 64-bit keys and 64-bit values (the wider types the
 * paper's tables are generic over, Sec. IV-B1 packed and AoS layouts).  Same
 * semantics as the 32-bit single-value table; reserved keys 0 (empty) and
 * 2^64 - 1 (tombstone).
 * ------------------------------------------------------------------------- */

struct Table64 {
  uint64_t capacity;
  std::unordered_map<uint64_t, uint64_t> map;
};

static bool reserved64(uint64_t k) { return k == 0 || k == ~0ull; }

void* orc64_create(uint64_t capacity) {
  Table64* t = new Table64();
  t->capacity = capacity;
  return t;
}

void orc64_destroy(void* h) { delete static_cast<Table64*>(h); }

uint64_t orc64_size(void* h) { return static_cast<Table64*>(h)->map.size(); }

void orc64_insert(void* h, const uint64_t* keys, const uint64_t* values, uint64_t n, uint8_t* status) {
  Table64* t = static_cast<Table64*>(h);
  for (uint64_t i = 0; i < n; ++i) {
    const uint64_t k = keys[i];
    uint8_t st;
    if (reserved64(k)) {
      st = ST_INVALID_KEY;
    } else {
      auto it = t->map.find(k);
      if (it != t->map.end()) { it->second = values[i]; st = ST_DUPLICATE; }
      else if (t->map.size() < t->capacity) { t->map.emplace(k, values[i]); st = ST_OK; }
      else st = ST_FULL;
    }
    if (status) status[i] = st;
  }
}

void orc64_retrieve(void* h, const uint64_t* keys, uint64_t n, uint64_t* values_out, uint8_t* found_out) {
  Table64* t = static_cast<Table64*>(h);
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t v = 0;
    uint8_t f = 0;
    if (!reserved64(keys[i])) {
      auto it = t->map.find(keys[i]);
      if (it != t->map.end()) { v = it->second; f = 1; }
    }
    values_out[i] = v;
    found_out[i] = f;
  }
}

void orc64_erase(void* h, const uint64_t* keys, uint64_t n, uint8_t* status) {
  Table64* t = static_cast<Table64*>(h);
  for (uint64_t i = 0; i < n; ++i) {
    uint8_t st;
    if (reserved64(keys[i])) st = ST_INVALID_KEY;
    else st = t->map.erase(keys[i]) ? ST_OK : ST_NOT_FOUND;
    if (status) status[i] = st;
  }
}

/* MurmurHash3's 64-bit finaliser (Appleby, public domain). */
uint64_t orc_fmix64(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return x;
}

/* Window of sequence step l for a 64-bit key: h1 and h2 are the low and high
 * halves of fmix64(k ^ seed); otherwise as orc_window_at. */
uint64_t orc64_window_at(uint64_t k, uint64_t l, uint64_t P, int scheme, uint64_t seed) {
  const uint64_t x = orc_fmix64(k ^ seed);
  const uint64_t w0 = reduce((uint32_t)x, P);
  if (scheme == SCHEME_LINEAR) return (w0 + l) % P;
  if (scheme == SCHEME_QUADRATIC) {
    unsigned __int128 tri = (unsigned __int128)l * (l + 1) / 2;
    return (uint64_t)((w0 + tri) % P);
  }
  const uint32_t h2 = (uint32_t)(x >> 32);
  uint64_t step;
  if (is_pow2(P)) step = (h2 & (P - 1)) | 1u;
  else step = 1 + (((uint64_t)h2 * (P - 1)) >> 32);
  unsigned __int128 s = (unsigned __int128)l * step;
  return (uint64_t)((w0 + s) % P);
}

/* Layout check of a dumped 64-bit table: P * W slots of two words (key, value).
 * Codes as orc_check_layout: 1 bad encoding (empty or tombstone slot with a
 * nonzero value word), 2 a key behind an empty slot of its sequence, 3 a key
 * stored twice, 4 a key where its sequence never reaches.  stats as there. */
int orc64_check_layout(const uint64_t* slots, uint64_t P, uint32_t W, int scheme, uint64_t seed, uint64_t* stats) {
  uint64_t bad = ~0ull;
  int code = 0;
  auto note = [&](uint64_t i, int c) {
    if (i < bad || (i == bad && c < code)) { bad = i; code = c; }
  };
  uint64_t live_n = 0, tombs = 0, maxw = 0, sumw = 0;
  std::unordered_map<uint64_t, uint64_t> where;
  const uint64_t C = P * W;
  for (uint64_t i = 0; i < C; ++i) {
    const uint64_t k = slots[2 * i], v = slots[2 * i + 1];
    if (k == 0) { if (v != 0) note(i, 1); continue; }
    if (k == ~0ull) { if (v != 0) note(i, 1); ++tombs; continue; }
    ++live_n;
    if (!where.emplace(k, i).second) { note(i, 3); continue; }
  }
  for (auto& kv : where) {
    const uint64_t k = kv.first, i = kv.second, tw = i / W;
    bool reached = false, empty_before = false;
    for (uint64_t l = 0; l < P; ++l) {
      const uint64_t w = orc64_window_at(k, l, P, scheme, seed);
      const uint64_t jmax = (w == tw) ? i - w * W : W;
      for (uint64_t j = 0; j < jmax && !empty_before; ++j) empty_before = slots[2 * (w * W + j)] == 0;
      if (w == tw) {
        if (empty_before) note(i, 2);
        maxw = std::max<uint64_t>(maxw, l + 1);
        sumw += l + 1;
        reached = true;
        break;
      }
    }
    if (!reached) note(i, 4);
  }
  stats[0] = live_n;
  stats[1] = tombs;
  stats[2] = maxw;
  stats[3] = sumw;
  stats[4] = bad;
  return code;
}

/* ------------------------------------------------------------------------- *
 * Bloom filter (split-block; the rule is stated in the header comment).
 * bits: B * words uint32 words, block j at words [j * words, (j + 1) * words).
 * ------------------------------------------------------------------------- */

static uint64_t bloom_block(uint32_t key, uint64_t B, uint64_t seed) {
  return reduce(orc_fmix32(key ^ (uint32_t)seed), B);
}

static uint32_t bloom_bit(uint32_t key, uint32_t i, uint64_t seed) {
  const uint32_t h2 = orc_fmix32((key ^ (uint32_t)(seed >> 32)) + 0x9E3779B9u);
  return orc_fmix32(h2 + i * 0x9E3779B9u) >> 27;
}

void orc_bloom_insert(uint32_t* bits, uint64_t B, uint32_t words, uint64_t seed, const uint32_t* keys, uint64_t n) {
  for (uint64_t x = 0; x < n; ++x) {
    const uint64_t blk = bloom_block(keys[x], B, seed);
    for (uint32_t i = 0; i < words; ++i) bits[blk * words + i] |= 1u << bloom_bit(keys[x], i, seed);
  }
}

void orc_bloom_query(const uint32_t* bits, uint64_t B, uint32_t words, uint64_t seed, const uint32_t* keys,
                     uint64_t n, uint8_t* out) {
  for (uint64_t x = 0; x < n; ++x) {
    const uint64_t blk = bloom_block(keys[x], B, seed);
    bool all = true;
    for (uint32_t i = 0; i < words; ++i) all = all && ((bits[blk * words + i] >> bloom_bit(keys[x], i, seed)) & 1u);
    out[x] = all ? 1 : 0;
  }
}

/* Block index of each key (to sample the blocks of a large filter). */
void orc_bloom_blocks(const uint32_t* keys, uint64_t n, uint64_t B, uint64_t seed, uint64_t* out) {
  for (uint64_t x = 0; x < n; ++x) out[x] = bloom_block(keys[x], B, seed);
}

/* Block index and the bit of every word of one key (for the oracle's own tests). */
void orc_bloom_positions(uint32_t key, uint64_t B, uint32_t words, uint64_t seed, uint64_t* block, uint32_t* bit) {
  *block = bloom_block(key, B, seed);
  for (uint32_t i = 0; i < words; ++i) bit[i] = bloom_bit(key, i, seed);
}

}  // extern "C"
