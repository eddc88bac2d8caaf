/*
 * hc.h -- C ABI of the MI355X (gfx950) cooperative-probing hash tables.
 *
 * The operations follow WarpCore (Juenger et al., arXiv 2009.07914):
 *   - open-addressing tables whose slots hold a key/value pair bit-packed into
 *     one 64-bit word, so a single 64-bit compare-and-swap stores both
 *     (Sec. IV-B1, packed AoS layout);
 *   - the Cooperative Probing Scheme: a group of g lanes loads one window of
 *     W consecutive slots, votes on it, and the lowest candidate slot is
 *     claimed with CAS; the start of each window comes from an outer probing
 *     scheme (Sec. IV-B2; linear, quadratic or double hashing of Sec. II);
 *   - host-callable bulk operations over device arrays, one group per input
 *     element (Sec. IV-B3), results written to caller-allocated device
 *     arrays (Sec. IV-B4), a two-pass count / prefix-sum / write retrieval of
 *     all values of a multi-value table (Sec. IV-B4), deletion by tombstone
 *     (Sec. IV-B5), asynchronous on a stream except where a value is returned
 *     to the host (Sec. IV-D).
 *
 * Conventions for every call:
 *   - Pointers named d_* are device memory owned by the caller; the library
 *     never frees them.  h_* pointers are host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls are ordered on that stream and return before the work completes,
 *     except calls with an h_* output, which synchronise the stream.
 *   - n == 0 is a no-op returning HC_OK.  A NULL required pointer, a bad
 *     group size or window gives HC_E_ARG and launches nothing.
 *   - `group` is the group size g (1, 2, 4, 8, 16, 32 or 64 lanes of a
 *     64-lane wavefront); 0 selects the table's default.  Results do not
 *     depend on g (Sec. IV-B2: a fixed window walked by any group size).
 *   - Keys 0 (empty indicator) and 0xFFFFFFFF (tombstone) are reserved;
 *     values are unrestricted.
 *   - Element outcomes go to the optional d_status array (uint8, one per
 *     input): HC_S_*.  A duplicate key is a warning, not an error.
 *   - Concurrency (Sec. IV-D): calls of the same kind, and reads, may
 *     overlap on one table (e.g. on several streams); a write call must not
 *     overlap a call of another kind on the same table.  Two calls are exempt
 *     and ordered by the library instead: hc_insert_grouped, and hc_insert on
 *     a bucket list table, run one after another per table on the device (each
 *     waits for the table's previous such call through an event, without
 *     blocking the host).  A handle is used by one host thread at a time.
 *   - Scratch memory: calls that need device workspace (multi-value and
 *     bucket list passes, grouped inserts, hc_stats) take it per call from a
 *     library-owned pool of the current device, ordered on the call's stream
 *     (hipMallocFromPoolAsync / hipFreeAsync): concurrent calls never share
 *     it and no call synchronises the device for it.  Freed blocks stay in
 *     the pool for later calls.  HC_E_NOMEM if the pool cannot grow.
 *   - Work counters: every stream that launches on a device gets its own
 *     pair of the library's work counters (the first 1024 streams per device;
 *     beyond that pairs are shared round-robin), so any number of calls may be
 *     in flight on different streams.  A graph captured from library calls uses
 *     its capturing stream's counters: replay it on that stream, not beside
 *     other work of that stream or beside another replay of itself (batch plans
 *     own their counters instead, see hc_batch_capture).
 *   - Errors: every call returns hc_err; hc_last_error() gives a message for
 *     the calling thread's last failure.  No C++ exception crosses the ABI.
 *     A device fault inside a kernel is not recoverable by the library.
 */
#ifndef HC_H
#define HC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hc_table_s* hc_table;

/* Table kinds (Sec. IV: SingleValueHashTable, MultiValueHashTable, CountingHashTable,
 * BucketListHashTable, made by hc_create_bucket_list; single-value tables of 64-bit keys and
 * values in the array-of-structures and structure-of-arrays layouts of Sec. IV-B1; HashSet). */
enum {
  HC_SINGLE_VALUE = 0,
  HC_MULTI_VALUE = 1,
  HC_COUNTING = 2,
  HC_BUCKET_LIST = 3,
  HC_SINGLE_VALUE_64 = 4,
  HC_HASH_SET = 5,
  HC_SINGLE_VALUE_64_SOA = 6
};

/* Outer probing schemes over windows (Sec. II):
 *   linear     w_l = (h + l) mod P
 *   quadratic  w_l = (h + l(l+1)/2) mod P, P a power of two (visits every window)
 *   double     w_l = (h + l s) mod P, s odd (P a power of two) or s in [1,P-1] (P prime) */
enum { HC_LINEAR = 0, HC_QUADRATIC = 1, HC_DOUBLE = 2 };

typedef enum {
  HC_OK = 0,
  HC_E_ARG = 1,     /* invalid argument */
  HC_E_NOMEM = 2,   /* device allocation failed */
  HC_E_KIND = 3,    /* operation not defined for this table kind */
  HC_E_DEVICE = 4   /* HIP runtime error */
} hc_err;

/* Per-element status codes written to d_status. */
enum {
  HC_S_OK = 0,          /* inserted a new key / erased */
  HC_S_DUPLICATE = 1,   /* key already present: value replaced (single-value) or count incremented */
  HC_S_FULL = 2,        /* no reusable slot in the whole probe sequence (Sec. II abort criterion) */
  HC_S_INVALID_KEY = 3, /* key is 0 or 0xFFFFFFFF; nothing done */
  HC_S_NOT_FOUND = 4    /* erase of an absent key */
};

typedef struct {
  uint32_t scheme;   /* HC_LINEAR / HC_QUADRATIC / HC_DOUBLE */
  uint32_t window;   /* W, slots per window: 8, 16, 32 or 64 (16 = one 128-byte line) */
  uint32_t group;    /* default group size g */
  uint32_t reserved; /* must be 0 */
  uint64_t seed;     /* hash seed: h(k) uses the low 32 bits, the double-hashing step the high 32 bits */
} hc_params;

typedef struct {
  uint32_t kind;
  uint32_t scheme;
  uint32_t window;       /* W */
  uint32_t group;        /* default g */
  uint64_t windows;      /* P: number of windows */
  uint64_t capacity;     /* C = P * W slots */
  uint64_t seed;
  uint64_t* d_slots;     /* the slot array: C uint64 words (key bits 0-31, value bits 32-63); 64-bit
                            tables 2C words (pairs, or C keys then C values); sets C uint32 keys */
} hc_table_info;

/* Fill *params with the defaults: double hashing, W = 16, g = 4, a fixed seed. */
void hc_default_params(hc_params* params);

/* Create a table of `kind` holding at least `capacity` slots on the current device.
 * The window count is P = ceil(capacity / W), rounded up to a power of two for
 * quadratic probing and to a prime for double hashing when P is not a power of two
 * (the cycle-free rule of Sec. IV-B2); hc_info reports the actual C = P * W.
 * The table starts empty.  params may be NULL (defaults).  Slots are allocated with
 * hipMalloc and owned by the table.  Errors: HC_E_ARG (bad kind/params, capacity 0,
 * P > 2^31), HC_E_NOMEM. */
hc_err hc_create(hc_table* out, uint32_t kind, uint64_t capacity, const hc_params* params);

/* Bytes of slot memory a table of this capacity and these params needs (8 * C after the
 * rounding of hc_create), for hc_create_in.  params may be NULL (defaults). */
hc_err hc_table_bytes(uint64_t capacity, const hc_params* params, uint64_t* h_out);

/* As hc_create, but the slot array is caller-owned device memory on the current device
 * (e.g. a torch tensor): d_slots must be 256-byte aligned and hold slot_bytes >= hc_table_bytes
 * bytes; it is cleared here (the call synchronises) and never freed by the library.  The caller
 * keeps it alive until hc_destroy.  Errors as hc_create, plus HC_E_ARG for a NULL, misaligned or
 * too small array. */
hc_err hc_create_in(hc_table* out, uint32_t kind, void* d_slots, uint64_t slot_bytes, uint64_t capacity,
                    const hc_params* params);

/* ---- single-value tables with 64-bit keys and values (Sec. IV-B1 wider types) ------
 * Kind HC_SINGLE_VALUE_64 (hc_create): slots of 16 bytes (key word, then value word), so a
 * window of W = 8 slots is one 128-byte line; group sizes g <= W.  Keys 0 and 2^64-1 are
 * reserved.  A claim is a 64-bit CAS of the key word followed by a relaxed atomic store of the
 * value word; a present key's value is replaced by such a store (status DUPLICATE).  Results,
 * statuses and errors as hc_insert / hc_retrieve / hc_erase with uint64 keys and values.
 * hc_size, hc_load_factor, hc_capacity, hc_info, hc_clear, hc_destroy apply; hc_dump_slots
 * copies 2*C uint64 words; hc_create_in needs 16 bytes per slot (hc_table_bytes counts 8).
 * The 32-bit entry points, hc_stats, hc_device_view, batches and the server return HC_E_KIND.
 *
 * Kind HC_SINGLE_VALUE_64_SOA: the same table in the structure-of-arrays layout: C key words,
 * then C value words, in one allocation of 16 * C bytes (hc_dump_slots copies the C keys, then
 * the C values).  Probing reads only key words (W = 16 keys: one 128-byte line) and a hit reads
 * one value word; the value is written after the key's CAS with a relaxed atomic store.  A
 * reader in the same launch as an insert may see the key before its value (the torn read of a
 * key-only CAS); a later launch sees whole pairs.  Same entry points, statuses and errors. */
hc_err hc_insert64(hc_table table, const uint64_t* d_keys, const uint64_t* d_values, uint64_t n, uint8_t* d_status,
                   uint32_t group, void* stream);
hc_err hc_retrieve64(hc_table table, const uint64_t* d_keys, uint64_t n, uint64_t* d_values_out,
                     uint8_t* d_found_out, uint32_t group, void* stream);
hc_err hc_erase64(hc_table table, const uint64_t* d_keys, uint64_t n, uint8_t* d_status, uint32_t group,
                  void* stream);

/* ---- HashSet (Sec. IV: a set of keys, each stored once) -----------------------------
 * Kind HC_HASH_SET (hc_create): slots of 4 bytes holding only the key, so a window of
 * W = 16 slots is one 64-byte line; group sizes g <= W.  Keys 0 and 0xFFFFFFFF are reserved.
 * The window sequence and hash are those of the 32-bit tables, so a key lands in the window a
 * single-value table of the same geometry would give it.  Entry points:
 *   hc_insert(set, keys, NULL, n, status, ...)      status OK (new key), DUPLICATE, FULL,
 *                                                   INVALID_KEY; d_values must be NULL
 *   hc_retrieve(set, keys, n, NULL, found, ...)     found[i] = 1 if keys[i] is in the set;
 *                                                   d_values_out must be NULL, d_found_out not
 *   hc_erase(set, keys, n, status, ...)             as for single-value tables
 * hc_size, hc_load_factor, hc_capacity, hc_info, hc_clear, hc_destroy apply; hc_dump_slots
 * copies C uint32 keys (C * 4 bytes); hc_create_in needs 4 bytes per slot.  hc_count_values,
 * hc_retrieve_all, hc_insert_grouped, hc_stats, hc_device_view, the 64-bit entry points,
 * batches and the server return HC_E_KIND. */

/* ---- Bloom filter (Sec. IV: answers set membership queries) ------------------------
 * The paper lists a BloomFilter without a design; this one is a split-block filter: the bit
 * array is B blocks of block_words 32-bit words (8, 16 or 32: 32, 64 or 128 bytes), and key x
 * sets one bit in every word of block reduce(h1(x), B): bit fmix32(h2(x) + i * 0x9E3779B9) >> 27
 * of word i, so k = block_words bits per key.  h1, h2 and reduce are the tables' (fmix32 of the
 * key with the seed's low / high half; mask for a power-of-two B, multiply-high otherwise).
 * Every 32-bit key is valid.  No false negatives; the false-positive rate with n keys is
 * sum_j Binomial(j; n, 1/B) (1 - (31/32)^j)^block_words.  A group of g lanes (power of two,
 * g <= block_words) takes one key; group is a tuning knob and never changes results.  Group 0
 * in a call means the filter's default; a default of 0 means one lane per word for inserts (the
 * block's atomic ORs leave as one request) and one lane per key for queries. */
typedef struct hc_bloom_s* hc_bloom;

typedef struct {
  uint32_t block_words; /* 8, 16 or 32 (bits per key) */
  uint32_t group;       /* default group size g; 0: per operation (insert: block_words, query: 1) */
  uint64_t seed;
} hc_bloom_params;

typedef struct {
  uint64_t blocks;      /* B */
  uint32_t block_words;
  uint32_t group;
  uint64_t seed;
  uint32_t* d_bits;     /* B * block_words uint32 words, block j at words [j * block_words, ...) */
} hc_bloom_info_t;

/* Defaults: 16 words (one 64-byte block, 16 bits per key), group 0 (per operation), a fixed seed. */
void hc_default_bloom_params(hc_bloom_params* params);
/* A cleared filter of at least `bits` bits (B = ceil(bits / (32 * block_words)) blocks,
 * B <= 2^32) on the current device; params may be NULL (defaults).  The call synchronises.
 * Errors: HC_E_ARG (bits 0, bad params), HC_E_NOMEM. */
hc_err hc_bloom_create(hc_bloom* out, uint64_t bits, const hc_bloom_params* params);
hc_err hc_bloom_destroy(hc_bloom filter);
/* Clear every bit (a fill kernel on the stream). */
hc_err hc_bloom_clear(hc_bloom filter, void* stream);
/* Add n keys (device array).  group 0 = the filter's default.  Concurrent inserts and
 * inserts racing with queries are allowed; a query sees a key inserted by an earlier launch. */
hc_err hc_bloom_insert(hc_bloom filter, const uint32_t* d_keys, uint64_t n, uint32_t group, void* stream);
/* d_found_out[i] = 1 if every bit of keys[i] is set, else 0. */
hc_err hc_bloom_contains(hc_bloom filter, const uint32_t* d_keys, uint64_t n, uint8_t* d_found_out, uint32_t group,
                         void* stream);
hc_err hc_bloom_info(hc_bloom filter, hc_bloom_info_t* h_out);
/* Copy the B * block_words words of the bit array into d_dst (device), on the stream. */
hc_err hc_bloom_dump(hc_bloom filter, uint32_t* d_dst, void* stream);

/* ---- bandwidth diagnostics (measurement support; not part of any table) -----------------
 * hc_diag_copy: copy `bytes` (a multiple of 16) from d_src to d_dst with 16-byte vector loads
 * and stores; hc_diag_read: read them (XOR-reduced into registers): the practical streaming
 * peaks.  hc_diag_gather: read n_lines lines of line_bytes
 * (32, 64 or 128) at pseudo-random line indices of the region [d_base, d_base + bytes) (d_base
 * aligned to line_bytes, at most 2^32 lines): the random-access ceiling a probe of a large table
 * pays.  hc_diag_atomic: n_ops atomics on pseudo-random 8-byte words of the region (8-byte aligned,
 * at most 2^32 words), one per lane: cas = 0 an OR without return (the region's bits change), cas
 * != 0 a CAS of 0 with return (zero words change): the rate of Bloom inserts and table claims.
 * d_sink is one device word the kernel may write.  All are asynchronous on the stream.
 * Errors: HC_E_ARG for NULL pointers, sizes or alignment as stated. */
hc_err hc_diag_copy(void* d_dst, const void* d_src, uint64_t bytes, void* stream);
hc_err hc_diag_read(const void* d_src, uint64_t bytes, uint32_t* d_sink, void* stream);
hc_err hc_diag_atomic(void* d_base, uint64_t bytes, uint32_t cas, uint64_t n_ops, uint32_t seed, uint32_t* d_sink,
                      void* stream);
hc_err hc_diag_gather(const void* d_base, uint64_t bytes, uint32_t line_bytes, uint64_t n_lines, uint32_t seed,
                      uint32_t* d_sink, void* stream);

/* ---- bucket list tables (Sec. IV-C) ------------------------------------------------
 * A multi-value table that stores each distinct key once: the key's slot in a
 * cooperative-probing table holds its number of values, and the values live in a list of
 * buckets in one preallocated pool.  Bucket i holds s_i values: s_0 = s0,
 * s_i = min(ceil(growth * s_{i-1}), smax) (the paper's growth rule, capped); every bucket
 * but the first begins with the pool offset of the bucket before it.  The first bucket of the
 * key in slot p is the s0 pool words at p * s0 (the first C * s0 pool words are reserved for
 * them); later buckets are allocated from the rest.  A key's values sit in its list in
 * insertion-ticket order.  Pool memory of erased keys' later buckets is not reused before
 * hc_clear (a first bucket is reused with its slot).
 *   hc_insert: pairs as for a multi-value table (status OK, FULL when the key table or the
 *              pool is full, INVALID_KEY); values are required.
 *   hc_retrieve: d_values_out = the key's number of values, found = key present.
 *   hc_count_values / hc_retrieve_all: as for multi-value tables (values in list order).
 *   hc_erase: removes the key and all its values.  hc_size: values stored.
 *   hc_insert_grouped: the same lists, one atomic per distinct key of the batch.
 * Not supported: batched launches and the server (HC_E_KIND). */
typedef struct {
  uint64_t pool_values;  /* pool size in 32-bit words (values and links), >= s0 * C; 0: (s0 + 3) * C */
  uint32_t s0;           /* first bucket size, >= 1 */
  uint32_t smax;         /* largest bucket size, s0 <= smax <= 2^24 */
  double growth;         /* growth factor lambda in [1, 64]; with 1 every bucket holds s0 (needs s0 = smax) */
} hc_bucket_params;

void hc_default_bucket_params(hc_bucket_params* params); /* pool 0 (s0 + 3 per slot), s0 1, smax 65536, growth 2 */

/* Create a bucket list table for at least key_capacity distinct keys (rounded as hc_create).
 * params / bparams may be NULL (defaults).  Errors: HC_E_ARG (bad parameters, a pool smaller
 * than s0 words per key slot or larger than 2^32 - 1 words, or a size ramp from s0 to smax
 * longer than 4096 buckets), HC_E_NOMEM. */
hc_err hc_create_bucket_list(hc_table* out, uint64_t key_capacity, const hc_params* params,
                             const hc_bucket_params* bparams);

typedef struct {
  uint64_t values;      /* values stored (hc_size) */
  uint64_t pool_used;   /* pool words in use: the C * s0 words of the first buckets, then the words
                           allocated (values, links and the unused tail of last buckets) */
  uint64_t pool_words;  /* pool size */
  uint32_t smax;
  uint32_t reserved;
} hc_bucket_usage_t;

/* Pool usage of a bucket list table (synchronises the stream); storage density follows from it. */
hc_err hc_bucket_usage(hc_table table, hc_bucket_usage_t* h_out, void* stream);

/* Copy the pool (pool_words uint32) and the per-slot last-bucket offsets (C uint32) to caller
 * device memory, on the stream (for inspection).  The last-bucket offset of slot p is meaningful
 * only for a key with more than one bucket; a key with one bucket has it at p * s0. */
hc_err hc_dump_buckets(hc_table table, uint32_t* d_pool_dst, uint32_t* d_last_dst, void* stream);

/* Release the table and its device memory (synchronises the device). */
hc_err hc_destroy(hc_table table);

/* Empty the table: every slot becomes the empty word, size becomes 0 (a fill kernel). */
hc_err hc_clear(hc_table table, void* stream);

/* Bulk insert of n elements (Sec. IV-B3), one group per element.
 *   single-value: insert (k, v); a present key keeps its slot and takes v (status DUPLICATE).
 *                 Within one call, which value of a repeated key survives is unspecified.
 *   multi-value:  store (k, v) as one more pair, even if identical pairs exist.
 *   counting:     d_values must be NULL; count(k) += 1 (mod 2^32), a new key starts at 1.
 * d_keys, d_values: n uint32 each.  d_status: optional, n uint8. */
hc_err hc_insert(hc_table table, const uint32_t* d_keys, const uint32_t* d_values, uint64_t n,
                 uint8_t* d_status, uint32_t group, void* stream);

/* Bulk retrieval (Sec. IV-B4): d_values_out[i] = value (single-value), count (counting)
 * or number of stored pairs (multi-value) of d_keys[i]; d_found_out[i] = 1 if present.
 * Absent and reserved keys give 0 / 0.  Either output may be NULL. */
hc_err hc_retrieve(hc_table table, const uint32_t* d_keys, uint64_t n, uint32_t* d_values_out,
                   uint8_t* d_found_out, uint32_t group, void* stream);

/* Bulk deletion by tombstone (Sec. IV-B5).  Single-value / counting: remove the key
 * (OK, or NOT_FOUND if absent).  Multi-value: remove every pair of the key; with the
 * same key repeated in one call the number of removed pairs is exact but which of
 * the repeats report OK is unspecified.  d_status optional. */
hc_err hc_erase(hc_table table, const uint32_t* d_keys, uint64_t n, uint8_t* d_status, uint32_t group,
                void* stream);

/* Multi-value pass 1 (Sec. IV-B4): d_offsets (n+1 uint64) receives the exclusive prefix sum
 * of the per-query value counts, d_offsets[n] = total; d_counts (optional, n uint32) the
 * counts themselves; *h_total (optional) the total, which synchronises the stream.
 * A query still open after 64 windows is handed to rounds in which blocks of 1024 threads scan
 * segments of its window sequence in parallel (keys with very many values); the hand-over list
 * holds n/16 + 1024 queries, past which groups walk on by themselves.  Workspace (per call,
 * from the pool): 8 bytes per 2048 queries for the scan plus 32 bytes per hand-over entry.
 * Multi-value and bucket list tables (HC_E_KIND otherwise). */
hc_err hc_count_values(hc_table table, const uint32_t* d_keys, uint64_t n, uint32_t* d_counts,
                       uint64_t* d_offsets, uint64_t* h_total, uint32_t group, void* stream);

/* hc_count_values for callers that cannot allocate device memory (code being captured into a
 * HIP graph, serving loops and harnesses that forbid allocation): the same arguments, results
 * and errors, but the scratch memory (scan tile sums, long-query list) is a fixed 16 MiB array
 * of the library on each GPU, held until the process ends, and the call allocates nothing.
 * Limits: n <= 2^28 (HC_E_ARG beyond); the long-query list holds min(n/16 + 1024, about
 * 490,000) entries, past which groups walk on by themselves (results are the same).  Every
 * call on one GPU shares that GPU's array: calls that overlap on one GPU (other streams, other
 * host threads) race and must be serialised by the caller.  The first call on a device looks
 * the array's address up once (no allocation). */
hc_err hc_count_values_noalloc(hc_table table, const uint32_t* d_keys, uint64_t n, uint32_t* d_counts,
                               uint64_t* d_offsets, uint64_t* h_total, uint32_t group, void* stream);

/* Multi-value pass 2 (Sec. IV-B4): writes the values of d_keys[i] to
 * d_values_out[d_offsets[i] .. d_offsets[i+1]); the order inside a segment is unspecified.
 * d_offsets must come from hc_count_values on the same keys with no write call in between;
 * writes never leave a segment.  Long queries as in hc_count_values (40 bytes of workspace per
 * hand-over entry).  Multi-value and bucket list tables. */
hc_err hc_retrieve_all(hc_table table, const uint32_t* d_keys, uint64_t n, const uint64_t* d_offsets,
                       uint32_t* d_values_out, uint32_t group, void* stream);

/* Insert of n keys grouped by key, for batches in which some keys repeat very often (not in the
 * paper).  The batch is sorted by key in a per-call workspace (about 48 bytes per element, from the
 * pool) and handled run by run:
 *  - multi-value tables: the paper's per-pair insert, hc_insert, makes the i-th copy of a key scan past
 *    the i-1 earlier ones, so a key with m copies costs about m^2/(2W) window visits (Sec. V-B); here
 *    each key's run claims its slots in one pass along its window sequence (long runs spread over the
 *    whole device).  The stored multiset, the layout invariant and every later result equal those of
 *    hc_insert.  d_values: n values, pair i = (d_keys[i], d_values[i]).
 *  - counting tables: each distinct key is inserted once, its count raised by its number of
 *    occurrences (one atomic per distinct key instead of one per occurrence).  d_values must be NULL.
 *  - bucket list tables: each run of one key takes its tickets with one atomic, then buckets are
 *    allocated and values placed as in hc_insert (same lists; values of a run in batch order).
 * Keys 0 and 0xFFFFFFFF are skipped; elements that find no reusable slot are dropped (hc_size tells
 * how many pairs / distinct keys are stored).  No per-element status.  n < 2^32.  Single-value
 * tables: HC_E_KIND.  Workspace: about 48 bytes per element (74 for bucket lists). */
hc_err hc_insert_grouped(hc_table table, const uint32_t* d_keys, const uint32_t* d_values, uint64_t n, void* stream);

/* Live entries (single-value / counting: keys; multi-value: pairs).  Synchronises the stream. */
hc_err hc_size(hc_table table, uint64_t* h_out, void* stream);

/* size / capacity (Sec. II load factor; tombstones are not counted).  Synchronises the stream. */
hc_err hc_load_factor(hc_table table, double* h_out, void* stream);

/* Actual capacity C (after rounding). */
hc_err hc_capacity(hc_table table, uint64_t* h_out);

/* Table geometry and the device address of its slot array. */
hc_err hc_info(hc_table table, hc_table_info* h_out);

/* Full scan of the slot array (a diagnostic, not on the hot path).  The probe length of a
 * live slot is the number of windows a retrieval of its key visits up to and including the
 * slot's window: its index l in the key's window sequence (Sec. II), plus one.  It grows with
 * the load factor (Sec. IV-B); live counts the same entries as hc_size.  cas_fails is not from
 * the scan: it counts, since hc_create or the last hc_clear, the claim CASes of per-element
 * inserts (hc_insert, batched launches and the device-side insert) that found their slot
 * changed by another insert -- the collisions Sec. IV-B2 names as the cost of concurrent
 * insertion.  Each such failure is followed by a retry at the next candidate or an update. */
#define HC_PROBE_BUCKETS 16
typedef struct {
  uint64_t live;        /* slots holding a key */
  uint64_t tombstones;  /* erased slots (Sec. IV-B5) */
  uint64_t empty;
  uint64_t max_probe;   /* largest probe length over live slots (<= P) */
  uint64_t probe_sum;   /* sum of probe lengths over live slots */
  uint64_t probe_hist[HC_PROBE_BUCKETS];  /* live slots with probe length in [2^b, 2^(b+1)); last bucket open */
  uint64_t cas_fails;   /* failed claim CASes of inserts since create / clear */
} hc_table_stats;
/* Synchronises the stream.  Errors: HC_E_ARG (NULL output), HC_E_NOMEM. */
hc_err hc_stats(hc_table table, hc_table_stats* h_out, void* stream);

/* The table's device view for user kernels (the device-side API in
 * paper_2009_07914_amd/csrc/hc_device_api.hpp: hc::dev::insert / retrieve / erase / for_all,
 * called by groups of G lanes from any kernel).  h_view receives a hc::TableView (defined in
 * hc_device.hpp) by value; bytes must be its size.  The view stays valid until hc_destroy. */
hc_err hc_device_view(hc_table table, void* h_view, uint64_t bytes);

/* Copy the slot array into caller memory d_dst (device), on the stream: C uint64 words (2C for
 * 64-bit tables, C/2 for sets, whose C 4-byte keys fill them). */
hc_err hc_dump_slots(hc_table table, uint64_t* d_dst, void* stream);

/* ---- batched launches over many tables ------------------------------------------
 * Not in the paper (its bulk calls take one table each, Sec. IV-B3); built from the
 * same per-element operations and the concurrency rules of Sec. IV-D.
 *
 * A batch is an ordered list of operations on single-value or counting tables.
 * Operations on one table run in list order, except that consecutive operations of
 * the same kind on a table run concurrently (Sec. IV-D: same-kind overlap is valid);
 * operations on different tables are independent.  The list is split into phases
 * (a table's next phase starts where its operation kind changes); each phase is one
 * persistent kernel per distinct (kind, group size, window) in it, on one stream,
 * in which wavefronts take chunks of any table's elements from a shared counter.
 * Results are exactly those of the same calls made one by one in list order, except
 * where concurrent same-kind writes of one phase touch the same key (then, as for one
 * call with a repeated key, which write wins is unspecified). */

enum { HC_OP_INSERT = 0, HC_OP_RETRIEVE = 1, HC_OP_ERASE = 2 };

typedef struct {
  hc_table table;            /* single-value or counting table (HC_E_KIND otherwise) */
  uint32_t op;               /* HC_OP_* */
  uint32_t group;            /* group size g; 0 = the table's default */
  const uint32_t* d_keys;    /* n keys */
  const uint32_t* d_values;  /* insert into a single-value table: n values; NULL otherwise */
  uint32_t* d_values_out;    /* retrieve: n values (or counts); optional */
  uint8_t* d_flags;          /* optional: n status codes (insert, erase) or found flags (retrieve) */
  uint64_t n;
} hc_batch_op;

typedef struct hc_batch_s* hc_batch;

/* Build a launch plan for `count` operations: validates them (HC_E_ARG / HC_E_KIND,
 * nothing allocated on error), assigns phases and uploads the device descriptors
 * (allocates device memory; synchronous).  The plan keeps the pointers it was given:
 * the caller keeps those buffers alive and unchanged in size while it is launched.
 * All tables must live on the current device. */
hc_err hc_batch_create(hc_batch* out, const hc_batch_op* ops, uint32_t count);

/* Flags of hc_batch_create_flags. */
enum { HC_BATCH_ONE_LAUNCH = 1 };
/* Longest wait of a one-launch plan for a table's previous phase, in milliseconds. */
#define HC_BATCH_WAIT_MS 20000

/* hc_batch_create with flags (0: the same plan).  HC_BATCH_ONE_LAUNCH runs every phase in
 * ONE persistent launch instead of one launch per phase: wavefronts take the chunks of all
 * phases from one counter in phase order, and a chunk of a table's later phase first waits,
 * on the device, until every chunk of that table's previous phase has finished (a completion
 * counter per table and phase, written after a device-scope release and read before a
 * device-scope acquire).  Tables that finish early are queried while others are still being
 * built; results are those of the phased plan.  Every operation of such a plan must use the
 * same group size and window (HC_E_ARG otherwise).  Waiting cannot deadlock (the chunks waited
 * for were taken earlier by running wavefronts, which never wait for later chunks); a wait
 * still ends after HC_BATCH_WAIT_MS, and is then counted as abandoned (the results of that
 * launch are not valid) -- a phase of one table that runs longer than that must use the
 * phased plan.  Launch, capture and replay rules are those of hc_batch_create. */
hc_err hc_batch_create_flags(hc_batch* out, const hc_batch_op* ops, uint32_t count, uint32_t flags);

/* Number of waits of a one-launch plan abandoned so far, over all its launches (0 for
 * other plans); synchronises the device first. */
hc_err hc_batch_abandoned_waits(hc_batch batch, uint64_t* h_count);

/* Enqueue every phase of the plan on `stream` (asynchronous; no allocation and no
 * memset, so it may be captured into a graph).  Each launch of the plan uses work
 * counters that belong to the plan (allocated by hc_batch_create and reset by the
 * launch itself), never the counters other calls take, so launches of other plans and
 * other calls may run beside it on other streams; two launches of one plan (or of its
 * captured graph) must not run concurrently. */
hc_err hc_batch_launch(hc_batch batch, void* stream);

/* Number of phases and of kernel launches per hc_batch_launch. */
hc_err hc_batch_info(hc_batch batch, uint32_t* h_phases, uint32_t* h_launches);

/* Release the plan's device memory (synchronises the device). */
hc_err hc_batch_destroy(hc_batch batch);

/* create + launch + synchronise the stream + destroy. */
hc_err hc_batch_run(const hc_batch_op* ops, uint32_t count, void* stream);

/* Capture hc_batch_launch(batch) into an instantiated hipGraphExec (returned as
 * void*); replay it with hc_graph_launch.  The graph uses the plan's own work counters:
 * replays of it must not overlap each other or a hc_batch_launch of the same plan, and
 * the plan must outlive the graph. */
hc_err hc_batch_capture(hc_batch batch, void** h_graph_exec);
hc_err hc_graph_launch(void* graph_exec, void* stream);
hc_err hc_graph_destroy(void* graph_exec);

/* ---- serving loop -----------------------------------------------------------------
 * Not in the paper (built from the bulk calls and the concurrency rules of Sec. IV-D).
 * A server owns a worker thread that admits requests (host-side key/value buffers on
 * resident single-value or counting tables) in arrival order while its device staging
 * ring (the admission budget) has room, coalesces everything admitted at once into one
 * batched launch group (whose phases keep every table's operations in arrival order),
 * overlaps the input/output copies of a group with the kernels of its neighbours on
 * rotating streams, and makes a group's kernels wait on the device for the unfinished
 * earlier groups that share one of its tables (groups on disjoint tables run side by
 * side, and may complete out of arrival order).  Every request's results equal those of
 * running the requests one by one in arrival order, except where requests admitted into
 * one group write the same key of one table with the same kind of operation: those
 * writes run in one launch (one epoch), and the results are those of one of their
 * orders.  For single-value inserts of key k with values v1..vm in one epoch: the value
 * left is one of v1..vm; if k was absent before, exactly one of those inserts reports OK
 * and the others DUPLICATE, else all report DUPLICATE.  Counting inserts: counts are
 * exact (addition commutes), statuses as above.  Erases: if k was present, exactly one
 * reports OK and the others NOT_FOUND.  A retrieve that follows in arrival order sees the
 * value left by the epoch.
 * Host buffers should be pinned (hipHostMalloc) for asynchronous copies; they must
 * stay valid until the request completes. */

typedef struct hc_server_s* hc_server;

typedef struct {
  uint64_t staging_bytes;       /* device staging ring = admission budget (>= 1 MiB); at most half
                                   the HBM free at creation (a larger request is cut to that) */
  uint64_t max_group_ops;       /* most elements coalesced into one launch group (a larger request
                                   forms a group alone); 0 = no limit */
  uint32_t max_group_requests;  /* most requests per launch group; 0 = 1024 */
  uint32_t streams;             /* streams rotated over launch groups; 0 = 3 */
  uint32_t serial;              /* 1: one request at a time, each waiting for the previous one */
  uint32_t reserved;
} hc_server_params;

typedef struct {
  hc_table table;
  uint32_t op;                  /* HC_OP_* */
  uint32_t group;               /* group size; 0 = the table's default */
  const uint32_t* h_keys;       /* n keys */
  const uint32_t* h_values;     /* insert into a single-value table: n values; NULL otherwise */
  uint32_t* h_values_out;       /* retrieve: n values (counts); optional */
  uint8_t* h_flags;             /* optional: status (insert, erase) or found (retrieve) */
  uint64_t n;
} hc_request;

typedef struct {
  uint64_t submitted, completed, launch_groups, ops_completed, staging_in_use;
  uint64_t staging_bytes;       /* the admission budget in use (staging ring size) */
} hc_server_counts;

/* Defaults: 1 GiB staging, 2^22 elements and 1024 requests per group, 3 streams. */
void hc_default_server_params(hc_server_params* params);

/* Create a server on the current device (allocates its staging ring, streams and a
 * worker thread).  params may be NULL. */
hc_err hc_server_create(hc_server* out, const hc_server_params* params);

/* Queue a request; returns at once with a ticket.  HC_E_ARG / HC_E_KIND for invalid
 * requests, HC_E_ARG if the request can never fit the staging ring. */
hc_err hc_server_submit(hc_server server, const hc_request* req, uint64_t* h_ticket);

/* Non-blocking status of a ticket; latency = completion - submission (microseconds),
 * -1 while pending. */
hc_err hc_server_query(hc_server server, uint64_t ticket, int* h_done, double* h_latency_us);

/* Block until the ticket completes / until every submitted request completes. */
hc_err hc_server_wait(hc_server server, uint64_t ticket);
hc_err hc_server_drain(hc_server server);

hc_err hc_server_stats(hc_server server, hc_server_counts* h_out);

/* Finish the queued work, stop the worker and release everything. */
hc_err hc_server_destroy(hc_server server);

/* Static text for an error code, and the calling thread's last error message. */
const char* hc_error_string(hc_err err);
const char* hc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HC_H */
