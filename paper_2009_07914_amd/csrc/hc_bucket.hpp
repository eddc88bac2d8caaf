// Bucket list hash table (Sec. IV-C): keys in a cooperative-probing table whose
// slot value is the key's number of values; the values in a list of buckets
// taken from one preallocated pool (see hc_bucket.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hc.h"
#include "hc_device.hpp"

namespace hc {

constexpr int KIND_BUCKET = 3;
constexpr uint32_t BL_MAX_RAMP = 4096;  // bucket sizes listed before the cap is reached, at most

// Device view of the bucket lists of one table.
struct BucketView {
  const uint64_t* cum;             // cum[i] = S(i), values held by buckets 0..i-1, for i = 0..m
  uint32_t m;                      // buckets before sizes reach smax (bucket m onward holds smax values)
  uint32_t smax;
  uint32_t* pool;                  // bucket pool, 32-bit words
  uint64_t pool_cap;               // words
  uint64_t s0;                     // size of bucket 0: slot p's bucket 0 is the words [p * s0, (p + 1) * s0)
  uint64_t bump;                   // C * s0: later buckets are allocated from here on
  unsigned long long* pool_next;   // words allocated after `bump`
  // per key slot, one 16-byte record, written by the allocation pass of a batch that gives the
  // key more than bucket 0 can hold, read by placement and the list walks (one line each):
  //   x = buckets the key holds (low 32; 0 after hc_clear or an erase: none recorded)
  //       | buckets it held before that batch (high 32)
  //   y = pool offset of the key's last bucket (low 32; meaningful once the key has more than
  //       one bucket) | first bucket that batch allocated (high 32: BL_NONE if none, BL_CUT if
  //       the pool ran out)
  ulonglong2* meta;
};

constexpr uint32_t BL_NONE = 0xFFFFFFFFu;
constexpr uint32_t BL_CUT = 0xFFFFFFFEu;  // never a bucket offset: a bucket takes >= 2 words below 2^32

// Bucket sizes s_0 = s0, s_i = min(ceil(growth * s_{i-1}), smax): the ramp up to
// the cap, as cumulative sums (host side).  Returns false if the ramp is longer
// than BL_MAX_RAMP buckets.
bool bucket_ramp(uint32_t s0, double growth, uint32_t smax, uint64_t* cum, uint32_t* m);

// Phase 1..3 of a bulk insert of n pairs (keys, values) into a bucket list table.
// Workspace: bl_insert_workspace(n) bytes.  status optional.
uint64_t bl_insert_workspace(uint64_t n);
hc_err launch_bl_insert(const TableView& t, const BucketView& b, uint32_t G, uint32_t W, const uint32_t* keys,
                        const uint32_t* values, uint64_t n, uint8_t* status, void* ws, hipStream_t s);
// The phases separately (grouped insert): tickets of n elements (n_dev non-NULL: *n_dev
// elements, n an upper bound) with incr[i] values each (NULL: 1); values non-NULL (per-pair
// inserts, incr NULL): a pair that claims a new key stores its value in bucket 0 at once;
// tickets of the pairs of a sorted batch from those of its runs; allocation and placement.
hc_err launch_bl_tickets(const TableView& t, const BucketView& b, uint32_t G, uint32_t W, const uint32_t* keys,
                         const uint32_t* incr, const uint32_t* values, uint64_t n, const uint64_t* n_dev,
                         uint64_t* pos, uint32_t* ticket, uint8_t* st, hipStream_t s);
hc_err launch_bl_expand(const uint64_t* scan, const uint64_t* starts, uint64_t n, const uint64_t* rpos,
                        const uint32_t* rticket, const uint8_t* rst, uint64_t* pos, uint32_t* ticket, uint8_t* st,
                        hipStream_t s);
hc_err launch_bl_finish(const TableView& t, const BucketView& b, const uint32_t* values, uint64_t n,
                        const uint64_t* pos, const uint32_t* ticket, const uint8_t* st, uint8_t* status,
                        hipStream_t s);
// Counts of keys (into offsets[i], and counts[i] when given), before the scan.
hc_err launch_bl_count(const TableView& t, uint32_t G, uint32_t W, const uint32_t* keys, uint64_t n, uint32_t* counts,
                       uint64_t* offsets, hipStream_t s);
// Values of keys into out[offsets[i] .. offsets[i+1]); lists longer than BL_LONG_LIST
// values are copied by whole blocks.  Workspace: bl_write_workspace(n) bytes.
constexpr uint64_t BL_LONG_LIST = 1024;
// Phase states beside ST_OK (a candidate for allocating its key's new buckets): BL_PLACED, the
// value is already stored (the pair claimed its key's slot and bucket 0); BL_FOLLOW, the pair
// only places its value (a pair of a sorted run other than the run's last); BL_ALLOC, the pair
// held its key's last ticket and allocated (it also fixes the count if the pool ran out).
constexpr uint8_t BL_PLACED = 0x80;
constexpr uint8_t BL_FOLLOW = 0x81;
constexpr uint8_t BL_ALLOC = 0x82;
uint64_t bl_write_workspace(uint64_t n);
hc_err launch_bl_write(const TableView& t, const BucketView& b, uint32_t G, uint32_t W, const uint32_t* keys,
                       uint64_t n, const uint64_t* offsets, uint32_t* out, void* ws, hipStream_t s);
hc_err launch_bl_erase(const TableView& t, const BucketView& b, uint32_t G, uint32_t W, const uint32_t* keys,
                       uint64_t n, uint8_t* status, hipStream_t s);
// Every slot's record says "no buckets" (a fill kernel).
hc_err launch_bl_reset(const BucketView& b, uint64_t C, hipStream_t s);
// Last-bucket offset of every slot (the low words of the records) into dst[0..C).
hc_err launch_bl_dump_last(const BucketView& b, uint64_t C, uint32_t* dst, hipStream_t s);

}  // namespace hc
