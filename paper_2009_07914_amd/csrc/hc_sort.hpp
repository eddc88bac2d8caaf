// Device-wide primitives used by the grouped multi-value path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hc.h"

namespace hc {

// In-place exclusive scan of a[0..n) (uint64), writing a[n] = total.  `tiles` is
// a workspace of scan_tiles_needed(n) entries.
uint64_t scan_tiles_needed(uint64_t n);
hc_err exclusive_scan_inplace(uint64_t* a, uint64_t n, uint64_t* tiles, hipStream_t stream);

// Stable sort of (keys, vals) by key, in place (keys_tmp / vals_tmp: n entries
// each; hist: sort_pairs_workspace(n) entries; scan_tiles: scan_tiles_needed of
// the histogram size).  vals and vals_tmp both NULL: keys only.
uint64_t sort_pairs_workspace(uint64_t n);
hc_err sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp, uint32_t* vals_tmp, uint64_t n,
                  uint64_t* hist, uint64_t* scan_tiles, hipStream_t stream);

}  // namespace hc
