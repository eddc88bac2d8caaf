// Single-value table with 64-bit keys and values (see hc_wide.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hc.h"
#include "hc_device.hpp"

namespace hc {

enum : int { WIDE_INSERT = 0, WIDE_RETRIEVE = 1, WIDE_ERASE = 2 };

// insert: keys, values -> flags (status, optional); retrieve: keys -> values_out, flags (found);
// erase: keys -> flags (status, optional).  G <= W.  soa: structure-of-arrays layout (C key
// words, then C value words), else 16-byte slots.
hc_err launch_wide(int op, bool soa, const TableView& t, uint32_t G, uint32_t W, const uint64_t* keys,
                   const uint64_t* values, uint64_t n, uint64_t* values_out, uint8_t* flags, hipStream_t s);

}  // namespace hc
