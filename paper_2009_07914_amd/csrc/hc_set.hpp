// HashSet of 32-bit keys (see hc_set.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hc.h"
#include "hc_device.hpp"

namespace hc {

enum : int { SET_INSERT = 0, SET_CONTAINS = 1, SET_ERASE = 2 };

// insert: keys -> flags (status, optional); contains: keys -> flags (found, required);
// erase: keys -> flags (status, optional).  t.slots holds P * W 32-bit keys; G <= W.
hc_err launch_set(int op, const TableView& t, uint32_t G, uint32_t W, const uint32_t* keys, uint64_t n,
                  uint8_t* flags, hipStream_t s);

}  // namespace hc
