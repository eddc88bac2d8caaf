// Grouped multi-value insert and long-query continuation (see hc_group.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hc.h"
#include "hc_device.hpp"

namespace hc {

constexpr uint64_t HEAVY_RUN = 2048;   // runs at least this long are claimed by a whole block
constexpr uint32_t LONG_BUDGET = 64;   // windows a group scans before handing a query over

uint64_t grouped_workspace_bytes(uint64_t n);
hc_err launch_grouped_insert(const TableView& t, uint32_t W, const uint32_t* keys, const uint32_t* values, uint64_t n,
                             void* ws, hipStream_t s);
hc_err launch_zero_u64(unsigned long long* p, uint32_t count, hipStream_t s);
hc_err launch_long_count(const TableView& t, uint32_t W, const uint32_t* keys, const uint64_t* list,
                         const unsigned long long* nlong, uint64_t max_long, uint32_t budget, uint64_t* offsets,
                         uint32_t* counts, hipStream_t s);
hc_err launch_long_write(const TableView& t, uint32_t W, const uint32_t* keys, const uint64_t* list,
                         const unsigned long long* nlong, uint64_t max_long, uint32_t budget, const uint64_t* offsets,
                         uint32_t* out, hipStream_t s);

}  // namespace hc
