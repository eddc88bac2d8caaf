// Full-scan statistics of a table (see hc_stats.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "hc.h"
#include "hc_device.hpp"

namespace hc {

constexpr int STATS_BUCKETS = 16;  // must match HC_PROBE_BUCKETS

// d_out: 5 + STATS_BUCKETS zeroed words (live, tombstones, empty, max probe, probe sum, histogram).
hc_err launch_stats(const TableView& t, uint32_t W, unsigned long long* d_out, hipStream_t s);

}  // namespace hc
