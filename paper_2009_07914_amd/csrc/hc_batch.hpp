// Device descriptor of one operation of a batched launch.
#pragma once

#include "hc.h"
#include "hc_device.hpp"

namespace hc {

// Operation kinds of batched launches (BATCH_COUNT: insert into a counting table).
enum : uint32_t { BATCH_INSERT = 0, BATCH_RETRIEVE = 1, BATCH_ERASE = 2, BATCH_COUNT = 3 };

struct BatchDesc {
  TableView t;
  const uint32_t* keys;
  const uint32_t* values;   // insert into a single-value table
  uint32_t* values_out;     // retrieve (optional)
  uint8_t* flags;           // status (insert / erase) or found (retrieve); optional
  uint64_t n;
  uint32_t chunk;           // elements per chunk
  uint32_t op;              // BATCH_*
};

// One persistent launch over descs[0..ndesc) (device arrays, all of operation
// kind `op`, group size G and window W) on `stream`.
hc_err launch_batch(uint32_t op, uint32_t G, uint32_t W, const BatchDesc* d_descs, const uint64_t* d_chunk_start,
                    uint32_t ndesc, uint64_t total_chunks, hipStream_t stream);

}  // namespace hc
