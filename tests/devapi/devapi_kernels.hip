// User kernels built on the device-side API (test support): a fused k-mer
// counter (DNA read -> 2-bit k-mer codes -> counting-table inserts in one
// kernel, the producer-kernel fusion the device API exists for), a fused k-mer
// index (the same codes inserted with their read positions into a multi-value
// table from one kernel, the shape of the paper's Sec. V-C database build), group
// lookups, group inserts with statuses, a per-key for_each collection of values
// and a for_all export of every stored pair.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hc_device_api.hpp"

namespace {

constexpr int G = 4;
constexpr int BLK = 256;

// Base codes A,C,G,T = 0..3 (input bytes are already 0..3).  The k-mer starting at
// position i is sum_j seq[i+j] * 4^(k-1-j); key = code + 1 (never 0, < 2^31 for k <= 15).
template <int W>
__global__ __launch_bounds__(BLK) void k_count_kmers(hc::TableView t, const uint8_t* __restrict__ seq,
                                                     uint64_t positions, uint32_t k) {
  const uint64_t groups = (uint64_t)gridDim.x * (BLK / G);
  for (uint64_t i = (uint64_t)blockIdx.x * (BLK / G) + threadIdx.x / G; i < positions; i += groups) {
    uint32_t code = 0;
    for (uint32_t j = 0; j < k; ++j) code = (code << 2) | seq[i + j];
    hc::dev::insert<G, W, hc::KIND_COUNT>(t, code + 1u);  // groups of a wavefront may diverge here
  }
}

// (k-mer code + 1, position) pairs into a multi-value table.
template <int W>
__global__ __launch_bounds__(BLK) void k_index_kmers(hc::TableView t, const uint8_t* __restrict__ seq,
                                                     uint64_t positions, uint32_t k, uint8_t* __restrict__ status) {
  const uint64_t groups = (uint64_t)gridDim.x * (BLK / G);
  for (uint64_t i = (uint64_t)blockIdx.x * (BLK / G) + threadIdx.x / G; i < positions; i += groups) {
    uint32_t code = 0;
    for (uint32_t j = 0; j < k; ++j) code = (code << 2) | seq[i + j];
    const uint8_t st = hc::dev::insert<G, W, hc::KIND_MULTI>(t, code + 1u, (uint32_t)i);
    if (threadIdx.x % G == 0) status[i] = st;
  }
}

// Every value of keys[i] written to out[offsets[i] + j] by for_each (at most
// offsets[i+1] - offsets[i] of them); counts[i] = the number for_each reports.
template <int W>
__global__ __launch_bounds__(BLK) void k_collect(hc::TableView t, const uint32_t* __restrict__ keys, uint64_t n,
                                                 const uint64_t* __restrict__ offsets, uint32_t* __restrict__ out,
                                                 uint32_t* __restrict__ counts) {
  const uint64_t groups = (uint64_t)gridDim.x * (BLK / G);
  for (uint64_t i = (uint64_t)blockIdx.x * (BLK / G) + threadIdx.x / G; i < n; i += groups) {
    const uint64_t base = offsets[i], room = offsets[i + 1] - offsets[i];
    const uint32_t c = hc::dev::for_each<G, W>(t, keys[i], [&](uint32_t v, uint32_t j) {
      if (j < room) out[base + j] = v;
    });
    if (threadIdx.x % G == 0) counts[i] = c;
  }
}

template <int W>
__global__ __launch_bounds__(BLK) void k_lookup(hc::TableView t, const uint32_t* __restrict__ keys, uint64_t n,
                                                uint32_t* __restrict__ vals, uint8_t* __restrict__ found) {
  const uint64_t groups = (uint64_t)gridDim.x * (BLK / G);
  for (uint64_t i = (uint64_t)blockIdx.x * (BLK / G) + threadIdx.x / G; i < n; i += groups) {
    uint32_t v = 0;
    const bool f = hc::dev::retrieve<G, W>(t, keys[i], v);
    if (threadIdx.x % G == 0) {
      vals[i] = v;
      found[i] = f;
    }
  }
}

template <int W>
__global__ __launch_bounds__(BLK) void k_insert(hc::TableView t, const uint32_t* __restrict__ keys,
                                                const uint32_t* __restrict__ values, uint64_t n,
                                                uint8_t* __restrict__ status) {
  const uint64_t groups = (uint64_t)gridDim.x * (BLK / G);
  for (uint64_t i = (uint64_t)blockIdx.x * (BLK / G) + threadIdx.x / G; i < n; i += groups) {
    const uint8_t st = hc::dev::insert<G, W, hc::KIND_SINGLE>(t, keys[i], values[i]);
    if (threadIdx.x % G == 0) status[i] = st;
  }
}

struct Export {
  uint32_t* keys;
  uint32_t* vals;
  unsigned long long* n;
  __device__ void operator()(uint32_t k, uint32_t v) const {
    const unsigned long long e = atomicAdd(n, 1ull);
    keys[e] = k;
    vals[e] = v;
  }
};

unsigned grid_of(uint64_t items) {
  const uint64_t g = (items + (BLK / G) - 1) / (BLK / G);
  return (unsigned)(g < 2048 ? (g ? g : 1) : 2048);
}

}  // namespace

extern "C" {

// view: the bytes hc_device_view() filled; window: the table's W (16 only here).
int devapi_count_kmers(const void* view, uint32_t window, const uint8_t* d_seq, uint64_t len, uint32_t k,
                       void* stream) {
  if (window != 16 || k == 0 || k > 15 || len < k) return 1;
  const hc::TableView t = *static_cast<const hc::TableView*>(view);
  const uint64_t positions = len - k + 1;
  hipLaunchKernelGGL(k_count_kmers<16>, dim3(grid_of(positions)), dim3(BLK), 0, (hipStream_t)stream, t, d_seq,
                     positions, k);
  return hipGetLastError() == hipSuccess ? 0 : 2;
}

int devapi_index_kmers(const void* view, uint32_t window, const uint8_t* d_seq, uint64_t len, uint32_t k,
                       uint8_t* d_status, void* stream) {
  if (window != 16 || k == 0 || k > 15 || len < k) return 1;
  const hc::TableView t = *static_cast<const hc::TableView*>(view);
  const uint64_t positions = len - k + 1;
  hipLaunchKernelGGL(k_index_kmers<16>, dim3(grid_of(positions)), dim3(BLK), 0, (hipStream_t)stream, t, d_seq,
                     positions, k, d_status);
  return hipGetLastError() == hipSuccess ? 0 : 2;
}

int devapi_collect(const void* view, uint32_t window, const uint32_t* d_keys, uint64_t n, const uint64_t* d_offsets,
                   uint32_t* d_out, uint32_t* d_counts, void* stream) {
  if (window != 16) return 1;
  const hc::TableView t = *static_cast<const hc::TableView*>(view);
  hipLaunchKernelGGL(k_collect<16>, dim3(grid_of(n)), dim3(BLK), 0, (hipStream_t)stream, t, d_keys, n, d_offsets,
                     d_out, d_counts);
  return hipGetLastError() == hipSuccess ? 0 : 2;
}

int devapi_lookup(const void* view, uint32_t window, const uint32_t* d_keys, uint64_t n, uint32_t* d_vals,
                  uint8_t* d_found, void* stream) {
  if (window != 16) return 1;
  const hc::TableView t = *static_cast<const hc::TableView*>(view);
  hipLaunchKernelGGL(k_lookup<16>, dim3(grid_of(n)), dim3(BLK), 0, (hipStream_t)stream, t, d_keys, n, d_vals, d_found);
  return hipGetLastError() == hipSuccess ? 0 : 2;
}

int devapi_insert(const void* view, uint32_t window, const uint32_t* d_keys, const uint32_t* d_vals, uint64_t n,
                  uint8_t* d_status, void* stream) {
  if (window != 16) return 1;
  const hc::TableView t = *static_cast<const hc::TableView*>(view);
  hipLaunchKernelGGL(k_insert<16>, dim3(grid_of(n)), dim3(BLK), 0, (hipStream_t)stream, t, d_keys, d_vals, n,
                     d_status);
  return hipGetLastError() == hipSuccess ? 0 : 2;
}

// d_keys / d_vals: capacity entries each; *d_n (zeroed by the caller) receives the count.
int devapi_export(const void* view, uint32_t window, uint32_t* d_keys, uint32_t* d_vals, unsigned long long* d_n,
                  void* stream) {
  const hc::TableView t = *static_cast<const hc::TableView*>(view);
  hipLaunchKernelGGL(hc::dev::for_all<Export>, dim3(1024), dim3(256), 0, (hipStream_t)stream, t, window,
                     Export{d_keys, d_vals, d_n});
  return hipGetLastError() == hipSuccess ? 0 : 2;
}

uint64_t devapi_view_bytes(void) { return sizeof(hc::TableView); }

}  // extern "C"
