// Bandwidth diagnostics for the measurement: a streaming copy and a streaming
// read (the practical HBM peaks), a gather of random lines (the random-access
// ceiling that every probe of a table larger than the caches pays) and random
// atomics (the rate of claims and Bloom ORs).  Not part of the tables.
#include "hc_device.hpp"
#include "hc_launch.hpp"

namespace hc {

typedef uint32_t v4u __attribute__((ext_vector_type(4)));

// Streaming accesses that are not kept in the caches (nontemporal).
__device__ __forceinline__ uint4 stream_load(const uint4* p) {
  const v4u v = __builtin_nontemporal_load(reinterpret_cast<const v4u*>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void stream_store(uint4 a, uint4* p) {
  const v4u v = {a.x, a.y, a.z, a.w};
  __builtin_nontemporal_store(v, reinterpret_cast<v4u*>(p));
}

constexpr int COPY_UNROLL = 8;   // 16-byte vectors per thread in flight
constexpr int READ_UNROLL = 16;  // a block reads 256 * 16 consecutive vectors (64 KiB) per step

// Grid-stride copy, COPY_UNROLL nontemporal loads issued before their stores.
__global__ __launch_bounds__(BLOCK) void k_diag_copy(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                                     uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * BLOCK;
  uint64_t i = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
  for (; i + (COPY_UNROLL - 1) * stride < n; i += COPY_UNROLL * stride) {
    uint4 a[COPY_UNROLL];
#pragma unroll
    for (int u = 0; u < COPY_UNROLL; ++u) a[u] = stream_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < COPY_UNROLL; ++u) stream_store(a[u], dst + i + u * stride);
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

// XOR of all 16-byte vectors (read-only streaming); stored only if it hits a marker.  Each block
// takes whole 64 KiB chunks (blockIdx, then every gridDim-th), READ_UNROLL nontemporal loads per
// thread in flight.
__global__ __launch_bounds__(BLOCK) void k_diag_read(const uint4* __restrict__ src, uint64_t n,
                                                     uint32_t* __restrict__ sink) {
  constexpr uint64_t CHUNK = (uint64_t)BLOCK * READ_UNROLL;
  uint32_t acc = 0;
  for (uint64_t c = blockIdx.x; c * CHUNK < n; c += gridDim.x) {
    const uint64_t b = c * CHUNK + threadIdx.x;
    if (c * CHUNK + CHUNK <= n) {
      uint4 a[READ_UNROLL];
#pragma unroll
      for (int u = 0; u < READ_UNROLL; ++u) a[u] = stream_load(src + b + u * BLOCK);
#pragma unroll
      for (int u = 0; u < READ_UNROLL; ++u) acc ^= a[u].x ^ a[u].y ^ a[u].z ^ a[u].w;
    } else {
      for (int u = 0; u < READ_UNROLL; ++u)
        if (b + u * BLOCK < n) {
          const uint4 a = src[b + u * BLOCK];
          acc ^= a.x ^ a.y ^ a.z ^ a.w;
        }
    }
  }
  if (acc == 0x9E3779B9u) sink[0] = acc;
}

// LPL lanes read one line of 16 * LPL bytes; line i of the launch is
// fmix32-mixed from (seed, i) and reduced to [0, lines) by multiply-high.
template <int LPL>
__global__ __launch_bounds__(BLOCK) void k_diag_gather(const uint4* __restrict__ base, uint64_t lines, uint64_t n,
                                                       uint32_t seed, uint32_t* __restrict__ sink) {
  const uint32_t r = __lane_id() & (LPL - 1);
  const uint64_t groups = (uint64_t)gridDim.x * (BLOCK / LPL);
  uint32_t acc = 0;
  for (uint64_t i = ((uint64_t)blockIdx.x * BLOCK + threadIdx.x) / LPL; i < n; i += groups) {
    const uint32_t h = fmix32((uint32_t)i ^ fmix32(seed + (uint32_t)(i >> 32)));
    const uint64_t line = ((uint64_t)h * lines) >> 32;
    const uint4 q = base[line * LPL + r];
    acc ^= q.x ^ q.y ^ q.z ^ q.w;
  }
  if (acc == 0x9E3779B9u) sink[0] = acc;  // keeps the loads; practically never stores
}

// One atomic per lane on a pseudo-random 8-byte word of [base, base + words):
// an OR without return (as a Bloom insert) or a CAS with return (as a table
// claim).  The words are random, so nearly every atomic hits its own line.
template <bool CAS>
__global__ __launch_bounds__(BLOCK) void k_diag_atomic(unsigned long long* __restrict__ base, uint64_t words,
                                                       uint64_t n, uint32_t seed, uint32_t* __restrict__ sink) {
  const uint64_t stride = (uint64_t)gridDim.x * BLOCK;
  uint32_t acc = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride) {
    const uint32_t h = fmix32((uint32_t)i ^ fmix32(seed + (uint32_t)(i >> 32)));
    unsigned long long* p = base + (((uint64_t)h * words) >> 32);
    if constexpr (CAS) {
      acc ^= (uint32_t)atomicCAS(p, 0ull, (unsigned long long)(i | 1));
    } else {
      atomicOr(p, 1ull << (h & 63));
    }
  }
  if (acc == 0x9E3779B9u) sink[0] = acc;
}

}  // namespace hc

using namespace hc;

extern "C" {

hc_err hc_diag_copy(void* d_dst, const void* d_src, uint64_t bytes, void* stream) {
  if (d_dst == nullptr || d_src == nullptr) return fail(HC_E_ARG, "dst or src is NULL");
  if (bytes % 16 != 0) return fail(HC_E_ARG, "bytes %llu is not a multiple of 16", (unsigned long long)bytes);
  const uint64_t n = bytes / 16;
  if (n == 0) return HC_OK;
  // 32 blocks per CU: the fastest of 4-32 measured for a 1 GiB copy
  const uint64_t want = (n + BLOCK - 1) / BLOCK, cap = (uint64_t)device_cu_count() * 32;
  const unsigned grid = (unsigned)(want < cap ? want : cap);
  hipLaunchKernelGGL(k_diag_copy, dim3(grid), dim3(BLOCK), 0, (hipStream_t)stream, static_cast<uint4*>(d_dst),
                     static_cast<const uint4*>(d_src), n);
  return check_launch("diagnostic copy");
}

hc_err hc_diag_read(const void* d_src, uint64_t bytes, uint32_t* d_sink, void* stream) {
  if (d_src == nullptr || d_sink == nullptr) return fail(HC_E_ARG, "src or sink is NULL");
  if (bytes % 16 != 0) return fail(HC_E_ARG, "bytes %llu is not a multiple of 16", (unsigned long long)bytes);
  const uint64_t n = bytes / 16;
  if (n == 0) return HC_OK;
  // 8 blocks per CU: the fastest of 4-32 measured for a 1 GiB read
  const uint64_t chunks = (n + (uint64_t)BLOCK * READ_UNROLL - 1) / ((uint64_t)BLOCK * READ_UNROLL);
  const uint64_t cap = (uint64_t)device_cu_count() * 8;
  const unsigned grid = (unsigned)(chunks < cap ? chunks : cap);
  hipLaunchKernelGGL(k_diag_read, dim3(grid), dim3(BLOCK), 0, (hipStream_t)stream, static_cast<const uint4*>(d_src), n,
                     d_sink);
  return check_launch("diagnostic read");
}

hc_err hc_diag_atomic(void* d_base, uint64_t bytes, uint32_t cas, uint64_t n_ops, uint32_t seed, uint32_t* d_sink,
                      void* stream) {
  if (d_base == nullptr || d_sink == nullptr) return fail(HC_E_ARG, "base or sink is NULL");
  if ((reinterpret_cast<uintptr_t>(d_base) & 7) != 0) return fail(HC_E_ARG, "base is not 8-byte aligned");
  const uint64_t words = bytes / 8;
  if (words == 0 || words > (1ull << 32)) return fail(HC_E_ARG, "region holds %llu words", (unsigned long long)words);
  if (n_ops == 0) return HC_OK;
  auto* base = static_cast<unsigned long long*>(d_base);
  if (cas) {
    hipLaunchKernelGGL(k_diag_atomic<true>, dim3(grid_for(k_diag_atomic<true>, n_ops, 1)), dim3(BLOCK), 0,
                       (hipStream_t)stream, base, words, n_ops, seed, d_sink);
  } else {
    hipLaunchKernelGGL(k_diag_atomic<false>, dim3(grid_for(k_diag_atomic<false>, n_ops, 1)), dim3(BLOCK), 0,
                       (hipStream_t)stream, base, words, n_ops, seed, d_sink);
  }
  return check_launch("diagnostic atomics");
}

hc_err hc_diag_gather(const void* d_base, uint64_t bytes, uint32_t line_bytes, uint64_t n_lines, uint32_t seed,
                      uint32_t* d_sink, void* stream) {
  if (d_base == nullptr || d_sink == nullptr) return fail(HC_E_ARG, "base or sink is NULL");
  if (line_bytes != 32 && line_bytes != 64 && line_bytes != 128)
    return fail(HC_E_ARG, "line bytes %u is not 32, 64 or 128", line_bytes);
  const uint64_t lines = bytes / line_bytes;
  if (lines == 0 || lines > (1ull << 32)) return fail(HC_E_ARG, "region holds %llu lines", (unsigned long long)lines);
  if ((reinterpret_cast<uintptr_t>(d_base) & (line_bytes - 1)) != 0) return fail(HC_E_ARG, "base is not line aligned");
  if (n_lines == 0) return HC_OK;
  const uint4* base = static_cast<const uint4*>(d_base);
  hipStream_t s = (hipStream_t)stream;
  switch (line_bytes) {
    case 32:
      hipLaunchKernelGGL(k_diag_gather<2>, dim3(grid_for(k_diag_gather<2>, n_lines, 2)), dim3(BLOCK), 0, s, base, lines,
                         n_lines, seed, d_sink);
      break;
    case 64:
      hipLaunchKernelGGL(k_diag_gather<4>, dim3(grid_for(k_diag_gather<4>, n_lines, 4)), dim3(BLOCK), 0, s, base, lines,
                         n_lines, seed, d_sink);
      break;
    default:
      hipLaunchKernelGGL(k_diag_gather<8>, dim3(grid_for(k_diag_gather<8>, n_lines, 8)), dim3(BLOCK), 0, s, base, lines,
                         n_lines, seed, d_sink);
  }
  return check_launch("diagnostic gather");
}

}  // extern "C"
