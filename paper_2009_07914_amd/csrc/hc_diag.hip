// Bandwidth diagnostics for the measurement: a streaming copy and a streaming
// read (the practical HBM peaks), a gather of random lines (the random-access
// ceiling that every probe of a table larger than the caches pays) and random
// atomics (the rate of claims and Bloom ORs).  Not part of the tables.
#include "hc_device.hpp"
#include "hc_launch.hpp"

namespace hc {

// Four 16-byte vectors per thread per step, all loads issued before the stores.
__global__ __launch_bounds__(BLOCK) void k_diag_copy(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                                     uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * BLOCK;
  uint64_t i = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = d;
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

// XOR of all 16-byte vectors (read-only streaming); stored only if it hits a marker.
__global__ __launch_bounds__(BLOCK) void k_diag_read(const uint4* __restrict__ src, uint64_t n,
                                                     uint32_t* __restrict__ sink) {
  const uint64_t stride = (uint64_t)gridDim.x * BLOCK;
  uint32_t acc = 0;
  uint64_t i = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    acc ^= (a.x ^ a.y ^ a.z ^ a.w) ^ (b.x ^ b.y ^ b.z ^ b.w) ^ (c.x ^ c.y ^ c.z ^ c.w) ^ (d.x ^ d.y ^ d.z ^ d.w);
  }
  for (; i < n; i += stride) {
    const uint4 a = src[i];
    acc ^= a.x ^ a.y ^ a.z ^ a.w;
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
  const unsigned grid = grid_for(k_diag_copy, n, 1);
  hipLaunchKernelGGL(k_diag_copy, dim3(grid), dim3(BLOCK), 0, (hipStream_t)stream, static_cast<uint4*>(d_dst),
                     static_cast<const uint4*>(d_src), n);
  return check_launch("diagnostic copy");
}

hc_err hc_diag_read(const void* d_src, uint64_t bytes, uint32_t* d_sink, void* stream) {
  if (d_src == nullptr || d_sink == nullptr) return fail(HC_E_ARG, "src or sink is NULL");
  if (bytes % 16 != 0) return fail(HC_E_ARG, "bytes %llu is not a multiple of 16", (unsigned long long)bytes);
  const uint64_t n = bytes / 16;
  if (n == 0) return HC_OK;
  const unsigned grid = grid_for(k_diag_read, n, 1);
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
