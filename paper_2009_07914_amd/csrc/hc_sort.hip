// Stable LSD radix sort of (key, value) pairs by 32-bit key: four passes of one
// 8-bit digit.  Each pass: per-tile digit histograms, an exclusive scan of the
// digit-major histogram table (global offsets of every (digit, tile)), then a
// scatter in which each tile ranks its elements stably (lanes with equal digits
// found with eight wavefront ballots, per-wavefront digit counts in LDS ordering
// the wavefronts and rounds), sorts them by digit in LDS and writes each digit's
// run with contiguous stores.  Used to group equal keys before a grouped
// multi-value insert.
#include "hc_launch.hpp"
#include "hc_sort.hpp"

namespace hc {

constexpr int RS_THREADS = 256;
constexpr int RS_ROUNDS = 16;                       // elements per thread per tile
constexpr uint64_t RS_TILE = (uint64_t)RS_THREADS * RS_ROUNDS;
constexpr int RS_WAVES = RS_THREADS / 64;

__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint32_t* __restrict__ keys, uint64_t n, int shift,
                                                        uint64_t* __restrict__ hist, uint64_t ntiles) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const uint64_t i = base + (uint64_t)r * RS_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(uint64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];  // digit-major
}

// The tile's elements are ranked stably within their digit (round by round:
// ballots give ranks inside a wavefront, LDS counts order the wavefronts and
// the rounds), placed in digit order in LDS, and written out by consecutive
// threads, so each digit's run of the tile leaves as contiguous stores.
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const uint32_t* __restrict__ keys_in,
                                                           const uint32_t* __restrict__ vals_in, uint64_t n,
                                                           int shift, const uint64_t* __restrict__ offs,
                                                           uint64_t ntiles, uint32_t* __restrict__ keys_out,
                                                           uint32_t* __restrict__ vals_out) {
  __shared__ uint32_t lrun[256];              // elements of each digit ranked so far in this tile
  __shared__ uint32_t loff[256];              // first position of each digit in the tile's sorted order
  __shared__ uint32_t wcnt[RS_WAVES][256];    // this round's count per wavefront and digit
  __shared__ uint32_t skeys[RS_TILE], svals[RS_TILE];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const bool with_vals = vals_in != nullptr;
  lrun[t] = 0;
  uint32_t k[RS_ROUNDS], v[RS_ROUNDS], rank[RS_ROUNDS];
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const uint64_t i = base + (uint64_t)r * RS_THREADS + t;
    k[r] = i < n ? keys_in[i] : 0u;
    v[r] = (with_vals && i < n) ? vals_in[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w) wcnt[w][t] = 0;
    __syncthreads();
    const bool valid = base + (uint64_t)r * RS_THREADS + t < n;
    const uint32_t d = (k[r] >> shift) & 255u;
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t m = __ballot(valid && ((d >> b) & 1u));
      same &= ((d >> b) & 1u) ? m : ~m;
    }
    const uint32_t rank_w = (uint32_t)__popcll(same & below);
    if (valid && rank_w == 0) wcnt[wave][d] = (uint32_t)__popcll(same);  // the digit's first lane
    __syncthreads();
    uint32_t rk = lrun[d] + rank_w;
    for (int w = 0; w < wave; ++w) rk += wcnt[w][d];
    rank[r] = rk;
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w) add += wcnt[w][t];
    lrun[t] += add;
  }
  __syncthreads();
  // exclusive scan of the tile's digit counts (256 digits, one per thread)
  {
    const uint32_t c = lrun[t];
    uint32_t x = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    if (lane == 63) wcnt[0][wave] = x;  // wavefront totals
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w) before += wcnt[0][w];
    loff[t] = before + x - c;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    if (base + (uint64_t)r * RS_THREADS + t < n) {
      const uint32_t p = loff[(k[r] >> shift) & 255u] + rank[r];
      skeys[p] = k[r];
      if (with_vals) svals[p] = v[r];
    }
  }
  __syncthreads();
  const uint32_t count = (uint32_t)(n - base < RS_TILE ? n - base : RS_TILE);
  for (uint32_t p = t; p < count; p += RS_THREADS) {
    const uint32_t kk = skeys[p], d = (kk >> shift) & 255u;
    const uint64_t pos = offs[(uint64_t)d * ntiles + blockIdx.x] + (p - loff[d]);
    keys_out[pos] = kk;
    if (with_vals) vals_out[pos] = svals[p];
  }
}

uint64_t sort_pairs_workspace(uint64_t n) {
  const uint64_t ntiles = (n + RS_TILE - 1) / RS_TILE;
  return 256 * ntiles + 1;  // uint64 histogram entries (+ total)
}

hc_err sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp, uint32_t* vals_tmp, uint64_t n,
                  uint64_t* hist, uint64_t* scan_tiles, hipStream_t stream) {
  if (n == 0) return HC_OK;
  const uint64_t ntiles = (n + RS_TILE - 1) / RS_TILE;
  uint32_t *ki = keys, *vi = vals, *ko = keys_tmp, *vo = vals_tmp;
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 8 * pass;
    hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)ntiles), dim3(RS_THREADS), 0, stream, ki, n, shift, hist, ntiles);
    if (hc_err r = check_launch("sort histogram"); r != HC_OK) return r;
    if (hc_err r = exclusive_scan_inplace(hist, 256 * ntiles, scan_tiles, stream); r != HC_OK) return r;
    hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)ntiles), dim3(RS_THREADS), 0, stream, ki, vi, n, shift, hist,
                       ntiles, ko, vo);
    if (hc_err r = check_launch("sort scatter"); r != HC_OK) return r;
    uint32_t* tk = ki;
    ki = ko;
    ko = tk;
    uint32_t* tv = vi;
    vi = vo;
    vo = tv;
  }
  return HC_OK;  // four passes: the sorted pairs are back in keys / vals
}

}  // namespace hc
