// Full scan of a table's slot array: live / tombstone / empty counts and, for
// every live slot, how many windows a retrieval of its key visits before
// reaching it (its sequence index l, plus one).  The scan cross-checks the
// table's size counter (Sec. II: load factor = live entries / capacity) and
// measures probe lengths (Sec. IV-B: they grow with the load factor).
//
// The sequence index of window w for key k is found in closed form from the
// window sequence (Sec. II probing schemes):
//   linear     w = h + l            ->  l = w - h                 (mod P)
//   double     w = h + l*s          ->  l = (w - h) * s^-1        (mod P)
//   quadratic  w = h + l(l+1)/2     ->  (2l+1)^2 = 8(w - h) + 1   (mod 8P)
// The inverse of an odd s modulo 2^m comes from Newton's iteration
// x <- x(2 - s x), each step doubling the correct low bits; modulo a prime P
// it is s^(P-2) (Fermat).  The square root modulo 2^j of a number that is 1
// mod 8 is lifted one bit at a time: if x^2 = a (mod 2^i) but not mod 2^(i+1),
// then x + 2^(i-1) is a root mod 2^(i+1) (i >= 3).
#include "hc_launch.hpp"
#include "hc_stats.hpp"

namespace hc {

constexpr int STATS_WORDS = 5 + STATS_BUCKETS;  // live, tomb, empty, max, sum, histogram

__device__ __forceinline__ uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) { return (a * b) % m; }  // a, b < 2^31

__device__ __forceinline__ uint64_t inverse_mod(uint32_t s, const TableView& t) {
  if (t.pow2) {
    uint64_t x = s;  // correct to 3 bits for odd s
#pragma unroll
    for (int i = 0; i < 5; ++i) x = x * (2 - (uint64_t)s * x);
    return x & t.pmask;
  }
  uint64_t r = 1, b = s % t.P, e = t.P - 2;
  while (e) {
    if (e & 1) r = mulmod(r, b, t.P);
    b = mulmod(b, b, t.P);
    e >>= 1;
  }
  return r;
}

// l in [0, P) with l(l+1)/2 = d (mod P), P = 2^m.
__device__ __forceinline__ uint64_t triangular_index(uint64_t d, const TableView& t) {
  const uint64_t P = t.P;
  const int m = 63 - __clzll(P);
  const int j = m + 3;
  const uint64_t mod = 1ull << j, a = (8 * d + 1) & (mod - 1);
  uint64_t x = 1;
  for (int i = 3; i < j; ++i)
    if ((((x * x) - a) >> i) & 1ull) x += 1ull << (i - 1);
  // the roots are +-x and +-x + 2^(j-1); l = (root - 1) / 2 taken mod P
  const uint64_t roots[4] = {x, (mod - x) & (mod - 1), (x + (mod >> 1)) & (mod - 1),
                             (mod - x + (mod >> 1)) & (mod - 1)};
  for (int r = 0; r < 4; ++r) {
    const uint64_t l = ((roots[r] - 1) >> 1) & (P - 1);
    if (((l * (l + 1) / 2) & (P - 1)) == d) return l;
  }
  return ~0ull;  // unreachable: triangular numbers are a permutation modulo 2^m
}

__device__ __forceinline__ uint64_t seq_index(const TableView& t, uint32_t k, uint32_t w) {
  Seq s;
  seq_start(t, k, s);
  const uint64_t d = (w >= s.w) ? (uint64_t)(w - s.w) : (uint64_t)w + t.P - s.w;
  if (t.scheme == SCHEME_LINEAR) return d;
  if (t.scheme == SCHEME_DOUBLE) {
    const uint64_t inv = inverse_mod(s.step, t);
    return t.pow2 ? ((d * inv) & t.pmask) : mulmod(d, inv, t.P);
  }
  return triangular_index(d, t);
}

__global__ __launch_bounds__(256) void k_stats(TableView t, uint32_t W, unsigned long long* __restrict__ out) {
  __shared__ unsigned long long acc[STATS_WORDS];
  if (threadIdx.x < STATS_WORDS) acc[threadIdx.x] = 0ull;
  __syncthreads();
  const uint64_t C = (uint64_t)t.P * W;
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  unsigned long long live = 0, tomb = 0, empty = 0, mx = 0, sum = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < C; i += stride) {
    const uint32_t k = slot_key(t.slots[i]);
    if (k == KEY_EMPTY) {
      ++empty;
    } else if (k == KEY_TOMB) {
      ++tomb;
    } else {
      ++live;
      const uint64_t v = seq_index(t, k, (uint32_t)(i / W)) + 1;  // windows visited
      mx = v > mx ? v : mx;
      sum += v;
      int b = 63 - __clzll(v);
      if (b >= STATS_BUCKETS) b = STATS_BUCKETS - 1;
      atomicAdd(&acc[5 + b], 1ull);
    }
  }
  atomicAdd(&acc[0], live);
  atomicAdd(&acc[1], tomb);
  atomicAdd(&acc[2], empty);
  atomicMax(&acc[3], mx);
  atomicAdd(&acc[4], sum);
  __syncthreads();
  if (threadIdx.x < STATS_WORDS) {
    if (threadIdx.x == 3) atomicMax(out + 3, acc[3]);
    else if (acc[threadIdx.x]) atomicAdd(out + threadIdx.x, acc[threadIdx.x]);
  }
}

hc_err launch_stats(const TableView& t, uint32_t W, unsigned long long* d_out, hipStream_t s) {
  const uint64_t C = (uint64_t)t.P * W;
  uint64_t blocks = (C + 255) / 256;
  const uint64_t cap = (uint64_t)device_cu_count() * 8;
  if (blocks > cap) blocks = cap;
  hipLaunchKernelGGL(k_stats, dim3((unsigned)(blocks ? blocks : 1)), dim3(256), 0, s, t, W, d_out);
  return check_launch("stats");
}

}  // namespace hc
