/*
 * Seeded synthetic input generators.
 *
 * This file produces workload inputs only (keys, values, query orders, Zipf
 * ranks).  It holds none of the hash-table arithmetic: no table hash, no probe
 * sequence, no slot codec.  Both the GPU path's tests/benchmarks and the CPU
 * oracle's tests draw their inputs from here, so that the two sides see the
 * same data without sharing any code of the method itself.
 *
 * Published definitions used:
 *   - SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
 *     generators", OOPSLA 2014): state += 0x9E3779B97F4A7C15, then the
 *     variant-13 style finaliser with multipliers 0xBF58476D1CE4E5B9 and
 *     0x94D049BB133111EB and shifts 30, 27, 31.  The i-th output (i >= 0) of
 *     a stream seeded with s is mix(s + (i + 1) * gamma), which makes the
 *     generator counter-based and trivially parallel.
 *   - A balanced Feistel network (Luby & Rackoff) is a bijection for any
 *     round function; restricting it to a sub-range by "cycle walking"
 *     (Black & Rogaway, "Ciphers with arbitrary finite domains", 2002) keeps it
 *     a bijection on that sub-range.
 *   - Zipf(s) over ranks 1..N by inversion of the exact CDF
 *     F(r) = sum_{j<=r} j^-s / H_{N,s}.
 */
#include <stdint.h>
#include <stdlib.h>
#include <math.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* i-th output (0-based) of the SplitMix64 stream seeded with `seed`. */
static inline uint64_t sm_at(uint64_t seed, uint64_t i) {
  return sm_mix(seed + (i + 1) * GAMMA);
}

uint64_t gen_splitmix64_at(uint64_t seed, uint64_t i) { return sm_at(seed, i); }

/* ---- keyed Feistel permutation on b-bit integers (b even, 2..64) -------- */
typedef struct {
  unsigned half;        /* bits per half */
  uint64_t mask;        /* (1 << half) - 1 */
  uint64_t rk[4];       /* round keys */
} feistel_t;

static void feistel_init(feistel_t* f, uint64_t seed, unsigned bits) {
  f->half = bits / 2;
  f->mask = (f->half >= 64) ? ~0ULL : ((1ULL << f->half) - 1);
  for (int r = 0; r < 4; ++r) f->rk[r] = sm_at(seed, 1000 + (uint64_t)r);
}

static inline uint64_t feistel_apply(const feistel_t* f, uint64_t x) {
  uint64_t L = (x >> f->half) & f->mask, R = x & f->mask;
  for (int r = 0; r < 4; ++r) {
    uint64_t t = L ^ (sm_mix(R ^ f->rk[r]) & f->mask);
    L = R;
    R = t;
  }
  return (L << f->half) | R;
}

/*
 * gen_keys: out[i] = perm_seed(start + i), i in [0, count).
 * perm_seed is a bijection of [1, 2^32 - 2] onto itself (a 32-bit Feistel
 * network restricted by cycle walking), so keys drawn from disjoint index
 * ranges are distinct and disjoint, and never equal 0 or 2^32 - 1.
 * Returns 0, or -1 if the index range leaves [1, 2^32 - 2].
 */
int gen_keys(uint64_t seed, uint64_t start, uint64_t count, uint32_t* out) {
  if (count == 0) return 0;
  if (start < 1 || start + count - 1 > 0xFFFFFFFEULL) return -1;
  feistel_t f;
  feistel_init(&f, seed ^ 0x6b65797366656973ULL, 32);
  #pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)count; ++i) {
    uint64_t y = start + (uint64_t)i;
    do { y = feistel_apply(&f, y); } while (y == 0 || y == 0xFFFFFFFFULL);
    out[i] = (uint32_t)y;
  }
  return 0;
}

/* gen_values: out[i] = low 32 bits of the i-th SplitMix64 output. */
void gen_values(uint64_t seed, uint64_t count, uint32_t* out) {
  #pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)count; ++i) out[i] = (uint32_t)sm_at(seed, (uint64_t)i);
}

/* gen_uniform: out[i] uniform on [lo, hi] (inclusive), by 64x64->128 multiply-high. */
void gen_uniform(uint64_t seed, uint32_t lo, uint32_t hi, uint64_t count, uint32_t* out) {
  uint64_t span = (uint64_t)hi - lo + 1;
  #pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)count; ++i) {
    unsigned __int128 p = (unsigned __int128)sm_at(seed, (uint64_t)i) * span;
    out[i] = lo + (uint32_t)(p >> 64);
  }
}

/*
 * gen_permutation: out[j] = pi(j) for j in [0, n), pi a seeded bijection of
 * [0, n) (Feistel on the next even bit width >= log2 n, cycle-walked into
 * [0, n)).  Used to shuffle query batches without a sequential shuffle.
 */
void gen_permutation(uint64_t seed, uint64_t n, uint64_t* out) {
  if (n == 0) return;
  unsigned bits = 2;
  while (bits < 64 && (1ULL << bits) < n) bits += 2;
  feistel_t f;
  feistel_init(&f, seed ^ 0x7065726d75746531ULL, bits);
  #pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < (int64_t)n; ++j) {
    uint64_t y = (uint64_t)j;
    do { y = feistel_apply(&f, y); } while (y >= n);
    out[j] = y;
  }
}

/* gen_gather_u32: out[j] = in[idx[j]] (helper to apply a permutation). */
void gen_gather_u32(const uint32_t* in, const uint64_t* idx, uint64_t n, uint32_t* out) {
  #pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < (int64_t)n; ++j) out[j] = in[idx[j]];
}

/*
 * gen_zipf_ranks: out[i] in [1, N], P(r) = r^-s / H_{N,s}, by inverse CDF.
 * The CDF table (N doubles) is built in index order, sum in fp64.
 * Returns 0, or -1 on allocation failure / bad arguments.
 */
int gen_zipf_ranks(uint64_t seed, uint32_t N, double s, uint64_t count, uint32_t* out) {
  if (N == 0) return -1;
  double* cdf = (double*)malloc(sizeof(double) * (size_t)N);
  if (!cdf) return -1;
  double acc = 0.0;
  for (uint32_t r = 1; r <= N; ++r) { acc += pow((double)r, -s); cdf[r - 1] = acc; }
  for (uint32_t r = 0; r < N; ++r) cdf[r] /= acc;
  cdf[N - 1] = 1.0;
  #pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)count; ++i) {
    /* u uniform in [0, 1) with 53 random bits */
    double u = (double)(sm_at(seed, (uint64_t)i) >> 11) * (1.0 / 9007199254740992.0);
    uint32_t lo = 0, hi = N - 1;             /* smallest r with cdf[r] > u */
    while (lo < hi) {
      uint32_t mid = lo + (hi - lo) / 2;
      if (cdf[mid] > u) hi = mid; else lo = mid + 1;
    }
    out[i] = lo + 1;
  }
  free(cdf);
  return 0;
}

/* gen_zipf_pmf: pmf[r-1] = r^-s / H_{N,s} (for goodness-of-fit tests). */
void gen_zipf_pmf(uint32_t N, double s, double* pmf) {
  double acc = 0.0;
  for (uint32_t r = 1; r <= N; ++r) { pmf[r - 1] = pow((double)r, -s); acc += pmf[r - 1]; }
  for (uint32_t r = 0; r < N; ++r) pmf[r] /= acc;
}
