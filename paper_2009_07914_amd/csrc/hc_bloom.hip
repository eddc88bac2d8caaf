// Bloom filter answering set membership queries (Sec. IV lists it among the
// structures built on the tables' principles; the paper gives no design).
//
// Split-block layout: the bit array is B blocks of `words` 32-bit words (8, 16
// or 32: 32, 64 or 128 bytes), so a key touches one block, one line of HBM,
// instead of k scattered lines.  Key x selects block reduce(h1(x), B) (h1, h2
// and the reduction are the tables' hash and window reduction) and sets one bit
// in every word of it: bit fmix32(h2(x) + i * 0x9E3779B9) >> 27 of word i, so
// k = words bits per key.  With one bit per word the words of a block fill
// independently, which gives the filter an exact false-positive rate.
//
// Cooperation follows the tables' groups (Sec. IV-B2): a group of G lanes takes
// one key, lane r owning the block's words [r * words/G, (r+1) * words/G).
// Insert: each lane ORs its words' bits in with atomic ORs (no return value; word
// pairs as one 64-bit OR).
// Query: each lane loads its words (vector loads) and checks its bits; the key
// is reported present iff every lane's bits are all set (a group ballot).
#include <new>

#include "hc_device.hpp"
#include "hc_launch.hpp"

namespace hc {

struct BloomView {
  uint32_t* bits;
  uint64_t B;     // blocks
  uint32_t pow2;  // B is a power of two
  uint32_t seed_lo, seed_hi;
};

struct BloomKey {
  uint64_t block;
  uint32_t h2;
  __device__ __forceinline__ BloomKey(const BloomView& f, uint32_t x) {
    const uint32_t h1 = fmix32(x ^ f.seed_lo);
    h2 = fmix32((x ^ f.seed_hi) + 0x9E3779B9u);
    block = f.pow2 ? (h1 & (f.B - 1)) : (((uint64_t)h1 * f.B) >> 32);
  }
  // Masks of words [first, first + WPL) of the block: one bit each.
  template <int WPL>
  __device__ __forceinline__ void masks(uint32_t first, uint32_t (&m)[WPL]) const {
#pragma unroll
    for (int j = 0; j < WPL; ++j) m[j] = 1u << (fmix32(h2 + (first + j) * 0x9E3779B9u) >> 27);
  }
};

template <int G, int WORDS>
__global__ __launch_bounds__(BLOCK) void k_bloom_insert(BloomView f, const uint32_t* __restrict__ keys, uint64_t n) {
  constexpr int WPL = WORDS / G;
  const uint32_t r = __lane_id() & (G - 1);
  const uint64_t groups = (uint64_t)gridDim.x * (BLOCK / G);
  for (uint64_t i = ((uint64_t)blockIdx.x * BLOCK + threadIdx.x) / G; i < n; i += groups) {
    const BloomKey key(f, keys[i]);
    uint32_t m[WPL];
    key.masks<WPL>(r * WPL, m);
    uint32_t* blk = f.bits + key.block * WORDS + r * WPL;
    if constexpr (WPL % 2 == 0) {  // word pairs as 64-bit atomic ORs: half the atomic lanes per key
#pragma unroll
      for (int j = 0; j < WPL; j += 2)
        atomicOr(reinterpret_cast<unsigned long long*>(blk + j), (unsigned long long)m[j] | ((unsigned long long)m[j + 1] << 32));
    } else {
      atomicOr(blk, m[0]);
    }
  }
}

template <int G, int WORDS>
__global__ __launch_bounds__(BLOCK) void k_bloom_contains(BloomView f, const uint32_t* __restrict__ keys, uint64_t n,
                                                          uint8_t* __restrict__ found_out) {
  constexpr int WPL = WORDS / G;
  GroupCtx<G> g;
  const uint64_t groups = (uint64_t)gridDim.x * (BLOCK / G);
  for (uint64_t i = ((uint64_t)blockIdx.x * BLOCK + threadIdx.x) / G; i < n; i += groups) {
    const BloomKey key(f, keys[i]);
    uint32_t m[WPL], w[WPL];
    key.masks<WPL>(g.glane * WPL, m);
    const uint32_t* blk = f.bits + key.block * WORDS + g.glane * WPL;
    if constexpr (WPL % 4 == 0) {
#pragma unroll
      for (int j = 0; j < WPL / 4; ++j) {
        const uint4 q = reinterpret_cast<const uint4*>(blk)[j];
        w[4 * j] = q.x;
        w[4 * j + 1] = q.y;
        w[4 * j + 2] = q.z;
        w[4 * j + 3] = q.w;
      }
    } else if constexpr (WPL == 2) {
      const uint2 q = *reinterpret_cast<const uint2*>(blk);
      w[0] = q.x;
      w[1] = q.y;
    } else {
      w[0] = blk[0];
    }
    bool ok = true;
#pragma unroll
    for (int j = 0; j < WPL; ++j) ok = ok && (w[j] & m[j]) == m[j];
    const bool all = g.bits(!ok) == 0;
    if (g.glane == 0) found_out[i] = all ? 1 : 0;
  }
}

// Zero n 16-byte vectors (a kernel, so a caller may capture a clear in a graph).
__global__ __launch_bounds__(BLOCK) void k_bloom_zero(uint4* __restrict__ p, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * BLOCK;
  for (uint64_t i = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

static hc_err launch_bloom_zero(uint32_t* bits, uint64_t words, hipStream_t s) {
  const uint64_t n = words / 4;  // words = blocks * (8, 16 or 32): a multiple of 4
  uint64_t blocks = (n + BLOCK - 1) / BLOCK;
  const uint64_t cap = (uint64_t)device_cu_count() * 16;
  if (blocks > cap) blocks = cap;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_bloom_zero, dim3((unsigned)blocks), dim3(BLOCK), 0, s, reinterpret_cast<uint4*>(bits), n);
  return check_launch("Bloom clear");
}

template <int G, int WORDS, typename F>
static hc_err bloom_call(F&& f) {
  if constexpr (G <= WORDS) return f(ic<G>{}, ic<WORDS>{});
  return fail(HC_E_ARG, "group size %d over %d words per block", G, WORDS);
}

template <int WORDS, typename F>
static hc_err dispatch_bloom_g(uint32_t G, F&& f) {
  switch (G) {
    case 1: return bloom_call<1, WORDS>(f);
    case 2: return bloom_call<2, WORDS>(f);
    case 4: return bloom_call<4, WORDS>(f);
    case 8: return bloom_call<8, WORDS>(f);
    case 16: return bloom_call<16, WORDS>(f);
    case 32: return bloom_call<32, WORDS>(f);
    default: return fail(HC_E_ARG, "group size %u is not a power of two up to %d", G, WORDS);
  }
}

template <typename F>
static hc_err dispatch_bloom(uint32_t G, uint32_t words, F&& f) {
  if (G > words) return fail(HC_E_ARG, "group size %u over %u words per block", G, words);
  switch (words) {
    case 8: return dispatch_bloom_g<8>(G, f);
    case 16: return dispatch_bloom_g<16>(G, f);
    case 32: return dispatch_bloom_g<32>(G, f);
    default: return fail(HC_E_ARG, "block words %u is not 8, 16 or 32", words);
  }
}

}  // namespace hc

using namespace hc;

struct hc_bloom_s {
  int device = 0;
  uint32_t* bits = nullptr;
  uint64_t blocks = 0;
  uint32_t words = 0, group = 0;
  uint64_t seed = 0;
};

static BloomView bloom_view(const hc_bloom_s* b) {
  BloomView v;
  v.bits = b->bits;
  v.B = b->blocks;
  v.pow2 = (b->blocks & (b->blocks - 1)) == 0;
  v.seed_lo = (uint32_t)b->seed;
  v.seed_hi = (uint32_t)(b->seed >> 32);
  return v;
}

static hc_err bloom_device(hc_bloom b) {
  if (b == nullptr) return fail(HC_E_ARG, "Bloom filter handle is NULL");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(HC_E_DEVICE, "hipGetDevice failed");
  if (cur != b->device) {
    const hipError_t e = hipSetDevice(b->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  }
  return HC_OK;
}

// Group 0 (in the call and in the filter's default): per operation, the fastest
// measured: inserts one lane per word (the block's atomic ORs leave as one
// request), queries one lane per key (a 64-byte block is one vector load).
static hc_err bloom_group(hc_bloom b, uint32_t group, bool insert, uint32_t* out) {
  uint32_t g = group ? group : b->group;
  if (g == 0) g = insert ? b->words : 1;
  if (g == 0 || (g & (g - 1)) != 0 || g > b->words)
    return fail(HC_E_ARG, "group size %u is not a power of two in [1, %u]", g, b->words);
  *out = g;
  return HC_OK;
}

extern "C" {

void hc_default_bloom_params(hc_bloom_params* p) {
  if (p == nullptr) return;
  p->block_words = 16;
  p->group = 0;
  p->seed = 0x9E3779B97F4A7C15ull;
}

hc_err hc_bloom_create(hc_bloom* out, uint64_t bits, const hc_bloom_params* params) {
  if (out == nullptr) return fail(HC_E_ARG, "out is NULL");
  *out = nullptr;
  hc_bloom_params p;
  hc_default_bloom_params(&p);
  if (params != nullptr) p = *params;
  if (p.block_words != 8 && p.block_words != 16 && p.block_words != 32)
    return fail(HC_E_ARG, "block words %u is not 8, 16 or 32", p.block_words);
  if ((p.group & (p.group - 1)) != 0 || p.group > p.block_words)
    return fail(HC_E_ARG, "group size %u is not a power of two in [1, %u]", p.group, p.block_words);
  if (bits == 0) return fail(HC_E_ARG, "bits is 0");
  const uint64_t per = 32ull * p.block_words;
  const uint64_t blocks = (bits + per - 1) / per;
  if (blocks > (1ull << 32)) return fail(HC_E_ARG, "more than 2^32 blocks");
  hc_bloom_s* b = new (std::nothrow) hc_bloom_s();
  if (b == nullptr) return fail(HC_E_NOMEM, "host allocation failed");
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return fail(HC_E_DEVICE, "hipGetDevice failed");
  }
  b->blocks = blocks;
  b->words = p.block_words;
  b->group = p.group;
  b->seed = p.seed;
  hipError_t e = hipMalloc((void**)&b->bits, blocks * p.block_words * 4);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    delete b;
    return fail(HC_E_NOMEM, "hipMalloc of %llu filter bytes failed", (unsigned long long)(blocks * p.block_words * 4));
  }
  hc_err rz = launch_bloom_zero(b->bits, blocks * p.block_words, nullptr);
  if (rz == HC_OK && (e = hipDeviceSynchronize()) != hipSuccess) rz = hip_fail(e, "hc_bloom_create: clear");
  if (rz != HC_OK) {
    (void)hipFree(b->bits);
    delete b;
    return rz;
  }
  *out = b;
  return HC_OK;
}

hc_err hc_bloom_destroy(hc_bloom b) {
  if (b == nullptr) return HC_OK;
  hc_err r = bloom_device(b);
  if (r != HC_OK) return r;
  const hipError_t e = hipDeviceSynchronize();
  (void)hipFree(b->bits);
  delete b;
  if (e != hipSuccess) return hip_fail(e, "hc_bloom_destroy: synchronise");
  return HC_OK;
}

hc_err hc_bloom_clear(hc_bloom b, void* stream) {
  hc_err r = bloom_device(b);
  if (r != HC_OK) return r;
  return launch_bloom_zero(b->bits, b->blocks * b->words, (hipStream_t)stream);
}

hc_err hc_bloom_insert(hc_bloom b, const uint32_t* d_keys, uint64_t n, uint32_t group, void* stream) {
  hc_err r = bloom_device(b);
  if (r != HC_OK) return r;
  uint32_t G;
  if ((r = bloom_group(b, group, true, &G)) != HC_OK) return r;
  if (n == 0) return HC_OK;
  if (d_keys == nullptr) return fail(HC_E_ARG, "keys is NULL");
  const BloomView v = bloom_view(b);
  return dispatch_bloom(G, b->words, [&](auto g, auto w) -> hc_err {
    constexpr int GG = decltype(g)::value, WW = decltype(w)::value;
    auto k = k_bloom_insert<GG, WW>;
    hipLaunchKernelGGL(k, dim3(grid_for(k, n, GG)), dim3(BLOCK), 0, (hipStream_t)stream, v, d_keys, n);
    return check_launch("Bloom insert");
  });
}

hc_err hc_bloom_contains(hc_bloom b, const uint32_t* d_keys, uint64_t n, uint8_t* d_found_out, uint32_t group,
                         void* stream) {
  hc_err r = bloom_device(b);
  if (r != HC_OK) return r;
  uint32_t G;
  if ((r = bloom_group(b, group, false, &G)) != HC_OK) return r;
  if (n == 0) return HC_OK;
  if (d_keys == nullptr || d_found_out == nullptr) return fail(HC_E_ARG, "keys or found is NULL");
  const BloomView v = bloom_view(b);
  return dispatch_bloom(G, b->words, [&](auto g, auto w) -> hc_err {
    constexpr int GG = decltype(g)::value, WW = decltype(w)::value;
    auto k = k_bloom_contains<GG, WW>;
    hipLaunchKernelGGL(k, dim3(grid_for(k, n, GG)), dim3(BLOCK), 0, (hipStream_t)stream, v, d_keys, n,
                       d_found_out);
    return check_launch("Bloom contains");
  });
}

hc_err hc_bloom_info(hc_bloom b, hc_bloom_info_t* out) {
  if (b == nullptr || out == nullptr) return fail(HC_E_ARG, "handle or out is NULL");
  out->blocks = b->blocks;
  out->block_words = b->words;
  out->group = b->group;
  out->seed = b->seed;
  out->d_bits = b->bits;
  return HC_OK;
}

hc_err hc_bloom_dump(hc_bloom b, uint32_t* d_dst, void* stream) {
  hc_err r = bloom_device(b);
  if (r != HC_OK) return r;
  if (d_dst == nullptr) return fail(HC_E_ARG, "dst is NULL");
  const hipError_t e =
      hipMemcpyAsync(d_dst, b->bits, b->blocks * b->words * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hc_bloom_dump");
  return HC_OK;
}

}  // extern "C"
