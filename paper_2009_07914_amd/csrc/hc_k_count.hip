// Counting insert with equal keys combined on chip before they reach the table.
//
// The counting table's insert (Sec. IV-B3, counting variant) raises a key's count by
// one 64-bit atomic add per occurrence.  Under key skew the occurrences of a hot key
// all serialise on one slot: a key that makes up 12% of 2^26 inserts is 8 M atomics
// on one word.  Here every block takes tiles of AGG_TILE consecutive keys, counts the
// equal keys of a tile in an LDS hash table, and upserts each distinct key of the tile
// once, with its multiplicity as the increment, through the per-element insert state
// machine (InsertUnique, counting kind: a present key takes one atomic add of
// multiplicity << 32, a new key is claimed with its multiplicity as the count).  A hot
// key then costs one atomic per tile instead of one per occurrence.
//
// Statuses keep the per-element meaning: of the occurrences of a key that is new to the
// table, exactly one reports OK (the one that created the key's LDS entry in the tile
// whose upsert claimed the slot) and the others DUPLICATE; occurrences of a present key
// report DUPLICATE; a key that finds no reusable slot reports FULL at every occurrence
// in its tile; reserved keys report INVALID_KEY and are not counted.
#include "hc_kernels.hpp"
#include "hc_launch.hpp"

namespace hc {

// 512 threads per block: a 2048-key tile (half the atomics per hot key of a 1024-key tile)
// with the LDS per wavefront and the registers per lane of 1024 keys over 256 threads; the
// kernel is held to 80 VGPRs (6 wavefronts per SIMD, 3 blocks per CU by LDS), spilling a few.
constexpr int AGG_BLOCK = 512;
constexpr int AGG_PER_THREAD = 4;
constexpr int AGG_TILE = AGG_BLOCK * AGG_PER_THREAD;  // keys per tile
constexpr int AGG_HASH = 2 * AGG_TILE;                // LDS hash slots: load at most 1/2
constexpr int AGG_HASH_BITS = 12;
constexpr int AGG_SLOTS_PER_THREAD = AGG_HASH / AGG_BLOCK;
static_assert((1 << AGG_HASH_BITS) == AGG_HASH, "hash size");
constexpr uint32_t AGG_NONE = 0xFFFFu;

// The insert state machine with the size and failed-CAS counts kept per lane over all
// tiles and added once at the end of the kernel.
template <int G, int W>
struct AggUpsert : InsertUnique<G, W, KIND_COUNT> {
  __device__ __forceinline__ void end() {}
};

// Block-wide exclusive scan of one value per thread (AGG_BLOCK threads).
__device__ __forceinline__ uint32_t agg_block_scan(uint32_t x, uint32_t* total, uint32_t* wsum) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t incl = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < AGG_BLOCK / 64; ++w) {
    const uint32_t v = wsum[w];
    before += (w < wave) ? v : 0u;
    all += v;
  }
  __syncthreads();
  *total = all;
  return before + incl - x;
}

template <int G, int W>
__global__ __launch_bounds__(AGG_BLOCK, 6) void k_count_agg(TableView t, WorkCtl ctl, const uint32_t* __restrict__ keys,
                                                     uint64_t n, uint8_t* __restrict__ status) {
  __shared__ uint32_t hkey[AGG_HASH];  // tile keys; after compaction the distinct keys in [0, m)
  __shared__ uint32_t hcnt[AGG_HASH];  // multiplicities, compacted likewise
  __shared__ uint16_t hpos[AGG_HASH];  // compact index of each used hash slot
  __shared__ uint8_t cres[AGG_TILE];   // upsert status of each distinct key
  __shared__ uint32_t wsum[AGG_BLOCK / 64];
  __shared__ unsigned long long s_tile;

  AggUpsert<G, W> op;
  op.t = t;
  op.keys = hkey;
  op.values = hcnt;
  op.status = cres;
  const uint64_t ntiles = (n + AGG_TILE - 1) / AGG_TILE;
  const int wave = threadIdx.x >> 6;
  for (;;) {
    if (threadIdx.x == 0) s_tile = atomicAdd(ctl.counters, 1ull);
#pragma unroll
    for (int j = 0; j < AGG_SLOTS_PER_THREAD; ++j) {
      hkey[j * AGG_BLOCK + threadIdx.x] = 0u;
      hcnt[j * AGG_BLOCK + threadIdx.x] = 0u;
    }
    __syncthreads();
    const uint64_t tile = s_tile;
    if (tile >= ntiles) break;
    const uint64_t base = tile * AGG_TILE;

    // 1. count the tile's keys in the LDS hash table (linear probing; at most AGG_TILE keys
    //    in AGG_HASH slots, so every key finds its slot)
    uint32_t slot[AGG_PER_THREAD];
    uint32_t creator = 0;  // bit j: this thread's j-th key created its entry
#pragma unroll
    for (int j = 0; j < AGG_PER_THREAD; ++j) {
      const uint64_t i = base + (uint64_t)j * AGG_BLOCK + threadIdx.x;
      slot[j] = AGG_NONE;
      if (i >= n) continue;
      const uint32_t k = keys[i];
      if (reserved_key(k)) {
        if (status != nullptr) status[i] = ST_INVALID_KEY;
        continue;
      }
      uint32_t hs = (k * 0x9E3779B1u) >> (32 - AGG_HASH_BITS);
      for (;;) {
        const uint32_t prev = atomicCAS(&hkey[hs], 0u, k);
        if (prev == 0u) {
          creator |= 1u << j;
          break;
        }
        if (prev == k) break;
        hs = (hs + 1) & (AGG_HASH - 1);
      }
      atomicAdd(&hcnt[hs], 1u);
      slot[j] = hs;
    }
    __syncthreads();

    // 2. compact the used slots, in slot order, to [0, m)
    uint32_t ck[AGG_SLOTS_PER_THREAD], cc[AGG_SLOTS_PER_THREAD];
    uint32_t used = 0;
#pragma unroll
    for (int j = 0; j < AGG_SLOTS_PER_THREAD; ++j) {
      ck[j] = hkey[threadIdx.x * AGG_SLOTS_PER_THREAD + j];
      cc[j] = hcnt[threadIdx.x * AGG_SLOTS_PER_THREAD + j];
      used += ck[j] != 0u;
    }
    uint32_t m = 0;
    uint32_t pos = agg_block_scan(used, &m, wsum);  // its barriers order the reads above before the writes
#pragma unroll
    for (int j = 0; j < AGG_SLOTS_PER_THREAD; ++j) {
      if (ck[j] != 0u) {
        hkey[pos] = ck[j];
        hcnt[pos] = cc[j];
        hpos[threadIdx.x * AGG_SLOTS_PER_THREAD + j] = (uint16_t)pos;
        ++pos;
      }
    }
    __syncthreads();

    // 3. upsert the m distinct keys: each wavefront an eighth of them, groups in order
    const uint64_t lo = (uint64_t)m * wave / (AGG_BLOCK / 64), hi = (uint64_t)m * (wave + 1) / (AGG_BLOCK / 64);
    drive_range<G>(lo, hi, op);
    __syncthreads();

    // 4. per-element statuses from the distinct keys' outcomes
    if (status != nullptr) {
#pragma unroll
      for (int j = 0; j < AGG_PER_THREAD; ++j) {
        if (slot[j] == AGG_NONE) continue;
        const uint64_t i = base + (uint64_t)j * AGG_BLOCK + threadIdx.x;
        const uint8_t r = cres[hpos[slot[j]]];
        status[i] = (r == ST_OK && !((creator >> j) & 1u)) ? (uint8_t)ST_DUPLICATE : r;
      }
    }
  }
  wave_add_to(t.size + CTR_SIZE, op.added);
  wave_add_to(t.size + CTR_CAS_FAILS, op.fails);
  if (threadIdx.x == 0) {
    if (atomicAdd(ctl.counters + 1, 1ull) == (unsigned long long)gridDim.x - 1) {  // every tile is taken
      atomicExch(ctl.counters, 0ull);
      atomicExch(ctl.counters + 1, 0ull);
    }
  }
}

hc_err launch_count_insert(const TableView& t, uint32_t G, uint32_t W, const uint32_t* keys, uint64_t n,
                           uint8_t* status, hipStream_t stream) {
  return dispatch_gw(G, W, [&](auto g, auto w) -> hc_err {
    constexpr int GG = decltype(g)::value, WW = decltype(w)::value;
    auto k = k_count_agg<GG, WW>;
    const uint64_t ntiles = (n + AGG_TILE - 1) / AGG_TILE;
    const uint64_t per_cu = (uint64_t)blocks_per_cu_threads(reinterpret_cast<const void*>(k), AGG_BLOCK);
    const uint64_t cap = (uint64_t)device_cu_count() * per_cu;
    const unsigned grid = (unsigned)(ntiles < cap ? (ntiles ? ntiles : 1) : cap);
    WorkCtl ctl = work_for(0, GG, grid, stream);
    hipLaunchKernelGGL(k, dim3(grid), dim3(AGG_BLOCK), 0, stream, t, ctl, keys, n, status);
    return check_launch("counting insert");
  });
}

}  // namespace hc
