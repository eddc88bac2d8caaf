// Multi-value tables under heavy key skew.
//
// The paper's multi-value insert stores every pair at the first reusable
// position of its key's window sequence (Sec. IV-B3), so the i-th copy of a key
// scans past the i-1 earlier ones: a key with m copies costs about m^2/(2W)
// window visits, and retrieving it scans about m/W windows (Sec. V-B: throughput
// degrades with the number of values per key).  Two additions keep the same
// stored multiset and the same layout invariant (no empty position before any
// stored position of a key) while removing the quadratic term:
//   * grouped insert: pairs are sorted by key; each run of one key claims its m
//     slots in one pass along the sequence (a wavefront per run, or a whole block
//     of 1024 threads for runs of at least HEAVY pairs), claiming reusable slots in
//     sequence order with a CAS to a placeholder and then writing the run's values
//     in the order of the successful claims;
//   * long queries: count and write passes give up after `budget` windows and
//     hand the query to a kernel in which a block of 1024 threads scans 4096 slots
//     per step.
#include "hc_group.hpp"
#include "hc_kernels.hpp"
#include "hc_launch.hpp"
#include "hc_sort.hpp"

namespace hc {

constexpr int GB = 1024;              // threads per block of the run / long-query kernels
constexpr int GB_WAVES = GB / 64;
constexpr int GB_SPL = 4;             // slots per lane in block mode
constexpr uint32_t RUN_GRAB = 16;     // light runs taken per wavefront atomic

struct KeySeq {
  uint32_t w0, step;
};

__device__ __forceinline__ KeySeq key_seq(const TableView& t, uint32_t k) {
  Seq s;
  seq_start(t, k, s);
  return {s.w, s.step};
}

// Window of sequence index l: the closed forms of seq_next.
__device__ __forceinline__ uint32_t window_at(const TableView& t, const KeySeq& q, uint64_t l) {
  uint64_t off;
  if (t.scheme == SCHEME_LINEAR) off = l;
  else if (t.scheme == SCHEME_QUADRATIC) off = l * (l + 1) / 2;
  else off = l * (uint64_t)q.step;
  if (t.pow2) return (uint32_t)((q.w0 + off) & t.pmask);
  return (uint32_t)((q.w0 + off) % t.P);
}

// Block-wide exclusive scan (GB threads); *total gets the sum.  lds: GB_WAVES words.
__device__ __forceinline__ uint32_t block_scan(uint32_t x, uint32_t* total, uint32_t* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t incl = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) lds[wave] = incl;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < GB_WAVES; ++w) {
    const uint32_t v = lds[w];
    before += (w < wave) ? v : 0u;
    all += v;
  }
  __syncthreads();
  *total = all;
  return before + incl - x;
}

// ---- grouped insert -------------------------------------------------------------

// Claim m slots for key k with a whole block; the run's values are vals[0..m).
template <int W>
__device__ void claim_run_block(const TableView& t, uint32_t k, const uint32_t* __restrict__ vals, uint64_t m,
                                uint64_t& added, uint32_t* lds) {
  constexpr uint32_t WPS_B = GB * GB_SPL / W;  // sequence windows per step
  const KeySeq q = key_seq(t, k);
  const uint32_t widx = (threadIdx.x * GB_SPL) / W, j0 = (threadIdx.x * GB_SPL) % W;
  uint64_t claimed = 0;
  for (uint64_t lbase = 0; claimed < m && lbase < t.P; lbase += WPS_B) {
    const uint64_t l = lbase + widx;
    uint64_t first = 0, word[GB_SPL];
    uint32_t reuse = 0, emptym = 0;
    if (l < t.P) {
      first = (uint64_t)window_at(t, q, l) * W + j0;
      load_slots<GB_SPL>(t.slots, first, word);
#pragma unroll
      for (int j = 0; j < GB_SPL; ++j) {
        const uint32_t key = slot_key(word[j]);
        emptym |= (uint32_t)(key == KEY_EMPTY) << j;
        reuse |= (uint32_t)(key == KEY_EMPTY || key == KEY_TOMB) << j;
      }
    }
    for (;;) {  // attempted slots leave `reuse`, so every round shrinks it
      uint32_t tot;
      const uint32_t ex = block_scan((uint32_t)__popc(reuse), &tot, lds);
      if (tot == 0) break;
      const uint64_t need = m - claimed;
      uint32_t succ = 0, tried = 0, rank = ex;
#pragma unroll
      for (int j = 0; j < GB_SPL; ++j) {
        if ((reuse >> j) & 1u) {
          if (rank < need) {
            const uint64_t expect = ((emptym >> j) & 1u) ? WORD_EMPTY : WORD_TOMB;
            const uint64_t r = atomicCAS((unsigned long long*)&t.slots[first + j], (unsigned long long)expect,
                                         (unsigned long long)make_slot(k, 0u));
            succ |= (uint32_t)(r == expect) << j;
            tried |= 1u << j;
          }
          ++rank;
        }
      }
      reuse &= ~tried;
      uint32_t stot;
      const uint32_t sex = block_scan((uint32_t)__popc(succ), &stot, lds);
      uint32_t rr = 0;
#pragma unroll
      for (int j = 0; j < GB_SPL; ++j) {
        if ((succ >> j) & 1u) {
          atomicExch((unsigned long long*)&t.slots[first + j],
                     (unsigned long long)make_slot(k, vals[claimed + sex + rr]));
          ++rr;
        }
      }
      claimed += stot;
      if (claimed >= m) break;
    }
  }
  if (threadIdx.x == 0) added += claimed;
}

// Claim m slots for key k with one wavefront (one slot per lane).
template <int W>
__device__ void claim_run_wave(const TableView& t, uint32_t k, const uint32_t* __restrict__ vals, uint64_t m,
                               uint64_t& added) {
  constexpr uint32_t WPS_W = 64 / W;  // W <= 64
  const uint32_t lane = __lane_id();
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const KeySeq q = key_seq(t, k);
  const uint32_t widx = lane / W, j = lane % W;
  uint64_t claimed = 0;
  for (uint64_t lbase = 0; claimed < m && lbase < t.P; lbase += WPS_W) {
    const uint64_t l = lbase + widx;
    uint64_t idx = 0, word = 0;
    bool reuse = false;
    if (l < t.P) {
      idx = (uint64_t)window_at(t, q, l) * W + j;
      word = t.slots[idx];
      const uint32_t key = slot_key(word);
      reuse = key == KEY_EMPTY || key == KEY_TOMB;
    }
    for (;;) {
      const uint64_t bal = __ballot(reuse);
      if (bal == 0) break;
      const uint64_t need = m - claimed;
      const uint32_t rank = (uint32_t)__popcll(bal & below);
      bool ok = false;
      if (reuse && rank < need) {
        const uint64_t expect = (slot_key(word) == KEY_EMPTY) ? WORD_EMPTY : WORD_TOMB;
        const uint64_t r = atomicCAS((unsigned long long*)&t.slots[idx], (unsigned long long)expect,
                                     (unsigned long long)make_slot(k, 0u));
        ok = r == expect;
        reuse = false;
      }
      const uint64_t sb = __ballot(ok);
      if (ok)
        atomicExch((unsigned long long*)&t.slots[idx],
                   (unsigned long long)make_slot(k, vals[claimed + __popcll(sb & below)]));
      claimed += (uint64_t)__popcll(sb);
      if (claimed >= m) break;
    }
  }
  if (lane == 0) added += claimed;
}

__global__ __launch_bounds__(256) void k_run_flags(const uint32_t* __restrict__ keys, uint64_t n,
                                                   uint64_t* __restrict__ flags, unsigned long long* nheavy) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i == 0) *nheavy = 0ull;
  if (i < n) flags[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1ull : 0ull;
}

// scan[i] = runs before element i (exclusive scan of the flags), scan[n] = runs.
__global__ __launch_bounds__(256) void k_run_starts(const uint64_t* __restrict__ scan, uint64_t n,
                                                    uint64_t* __restrict__ starts) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n && scan[i + 1] != scan[i]) starts[scan[i]] = i;
  if (i == n) starts[scan[n]] = n;
}

__global__ __launch_bounds__(256) void k_heavy_list(const uint64_t* __restrict__ starts,
                                                    const uint64_t* __restrict__ nruns, uint64_t max_runs,
                                                    uint32_t* __restrict__ heavy, unsigned long long* nheavy) {
  const uint64_t r = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (r < max_runs && r < *nruns && starts[r + 1] - starts[r] >= HEAVY_RUN)
    heavy[atomicAdd(nheavy, 1ull)] = (uint32_t)r;
}

template <int W>
__global__ __launch_bounds__(GB) void k_claim_runs(TableView t, WorkCtl ctl, const uint32_t* __restrict__ keys,
                                                   const uint32_t* __restrict__ vals,
                                                   const uint64_t* __restrict__ starts,
                                                   const uint64_t* __restrict__ nruns,
                                                   const uint32_t* __restrict__ heavy,
                                                   const unsigned long long* __restrict__ nheavy) {
  __shared__ uint32_t lds[GB_WAVES];
  __shared__ unsigned long long s_item;
  const uint64_t R = *nruns, H = *nheavy;
  uint64_t added = 0;
  for (;;) {  // heavy runs, one block each, biggest work first in list order
    if (threadIdx.x == 0) s_item = atomicAdd(ctl.counters, 1ull);
    __syncthreads();
    const uint64_t h = s_item;
    __syncthreads();
    if (h >= H) break;
    const uint64_t r = heavy[h], st = starts[r], m = starts[r + 1] - st;
    const uint32_t k = keys[st];
    if (!reserved_key(k)) claim_run_block<W>(t, k, vals + st, m, added, lds);
  }
  const uint32_t lane = __lane_id();
  for (;;) {  // light runs, one wavefront each, RUN_GRAB runs per atomic
    unsigned long long c = 0;
    if (lane == 0) c = atomicAdd(ctl.counters + 2, 1ull);
    c = __builtin_amdgcn_readfirstlane((uint32_t)c);
    const uint64_t r0 = (uint64_t)c * RUN_GRAB;
    if (r0 >= R) break;
    for (uint64_t r = r0; r < r0 + RUN_GRAB && r < R; ++r) {
      const uint64_t st = starts[r], m = starts[r + 1] - st;
      const uint32_t k = keys[st];
      if (m < HEAVY_RUN && !reserved_key(k)) claim_run_wave<W>(t, k, vals + st, m, added);
    }
  }
  __syncthreads();
  wave_add_to(t.size, (long long)added);
  if (threadIdx.x == 0) {
    if (atomicAdd(ctl.counters + 1, 1ull) == (unsigned long long)gridDim.x - 1) {
      atomicExch(ctl.counters, 0ull);
      atomicExch(ctl.counters + 1, 0ull);
      atomicExch(ctl.counters + 2, 0ull);
    }
  }
}

// ---- long queries -----------------------------------------------------------------

__global__ __launch_bounds__(256) void k_zero_u64(unsigned long long* p, uint32_t count) {
  if (threadIdx.x < count) p[threadIdx.x] = 0ull;
}

// Continue the count of long queries from window `budget`: offsets[i] holds the
// count so far and receives the full count (counts[i] too when given).
template <int W>
__global__ __launch_bounds__(GB) void k_long_count(TableView t, WorkCtl ctl, const uint32_t* __restrict__ keys,
                                                   const uint64_t* __restrict__ list,
                                                   const unsigned long long* __restrict__ nlong, uint32_t budget,
                                                   uint64_t* __restrict__ offsets, uint32_t* __restrict__ counts) {
  constexpr uint32_t WPS_B = GB * GB_SPL / W;
  __shared__ uint32_t lds[GB_WAVES];
  __shared__ unsigned long long s_item;
  __shared__ uint32_t s_first_empty;
  const uint64_t L = *nlong;
  const uint32_t widx = (threadIdx.x * GB_SPL) / W, j0 = (threadIdx.x * GB_SPL) % W;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(ctl.counters, 1ull);
    __syncthreads();
    const uint64_t it = s_item;
    __syncthreads();
    if (it >= L) break;
    const uint64_t i = list[it];
    const uint32_t k = keys[i];
    const KeySeq q = key_seq(t, k);
    uint64_t cnt = offsets[i];
    for (uint64_t lbase = budget; lbase < t.P; lbase += WPS_B) {
      if (threadIdx.x == 0) s_first_empty = 0xFFFFFFFFu;
      __syncthreads();
      const uint64_t l = lbase + widx;
      uint32_t matches = 0;
      if (l < t.P) {
        uint64_t word[GB_SPL];
        load_slots<GB_SPL>(t.slots, (uint64_t)window_at(t, q, l) * W + j0, word);
        bool empty = false;
#pragma unroll
        for (int j = 0; j < GB_SPL; ++j) {
          matches += slot_key(word[j]) == k;
          empty |= slot_key(word[j]) == KEY_EMPTY;
        }
        if (empty) atomicMin(&s_first_empty, widx);
      }
      __syncthreads();
      const uint32_t fe = s_first_empty;
      uint32_t tot;
      block_scan((l < t.P && widx <= fe) ? matches : 0u, &tot, lds);
      cnt += tot;
      if (fe != 0xFFFFFFFFu) break;
    }
    if (threadIdx.x == 0) {
      offsets[i] = cnt;
      if (counts != nullptr) counts[i] = (uint32_t)cnt;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (atomicAdd(ctl.counters + 1, 1ull) == (unsigned long long)gridDim.x - 1) {
      atomicExch(ctl.counters, 0ull);
      atomicExch(ctl.counters + 1, 0ull);
    }
  }
}

// Continue the write of long queries from window `budget`: list holds (i, written).
template <int W>
__global__ __launch_bounds__(GB) void k_long_write(TableView t, WorkCtl ctl, const uint32_t* __restrict__ keys,
                                                   const uint64_t* __restrict__ list,
                                                   const unsigned long long* __restrict__ nlong, uint32_t budget,
                                                   const uint64_t* __restrict__ offsets, uint32_t* __restrict__ out) {
  constexpr uint32_t WPS_B = GB * GB_SPL / W;
  __shared__ uint32_t lds[GB_WAVES];
  __shared__ unsigned long long s_item;
  __shared__ uint32_t s_first_empty;
  const uint64_t L = *nlong;
  const uint32_t widx = (threadIdx.x * GB_SPL) / W, j0 = (threadIdx.x * GB_SPL) % W;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(ctl.counters, 1ull);
    __syncthreads();
    const uint64_t it = s_item;
    __syncthreads();
    if (it >= L) break;
    const uint64_t i = list[2 * it];
    uint64_t written = list[2 * it + 1];
    const uint32_t k = keys[i];
    const KeySeq q = key_seq(t, k);
    const uint64_t base = offsets[i], limit = offsets[i + 1] - base;
    for (uint64_t lbase = budget; lbase < t.P && written < limit; lbase += WPS_B) {
      if (threadIdx.x == 0) s_first_empty = 0xFFFFFFFFu;
      __syncthreads();
      const uint64_t l = lbase + widx;
      uint64_t word[GB_SPL];
      uint32_t mm = 0;
      if (l < t.P) {
        load_slots<GB_SPL>(t.slots, (uint64_t)window_at(t, q, l) * W + j0, word);
        bool empty = false;
#pragma unroll
        for (int j = 0; j < GB_SPL; ++j) {
          mm |= (uint32_t)(slot_key(word[j]) == k) << j;
          empty |= slot_key(word[j]) == KEY_EMPTY;
        }
        if (empty) atomicMin(&s_first_empty, widx);
      }
      __syncthreads();
      const uint32_t fe = s_first_empty;
      if (!(l < t.P && widx <= fe)) mm = 0;
      uint32_t tot;
      uint64_t rank = written + block_scan((uint32_t)__popc(mm), &tot, lds);
#pragma unroll
      for (int j = 0; j < GB_SPL; ++j) {
        if ((mm >> j) & 1u) {
          if (rank < limit) out[base + rank] = slot_value(word[j]);
          ++rank;
        }
      }
      written += tot;
      if (fe != 0xFFFFFFFFu) break;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (atomicAdd(ctl.counters + 1, 1ull) == (unsigned long long)gridDim.x - 1) {
      atomicExch(ctl.counters, 0ull);
      atomicExch(ctl.counters + 1, 0ull);
    }
  }
}

// ---- host side ----------------------------------------------------------------------

template <typename F>
static hc_err dispatch_w(uint32_t W, F&& f) {
  switch (W) {
    case 8: return f(ic<8>{});
    case 16: return f(ic<16>{});
    case 32: return f(ic<32>{});
    case 64: return f(ic<64>{});
  }
  return fail(HC_E_ARG, "window %u is not one of 8, 16, 32, 64", W);
}

static unsigned block_grid(const void* kernel, uint64_t items) {
  const uint64_t cap = (uint64_t)device_cu_count() * (uint64_t)blocks_per_cu_threads(kernel, GB);
  const uint64_t g = items < cap ? items : cap;
  return (unsigned)(g == 0 ? 1 : g);
}

uint64_t grouped_workspace_bytes(uint64_t n) {
  const uint64_t hist = sort_pairs_workspace(n);
  const uint64_t scan_n = (hist > n + 1 ? hist : n + 1);
  return 16 * n + 8 * hist + 8 * scan_tiles_needed(scan_n) + 8 * (n + 1) + 8 * (n + 2) + 4 * (n / HEAVY_RUN + 1) +
         256 + 6 * 256;
}

hc_err launch_grouped_insert(const TableView& t, uint32_t W, const uint32_t* keys, const uint32_t* values, uint64_t n,
                             void* ws, hipStream_t s) {
  if (n == 0) return HC_OK;
  auto align = [](uint64_t x) { return (x + 255) & ~255ull; };
  char* p = (char*)ws;
  uint32_t* kc = (uint32_t*)p; p += align(4 * n);
  uint32_t* vc = (uint32_t*)p; p += align(4 * n);
  uint32_t* kt = (uint32_t*)p; p += align(4 * n);
  uint32_t* vt = (uint32_t*)p; p += align(4 * n);
  const uint64_t hist_n = sort_pairs_workspace(n);
  uint64_t* hist = (uint64_t*)p; p += align(8 * hist_n);
  const uint64_t scan_n = (hist_n > n + 1 ? hist_n : n + 1);
  uint64_t* tiles = (uint64_t*)p; p += align(8 * scan_tiles_needed(scan_n));
  uint64_t* flags = (uint64_t*)p; p += align(8 * (n + 1));
  uint64_t* starts = (uint64_t*)p; p += align(8 * (n + 2));
  uint32_t* heavy = (uint32_t*)p; p += align(4 * (n / HEAVY_RUN + 1));
  unsigned long long* nheavy = (unsigned long long*)p;
  hipError_t e = hipMemcpyAsync(kc, keys, 4 * n, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(vc, values, 4 * n, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return fail(HC_E_DEVICE, "grouped insert copy: %s", hipGetErrorString(e));
  if (hc_err r = sort_pairs(kc, vc, kt, vt, n, hist, tiles, s); r != HC_OK) return r;
  const unsigned g256 = (unsigned)((n + 256) / 256);
  hipLaunchKernelGGL(k_run_flags, dim3(g256), dim3(256), 0, s, kc, n, flags, nheavy);
  if (hc_err r = check_launch("run flags"); r != HC_OK) return r;
  if (hc_err r = exclusive_scan_inplace(flags, n, tiles, s); r != HC_OK) return r;
  hipLaunchKernelGGL(k_run_starts, dim3(g256), dim3(256), 0, s, flags, n, starts);
  if (hc_err r = check_launch("run starts"); r != HC_OK) return r;
  hipLaunchKernelGGL(k_heavy_list, dim3(g256), dim3(256), 0, s, starts, flags + n, n, heavy, nheavy);
  if (hc_err r = check_launch("heavy runs"); r != HC_OK) return r;
  return dispatch_w(W, [&](auto w) -> hc_err {
    constexpr int WW = decltype(w)::value;
    auto k = k_claim_runs<WW>;
    const unsigned grid = block_grid(reinterpret_cast<const void*>(k), ~0ull);
    WorkCtl ctl = work_for(0, 64, grid * (GB / 256));  // a launch slot (counters 0..2 reset by the kernel)
    hipLaunchKernelGGL(k, dim3(grid), dim3(GB), 0, s, t, ctl, kc, vc, starts, flags + n, heavy, nheavy);
    return check_launch("claim runs");
  });
}

hc_err launch_zero_u64(unsigned long long* p, uint32_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(256), 0, s, p, count);
  return check_launch("zero");
}

hc_err launch_long_count(const TableView& t, uint32_t W, const uint32_t* keys, const uint64_t* list,
                         const unsigned long long* nlong, uint64_t max_long, uint32_t budget, uint64_t* offsets,
                         uint32_t* counts, hipStream_t s) {
  return dispatch_w(W, [&](auto w) -> hc_err {
    constexpr int WW = decltype(w)::value;
    auto k = k_long_count<WW>;
    const unsigned grid = block_grid(reinterpret_cast<const void*>(k), max_long);
    WorkCtl ctl = work_for(0, 64, grid * (GB / 256));
    hipLaunchKernelGGL(k, dim3(grid), dim3(GB), 0, s, t, ctl, keys, list, nlong, budget, offsets, counts);
    return check_launch("long count");
  });
}

hc_err launch_long_write(const TableView& t, uint32_t W, const uint32_t* keys, const uint64_t* list,
                         const unsigned long long* nlong, uint64_t max_long, uint32_t budget, const uint64_t* offsets,
                         uint32_t* out, hipStream_t s) {
  return dispatch_w(W, [&](auto w) -> hc_err {
    constexpr int WW = decltype(w)::value;
    auto k = k_long_write<WW>;
    const unsigned grid = block_grid(reinterpret_cast<const void*>(k), max_long);
    WorkCtl ctl = work_for(0, 64, grid * (GB / 256));
    hipLaunchKernelGGL(k, dim3(grid), dim3(GB), 0, s, t, ctl, keys, list, nlong, budget, offsets, out);
    return check_launch("long write");
  });
}

}  // namespace hc
