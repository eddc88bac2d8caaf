// C ABI of the cooperative-probing hash tables: handles, allocation, argument
// checks, stream ordering, the prefix sum of the multi-value count pass and the
// table fill kernel.  Kernels of the bulk operations live in hc_k_*.hip.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <algorithm>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "hc.h"
#include "hc_batch.hpp"
#include "hc_bucket.hpp"
#include "hc_set.hpp"
#include "hc_wide.hpp"
#include "hc_device.hpp"
#include "hc_group.hpp"
#include "hc_stats.hpp"
#include "hc_launch.hpp"
#include "hc_sort.hpp"

struct hc_batch_s {
  int device = 0;
  uint32_t phases = 0;
  std::vector<hc::PlanLaunch> launches;  // in phase order
  hc::BatchDesc* d_descs = nullptr;
  uint64_t* d_chunk_start = nullptr;
  // work counters of the plan's own launches (not the shared launch-slot ring), so a
  // captured graph never shares counters with launches made outside it
  unsigned long long* d_counters = nullptr;
  uint32_t gates = 0;       // one-launch plans: completion counters after the launch counters
  uint64_t wait_ticks = 0;  // device clock ticks after which a completion wait is abandoned
};

struct hc_table_s {
  int device;
  uint32_t kind, scheme, window, group;
  uint64_t P, C, seed;
  uint64_t* slots;
  unsigned long long* d_size;  // counter block: size, bucket pool, failed claim CASes
  bool owns_slots;        // false: caller-owned slot array (hc_create_in)
  // grouped and bucket list inserts of one table run one after another: each waits on the
  // device for the event recorded after the previous one, whatever stream it is issued on
  hipEvent_t order_ev = nullptr;
  bool order_pending = false;
  // bucket list tables (kind HC_BUCKET_LIST)
  uint64_t* d_cum = nullptr;       // cumulative bucket sizes of the ramp
  uint32_t bl_m = 0, bl_smax = 0, bl_s0 = 1;
  uint32_t* d_pool = nullptr;
  uint64_t pool_cap = 0;
  ulonglong2* d_meta = nullptr;  // per slot: buckets held (and before the latest batch), last and first new bucket
};

namespace hc {

// ---- table fill ----------------------------------------------------------------

__global__ __launch_bounds__(BLOCK) void k_fill_empty(ulonglong2* __restrict__ slots, uint64_t pairs,
                                                      unsigned long long* __restrict__ size) {
  const uint64_t stride = (uint64_t)gridDim.x * BLOCK;
  const ulonglong2 z = {0ull, 0ull};
  for (uint64_t i = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; i < pairs; i += stride) slots[i] = z;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    size[CTR_SIZE] = 0ull;
    size[CTR_CAS_FAILS] = 0ull;
  }
}

// ---- exclusive prefix sum, in place, n counts -> n+1 offsets --------------------
// Three launches: per-tile sums, one-block scan of the tile sums (also writing
// offsets[n] = total), per-tile scan plus the tile's prefix.

constexpr int SCAN_ITEMS = 8;
constexpr uint64_t SCAN_TILE = (uint64_t)BLOCK * SCAN_ITEMS;

// Block-wide exclusive scan of one value per thread; returns the prefix, *total the sum.
__device__ uint64_t block_exclusive_scan(uint64_t x, uint64_t* total) {
  __shared__ uint64_t wave_tot[BLOCK / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t incl = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t lo = __shfl_up((uint32_t)incl, d, 64);
    const uint32_t hi = __shfl_up((uint32_t)(incl >> 32), d, 64);
    if (lane >= d) incl += (uint64_t)lo | ((uint64_t)hi << 32);
  }
  if (lane == 63) wave_tot[wave] = incl;
  __syncthreads();
  uint64_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < BLOCK / 64; ++w) {
    if (w < wave) before += wave_tot[w];
    all += wave_tot[w];
  }
  __syncthreads();
  *total = all;
  return before + incl - x;
}

// Tile sums: coalesced loads (a sum does not care about order), one block reduction.
__global__ __launch_bounds__(BLOCK) void k_scan_tile_sums(const uint64_t* __restrict__ a, uint64_t n,
                                                          uint64_t* __restrict__ tiles) {
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + threadIdx.x;
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) {
    const uint64_t i = base + (uint64_t)j * BLOCK;
    if (i < n) s += a[i];
  }
  uint64_t total;
  block_exclusive_scan(s, &total);
  if (threadIdx.x == 0) tiles[blockIdx.x] = total;
}

__global__ __launch_bounds__(BLOCK) void k_scan_tiles(uint64_t* __restrict__ tiles, uint64_t ntiles,
                                                      uint64_t* __restrict__ offsets, uint64_t n) {
  uint64_t carry = 0;
  for (uint64_t c = 0; c < ntiles; c += SCAN_TILE) {
    const uint64_t base = c + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint64_t v[SCAN_ITEMS];
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
      v[j] = (base + j < ntiles) ? tiles[base + j] : 0;
      s += v[j];
    }
    uint64_t total;
    uint64_t p = carry + block_exclusive_scan(s, &total);
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
      if (base + j < ntiles) tiles[base + j] = p;
      p += v[j];
    }
    carry += total;
  }
  if (threadIdx.x == 0) offsets[n] = carry;
}

// Apply: the tile goes through LDS so that global loads and stores are coalesced while each
// thread scans SCAN_ITEMS consecutive elements.
__global__ __launch_bounds__(BLOCK) void k_scan_apply(uint64_t* __restrict__ a, uint64_t n,
                                                      const uint64_t* __restrict__ tiles) {
  __shared__ uint64_t buf[SCAN_TILE];
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) {
    const uint64_t i = base + (uint64_t)j * BLOCK + threadIdx.x;
    buf[j * BLOCK + threadIdx.x] = i < n ? a[i] : 0;
  }
  __syncthreads();
  uint64_t v[SCAN_ITEMS];
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) {
    v[j] = buf[threadIdx.x * SCAN_ITEMS + j];
    s += v[j];
  }
  uint64_t total;
  uint64_t p = tiles[blockIdx.x] + block_exclusive_scan(s, &total);
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) {
    buf[threadIdx.x * SCAN_ITEMS + j] = p;
    p += v[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) {
    const uint64_t i = base + (uint64_t)j * BLOCK + threadIdx.x;
    if (i < n) a[i] = buf[j * BLOCK + threadIdx.x];
  }
}

uint64_t scan_tiles_needed(uint64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

hc_err exclusive_scan_inplace(uint64_t* a, uint64_t n, uint64_t* tiles, hipStream_t s) {
  const uint64_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (n > 0) {
    hipLaunchKernelGGL(k_scan_tile_sums, dim3((unsigned)ntiles), dim3(BLOCK), 0, s, a, n, tiles);
    if (hc_err r = check_launch("scan tile sums"); r != HC_OK) return r;
  }
  hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(BLOCK), 0, s, tiles, ntiles, a, n);
  if (hc_err r = check_launch("scan tiles"); r != HC_OK) return r;
  if (n > 0) {
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)ntiles), dim3(BLOCK), 0, s, a, n, tiles);
    if (hc_err r = check_launch("scan apply"); r != HC_OK) return r;
  }
  return HC_OK;
}

// Ordered inserts (grouped, bucket list): wait for the table's previous one, on the device.
static hc_err order_begin(hc_table_s* t, hipStream_t s) {
  if (t->order_ev == nullptr) {
    const hipError_t e = hipEventCreateWithFlags(&t->order_ev, hipEventDisableTiming);
    if (e != hipSuccess) {
      t->order_ev = nullptr;
      return hip_fail(e, "ordering event");
    }
  }
  if (t->order_pending) {
    const hipError_t e = hipStreamWaitEvent(s, t->order_ev, 0);
    if (e != hipSuccess) return hip_fail(e, "ordering wait");
  }
  return HC_OK;
}

static hc_err order_end(hc_table_s* t, hipStream_t s, hc_err r) {
  if (r != HC_OK) return r;
  const hipError_t e = hipEventRecord(t->order_ev, s);
  if (e != hipSuccess) return hip_fail(e, "ordering record");
  t->order_pending = true;
  return HC_OK;
}

static bool is_wide(uint32_t kind) { return kind == HC_SINGLE_VALUE_64 || kind == HC_SINGLE_VALUE_64_SOA; }

static uint64_t slot_bytes(uint32_t kind) { return is_wide(kind) ? 16 : kind == HC_HASH_SET ? 4 : 8; }

static BucketView bview_of(const hc_table_s* t) {
  BucketView b{};
  b.cum = t->d_cum;
  b.m = t->bl_m;
  b.smax = t->bl_smax;
  b.pool = t->d_pool;
  b.pool_cap = t->pool_cap;
  b.s0 = t->bl_s0;
  b.bump = t->C * t->bl_s0;     // the first C * s0 words hold the slots' first buckets
  b.pool_next = t->d_size + 1;  // the size counter and the pool counter share one allocation
  b.meta = t->d_meta;
  return b;
}

// 32-bit entry points on a 64-bit table.
static hc_err not_wide(hc_table t, const char* what) {
  if (t != nullptr && is_wide(t->kind))
    return fail(HC_E_KIND, "%s: 64-bit tables take hc_insert64 / hc_retrieve64 / hc_erase64", what);
  return HC_OK;
}

// Table-only entry points on a set.
static hc_err not_set(hc_table t, const char* what) {
  if (t != nullptr && t->kind == HC_HASH_SET)
    return fail(HC_E_KIND, "%s: sets take hc_insert / hc_retrieve / hc_erase", what);
  return HC_OK;
}

static TableView view_of(const hc_table_s* t) {
  TableView v;
  v.slots = t->slots;
  v.size = t->d_size;
  v.P = (uint32_t)t->P;
  v.pow2 = (t->P & (t->P - 1)) == 0;
  v.pmask = v.pow2 ? (uint32_t)(t->P - 1) : 0u;
  v.scheme = t->scheme;
  v.seed_lo = (uint32_t)t->seed;
  v.seed_hi = (uint32_t)(t->seed >> 32);
  return v;
}

static bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }

static bool is_prime(uint64_t x) {
  if (x < 2) return false;
  if (x % 2 == 0) return x == 2;
  for (uint64_t d = 3; d * d <= x; d += 2)
    if (x % d == 0) return false;
  return true;
}

static hc_err check_table(hc_table t) {
  if (t == nullptr) return fail(HC_E_ARG, "table handle is NULL");
  return HC_OK;
}

static hc_err resolve_group(hc_table t, uint32_t group, uint32_t* out) {
  const uint32_t g = group ? group : t->group;
  if (!is_pow2(g) || g > 64) return fail(HC_E_ARG, "group size %u is not a power of two in [1, 64]", g);
  *out = g;
  return HC_OK;
}

static hc_err set_device(hc_table t) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(HC_E_DEVICE, "hipGetDevice failed");
  if (cur != t->device) {
    const hipError_t e = hipSetDevice(t->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  }
  return HC_OK;
}

}  // namespace hc

namespace hc {

struct PlanItem {
  uint32_t phase, op, G, W;
  uint32_t index;  // into ops
};

// Chunk size of an operation of n elements with group size G in a launch whose
// per-wavefront share is per_wave elements: about two chunks per resident wavefront
// over the whole launch, between one element per group and 64 elements per group of a
// wavefront.
static uint32_t chunk_of(uint64_t n, uint32_t G, uint64_t per_wave) {
  const uint64_t gpw = 64 / G;
  uint64_t ch = per_wave < gpw ? gpw : per_wave;
  if (ch > 64 * gpw) ch = 64 * gpw;
  return (uint32_t)(n < ch ? n : ch);
}

// Every phase in one launch (items with phases assigned, list order kept): descriptors in
// (phase, list) order; a table's descriptors in phase p wait for the completion counter of
// the table's latest earlier phase that has elements, and post to their own (table, phase)
// counter if a later phase of the table waits for it.
static hc_err build_one_launch(const hc_batch_op* ops, std::vector<PlanItem>& items, uint32_t phases,
                               PlanHost* out) {
  out->phases = phases;
  if (items.empty()) return HC_OK;
  for (const PlanItem& x : items)
    if (x.G != items[0].G || x.W != items[0].W)
      return fail(HC_E_ARG, "a one-launch plan needs one group size and window for every operation "
                            "(op %u has g = %u, W = %u; op %u has g = %u, W = %u)",
                  items[0].index, items[0].G, items[0].W, x.index, x.G, x.W);
  std::stable_sort(items.begin(), items.end(),
                   [](const PlanItem& a, const PlanItem& b) { return a.phase < b.phase; });
  const uint64_t waves = (uint64_t)device_cu_count() * 32;
  uint64_t total = 0;
  for (const PlanItem& x : items) total += ops[x.index].n;
  const uint64_t per_wave = (total + 2 * waves - 1) / (2 * waves);
  // (table, phase) groups: own completion counter and the counter they wait for
  struct Group {
    uint32_t phase, gate, wait;
  };
  std::unordered_map<const hc_table_s*, Group> cur;  // each table's latest group so far
  std::vector<uint64_t> gate_chunks;                 // chunks per counter
  std::vector<uint8_t> gate_used;                    // a later group waits for it
  uint64_t chunks = 0;
  for (const PlanItem& x : items) {
    const hc_batch_op& o = ops[x.index];
    auto it = cur.find(o.table);
    if (it == cur.end() || it->second.phase != x.phase) {  // a new (table, phase) group
      const uint32_t prev = it == cur.end() ? NO_GATE : it->second.gate;
      if (prev != NO_GATE) gate_used[prev] = 1;
      cur[o.table] = Group{x.phase, (uint32_t)gate_chunks.size(), prev};
      gate_chunks.push_back(0);
      gate_used.push_back(0);
      it = cur.find(o.table);
    }
    BatchDesc d;
    d.t = view_of(o.table);
    d.keys = o.d_keys;
    d.values = o.d_values;
    d.values_out = o.d_values_out;
    d.flags = o.d_flags;
    d.n = o.n;
    d.chunk = chunk_of(o.n, x.G, per_wave);
    d.op = x.op;
    d.variant = MIXED_NONE;
    d.pad = 0;
    d.gate_need = 0;
    d.gate_wait = it->second.wait;
    d.gate_post = it->second.gate;
    const uint64_t nch = (o.n + d.chunk - 1) / d.chunk;
    gate_chunks[it->second.gate] += nch;
    out->descs.push_back(d);
    out->cs.push_back(chunks);
    chunks += nch;
  }
  out->cs.push_back(chunks);
  // counters nobody waits for are dropped; the others get compact ids
  std::vector<uint32_t> id(gate_chunks.size(), NO_GATE);
  uint32_t ngates = 0;
  for (size_t g = 0; g < gate_chunks.size(); ++g)
    if (gate_used[g]) id[g] = ngates++;
  for (BatchDesc& d : out->descs) {
    if (d.gate_wait != NO_GATE) {
      d.gate_need = gate_chunks[d.gate_wait];
      d.gate_wait = id[d.gate_wait];
    }
    d.gate_post = id[d.gate_post];
  }
  out->gates = ngates;
  PlanLaunch L;
  L.op = BATCH_ALL;
  L.G = items[0].G;
  L.W = items[0].W;
  L.first_desc = 0;
  L.ndesc = (uint32_t)out->descs.size();
  L.cs_offset = 0;
  L.total_chunks = chunks;
  out->launches.push_back(L);
  return HC_OK;
}

// Validate `ops`, assign phases (a table's phase advances where its operation kind
// changes) and lay out the per-launch descriptor groups on the host.
hc_err build_plan(const hc_batch_op* ops, uint32_t count, int dev, PlanHost* out, bool one_launch) {
  out->descs.clear();
  out->cs.clear();
  out->launches.clear();
  out->phases = 0;
  out->gates = 0;
  if (count > 0 && ops == nullptr) return fail(HC_E_ARG, "ops is NULL");
  std::vector<PlanItem> items;
  items.reserve(count);
  std::unordered_map<const hc_table_s*, std::pair<uint32_t, uint32_t>> last;  // table -> (phase, op)
  uint32_t phases = 0;
  for (uint32_t j = 0; j < count; ++j) {
    const hc_batch_op& o = ops[j];
    if (o.table == nullptr) return fail(HC_E_ARG, "op %u: table is NULL", j);
    const hc_table_s* t = o.table;
    if (t->kind == HC_MULTI_VALUE || t->kind == HC_BUCKET_LIST || is_wide(t->kind) || t->kind == HC_HASH_SET)
      return fail(HC_E_KIND, "op %u: batched operations take single-value or counting tables", j);
    if (t->device != dev) return fail(HC_E_ARG, "op %u: table lives on device %d, current device is %d", j, t->device, dev);
    if (o.op > HC_OP_ERASE) return fail(HC_E_ARG, "op %u: unknown operation %u", j, o.op);
    uint32_t g;
    if (hc_err r = resolve_group(o.table, o.group, &g); r != HC_OK) return r;
    if (o.n > 0 && o.d_keys == nullptr) return fail(HC_E_ARG, "op %u: keys is NULL", j);
    uint32_t bop = o.op == HC_OP_RETRIEVE ? BATCH_RETRIEVE : o.op == HC_OP_ERASE ? BATCH_ERASE : BATCH_INSERT;
    if (o.op == HC_OP_INSERT) {
      if (t->kind == HC_COUNTING) {
        if (o.d_values != nullptr) return fail(HC_E_ARG, "op %u: counting tables take no values", j);
        bop = BATCH_COUNT;
      } else if (o.n > 0 && o.d_values == nullptr) {
        return fail(HC_E_ARG, "op %u: values is NULL", j);
      }
    }
    uint32_t phase = 0;
    auto it = last.find(t);
    if (it != last.end()) phase = it->second.first + (it->second.second == o.op ? 0u : 1u);
    last[t] = {phase, o.op};
    if (phase + 1 > phases) phases = phase + 1;
    if (o.n > 0) items.push_back({phase, bop, g, t->window, j});
  }
  if (one_launch) return build_one_launch(ops, items, phases, out);
  // Launches: one per (phase, kind, G, W) group, list order kept inside each group.
  // Where a (phase, kind) has several pairs, those of the mixed-launch set share one
  // mixed launch (G = W = 0 below); pairs outside the set keep launches of their own.
  auto pair_key = [](const PlanItem& x) { return (x.G << 8) | x.W; };
  std::stable_sort(items.begin(), items.end(), [](const PlanItem& a, const PlanItem& b) {
    if (a.phase != b.phase) return a.phase < b.phase;
    return a.op < b.op;
  });
  std::vector<uint8_t> mixed(items.size(), 0);
  for (size_t a = 0; a < items.size();) {
    size_t e = a;
    bool several = false;
    while (e < items.size() && items[e].phase == items[a].phase && items[e].op == items[a].op) {
      several |= pair_key(items[e]) != pair_key(items[a]);
      ++e;
    }
    if (several)
      for (size_t q = a; q < e; ++q) mixed[q] = mixed_variant(items[q].G, items[q].W) != MIXED_NONE;
    a = e;
  }
  std::vector<size_t> order(items.size());
  for (size_t q = 0; q < order.size(); ++q) order[q] = q;
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
    const PlanItem &a = items[x], &b = items[y];
    if (a.phase != b.phase) return a.phase < b.phase;
    if (a.op != b.op) return a.op < b.op;
    if (mixed[x] != mixed[y]) return mixed[x] > mixed[y];
    return mixed[x] ? false : pair_key(a) < pair_key(b);
  });
  const uint64_t waves = (uint64_t)device_cu_count() * 32;
  out->phases = phases;
  for (size_t a = 0; a < order.size();) {
    const PlanItem& f = items[order[a]];
    const bool mix = mixed[order[a]] != 0;
    size_t e = a;
    while (e < order.size()) {
      const PlanItem& x = items[order[e]];
      if (x.phase != f.phase || x.op != f.op || (mixed[order[e]] != 0) != mix) break;
      if (!mix && pair_key(x) != pair_key(f)) break;
      ++e;
    }
    PlanLaunch L;
    L.op = f.op;
    L.G = mix ? 0 : f.G;
    L.W = mix ? 0 : f.W;
    L.first_desc = (uint32_t)out->descs.size();
    L.ndesc = (uint32_t)(e - a);
    L.cs_offset = out->cs.size();
    uint64_t total = 0;
    for (size_t q = a; q < e; ++q) total += ops[items[order[q]].index].n;
    const uint64_t per_wave = (total + 2 * waves - 1) / (2 * waves);
    uint64_t chunks = 0;
    for (size_t q = a; q < e; ++q) {
      const PlanItem& x = items[order[q]];
      const hc_batch_op& o = ops[x.index];
      BatchDesc d;
      d.t = view_of(o.table);
      d.keys = o.d_keys;
      d.values = o.d_values;
      d.values_out = o.d_values_out;
      d.flags = o.d_flags;
      d.n = o.n;
      d.chunk = chunk_of(o.n, x.G, per_wave);
      d.op = L.op;
      d.variant = mix ? mixed_variant(x.G, x.W) : MIXED_NONE;
      d.gate_post = d.gate_wait = NO_GATE;
      d.pad = 0;
      d.gate_need = 0;
      out->descs.push_back(d);
      out->cs.push_back(chunks);
      chunks += (o.n + d.chunk - 1) / d.chunk;
    }
    out->cs.push_back(chunks);
    L.total_chunks = chunks;
    out->launches.push_back(L);
    a = e;
  }
  return HC_OK;
}

hc_err launch_plan(const std::vector<PlanLaunch>& launches, const BatchDesc* d_descs, const uint64_t* d_cs,
                   unsigned long long* counters, hipStream_t stream, uint32_t gates, uint64_t wait_ticks) {
  for (size_t j = 0; j < launches.size(); ++j) {
    const PlanLaunch& L = launches[j];
    unsigned long long* c = counters ? counters + j * PLAN_COUNTER_STRIDE : nullptr;
    if (L.op == BATCH_ALL) {
      unsigned long long* extra = counters ? counters + launches.size() * PLAN_COUNTER_STRIDE : nullptr;
      hc_err r = launch_batch_one(L.G, L.W, d_descs + L.first_desc, d_cs + L.cs_offset, L.ndesc, L.total_chunks, c,
                                  extra ? extra + PLAN_COUNTER_STRIDE : nullptr, gates, extra, wait_ticks, stream);
      if (r != HC_OK) return r;
      continue;
    }
    hc_err r = L.G == 0 ? launch_batch_mixed(L.op, d_descs + L.first_desc, d_cs + L.cs_offset, L.ndesc,
                                             L.total_chunks, c, stream)
                        : launch_batch(L.op, L.G, L.W, d_descs + L.first_desc, d_cs + L.cs_offset, L.ndesc,
                                       L.total_chunks, c, stream);
    if (r != HC_OK) return r;
  }
  return HC_OK;
}

}  // namespace hc

namespace hc {

// Workspace of a count pass: the scan's tile sums, then the long-query state (multi-value
// tables, `cap` hand-over entries).
static uint64_t count_values_ws_bytes(uint64_t n, uint64_t cap) {
  const uint64_t tiles = (8 * scan_tiles_needed(n) + 255) & ~255ull;
  return tiles + (cap ? long_workspace_bytes(cap, 0) : 0);
}

// Count pass and exclusive scan of hc_count_values in the workspace `ws` (count_values_ws_bytes).
static hc_err count_values_in(hc_table_s* t, const uint32_t* d_keys, uint64_t n, uint32_t* d_counts,
                              uint64_t* d_offsets, uint32_t g, void* ws, uint64_t cap, hipStream_t s) {
  hc_err r = HC_OK;
  uint64_t* tiles = static_cast<uint64_t*>(ws);
  void* lws = static_cast<char*>(ws) + ((8 * scan_tiles_needed(n) + 255) & ~255ull);
  if (n > 0 && t->kind == HC_BUCKET_LIST) {  // the count sits in the key's slot
    if ((r = launch_bl_count(view_of(t), g, t->window, d_keys, n, d_counts, d_offsets, s)) != HC_OK) return r;
  } else if (n > 0) {
    // queries still open after LONG_BUDGET windows are finished by block-wide segment rounds
    const LongState ls = long_layout(lws, cap, 0);
    if ((r = launch_zero_u64((unsigned long long*)ls.nlong, 1, s)) != HC_OK) return r;
    if ((r = launch_count_multi(view_of(t), g, t->window, d_keys, n, d_counts, d_offsets, nullptr, LONG_BUDGET,
                                ls.entries, (unsigned long long*)ls.nlong, cap, s)) != HC_OK)
      return r;
    if ((r = launch_long_queries(view_of(t), t->window, 0, d_keys, ls, n, LONG_BUDGET, d_offsets, d_counts, nullptr,
                                 s)) != HC_OK)
      return r;
  }
  return exclusive_scan_inplace(d_offsets, n, tiles, s);
}

}  // namespace hc

using namespace hc;

extern "C" {

void hc_default_params(hc_params* p) {
  if (!p) return;
  p->scheme = HC_DOUBLE;
  p->window = 16;
  p->group = 4;
  p->reserved = 0;
  p->seed = 0x5EED0F0C0A5CAD1Eull;
}

// Validated parameters and the rounded window count P (Sec. IV-B2 cycle-free rule).
static hc_err table_geometry(uint64_t capacity, const hc_params* params, hc_params* p, uint64_t* P_out) {
  hc_default_params(p);
  if (params) *p = *params;
  if (p->scheme > 2) return fail(HC_E_ARG, "unknown probing scheme %u", p->scheme);
  if (!(p->window == 8 || p->window == 16 || p->window == 32 || p->window == 64))
    return fail(HC_E_ARG, "window %u is not one of 8, 16, 32, 64", p->window);
  if (!is_pow2(p->group) || p->group > 64)
    return fail(HC_E_ARG, "group size %u is not a power of two in [1, 64]", p->group);
  if (p->reserved != 0) return fail(HC_E_ARG, "params.reserved must be 0");
  if (capacity == 0) return fail(HC_E_ARG, "capacity must be positive");
  if (capacity > (1ull << 40)) return fail(HC_E_ARG, "capacity %llu too large", (unsigned long long)capacity);
  uint64_t P = (capacity + p->window - 1) / p->window;
  if (p->scheme == HC_QUADRATIC) {
    uint64_t q = 1;
    while (q < P) q <<= 1;
    P = q;
  } else if (p->scheme == HC_DOUBLE && !is_pow2(P)) {
    while (!is_prime(P)) ++P;
  }
  if (P > (1ull << 31)) return fail(HC_E_ARG, "window count %llu exceeds 2^31", (unsigned long long)P);
  *P_out = P;
  return HC_OK;
}

static hc_err create_table(hc_table* out, uint32_t kind, uint64_t capacity, const hc_params* params,
                           void* ext_slots, uint64_t ext_bytes) {
  if (out == nullptr) return fail(HC_E_ARG, "out is NULL");
  *out = nullptr;
  if (kind > HC_SINGLE_VALUE_64_SOA) return fail(HC_E_ARG, "unknown table kind %u", kind);
  hc_params p;
  uint64_t P = 0;
  if (hc_err r = table_geometry(capacity, params, &p, &P); r != HC_OK) return r;
  if (is_wide(kind) && p.group > p.window)
    return fail(HC_E_ARG, "64-bit tables need group <= window (group %u, window %u)", p.group, p.window);
  if (kind == HC_HASH_SET && p.group > p.window)
    return fail(HC_E_ARG, "sets need group <= window (group %u, window %u)", p.group, p.window);
  if (ext_slots != nullptr) {
    if ((reinterpret_cast<uintptr_t>(ext_slots) & 255) != 0) return fail(HC_E_ARG, "slot array is not 256-byte aligned");
    if (ext_bytes < P * p.window * slot_bytes(kind))
      return fail(HC_E_ARG, "slot array holds %llu bytes, the table needs %llu", (unsigned long long)ext_bytes,
                  (unsigned long long)(P * p.window * slot_bytes(kind)));
  }
  hc_table_s* t = new (std::nothrow) hc_table_s();
  if (!t) return fail(HC_E_NOMEM, "host allocation failed");
  if (hipGetDevice(&t->device) != hipSuccess) {
    delete t;
    return fail(HC_E_DEVICE, "hipGetDevice failed");
  }
  if (hc_err re = ensure_ring(t->device); re != HC_OK) {
    delete t;
    return re;
  }
  t->kind = kind;
  t->scheme = p.scheme;
  t->window = p.window;
  t->group = p.group;
  t->P = P;
  t->C = P * p.window;
  t->seed = p.seed;
  t->owns_slots = ext_slots == nullptr;
  if (ext_slots != nullptr) {
    t->slots = static_cast<uint64_t*>(ext_slots);
  } else {
    hipError_t e = hipMalloc((void**)&t->slots, t->C * slot_bytes(kind));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      delete t;
      return fail(HC_E_NOMEM, "hipMalloc of %llu slots failed: %s", (unsigned long long)t->C, hipGetErrorString(e));
    }
  }
  hipError_t e = hipMalloc((void**)&t->d_size, 256);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    if (t->owns_slots) (void)hipFree(t->slots);
    delete t;
    return fail(HC_E_NOMEM, "hipMalloc of the size counter failed");
  }
  hc_err r = hc_clear(t, nullptr);
  if (r == HC_OK) {
    e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) r = hip_fail(e, "hc_create: synchronise");
  }
  if (r != HC_OK) {
    if (t->owns_slots) (void)hipFree(t->slots);
    (void)hipFree(t->d_size);
    delete t;
    return r;
  }
  *out = t;
  return HC_OK;
}

hc_err hc_create(hc_table* out, uint32_t kind, uint64_t capacity, const hc_params* params) {
  if (kind == HC_BUCKET_LIST) {
    if (out) *out = nullptr;
    return fail(HC_E_ARG, "bucket list tables are made by hc_create_bucket_list");
  }
  return create_table(out, kind, capacity, params, nullptr, 0);
}

void hc_default_bucket_params(hc_bucket_params* p) {
  p->pool_values = 0;  // 0: s0 + 3 words per key slot
  p->s0 = 1;
  p->smax = 1u << 16;
  p->growth = 2.0;
}

hc_err hc_create_bucket_list(hc_table* out, uint64_t key_capacity, const hc_params* params,
                             const hc_bucket_params* bparams) {
  if (out == nullptr) return fail(HC_E_ARG, "out is NULL");
  *out = nullptr;
  hc_bucket_params bp;
  hc_default_bucket_params(&bp);
  if (bparams) bp = *bparams;
  if (bp.s0 == 0 || bp.smax < bp.s0 || bp.smax > (1u << 24))
    return fail(HC_E_ARG, "bucket sizes need 1 <= s0 <= smax <= 2^24 (s0 %u, smax %u)", bp.s0, bp.smax);
  if (!(bp.growth >= 1.0 && bp.growth <= 64.0)) return fail(HC_E_ARG, "growth factor must lie in [1, 64]");
  std::vector<uint64_t> cum(BL_MAX_RAMP + 1);
  uint32_t m = 0;
  if (!bucket_ramp(bp.s0, bp.growth, bp.smax, cum.data(), &m))
    return fail(HC_E_ARG, "bucket sizes take more than %u steps to reach smax", BL_MAX_RAMP);
  hc_table t = nullptr;
  hc_err r = create_table(&t, HC_BUCKET_LIST, key_capacity, params, nullptr, 0);
  if (r != HC_OK) return r;
  const uint64_t pool = bp.pool_values ? bp.pool_values : ((uint64_t)bp.s0 + 3) * t->C;
  if (pool > 0xFFFFFFFFull) {
    hc_destroy(t);
    return fail(HC_E_ARG, "pool of %llu words exceeds 2^32 - 1", (unsigned long long)pool);
  }
  if (pool < (uint64_t)bp.s0 * t->C) {
    const uint64_t need = (uint64_t)bp.s0 * t->C;
    hc_destroy(t);
    return fail(HC_E_ARG, "pool of %llu words is smaller than the first buckets of the %llu key slots (%llu words)",
                (unsigned long long)pool, (unsigned long long)(need / bp.s0), (unsigned long long)need);
  }
  t->bl_s0 = bp.s0;
  t->bl_m = m;
  t->bl_smax = bp.smax;
  t->pool_cap = pool;
  hipError_t e = hipMalloc((void**)&t->d_cum, (m + 1) * sizeof(uint64_t));
  if (e == hipSuccess) e = hipMalloc((void**)&t->d_pool, pool * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc((void**)&t->d_meta, t->C * sizeof(ulonglong2));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    hc_destroy(t);
    return fail(HC_E_NOMEM, "bucket list allocation failed");
  }
  e = hipMemcpy(t->d_cum, cum.data(), (m + 1) * sizeof(uint64_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hc_destroy(t);
    return hip_fail(e, "bucket sizes upload");
  }
  r = hc_clear(t, nullptr);
  if (r == HC_OK && (e = hipStreamSynchronize(nullptr)) != hipSuccess) r = hip_fail(e, "hc_create_bucket_list");
  if (r != HC_OK) {
    hc_destroy(t);
    return r;
  }
  *out = t;
  return HC_OK;
}

hc_err hc_bucket_usage(hc_table t, hc_bucket_usage_t* h_out, void* stream) {
  hc_err r = check_table(t);
  if (r != HC_OK) return r;
  if (h_out == nullptr) return fail(HC_E_ARG, "out is NULL");
  if (t->kind != HC_BUCKET_LIST) return fail(HC_E_KIND, "bucket usage needs a bucket list table");
  if ((r = set_device(t)) != HC_OK) return r;
  unsigned long long v[2] = {0, 0};
  hipError_t e = hipMemcpyAsync(v, t->d_size, sizeof v, hipMemcpyDeviceToHost, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hc_bucket_usage");
  h_out->values = v[0];
  const uint64_t used = t->C * t->bl_s0 + v[1];  // the slots' first buckets, then the allocated ones
  h_out->pool_used = used < t->pool_cap ? used : t->pool_cap;
  h_out->pool_words = t->pool_cap;
  h_out->smax = t->bl_smax;
  return HC_OK;
}

hc_err hc_dump_buckets(hc_table t, uint32_t* d_pool_dst, uint32_t* d_last_dst, void* stream) {
  hc_err r = check_table(t);
  if (r != HC_OK) return r;
  if (t->kind != HC_BUCKET_LIST) return fail(HC_E_KIND, "bucket dump needs a bucket list table");
  if (d_pool_dst == nullptr || d_last_dst == nullptr) return fail(HC_E_ARG, "destination is NULL");
  if ((r = set_device(t)) != HC_OK) return r;
  hipError_t e = hipMemcpyAsync(d_pool_dst, t->d_pool, t->pool_cap * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                                (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hc_dump_buckets");
  return launch_bl_dump_last(bview_of(t), t->C, d_last_dst, (hipStream_t)stream);
}

hc_err hc_create_in(hc_table* out, uint32_t kind, void* d_slots, uint64_t slot_bytes, uint64_t capacity,
                    const hc_params* params) {
  if (d_slots == nullptr) {
    if (out) *out = nullptr;
    return fail(HC_E_ARG, "slot array is NULL");
  }
  return create_table(out, kind, capacity, params, d_slots, slot_bytes);
}

hc_err hc_table_bytes(uint64_t capacity, const hc_params* params, uint64_t* h_out) {
  if (h_out == nullptr) return fail(HC_E_ARG, "out is NULL");
  hc_params p;
  uint64_t P = 0;
  if (hc_err r = table_geometry(capacity, params, &p, &P); r != HC_OK) return r;
  *h_out = P * p.window * sizeof(uint64_t);
  return HC_OK;
}

hc_err hc_destroy(hc_table t) {
  if (t == nullptr) return HC_OK;
  hc_err r = set_device(t);
  if (r != HC_OK) return r;
  hipError_t e = hipDeviceSynchronize();
  if (t->slots && t->owns_slots) (void)hipFree(t->slots);
  if (t->d_size) (void)hipFree(t->d_size);
  if (t->order_ev) (void)hipEventDestroy(t->order_ev);
  for (void* q : {(void*)t->d_cum, (void*)t->d_pool, (void*)t->d_meta})
    if (q) (void)hipFree(q);
  delete t;
  if (e != hipSuccess) return hip_fail(e, "hc_destroy: synchronise");
  return HC_OK;
}

hc_err hc_clear(hc_table t, void* stream) {
  hc_err r = check_table(t);
  if (r != HC_OK) return r;
  if ((r = set_device(t)) != HC_OK) return r;
  const uint64_t pairs = t->C * slot_bytes(t->kind) / 16;  // 16-byte stores; C = P * W with W >= 8: even
  uint64_t blocks = (pairs + BLOCK - 1) / BLOCK;
  const uint64_t cap = (uint64_t)device_cu_count() * 16;
  if (blocks > cap) blocks = cap;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_fill_empty, dim3((unsigned)blocks), dim3(BLOCK), 0, (hipStream_t)stream,
                     reinterpret_cast<ulonglong2*>(t->slots), pairs, t->d_size);
  if ((r = check_launch("clear")) != HC_OK) return r;
  if (t->kind == HC_BUCKET_LIST && t->d_meta != nullptr) {  // empty pool, records of no buckets (once allocated)
    if ((r = launch_zero_u64(t->d_size + 1, 1, (hipStream_t)stream)) != HC_OK) return r;
    if ((r = launch_bl_reset(bview_of(t), t->C, (hipStream_t)stream)) != HC_OK) return r;
  }
  return HC_OK;
}

hc_err hc_insert(hc_table t, const uint32_t* d_keys, const uint32_t* d_values, uint64_t n, uint8_t* d_status,
                 uint32_t group, void* stream) {
  hc_err r = check_table(t);
  if (r != HC_OK) return r;
  if ((r = not_wide(t, "hc_insert")) != HC_OK) return r;
  uint32_t g;
  if ((r = resolve_group(t, group, &g)) != HC_OK) return r;
  if (n == 0) return HC_OK;
  if (d_keys == nullptr) return fail(HC_E_ARG, "keys is NULL");
  if (t->kind == HC_HASH_SET) {
    if (d_values != nullptr) return fail(HC_E_ARG, "sets take no values");
    if ((r = set_device(t)) != HC_OK) return r;
    return launch_set(SET_INSERT, view_of(t), g, t->window, d_keys, n, d_status, (hipStream_t)stream);
  }
  if (t->kind == HC_COUNTING) {
    if (d_values != nullptr) return fail(HC_E_ARG, "counting tables take no values");
  } else if (d_values == nullptr) {
    return fail(HC_E_ARG, "values is NULL");
  }
  if ((r = set_device(t)) != HC_OK) return r;
  if (t->kind == HC_BUCKET_LIST) {
    hipStream_t s = (hipStream_t)stream;
    CallWs ws(s);
    if ((r = ws.get(bl_insert_workspace(n))) != HC_OK) return r;
    if ((r = order_begin(t, s)) != HC_OK) return r;
    return order_end(t, s, launch_bl_insert(view_of(t), bview_of(t), g, t->window, d_keys, d_values, n, d_status,
                                            ws.p, s));
  }
  return launch_insert(view_of(t), (int)t->kind, g, t->window, d_keys, d_values, n, d_status, (hipStream_t)stream);
}

hc_err hc_retrieve(hc_table t, const uint32_t* d_keys, uint64_t n, uint32_t* d_values_out, uint8_t* d_found_out,
                   uint32_t group, void* stream) {
  hc_err r = check_table(t);
  if (r != HC_OK) return r;
  if ((r = not_wide(t, "hc_retrieve")) != HC_OK) return r;
  uint32_t g;
  if ((r = resolve_group(t, group, &g)) != HC_OK) return r;
  if (n == 0) return HC_OK;
  if (d_keys == nullptr) return fail(HC_E_ARG, "keys is NULL");
  if (t->kind == HC_HASH_SET) {
    if (d_values_out != nullptr) return fail(HC_E_ARG, "sets return no values");
    if (d_found_out == nullptr) return fail(HC_E_ARG, "found is NULL");
  }
  if ((r = set_device(t)) != HC_OK) return r;
  if (t->kind == HC_HASH_SET)
    return launch_set(SET_CONTAINS, view_of(t), g, t->window, d_keys, n, d_found_out, (hipStream_t)stream);
  if (t->kind == HC_MULTI_VALUE)
    return launch_count_multi(view_of(t), g, t->window, d_keys, n, d_values_out, nullptr, d_found_out, 0xFFFFFFFFu,
                              nullptr, nullptr, 0, (hipStream_t)stream);
  return launch_retrieve(view_of(t), g, t->window, d_keys, n, d_values_out, d_found_out, (hipStream_t)stream);
}

hc_err hc_erase(hc_table t, const uint32_t* d_keys, uint64_t n, uint8_t* d_status, uint32_t group, void* stream) {
  hc_err r = check_table(t);
  if (r != HC_OK) return r;
  if ((r = not_wide(t, "hc_erase")) != HC_OK) return r;
  uint32_t g;
  if ((r = resolve_group(t, group, &g)) != HC_OK) return r;
  if (n == 0) return HC_OK;
  if (d_keys == nullptr) return fail(HC_E_ARG, "keys is NULL");
  if ((r = set_device(t)) != HC_OK) return r;
  if (t->kind == HC_BUCKET_LIST)
    return launch_bl_erase(view_of(t), bview_of(t), g, t->window, d_keys, n, d_status, (hipStream_t)stream);
  if (t->kind == HC_HASH_SET)
    return launch_set(SET_ERASE, view_of(t), g, t->window, d_keys, n, d_status, (hipStream_t)stream);
  return launch_erase(view_of(t), (int)t->kind, g, t->window, d_keys, n, d_status, (hipStream_t)stream);
}

// Argument checks shared by hc_count_values and hc_count_values_noalloc.
static hc_err count_values_args(hc_table t, const uint32_t* d_keys, uint64_t n, uint64_t* d_offsets, uint32_t group,
                                uint32_t* g) {
  hc_err r = check_table(t);
  if (r != HC_OK) return r;
  if ((r = not_wide(t, "hc_count_values")) != HC_OK) return r;
  if ((r = not_set(t, "hc_count_values")) != HC_OK) return r;
  if (t->kind != HC_MULTI_VALUE && t->kind != HC_BUCKET_LIST)
    return fail(HC_E_KIND, "count_values needs a multi-value or bucket list table");
  if ((r = resolve_group(t, group, g)) != HC_OK) return r;
  if (d_offsets == nullptr) return fail(HC_E_ARG, "offsets is NULL");
  if (n > 0 && d_keys == nullptr) return fail(HC_E_ARG, "keys is NULL");
  return set_device(t);
}

static hc_err count_values_total(const uint64_t* d_offsets, uint64_t n, uint64_t* h_total, hipStream_t s) {
  if (h_total == nullptr) return HC_OK;
  hipError_t e = hipMemcpyAsync(h_total, d_offsets + n, sizeof(uint64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "count_values: total");
  return HC_OK;
}

}  // extern "C"

namespace hc {

hc_err table_device(hc_table t, int* dev) {
  if (t == nullptr) return fail(HC_E_ARG, "table handle is NULL");
  *dev = t->device;
  return HC_OK;
}

hc_err count_values_into(hc_table t, const uint32_t* d_keys, uint64_t n, uint32_t* d_counts, uint64_t* d_offsets,
                         uint64_t* h_total, uint32_t group, void* ws, uint64_t ws_bytes, void* stream) {
  uint32_t g;
  hc_err r = count_values_args(t, d_keys, n, d_offsets, group, &g);
  if (r != HC_OK) return r;
  if (ws == nullptr || (reinterpret_cast<uintptr_t>(ws) & 255) != 0)
    return fail(HC_E_ARG, "workspace is NULL or not 256-byte aligned");
  const uint64_t tiles = count_values_ws_bytes(n, 0);
  if (tiles > ws_bytes)
    return fail(HC_E_ARG, "%llu queries need %llu workspace bytes for the scan, %llu given", (unsigned long long)n,
                (unsigned long long)tiles, (unsigned long long)ws_bytes);
  uint64_t cap = 0;
  if (t->kind == HC_MULTI_VALUE && n > 0) {
    cap = long_capacity(n);
    const uint64_t fit = (ws_bytes - tiles) > 2048 ? (ws_bytes - tiles - 2048) / 32 : 0;
    if (cap > fit) cap = fit;
    while (cap > 0 && count_values_ws_bytes(n, cap) > ws_bytes) --cap;
    if (cap == 0) return fail(HC_E_ARG, "workspace of %llu bytes holds no long-query entry", (unsigned long long)ws_bytes);
  }
  hipStream_t s = (hipStream_t)stream;
  if ((r = count_values_in(t, d_keys, n, d_counts, d_offsets, g, ws, cap, s)) != HC_OK) return r;
  return count_values_total(d_offsets, n, h_total, s);
}

}  // namespace hc

extern "C" {

hc_err hc_count_values(hc_table t, const uint32_t* d_keys, uint64_t n, uint32_t* d_counts, uint64_t* d_offsets,
                       uint64_t* h_total, uint32_t group, void* stream) {
  uint32_t g;
  hc_err r = count_values_args(t, d_keys, n, d_offsets, group, &g);
  if (r != HC_OK) return r;
  hipStream_t s = (hipStream_t)stream;
  CallWs ws(s);
  const uint64_t cap = t->kind == HC_MULTI_VALUE ? long_capacity(n) : 0;
  if ((r = ws.get(count_values_ws_bytes(n, cap))) != HC_OK) return r;
  if ((r = count_values_in(t, d_keys, n, d_counts, d_offsets, g, ws.p, cap, s)) != HC_OK) return r;
  return count_values_total(d_offsets, n, h_total, s);
}

hc_err hc_retrieve_all(hc_table t, const uint32_t* d_keys, uint64_t n, const uint64_t* d_offsets,
                       uint32_t* d_values_out, uint32_t group, void* stream) {
  hc_err r = check_table(t);
  if (r != HC_OK) return r;
  if ((r = not_wide(t, "hc_retrieve_all")) != HC_OK) return r;
  if ((r = not_set(t, "hc_retrieve_all")) != HC_OK) return r;
  if (t->kind != HC_MULTI_VALUE && t->kind != HC_BUCKET_LIST)
    return fail(HC_E_KIND, "retrieve_all needs a multi-value or bucket list table");
  uint32_t g;
  if ((r = resolve_group(t, group, &g)) != HC_OK) return r;
  if (n == 0) return HC_OK;
  if (d_keys == nullptr || d_offsets == nullptr) return fail(HC_E_ARG, "keys or offsets is NULL");
  if ((r = set_device(t)) != HC_OK) return r;
  hipStream_t s = (hipStream_t)stream;
  CallWs ws(s);
  if (t->kind == HC_BUCKET_LIST) {
    if ((r = ws.get(bl_write_workspace(n))) != HC_OK) return r;
    return launch_bl_write(view_of(t), bview_of(t), g, t->window, d_keys, n, d_offsets, d_values_out, ws.p, s);
  }
  const uint64_t cap = long_capacity(n);
  if ((r = ws.get(long_workspace_bytes(cap, 1))) != HC_OK) return r;
  const LongState ls = long_layout(ws.p, cap, 1);
  if ((r = launch_zero_u64((unsigned long long*)ls.nlong, 1, s)) != HC_OK) return r;
  if ((r = launch_write_multi(view_of(t), g, t->window, d_keys, n, d_offsets, d_values_out, LONG_BUDGET, ls.entries,
                              (unsigned long long*)ls.nlong, cap, s)) != HC_OK)
    return r;
  // the write rounds only read the offsets
  return launch_long_queries(view_of(t), t->window, 1, d_keys, ls, n, LONG_BUDGET, const_cast<uint64_t*>(d_offsets),
                             nullptr, d_values_out, s);
}

hc_err hc_insert_grouped(hc_table t, const uint32_t* d_keys, const uint32_t* d_values, uint64_t n, void* stream) {
  hc_err r = check_table(t);
  if (r != HC_OK) return r;
  if ((r = not_wide(t, "hc_insert_grouped")) != HC_OK) return r;
  if ((r = not_set(t, "hc_insert_grouped")) != HC_OK) return r;
  if (t->kind == HC_SINGLE_VALUE)
    return fail(HC_E_KIND, "grouped insert needs a multi-value, counting or bucket list table");
  if (n == 0) return HC_OK;
  if (d_keys == nullptr) return fail(HC_E_ARG, "keys is NULL");
  if (t->kind == HC_COUNTING) {
    if (d_values != nullptr) return fail(HC_E_ARG, "counting tables take no values");
  } else if (d_values == nullptr) {
    return fail(HC_E_ARG, "values is NULL");
  }
  if (n > 0xFFFFFFFFull) return fail(HC_E_ARG, "grouped insert takes at most 2^32-1 pairs");
  if ((r = set_device(t)) != HC_OK) return r;
  hipStream_t s = (hipStream_t)stream;
  CallWs ws(s);
  if (t->kind == HC_BUCKET_LIST) {
    if ((r = ws.get(bl_grouped_workspace_bytes(n))) != HC_OK) return r;
    if ((r = order_begin(t, s)) != HC_OK) return r;
    return order_end(t, s, launch_bl_grouped(view_of(t), bview_of(t), t->group, t->window, d_keys, d_values, n,
                                             ws.p, s));
  }
  if ((r = ws.get(grouped_workspace_bytes(n))) != HC_OK) return r;
  if ((r = order_begin(t, s)) != HC_OK) return r;
  return order_end(t, s, launch_grouped_insert(view_of(t), (int)t->kind, t->group, t->window, d_keys, d_values, n,
                                               ws.p, s));
}

static hc_err wide_call(hc_table t, int op, const uint64_t* keys, const uint64_t* values, uint64_t n,
                        uint64_t* values_out, uint8_t* flags, uint32_t group, void* stream) {
  hc_err r = check_table(t);
  if (r != HC_OK) return r;
  if (!is_wide(t->kind)) return fail(HC_E_KIND, "64-bit entry points need a 64-bit table");
  uint32_t g;
  if ((r = resolve_group(t, group, &g)) != HC_OK) return r;
  if (n == 0) return HC_OK;
  if (keys == nullptr) return fail(HC_E_ARG, "keys is NULL");
  if (op == WIDE_INSERT && values == nullptr) return fail(HC_E_ARG, "values is NULL");
  if ((r = set_device(t)) != HC_OK) return r;
  return launch_wide(op, t->kind == HC_SINGLE_VALUE_64_SOA, view_of(t), g, t->window, keys, values, n, values_out,
                     flags, (hipStream_t)stream);
}

hc_err hc_insert64(hc_table t, const uint64_t* d_keys, const uint64_t* d_values, uint64_t n, uint8_t* d_status,
                   uint32_t group, void* stream) {
  return wide_call(t, WIDE_INSERT, d_keys, d_values, n, nullptr, d_status, group, stream);
}

hc_err hc_retrieve64(hc_table t, const uint64_t* d_keys, uint64_t n, uint64_t* d_values_out, uint8_t* d_found_out,
                     uint32_t group, void* stream) {
  return wide_call(t, WIDE_RETRIEVE, d_keys, nullptr, n, d_values_out, d_found_out, group, stream);
}

hc_err hc_erase64(hc_table t, const uint64_t* d_keys, uint64_t n, uint8_t* d_status, uint32_t group, void* stream) {
  return wide_call(t, WIDE_ERASE, d_keys, nullptr, n, nullptr, d_status, group, stream);
}

hc_err hc_size(hc_table t, uint64_t* h_out, void* stream) {
  hc_err r = check_table(t);
  if (r != HC_OK) return r;
  if (h_out == nullptr) return fail(HC_E_ARG, "out is NULL");
  if ((r = set_device(t)) != HC_OK) return r;
  unsigned long long v = 0;
  hipError_t e = hipMemcpyAsync(&v, t->d_size, sizeof v, hipMemcpyDeviceToHost, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hc_size");
  *h_out = v;
  return HC_OK;
}

hc_err hc_load_factor(hc_table t, double* h_out, void* stream) {
  if (h_out == nullptr) return fail(HC_E_ARG, "out is NULL");
  uint64_t s = 0;
  hc_err r = hc_size(t, &s, stream);
  if (r != HC_OK) return r;
  *h_out = (double)s / (double)t->C;
  return HC_OK;
}

hc_err hc_capacity(hc_table t, uint64_t* h_out) {
  hc_err r = check_table(t);
  if (r != HC_OK) return r;
  if (h_out == nullptr) return fail(HC_E_ARG, "out is NULL");
  *h_out = t->C;
  return HC_OK;
}

hc_err hc_info(hc_table t, hc_table_info* h_out) {
  hc_err r = check_table(t);
  if (r != HC_OK) return r;
  if (h_out == nullptr) return fail(HC_E_ARG, "out is NULL");
  h_out->kind = t->kind;
  h_out->scheme = t->scheme;
  h_out->window = t->window;
  h_out->group = t->group;
  h_out->windows = t->P;
  h_out->capacity = t->C;
  h_out->seed = t->seed;
  h_out->d_slots = t->slots;
  return HC_OK;
}

hc_err hc_stats(hc_table t, hc_table_stats* h_out, void* stream) {
  hc_err r = check_table(t);
  if (r != HC_OK) return r;
  if ((r = not_wide(t, "hc_stats")) != HC_OK) return r;
  if ((r = not_set(t, "hc_stats")) != HC_OK) return r;
  if (h_out == nullptr) return fail(HC_E_ARG, "out is NULL");
  static_assert(HC_PROBE_BUCKETS == STATS_BUCKETS, "histogram width");
  static_assert(sizeof(hc_table_stats) == (6 + STATS_BUCKETS) * sizeof(uint64_t), "stats layout");
  if ((r = set_device(t)) != HC_OK) return r;
  hipStream_t s = (hipStream_t)stream;
  CallWs ws(s);
  if ((r = ws.get(sizeof(hc_table_stats))) != HC_OK) return r;
  unsigned long long* d = static_cast<unsigned long long*>(ws.p);
  if ((r = launch_zero_u64(d, 5 + STATS_BUCKETS, s)) != HC_OK) return r;
  if ((r = launch_stats(view_of(t), t->window, d, s)) != HC_OK) return r;
  hipError_t e = hipMemcpyAsync(h_out, d, (5 + STATS_BUCKETS) * sizeof(uint64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(&h_out->cas_fails, t->d_size + CTR_CAS_FAILS, sizeof(uint64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "hc_stats");
  return HC_OK;
}

hc_err hc_device_view(hc_table t, void* h_view, uint64_t bytes) {
  hc_err r = check_table(t);
  if (r != HC_OK) return r;
  if ((r = not_wide(t, "hc_device_view")) != HC_OK) return r;
  if ((r = not_set(t, "hc_device_view")) != HC_OK) return r;
  if (h_view == nullptr) return fail(HC_E_ARG, "view is NULL");
  if (bytes != sizeof(TableView)) return fail(HC_E_ARG, "view takes %zu bytes, not %llu", sizeof(TableView),
                                              (unsigned long long)bytes);
  const TableView v = view_of(t);
  std::memcpy(h_view, &v, sizeof v);
  return HC_OK;
}

hc_err hc_dump_slots(hc_table t, uint64_t* d_dst, void* stream) {
  hc_err r = check_table(t);
  if (r != HC_OK) return r;
  if (d_dst == nullptr) return fail(HC_E_ARG, "destination is NULL");
  if ((r = set_device(t)) != HC_OK) return r;
  hipError_t e = hipMemcpyAsync(d_dst, t->slots, t->C * slot_bytes(t->kind), hipMemcpyDeviceToDevice,
                                (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hc_dump_slots");
  return HC_OK;
}


hc_err hc_batch_create(hc_batch* out, const hc_batch_op* ops, uint32_t count) {
  return hc_batch_create_flags(out, ops, count, 0);
}

hc_err hc_batch_create_flags(hc_batch* out, const hc_batch_op* ops, uint32_t count, uint32_t flags) {
  if (out == nullptr) return fail(HC_E_ARG, "out is NULL");
  *out = nullptr;
  if ((flags & ~(uint32_t)HC_BATCH_ONE_LAUNCH) != 0) return fail(HC_E_ARG, "unknown batch flags 0x%x", flags);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(HC_E_DEVICE, "hipGetDevice failed");
  PlanHost plan;
  if (hc_err r = build_plan(ops, count, dev, &plan, (flags & HC_BATCH_ONE_LAUNCH) != 0); r != HC_OK) return r;
  uint64_t ticks = 0;
  if (flags & HC_BATCH_ONE_LAUNCH) {
    int khz = 0;
    const hipError_t e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess || khz <= 0) return fail(HC_E_DEVICE, "device clock rate unavailable");
    ticks = (uint64_t)khz * HC_BATCH_WAIT_MS;
  }
  hc_batch_s* b = new (std::nothrow) hc_batch_s();
  if (!b) return fail(HC_E_NOMEM, "host allocation failed");
  b->device = dev;
  b->phases = plan.phases;
  b->launches = plan.launches;
  b->gates = plan.gates;
  b->wait_ticks = ticks;
  if (!plan.descs.empty()) {
    const size_t cbytes = plan_counter_words(plan) * sizeof(unsigned long long);
    hipError_t e1 = hipMalloc((void**)&b->d_descs, plan.descs.size() * sizeof(BatchDesc));
    hipError_t e2 = e1 == hipSuccess ? hipMalloc((void**)&b->d_chunk_start, plan.cs.size() * sizeof(uint64_t)) : e1;
    hipError_t e3 = e2 == hipSuccess ? hipMalloc((void**)&b->d_counters, cbytes) : e2;
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
      (void)hipGetLastError();
      if (b->d_descs) (void)hipFree(b->d_descs);
      if (b->d_chunk_start) (void)hipFree(b->d_chunk_start);
      delete b;
      return fail(HC_E_NOMEM, "hipMalloc of batch descriptors failed");
    }
    hipError_t e = hipMemcpy(b->d_descs, plan.descs.data(), plan.descs.size() * sizeof(BatchDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(b->d_chunk_start, plan.cs.data(), plan.cs.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemsetAsync(b->d_counters, 0, cbytes, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
      (void)hipFree(b->d_descs);
      (void)hipFree(b->d_chunk_start);
      (void)hipFree(b->d_counters);
      delete b;
      return hip_fail(e, "batch descriptor upload");
    }
  }
  *out = b;
  return HC_OK;
}

hc_err hc_batch_launch(hc_batch b, void* stream) {
  if (b == nullptr) return fail(HC_E_ARG, "batch is NULL");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(HC_E_DEVICE, "hipGetDevice failed");
  if (cur != b->device) {
    const hipError_t e = hipSetDevice(b->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  }
  return launch_plan(b->launches, b->d_descs, b->d_chunk_start, b->d_counters, (hipStream_t)stream, b->gates,
                     b->wait_ticks);
}

hc_err hc_batch_abandoned_waits(hc_batch b, uint64_t* h_count) {
  if (b == nullptr || h_count == nullptr) return fail(HC_E_ARG, "batch or out is NULL");
  *h_count = 0;
  bool one = false;
  for (const PlanLaunch& L : b->launches) one |= L.op == BATCH_ALL;
  if (!one || b->d_counters == nullptr) return HC_OK;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(HC_E_DEVICE, "hipGetDevice failed");
  if (cur != b->device) {
    const hipError_t e = hipSetDevice(b->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  }
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess)
    e = hipMemcpy(h_count, b->d_counters + b->launches.size() * PLAN_COUNTER_STRIDE, sizeof(uint64_t),
                  hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hc_batch_abandoned_waits");
  return HC_OK;
}

hc_err hc_batch_info(hc_batch b, uint32_t* h_phases, uint32_t* h_launches) {
  if (b == nullptr) return fail(HC_E_ARG, "batch is NULL");
  if (h_phases) *h_phases = b->phases;
  if (h_launches) *h_launches = (uint32_t)b->launches.size();
  return HC_OK;
}

hc_err hc_batch_destroy(hc_batch b) {
  if (b == nullptr) return HC_OK;
  if (b->d_descs) (void)hipFree(b->d_descs);
  if (b->d_chunk_start) (void)hipFree(b->d_chunk_start);
  if (b->d_counters) (void)hipFree(b->d_counters);
  delete b;
  return HC_OK;
}

hc_err hc_batch_run(const hc_batch_op* ops, uint32_t count, void* stream) {
  hc_batch b = nullptr;
  hc_err r = hc_batch_create(&b, ops, count);
  if (r != HC_OK) return r;
  r = hc_batch_launch(b, stream);
  if (r == HC_OK) {
    const hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) r = hip_fail(e, "hc_batch_run: synchronise");
  }
  hc_batch_destroy(b);
  return r;
}

hc_err hc_batch_capture(hc_batch b, void** h_graph_exec) {
  if (b == nullptr || h_graph_exec == nullptr) return fail(HC_E_ARG, "batch or out is NULL");
  *h_graph_exec = nullptr;
  hipStream_t s = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "capture stream");
  hipGraph_t graph = nullptr;
  e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  hc_err r = HC_OK;
  if (e == hipSuccess) {
    r = hc_batch_launch(b, s);
    const hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (r == HC_OK && e2 != hipSuccess) r = hip_fail(e2, "end capture");
  } else {
    r = hip_fail(e, "begin capture");
  }
  hipGraphExec_t exec = nullptr;
  if (r == HC_OK) {
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) r = hip_fail(e, "graph instantiate");
  }
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(s);
  if (r == HC_OK) *h_graph_exec = (void*)exec;
  return r;
}

hc_err hc_graph_launch(void* graph_exec, void* stream) {
  if (graph_exec == nullptr) return fail(HC_E_ARG, "graph is NULL");
  const hipError_t e = hipGraphLaunch((hipGraphExec_t)graph_exec, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return HC_OK;
}

hc_err hc_graph_destroy(void* graph_exec) {
  if (graph_exec == nullptr) return HC_OK;
  const hipError_t e = hipGraphExecDestroy((hipGraphExec_t)graph_exec);
  if (e != hipSuccess) return hip_fail(e, "hipGraphExecDestroy");
  return HC_OK;
}

const char* hc_error_string(hc_err err) {
  switch (err) {
    case HC_OK: return "ok";
    case HC_E_ARG: return "invalid argument";
    case HC_E_NOMEM: return "device allocation failed";
    case HC_E_KIND: return "operation not defined for this table kind";
    case HC_E_DEVICE: return "HIP runtime error";
  }
  return "unknown error";
}

const char* hc_last_error(void) { return hc::last_error_text(); }

}  // extern "C"
