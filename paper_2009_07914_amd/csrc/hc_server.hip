// Serving loop: continuous batching of host-side requests onto resident tables.
//
// Not in the paper; built from its bulk operations (Sec. IV-B3/B4/B5) and its
// concurrency rules (Sec. IV-D).  A worker thread owns the device side:
//   * admission: requests are taken in arrival order while the device staging
//     ring (the admission budget, at most half the HBM free when the server is
//     created) has room for their inputs and outputs;
//   * coalescing: everything admitted at one moment becomes one launch group, a
//     batched plan whose phases keep each table's operations in arrival order;
//     same-kind writes of one group to one table run in one launch (one epoch):
//     where they touch the same key, the outcome is one of the arrival orders of
//     those writes (Sec. IV-D: concurrent same-kind operations are valid but
//     order-dependent);
//   * overlap: a group's input copies, kernels and output copies go to one of
//     several streams in rotation, so the copies of one group overlap the
//     kernels of its neighbours; a group's kernels wait (on the device) only for
//     the unfinished earlier groups that touch one of its tables, so groups on
//     disjoint tables also run their kernels side by side, while every table's
//     operations keep their arrival order across groups;
//   * completion: a group is done when the event after its output copies fires
//     (groups may finish out of order); a request's latency is that moment minus
//     its submission.  Staging memory is given back in admission order.
// In serial mode every request is its own group and starts only when the previous
// one has completed: the plain one-request-at-a-time path, for comparison.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hc.h"
#include "hc_batch.hpp"
#include "hc_launch.hpp"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  hc_request r;
  Clock::time_point arrival;
  Clock::time_point done_at;
  uint64_t bytes = 0;
  bool done = false;
};

struct Slot {  // per in-flight launch group
  hc::BatchDesc* d_descs = nullptr;
  uint64_t* d_cs = nullptr;
  hc::BatchDesc* h_descs = nullptr;  // pinned
  uint64_t* h_cs = nullptr;          // pinned
  hipEvent_t kernel_done = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
};

struct Group {
  std::vector<uint64_t> tickets;
  uint64_t ring_end = 0;
  uint64_t seq = 0;    // launch order
  int slot = -1;
  bool done = false;   // its requests are complete (it may still hold staging memory)
};

constexpr uint64_t ALIGN = 256;
inline uint64_t align_up(uint64_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

}  // namespace

struct hc_server_s {
  int device = 0;
  hc_server_params p{};
  bool serial = false;
  char* d_staging = nullptr;
  uint64_t head = 0, tail = 0;  // ring allocation counters (monotonic bytes)
  std::vector<hipStream_t> streams;
  std::vector<Slot> slots;
  uint32_t next_stream = 0;
  uint64_t next_seq = 0;
  std::unordered_map<const void*, uint64_t> table_last;  // table -> seq of the last group touching it

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> pending;
  std::vector<Request*> reqs;  // by ticket
  std::deque<Group> inflight;
  bool stop = false;
  uint32_t launching = 0;  // groups taken from `pending` but not yet in `inflight`
  hc_err error = HC_OK;
  std::string error_msg;
  uint64_t groups = 0, ops_done = 0, completed = 0;
  std::thread worker;

  // staging bytes of a request
  static uint64_t bytes_of(const hc_request& r) {
    uint64_t b = align_up(4 * r.n);
    if (r.op == HC_OP_INSERT && r.h_values) b += align_up(4 * r.n);
    if (r.op == HC_OP_RETRIEVE && r.h_values_out) b += align_up(4 * r.n);
    if (r.h_flags) b += align_up(r.n);
    return b;
  }

  // Reserve `bytes` contiguous ring bytes; returns the offset or UINT64_MAX if full.
  uint64_t ring_alloc(uint64_t bytes) {
    const uint64_t size = p.staging_bytes;
    if (head == tail) head = tail = 0;  // empty: start at offset 0, so any request up to `size` fits
    uint64_t h = head;
    const uint64_t pos = h % size;
    if (pos + bytes > size) h += size - pos;  // do not wrap inside an allocation
    if (h + bytes - tail > size) return UINT64_MAX;
    head = h + bytes;
    return h % size;
  }

  void run();
  bool retire();
  bool launch_group();
};

static hc_err server_fail(hc_server_s* s, hc_err e, const char* what, hipError_t he) {
  s->error = e;
  s->error_msg = std::string(what) + ": " + hipGetErrorString(he);
  return e;
}

// Complete the groups whose work has finished, in any order; give staging memory back
// over the prefix of finished groups (admission order).  Called with the lock held.
bool hc_server_s::retire() {
  bool any = false;
  for (Group& g : inflight) {
    if (g.done) continue;
    const hipError_t e = hipEventQuery(slots[g.slot].done);
    if (e == hipErrorNotReady) continue;
    if (e != hipSuccess) {
      server_fail(this, HC_E_DEVICE, "launch group", e);
      break;
    }
    const Clock::time_point now = Clock::now();
    for (uint64_t t : g.tickets) {
      Request* r = reqs[t];
      r->done = true;
      r->done_at = now;
      ops_done += r->r.n;
      ++completed;
    }
    g.done = true;
    slots[g.slot].busy = false;
    any = true;
  }
  while (!inflight.empty() && inflight.front().done) {
    tail = inflight.front().ring_end;
    inflight.pop_front();
  }
  if (any) cv_done.notify_all();
  return any;
}

// Admit the pending requests that fit and launch them as one group.  Lock held on
// entry; released while the group is enqueued.
bool hc_server_s::launch_group() {
  if (pending.empty()) return false;
  if (serial && !inflight.empty()) return false;
  int slot = -1;
  for (size_t i = 0; i < slots.size(); ++i)
    if (!slots[i].busy) {
      slot = (int)i;
      break;
    }
  if (slot < 0) return false;
  // gather in arrival order
  std::vector<uint64_t> take;
  std::vector<uint64_t> offs;
  uint64_t ops = 0;
  const uint64_t head0 = head;
  while (!pending.empty()) {
    Request* r = reqs[pending.front()];
    if (!take.empty()) {
      if (serial || take.size() >= p.max_group_requests) break;
      if (p.max_group_ops && ops + r->r.n > p.max_group_ops) break;
    }
    const uint64_t off = ring_alloc(r->bytes);
    if (off == UINT64_MAX) break;
    take.push_back(pending.front());
    offs.push_back(off);
    ops += r->r.n;
    pending.pop_front();
  }
  if (take.empty()) {
    head = head0;
    return false;
  }
  Slot& sl = slots[slot];
  sl.busy = true;
  Group g;
  g.tickets = take;
  g.ring_end = head;
  g.slot = slot;
  g.seq = next_seq++;
  hipStream_t st = streams[next_stream++ % streams.size()];
  // per-table order: the kernels wait for the unfinished earlier groups that share a table
  std::vector<hipEvent_t> waits;
  for (uint64_t tk : take) {
    const void* tab = reqs[tk]->r.table;
    auto it = table_last.find(tab);
    if (it != table_last.end()) {
      for (const Group& e : inflight)
        if (e.seq == it->second && !e.done) {
          const hipEvent_t ev = slots[e.slot].kernel_done;
          if (std::find(waits.begin(), waits.end(), ev) == waits.end()) waits.push_back(ev);
        }
    }
    table_last[tab] = g.seq;
  }
  ++launching;
  mu.unlock();

  hc_err err = HC_OK;
  hipError_t he = hipSuccess;
  std::vector<hc_batch_op> bops(take.size());
  struct Out {
    void* dst;
    const void* src;
    uint64_t bytes;
  };
  std::vector<Out> outs;
  for (size_t j = 0; j < take.size() && he == hipSuccess; ++j) {
    const hc_request& r = reqs[take[j]]->r;
    char* base = d_staging + offs[j];
    uint64_t o = 0;
    hc_batch_op& b = bops[j];
    std::memset(&b, 0, sizeof b);
    b.table = r.table;
    b.op = r.op;
    b.group = r.group;
    b.n = r.n;
    b.d_keys = reinterpret_cast<const uint32_t*>(base + o);
    he = hipMemcpyAsync(base + o, r.h_keys, 4 * r.n, hipMemcpyHostToDevice, st);
    o += align_up(4 * r.n);
    if (r.op == HC_OP_INSERT && r.h_values && he == hipSuccess) {
      b.d_values = reinterpret_cast<const uint32_t*>(base + o);
      he = hipMemcpyAsync(base + o, r.h_values, 4 * r.n, hipMemcpyHostToDevice, st);
      o += align_up(4 * r.n);
    }
    if (r.op == HC_OP_RETRIEVE && r.h_values_out) {
      b.d_values_out = reinterpret_cast<uint32_t*>(base + o);
      outs.push_back({r.h_values_out, base + o, 4 * r.n});
      o += align_up(4 * r.n);
    }
    if (r.h_flags) {
      b.d_flags = reinterpret_cast<uint8_t*>(base + o);
      outs.push_back({r.h_flags, base + o, r.n});
      o += align_up(r.n);
    }
  }
  hc::PlanHost plan;
  if (he == hipSuccess) err = hc::build_plan(bops.data(), (uint32_t)bops.size(), device, &plan);
  if (he == hipSuccess && err == HC_OK && !plan.descs.empty()) {
    std::memcpy(sl.h_descs, plan.descs.data(), plan.descs.size() * sizeof(hc::BatchDesc));
    std::memcpy(sl.h_cs, plan.cs.data(), plan.cs.size() * sizeof(uint64_t));
    he = hipMemcpyAsync(sl.d_descs, sl.h_descs, plan.descs.size() * sizeof(hc::BatchDesc), hipMemcpyHostToDevice, st);
    if (he == hipSuccess)
      he = hipMemcpyAsync(sl.d_cs, sl.h_cs, plan.cs.size() * sizeof(uint64_t), hipMemcpyHostToDevice, st);
  }
  for (size_t j = 0; j < waits.size() && he == hipSuccess && err == HC_OK; ++j)
    he = hipStreamWaitEvent(st, waits[j], 0);
  if (he == hipSuccess && err == HC_OK) err = hc::launch_plan(plan.launches, sl.d_descs, sl.d_cs, nullptr, st);
  if (he == hipSuccess && err == HC_OK) he = hipEventRecord(sl.kernel_done, st);
  for (size_t j = 0; j < outs.size() && he == hipSuccess && err == HC_OK; ++j)
    he = hipMemcpyAsync(outs[j].dst, outs[j].src, outs[j].bytes, hipMemcpyDeviceToHost, st);
  const hipError_t he_done = hipEventRecord(sl.done, st);  // recorded even after a failure, so the group retires
  if (he == hipSuccess) he = he_done;

  mu.lock();
  if (he != hipSuccess) server_fail(this, HC_E_DEVICE, "enqueue launch group", he);
  else if (err != HC_OK) {
    error = err;
    error_msg = hc_last_error();
  }
  ++groups;
  inflight.push_back(std::move(g));
  --launching;
  return true;
}

void hc_server_s::run() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lock(mu);
  for (;;) {
    const bool retired = retire();
    const bool launched = error == HC_OK && launch_group();
    if (stop && pending.empty() && inflight.empty()) break;
    if (error != HC_OK) {  // drop what cannot run; waiters see the error
      pending.clear();
      if (inflight.empty()) {
        cv_done.notify_all();
        if (stop) break;
        cv_work.wait(lock, [&] { return stop || !pending.empty(); });
        continue;
      }
    }
    if (!retired && !launched) {
      if (inflight.empty()) {
        cv_work.wait(lock, [&] { return stop || !pending.empty(); });
      } else {
        lock.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(5));
        lock.lock();
      }
    }
  }
}

extern "C" {

void hc_default_server_params(hc_server_params* p) {
  if (!p) return;
  p->staging_bytes = 1ull << 30;
  p->max_group_ops = 1ull << 22;  // a small request waits behind at most about 4 M elements
  p->max_group_requests = 1024;
  p->streams = 3;
  p->serial = 0;
}

hc_err hc_server_create(hc_server* out, const hc_server_params* params) {
  using hc::fail;
  if (out == nullptr) return fail(HC_E_ARG, "out is NULL");
  *out = nullptr;
  hc_server_params p;
  hc_default_server_params(&p);
  if (params) p = *params;
  if (p.staging_bytes < (1u << 20)) return fail(HC_E_ARG, "staging_bytes must be at least 1 MiB");
  if (p.max_group_requests == 0) p.max_group_requests = 1024;
  if (p.streams == 0) p.streams = 3;
  hc_server_s* s = new (std::nothrow) hc_server_s();
  if (!s) return fail(HC_E_NOMEM, "host allocation failed");
  s->p = p;
  s->serial = p.serial != 0;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return fail(HC_E_DEVICE, "hipGetDevice failed");
  }
  size_t free_b = 0, total_b = 0;
  hipError_t e = hipMemGetInfo(&free_b, &total_b);
  if (e != hipSuccess) {
    delete s;
    return hc::hip_fail(e, "hipMemGetInfo");
  }
  if (p.staging_bytes > free_b / 2) {  // the admission budget takes at most half the free HBM
    if (free_b / 2 < (1u << 20)) {
      delete s;
      return fail(HC_E_NOMEM, "%llu bytes of HBM free: too little for a staging ring", (unsigned long long)free_b);
    }
    s->p.staging_bytes = p.staging_bytes = (free_b / 2) & ~(uint64_t)(ALIGN - 1);
  }
  e = hipMalloc((void**)&s->d_staging, p.staging_bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    delete s;
    return fail(HC_E_NOMEM, "hipMalloc of %llu staging bytes failed", (unsigned long long)p.staging_bytes);
  }
  const size_t nslots = s->serial ? 1 : (size_t)p.streams + 1;
  const size_t max_desc = p.max_group_requests;
  const size_t max_cs = 2 * (size_t)p.max_group_requests + 8;
  s->slots.resize(nslots);
  for (auto& sl : s->slots) {
    if (e == hipSuccess) e = hipMalloc((void**)&sl.d_descs, max_desc * sizeof(hc::BatchDesc));
    if (e == hipSuccess) e = hipMalloc((void**)&sl.d_cs, max_cs * sizeof(uint64_t));
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_descs, max_desc * sizeof(hc::BatchDesc), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_cs, max_cs * sizeof(uint64_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.kernel_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
  }
  s->streams.resize(s->serial ? 1 : p.streams);
  for (auto& st : s->streams)
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    hc_server_destroy(s);
    return fail(HC_E_NOMEM, "server resources: %s", hipGetErrorString(e));
  }
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return HC_OK;
}

hc_err hc_server_submit(hc_server s, const hc_request* req, uint64_t* h_ticket) {
  using hc::fail;
  if (s == nullptr || req == nullptr) return fail(HC_E_ARG, "server or request is NULL");
  const hc_request& r = *req;
  if (r.table == nullptr) return fail(HC_E_ARG, "request table is NULL");
  if (r.op > HC_OP_ERASE) return fail(HC_E_ARG, "unknown operation %u", r.op);
  if (r.n > 0 && r.h_keys == nullptr) return fail(HC_E_ARG, "keys is NULL");
  hc_table_info info;
  if (hc_err e = hc_info(r.table, &info); e != HC_OK) return e;
  if (info.kind == HC_MULTI_VALUE || info.kind == HC_BUCKET_LIST || info.kind == HC_SINGLE_VALUE_64 ||
      info.kind == HC_SINGLE_VALUE_64_SOA || info.kind == HC_HASH_SET)
    return fail(HC_E_KIND, "requests take single-value or counting tables");
  if (r.group != 0 && (r.group > 64 || (r.group & (r.group - 1)) != 0))
    return fail(HC_E_ARG, "group size %u is not a power of two in [1, 64]", r.group);
  if (r.op == HC_OP_INSERT) {
    if (info.kind == HC_COUNTING && r.h_values != nullptr) return fail(HC_E_ARG, "counting tables take no values");
    if (info.kind == HC_SINGLE_VALUE && r.n > 0 && r.h_values == nullptr) return fail(HC_E_ARG, "values is NULL");
  }
  Request* q = new (std::nothrow) Request();
  if (!q) return fail(HC_E_NOMEM, "host allocation failed");
  q->r = r;
  q->bytes = hc_server_s::bytes_of(r);
  if (q->bytes > s->p.staging_bytes) {
    delete q;
    return fail(HC_E_ARG, "request needs %llu staging bytes, the server has %llu", (unsigned long long)q->bytes,
                (unsigned long long)s->p.staging_bytes);
  }
  q->arrival = Clock::now();
  std::lock_guard<std::mutex> lock(s->mu);
  if (s->error != HC_OK) {
    delete q;
    return fail(s->error, "server failed earlier: %s", s->error_msg.c_str());
  }
  const uint64_t t = s->reqs.size();
  s->reqs.push_back(q);
  if (r.n == 0) {
    q->done = true;
    q->done_at = q->arrival;
    ++s->completed;
  } else {
    s->pending.push_back(t);
    s->cv_work.notify_one();
  }
  if (h_ticket) *h_ticket = t;
  return HC_OK;
}

hc_err hc_server_query(hc_server s, uint64_t ticket, int* h_done, double* h_latency_us) {
  using hc::fail;
  if (s == nullptr) return fail(HC_E_ARG, "server is NULL");
  std::lock_guard<std::mutex> lock(s->mu);
  if (ticket >= s->reqs.size()) return fail(HC_E_ARG, "unknown ticket %llu", (unsigned long long)ticket);
  const Request* r = s->reqs[ticket];
  if (h_done) *h_done = r->done ? 1 : 0;
  if (h_latency_us)
    *h_latency_us = r->done ? std::chrono::duration<double, std::micro>(r->done_at - r->arrival).count() : -1.0;
  if (s->error != HC_OK && !r->done) return fail(s->error, "server failed: %s", s->error_msg.c_str());
  return HC_OK;
}

hc_err hc_server_wait(hc_server s, uint64_t ticket) {
  using hc::fail;
  if (s == nullptr) return fail(HC_E_ARG, "server is NULL");
  std::unique_lock<std::mutex> lock(s->mu);
  if (ticket >= s->reqs.size()) return fail(HC_E_ARG, "unknown ticket %llu", (unsigned long long)ticket);
  s->cv_done.wait(lock, [&] { return s->reqs[ticket]->done || s->error != HC_OK; });
  if (!s->reqs[ticket]->done) return fail(s->error, "server failed: %s", s->error_msg.c_str());
  return HC_OK;
}

hc_err hc_server_drain(hc_server s) {
  using hc::fail;
  if (s == nullptr) return fail(HC_E_ARG, "server is NULL");
  std::unique_lock<std::mutex> lock(s->mu);
  s->cv_done.wait(lock, [&] {
    return (s->pending.empty() && s->inflight.empty() && s->launching == 0) || s->error != HC_OK;
  });
  if (s->error != HC_OK) return fail(s->error, "server failed: %s", s->error_msg.c_str());
  return HC_OK;
}

hc_err hc_server_stats(hc_server s, hc_server_counts* h_out) {
  using hc::fail;
  if (s == nullptr || h_out == nullptr) return fail(HC_E_ARG, "server or out is NULL");
  std::lock_guard<std::mutex> lock(s->mu);
  h_out->submitted = s->reqs.size();
  h_out->completed = s->completed;
  h_out->launch_groups = s->groups;
  h_out->ops_completed = s->ops_done;
  h_out->staging_in_use = s->head - s->tail;
  h_out->staging_bytes = s->p.staging_bytes;
  return HC_OK;
}

hc_err hc_server_destroy(hc_server s) {
  if (s == nullptr) return HC_OK;
  {
    std::lock_guard<std::mutex> lock(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipDeviceSynchronize();
  for (auto& sl : s->slots) {
    if (sl.d_descs) (void)hipFree(sl.d_descs);
    if (sl.d_cs) (void)hipFree(sl.d_cs);
    if (sl.h_descs) (void)hipHostFree(sl.h_descs);
    if (sl.h_cs) (void)hipHostFree(sl.h_cs);
    if (sl.kernel_done) (void)hipEventDestroy(sl.kernel_done);
    if (sl.done) (void)hipEventDestroy(sl.done);
  }
  for (auto st : s->streams)
    if (st) (void)hipStreamDestroy(st);
  if (s->d_staging) (void)hipFree(s->d_staging);
  for (auto* r : s->reqs) delete r;
  delete s;
  return HC_OK;
}

}  // extern "C"
