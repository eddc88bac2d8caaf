"""Benchmark: bulk insert and bulk retrieval on a 2^28-slot single-value table at load 0.9.

One step = clear the table, insert n = floor(0.9 * 2^28) distinct uint32 keys with
uint32 values, then retrieve 2n queries (the n present keys and n absent keys,
shuffled).  Inputs are synthetic and seeded, resident in HBM before timing.
Kernel times come from HIP events on the stream the library launches on.

Prints ONE JSON line.  `value` is the whole step's rate in G operations/s
(inserts + retrievals); the per-phase rates, p50/p99 phase latencies, the HBM
roofline of the dominant kernel and the CPU oracle's rate sit beside it.

Algorithmic bytes per operation (what the method must move; windows per
operation from the sequential probing model at this load, double hashing,
W = 16, used for every configuration so extra probing earns no credit):
  insert    8 + 128 * 1.109 + 128                      = 277.95 B
  retrieve  present 9 + 128 * 1.109, absent 9 + 128 * 2.127, 50/50 mix = 216.1 B
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
W_HIT, W_MISS = 1.109, 2.127            # windows per present / absent key at load 0.9
B_INSERT = 8 + 128 * W_HIT + 128        # key+value in, windows read, claimed line written back
B_RETRIEVE = 0.5 * (9 + 128 * W_HIT) + 0.5 * (9 + 128 * W_MISS)
KERNEL_NAMES = {"insert": "k_insert_unique", "retrieve": "k_retrieve"}


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="single", choices=["single", "batched", "serving", "multi", "sweep", "bucket", "wide", "set", "bloom"],
                    help="single: the 2^28-slot table (default); batched: 256 tables in one launch; "
                         "serving: Poisson request stream on 16 resident tables; multi: counting and "
                         "multi-value tables; sweep: load x scheme x group size on the 2^28-slot table; "
                         "bucket: bucket list tables on the multi-value workloads; wide: 64-bit keys and values")
    ap.add_argument("--loads", default="0.5,0.8,0.9,0.95,0.99", help="sweep: load factors")
    ap.add_argument("--requests", type=int, default=1500)
    ap.add_argument("--max-log2-request", type=int, default=24)
    ap.add_argument("--zipf", action="store_true", help="serving: Zipf(1.1) keys instead of uniform")
    ap.add_argument("--max-group-ops", type=int, default=1 << 22, help="serving: most elements per launch group (0: any)")
    ap.add_argument("--server-streams", type=int, default=3, help="serving: streams of the server")
    ap.add_argument("--tables", type=int, default=256)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--log2-capacity", type=int, default=28)
    ap.add_argument("--load", type=float, default=0.9)
    ap.add_argument("--scheme", default="double")
    ap.add_argument("--window", type=int, default=16)
    ap.add_argument("--group-insert", type=int, default=4)
    ap.add_argument("--group-query", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-log2", type=int, default=25)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run one device copy of this size (HBM counter calibration)")
    return ap.parse_args()


# Sources of the single-table insert and retrieve kernels and of their launch shape: a
# counter record taken with other contents of these files no longer describes the kernels.
KERNEL_SOURCES = ("hc_device.hpp", "hc_kernels.hpp", "hc_launch.hpp", "hc_launch.hip", "hc_k_insert.hip",
                  "hc_k_query.hip")


def _csrc_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2009_07914_amd", "csrc")
    for f in KERNEL_SOURCES:
        h.update(f.encode())
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def _traffic(kernel: str, workload: str):
    """HBM bytes per launch from committed counter runs, if they match the current kernels."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(p))[workload][kernel]
    except Exception:
        return None
    if rec.get("csrc_sha") != _csrc_hash():
        return None
    return rec.get("bytes_per_launch")


def _host_cpus():
    """(model name, logical CPUs of the host, CPUs this process may use): the affinity mask, further
    limited by a cgroup CPU quota where one is set."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0))
    try:
        quota, period = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if quota != "max":
            usable = max(1, min(usable, int(int(quota) // int(period))))
    except (OSError, ValueError):
        pass
    return model, os.cpu_count() or 1, usable


def _measured_frac(traffic_bytes, ms):
    if not traffic_bytes:
        return None
    return round(traffic_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)


def _cpu_baseline(w, log2n: int):
    """The oracle as it stands, single thread, on a bounded sample of the same workload."""
    import numpy as np
    import oracle

    m = 1 << log2n
    keys, vals = w["keys"][:m], w["values"][:m]
    q = np.concatenate([keys, w["absent"][:m]])
    t = oracle.OracleTable(oracle.SINGLE, 1 << 28)
    t0 = time.perf_counter()
    t.insert(keys, vals)
    t1 = time.perf_counter()
    t.retrieve(q)
    t2 = time.perf_counter()
    ops = keys.size + q.size
    model, nproc, usable = _host_cpus()
    return {"value": round(ops / (t2 - t0) / 1e9, 6), "unit": "G ops/s", "cores": 1, "kind": "oracle",
            "cpu_model": model, "nproc": nproc, "cpus_usable": usable,
            "sample": f"first 2^{log2n} keys inserted, then 2^{log2n + 1} queries (50/50 present/absent) "
                      f"of the same workload; insert {keys.size / (t1 - t0) / 1e6:.2f} M/s, "
                      f"retrieve {q.size / (t2 - t1) / 1e6:.2f} M/s, {t2 - t0:.1f} s"}


def _cpu_multicore(w, log2n: int):
    """The same sample on the oracle sharded by key hash across the host's cores (one independent oracle
    table per thread; the library call releases the interpreter lock): the analogue of a multi-core CPU
    hash map, reported beside the single-core baseline."""
    import threading

    import numpy as np
    import oracle

    model, nproc, threads = _host_cpus()  # every CPU this process may use
    m = 1 << log2n
    keys, vals = w["keys"][:m], w["values"][:m]
    q = np.concatenate([keys, w["absent"][:m]])
    shard_of = lambda k: ((k.astype(np.uint64) * np.uint64(0x9E3779B1)) >> np.uint64(16)) % np.uint64(threads)  # noqa: E731
    ks, qs = shard_of(keys), shard_of(q)
    parts = [(keys[ks == j], vals[ks == j], q[qs == j]) for j in range(threads)]
    tables = [oracle.OracleTable(oracle.SINGLE, 1 << 28) for _ in range(threads)]

    def phase(fn):
        ths = [threading.Thread(target=fn, args=(j,)) for j in range(threads)]
        t0 = time.perf_counter()
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        return time.perf_counter() - t0

    ti = phase(lambda j: tables[j].insert(parts[j][0], parts[j][1]))
    tr = phase(lambda j: tables[j].retrieve(parts[j][2]))
    ops = keys.size + q.size
    return {"value": round(ops / (ti + tr) / 1e9, 6), "unit": "G ops/s", "threads": threads,
            "cpu_model": model, "nproc": nproc,
            "kind": "oracle sharded by key hash, one table per thread",
            "sample": f"the single-core sample; insert {keys.size / ti / 1e6:.2f} M/s, "
                      f"retrieve {q.size / tr / 1e6:.2f} M/s"}


def main():
    args = _parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the tables run on one GPU (no sharding across GPUs); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "sweep":
        return bench_sweep(args)
    if args.workload == "bucket":
        return bench_bucket(args)
    if args.workload == "set":
        return bench_set(args)
    if args.workload == "bloom":
        return bench_bloom(args)
    if args.workload == "wide":
        return bench_wide(args)
    if args.workload == "multi":
        return bench_multi(args)
    import numpy as np
    import torch

    lib = os.path.join(ROOT, "paper_2009_07914_amd", "libhc.so")
    if not os.path.exists(lib):
        import __graft_entry__
        __graft_entry__.build()
    import gen
    import paper_2009_07914_amd as hc

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    cap = 1 << args.log2_capacity
    t_gen = time.perf_counter()
    w = gen.single_value_workload(cap, args.load, gen.SEED_BASE + 1)
    n = w["n"]
    print(f"# workload generated in {time.perf_counter() - t_gen:.1f} s: n={n}", file=sys.stderr, flush=True)

    table = hc.Table("single", cap, scheme=args.scheme, window=args.window, group=args.group_insert,
                     device=dev)
    keys = torch.from_numpy(w["keys"]).to(dev)
    vals = torch.from_numpy(w["values"]).to(dev)
    q = torch.from_numpy(w["queries"]).to(dev)
    vout = torch.empty(q.numel(), dtype=torch.uint32, device=dev)
    fout = torch.empty(q.numel(), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    def step(record=None):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        hc.hc_clear(table.handle, stream)
        ev[0].record(stream)
        hc.hc_insert(table.handle, keys, vals, None, args.group_insert, stream)
        ev[1].record(stream)
        ev[2].record(stream)
        hc.hc_retrieve(table.handle, q, vout, fout, args.group_query, stream)
        ev[3].record(stream)
        if record is not None:
            record.append(ev)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(evs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ins_ms = [e[0].elapsed_time(e[1]) for e in evs]
    ret_ms = [e[2].elapsed_time(e[3]) for e in evs]

    # parity on the timed outputs: size, and every query's value / found flag
    assert table.size() == n, "size mismatch after insert"
    f = fout.cpu().numpy()
    v = vout.cpu().numpy()
    src = w["query_src"]
    present = src < n                       # query j is (present ++ absent)[src[j]]
    assert np.array_equal(f.astype(bool), present), "found flags disagree with the key sets"
    assert np.array_equal(v[present], w["values"][src[present].astype(np.int64)]), "retrieved values disagree"
    assert not v[~present].any()
    del src, present, f, v

    ms_step = wall * 1000 / args.steps
    ins_avg, ret_avg = statistics.mean(ins_ms), statistics.mean(ret_ms)
    ins_gops = n / (ins_avg * 1e-3) / 1e9
    ret_gops = q.numel() / (ret_avg * 1e-3) / 1e9
    ins_gbs = n * B_INSERT / (ins_avg * 1e-3) / 1e9
    ret_gbs = q.numel() * B_RETRIEVE / (ret_avg * 1e-3) / 1e9
    dom = "insert" if sum(ins_ms) >= sum(ret_ms) else "retrieve"
    workload = f"single_value_l{args.log2_capacity}_a{args.load}"
    dom_gbs = ins_gbs if dom == "insert" else ret_gbs
    tr = _traffic(KERNEL_NAMES[dom], workload)

    def pct(xs, p):
        xs = sorted(xs)
        return xs[min(len(xs) - 1, int(round(p / 100 * (len(xs) - 1))))]

    out = {
        "metric": "G inserts/s and G retrievals/s at load 0.9 (uint32 k/v), % of HBM peak; p99 latency",
        "value": round((n + q.numel()) / (ms_step * 1e-3) / 1e9, 4),
        "unit": "G ops/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "single-value table, 2^%d slots (%d GiB), load %.2f, uint32 keys uniform distinct, "
                               "insert all then retrieve 50%% present / 50%% absent" %
                               (args.log2_capacity, (cap * 8) >> 30, args.load),
                   "capacity": table.capacity, "n_insert": n, "n_retrieve": q.numel(),
                   "scheme": args.scheme, "window": args.window,
                   "group_insert": args.group_insert, "group_query": args.group_query},
        "insert_gops": round(ins_gops, 4), "retrieve_gops": round(ret_gops, 4),
        "insert_ms": {"mean": round(ins_avg, 4), "p50": round(pct(ins_ms, 50), 4), "p99": round(pct(ins_ms, 99), 4)},
        "retrieve_ms": {"mean": round(ret_avg, 4), "p50": round(pct(ret_ms, 50), 4), "p99": round(pct(ret_ms, 99), 4)},
        "insert_hbm_frac": round(ins_gbs / HBM_PEAK_GBS, 4),
        "retrieve_hbm_frac": round(ret_gbs / HBM_PEAK_GBS, 4),
        # counter-measured DRAM bytes (FETCH_SIZE + WRITE_SIZE of the committed counter runs, when they
        # describe the current kernels) over the same kernel times: the model charges a whole 128-byte
        # line written back per claim, the memory system writes back the dirty 64-byte half
        "insert_hbm_frac_measured": _measured_frac(_traffic(KERNEL_NAMES["insert"], workload), ins_avg),
        "retrieve_hbm_frac_measured": _measured_frac(_traffic(KERNEL_NAMES["retrieve"], workload), ret_avg),
        "roofline": {"bound": "hbm", "kernel": KERNEL_NAMES[dom], "achieved": round(dom_gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(dom_gbs / HBM_PEAK_GBS, 4),
                     "traffic": tr},
        "cpu_baseline": None,
    }
    out["ceilings"] = _ceilings(hc, table, dev, stream)
    out["ceilings"]["retrieve_frac_of_gather128"] = round(ret_gbs / out["ceilings"]["gather128_gbs"], 4)
    out["ceilings"]["insert_frac_of_gather128"] = round(ins_gbs / out["ceilings"]["gather128_gbs"], 4)
    out["ceilings"]["insert_frac_of_atomic_cas"] = round(ins_gops / out["ceilings"]["atomic_cas_gops"], 4)
    if args.calibrate_copy_mib:
        a = torch.empty(args.calibrate_copy_mib << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
    del keys, vals, q, vout, fout
    table.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = _cpu_baseline(w, args.cpu_sample_log2)
        out["cpu_multicore"] = _cpu_multicore(w, args.cpu_sample_log2)
    print(json.dumps(out), flush=True)


def _ceilings(hc, table, dev, s):
    """Practical bandwidth ceilings of this GPU, measured with the library's diagnostic kernels: a streaming
    copy of 1 GiB (read + write bytes), a streaming read of it, and gathers of random 64- and 128-byte lines over the table's own
    2 GiB slot array (as many lines as it holds; no cache holds a useful share of it)."""
    import torch

    info = hc.hc_info(table.handle)
    nbytes = info.capacity * 8
    sink = torch.zeros(1, dtype=torch.uint32, device=dev)

    def timed(fn, reps=5):
        fn()
        ms = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            fn()
            b.record(s)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        return statistics.mean(ms)

    res = {}
    a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    res["copy_gbs"] = round(2 * a.numel() / timed(lambda: hc.hc_diag_copy(b, a, s)) / 1e6, 1)
    res["read_gbs"] = round(a.numel() / timed(lambda: hc.hc_diag_read(a, sink, s)) / 1e6, 1)
    del a, b
    for lb in (64, 128):
        n_lines = nbytes // lb
        ms = timed(lambda: hc.hc_diag_gather(info.d_slots, nbytes, lb, n_lines, sink, 0x5EED, s))
        res[f"gather{lb}_gbs"] = round(n_lines * lb / ms / 1e6, 1)
    # random atomics over a scratch region of the table's size: claims (CAS with return) and ORs
    region = torch.zeros(nbytes // 8, dtype=torch.int64, device=dev)
    n_ops = nbytes // 16
    res["atomic_cas_gops"] = round(n_ops / timed(lambda: hc.hc_diag_atomic(region, True, n_ops, sink, 7, s)) / 1e6, 2)
    res["atomic_or_gops"] = round(n_ops / timed(lambda: hc.hc_diag_atomic(region, False, n_ops, sink, 9, s)) / 1e6, 2)
    del region
    return res


def bench_batched(args):
    """Many independent single-value tables (capacities log-uniform in [2^10, 2^24], loads uniform in
    [0.6, 0.95]): build all, then query all 50/50, as (a) one launch per table and operation, with the
    default layout and with the autotuned one, (b) one batched plan (one launch per phase, or every phase
    in one gated launch), and (c) the plan replayed as a graph."""
    import numpy as np
    import torch

    lib = os.path.join(ROOT, "paper_2009_07914_amd", "libhc.so")
    if not os.path.exists(lib):
        import __graft_entry__
        __graft_entry__.build()
    import gen
    import paper_2009_07914_amd as hc
    from paper_2009_07914_amd import autotune

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    s = torch.cuda.current_stream()
    spec = gen.batched_tables_spec(args.tables, 10, 24, 0.6, 0.95, 16, gen.SEED_BASE + 3)
    sets = {}
    for label in ("default", "tuned"):
        tabs = []
        for sp in spec:
            cfg = dict(autotune.DEFAULT) if label == "default" else autotune.choose(sp["capacity"], sp["load"])
            t = hc.Table("single", sp["capacity"], scheme=cfg["scheme"], window=cfg["window"],
                         group=cfg["group_insert"], seed=sp["seed"], device=dev)
            tabs.append((t, cfg))
        sets[label] = tabs
    data = []
    for sp, (t, _) in zip(spec, sets["default"]):
        w = gen.single_value_workload(sp["capacity"], sp["load"], sp["seed"])
        k, v, q = (torch.from_numpy(w[x]).to(dev) for x in ("keys", "values", "queries"))
        vo = torch.empty(q.numel(), dtype=torch.uint32, device=dev)
        fo = torch.empty(q.numel(), dtype=torch.uint8, device=dev)
        data.append({"n": w["n"], "k": k, "v": v, "q": q, "vo": vo, "fo": fo, "src": w["query_src"],
                     "values": w["values"]})
    n_ins = sum(x["n"] for x in data)
    n_ret = sum(x["q"].numel() for x in data)
    ops_total = n_ins + n_ret

    def clear(tabs):
        for t, _ in tabs:
            hc.hc_clear(t.handle, s)

    def per_table(tabs):
        for (t, cfg), x in zip(tabs, data):
            hc.hc_insert(t.handle, x["k"], x["v"], None, cfg["group_insert"], s)
        for (t, cfg), x in zip(tabs, data):
            hc.hc_retrieve(t.handle, x["q"], x["vo"], x["fo"], cfg["group_query"], s)

    def plan(tabs, one_launch=False):
        ops = [(hc.hc_batch_op(t, hc.OP_INSERT, x["k"], x["v"], group=cfg["group_insert"]), [x["k"], x["v"]])
               for (t, cfg), x in zip(tabs, data)]
        ops += [(hc.hc_batch_op(t, hc.OP_RETRIEVE, x["q"], values_out=x["vo"], flags=x["fo"],
                                group=cfg["group_query"]), [x["q"], x["vo"], x["fo"]])
                for (t, cfg), x in zip(tabs, data)]
        return hc.Batch(ops, one_launch=one_launch)

    def timed(tabs, fn):
        ms = []
        for rep in range(args.warmup + args.steps):
            clear(tabs)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            fn()
            b.record(s)
            torch.cuda.synchronize()
            if rep >= args.warmup:
                ms.append(a.elapsed_time(b))
        return ms

    def check(tabs):
        for (t, _), x in zip(tabs, data):
            f = x["fo"].cpu().numpy()
            v = x["vo"].cpu().numpy()
            present = x["src"] < x["n"]
            assert np.array_equal(f.astype(bool), present), "found flags disagree"
            assert np.array_equal(v[present], x["values"][x["src"][present].astype(np.int64)]), "values disagree"
            assert t.size() == x["n"], "size disagrees"

    res = {}
    res["per_table_default"] = timed(sets["default"], lambda: per_table(sets["default"]))
    check(sets["default"])
    res["per_table_tuned"] = timed(sets["tuned"], lambda: per_table(sets["tuned"]))
    check(sets["tuned"])
    b_def = plan(sets["default"])
    res["batched_default"] = timed(sets["default"], lambda: b_def.launch(s))
    check(sets["default"])
    b_def.capture()
    res["graph_default"] = timed(sets["default"], lambda: b_def.replay(s))
    check(sets["default"])
    b_tun = plan(sets["tuned"])
    res["batched_tuned"] = timed(sets["tuned"], lambda: b_tun.launch(s))
    check(sets["tuned"])
    b_tun.capture()
    res["graph_tuned"] = timed(sets["tuned"], lambda: b_tun.replay(s))
    check(sets["tuned"])
    # default layouts, both phases in one launch: each table's queries wait on the device for its own
    # build only, so tables built early are queried while the others are still being built
    b_one = plan(sets["default"], one_launch=True)
    res["batched_one_launch"] = timed(sets["default"], lambda: b_one.launch(s))
    check(sets["default"])
    b_one.capture()
    res["graph_one_launch"] = timed(sets["default"], lambda: b_one.replay(s))
    check(sets["default"])
    assert b_one.abandoned_waits() == 0, "a completion wait was abandoned"

    def pct(xs, p):
        xs = sorted(xs)
        return xs[min(len(xs) - 1, int(round(p / 100 * (len(xs) - 1))))]

    summary = {k: {"ms_mean": round(statistics.mean(v), 4), "ms_p50": round(pct(v, 50), 4),
                   "ms_p99": round(pct(v, 99), 4), "gops": round(ops_total / (statistics.mean(v) * 1e-3) / 1e9, 4)}
               for k, v in res.items()}
    # the graph of the faster layout set: per-table tuned layouts need the mixed kernel (one launch for
    # several (g, W) pairs, fewer waves per SIMD) where they differ, the default layout one lean kernel
    best_label = min(("graph_default", "graph_tuned", "graph_one_launch"), key=lambda k: summary[k]["ms_mean"])
    best = summary[best_label]
    layouts = {}
    for _, cfg in sets["tuned"]:
        key = f"{cfg['scheme']}/W{cfg['window']}/g{cfg['group_insert']},{cfg['group_query']}"
        layouts[key] = layouts.get(key, 0) + 1
    out = {
        "metric": "G ops/s, build then 50/50 query of many tables: batched graph launch vs one launch per table",
        "value": best["gops"], "unit": "G ops/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": best["ms_mean"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"{args.tables} single-value tables, capacity log-uniform in [2^10, 2^24], "
                               f"load uniform in [0.6, 0.95], uint32 keys; build all then query present+absent",
                   "tables": args.tables, "plan": best_label[len("graph_"):],
                   "slots": sum(t.capacity for t, _ in sets["tuned" if best_label == "graph_tuned" else "default"]),
                   "n_insert": n_ins, "n_retrieve": n_ret, "tuned_layouts": layouts,
                   "plan_phases": b_tun.phases, "plan_launches_tuned": b_tun.launches,
                   "plan_launches_default": b_def.launches, "plan_launches_one_launch": b_one.launches},
        "modes": summary,
        "speedup_graph_vs_per_table_default": round(summary["per_table_default"]["ms_mean"] / best["ms_mean"], 3),
    }
    b_def.close()
    b_tun.close()
    b_one.close()
    print(json.dumps(out), flush=True)


def bench_multi(args):
    """Counting table: 2^26 keys drawn from Zipf(1.1) over 2^22 distinct k-mer-like keys into 2^27 slots,
    then the count of every one of the 2^22 keys.  Multi-value table: 2^26 pairs with keys uniform on
    1..2^26/r into 2^27 slots, then count / prefix sum / retrieve-all for the queries 1..2^26 (the
    paper's multiplicity workload), r in {1, 4, 16, 64}."""
    import numpy as np
    import torch

    lib = os.path.join(ROOT, "paper_2009_07914_amd", "libhc.so")
    if not os.path.exists(lib):
        import __graft_entry__
        __graft_entry__.build()
    import gen
    import paper_2009_07914_amd as hc

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    s = torch.cuda.current_stream()
    cap, n = 1 << 27, 1 << 26

    def ev_time(fn, reps):
        ms = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            pre = fn[0]
            if pre:
                pre()
            a.record(s)
            fn[1]()
            b.record(s)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        return ms

    reps = args.warmup + args.steps
    res = {}
    # ---- counting, Zipf(1.1)
    w = gen.multi_value_zipf_workload(n, 1 << 22, 1.1, gen.SEED_BASE + 2)
    keys = torch.from_numpy(w["keys"]).to(dev)
    q = torch.from_numpy(w["queries"]).to(dev)
    ct = hc.Table("counting", cap, scheme="double", window=16, group=4, device=dev)
    cnt = torch.empty(q.numel(), dtype=torch.uint32, device=dev)
    fnd = torch.empty(q.numel(), dtype=torch.uint8, device=dev)
    u, c = np.unique(w["keys"], return_counts=True)
    expect = np.zeros(q.numel(), dtype=np.uint32)
    pos = np.searchsorted(u, w["queries"])
    hit = (pos < u.size) & (u[np.minimum(pos, u.size - 1)] == w["queries"])
    expect[hit] = c[pos[hit]]
    # per-key insert: equal keys of each 2048-key tile are combined in LDS, then one upsert per
    # distinct key of the tile (the hottest key costs one atomic per tile, not one per occurrence)
    st_ct = torch.empty(n, dtype=torch.uint8, device=dev)
    ins = ev_time((ct.clear, lambda: hc.hc_insert(ct.handle, keys, None, None, args.group_insert, s)), reps)[args.warmup:]
    ins_st = ev_time((ct.clear, lambda: hc.hc_insert(ct.handle, keys, None, st_ct, args.group_insert, s)),
                     reps)[args.warmup:]
    hc.hc_retrieve(ct.handle, q, cnt, fnd, args.group_query, s)
    assert np.array_equal(cnt.cpu().numpy(), expect), "counts disagree with numpy.unique"
    assert int((st_ct == hc.S_OK).sum()) == u.size, "one OK status per distinct key"
    fails = ct.stats()["cas_fails"]
    # grouped insert: one insert per distinct key with its multiplicity
    gins = ev_time((ct.clear, lambda: hc.hc_insert_grouped(ct.handle, keys, None, s)), reps)[args.warmup:]
    ret = ev_time((None, lambda: hc.hc_retrieve(ct.handle, q, cnt, fnd, args.group_query, s)), reps)[args.warmup:]
    assert np.array_equal(cnt.cpu().numpy(), expect), "counts disagree with numpy.unique"
    assert ct.size() == u.size
    res["counting_zipf"] = {"insert_per_key_ms": round(statistics.mean(ins), 4),
                            "insert_per_key_status_ms": round(statistics.mean(ins_st), 4),
                            "insert_per_key_cas_fails": int(fails),
                            "insert_grouped_ms": round(statistics.mean(gins), 4),
                            "retrieve_ms": round(statistics.mean(ret), 4),
                            "insert_per_key_gops": round(n / statistics.mean(ins) / 1e6, 4),
                            "insert_grouped_gops": round(n / statistics.mean(gins) / 1e6, 4),
                            "retrieve_gops": round(q.numel() / statistics.mean(ret) / 1e6, 4),
                            "distinct_keys": int(u.size), "top_key_count": int(c.max())}
    del keys, q, cnt, fnd, ct, w, st_ct
    # ---- counting, keys uniform on 1..2^26 (few repeats): the cost of combining where it saves little
    w = gen.multi_value_uniform_r_workload(n, 1, gen.SEED_BASE + 4)
    keys = torch.from_numpy(w["keys"]).to(dev)
    ct = hc.Table("counting", cap, scheme="double", window=16, group=4, device=dev)
    ins = ev_time((ct.clear, lambda: hc.hc_insert(ct.handle, keys, None, None, args.group_insert, s)), reps)[args.warmup:]
    u = np.unique(w["keys"])
    assert ct.size() == u.size
    res["counting_uniform"] = {"insert_per_key_ms": round(statistics.mean(ins), 4),
                               "insert_per_key_gops": round(n / statistics.mean(ins) / 1e6, 4),
                               "distinct_keys": int(u.size)}
    del keys, ct, w
    # ---- multi-value, uniform multiplicity r
    mv = hc.Table("multi", cap, scheme="double", window=16, group=4, device=dev)
    for r in (1, 4, 16, 64):
        w = gen.multi_value_uniform_r_workload(n, r, gen.SEED_BASE + 20 + r)
        keys = torch.from_numpy(w["keys"]).to(dev)
        vals = torch.from_numpy(w["values"]).to(dev)
        q = torch.from_numpy(w["queries"]).to(dev)
        offs = torch.empty(n + 1, dtype=torch.uint64, device=dev)
        out = torch.empty(n, dtype=torch.uint32, device=dev)
        ins = ev_time((mv.clear, lambda: hc.hc_insert(mv.handle, keys, vals, None, 8, s)), reps)[args.warmup:]
        # grouped: sort, then one walk per run of equal keys (the table the queries below check)
        gins = ev_time((mv.clear, lambda: hc.hc_insert_grouped(mv.handle, keys, vals, s)), reps)[args.warmup:]
        cnt_ms = ev_time((None, lambda: hc.hc_count_values(mv.handle, q, offs, None, False, 4, s)), reps)[args.warmup:]
        wr_ms = ev_time((None, lambda: hc.hc_retrieve_all(mv.handle, q, offs, out, 4, s)), reps)[args.warmup:]
        off = offs.cpu().numpy()
        assert int(off[-1]) == n, "sum of counts must equal the number of stored pairs"
        # sampled segments against lexsort grouping of the inputs
        order = np.lexsort((w["values"], w["keys"]))
        sk, sv = w["keys"][order], w["values"][order]
        o = out.cpu().numpy()
        for qi in np.linspace(0, n - 1, 2000).astype(np.int64):
            key = w["queries"][qi]
            lo, hi = np.searchsorted(sk, key, "left"), np.searchsorted(sk, key, "right")
            seg = np.sort(o[off[qi]:off[qi + 1]])
            assert np.array_equal(seg, sv[lo:hi]), "segment disagrees"
        t_all = statistics.mean(cnt_ms) + statistics.mean(wr_ms)
        best = min(statistics.mean(ins), statistics.mean(gins))
        res[f"multi_uniform_r{r}"] = {"insert_ms": round(statistics.mean(ins), 4),
                                      "insert_grouped_ms": round(statistics.mean(gins), 4),
                                      "count_scan_ms": round(statistics.mean(cnt_ms), 4),
                                      "write_ms": round(statistics.mean(wr_ms), 4),
                                      "insert_gops": round(n / best / 1e6, 4),
                                      "retrieve_all_gops": round(n / t_all / 1e6, 4)}
        del keys, vals, q, offs, out, w
    # ---- multi-value, Zipf(1.1) keys: grouped insert, then every distinct key's values (long queries)
    w = gen.multi_value_zipf_workload(n, 1 << 22, 1.1, gen.SEED_BASE + 3)
    keys = torch.from_numpy(w["keys"]).to(dev)
    vals = torch.from_numpy(w["values"]).to(dev)
    q = torch.from_numpy(w["queries"]).to(dev)
    nq = q.numel()
    offs = torch.empty(nq + 1, dtype=torch.uint64, device=dev)
    out = torch.empty(n, dtype=torch.uint32, device=dev)
    ins = ev_time((mv.clear, lambda: hc.hc_insert_grouped(mv.handle, keys, vals, s)), reps)[args.warmup:]
    cnt_ms = ev_time((None, lambda: hc.hc_count_values(mv.handle, q, offs, None, False, 4, s)), reps)[args.warmup:]
    wr_ms = ev_time((None, lambda: hc.hc_retrieve_all(mv.handle, q, offs, out, 4, s)), reps)[args.warmup:]
    off = offs.cpu().numpy()
    assert int(off[-1]) == n, "sum of counts must equal the number of stored pairs"
    order = np.lexsort((w["values"], w["keys"]))
    sk, sv = w["keys"][order], w["values"][order]
    o = out.cpu().numpy()
    heavy = np.argsort(np.diff(off.astype(np.int64)))[-8:]  # the eight longest segments, plus a spread
    for qi in np.concatenate([heavy, np.linspace(0, nq - 1, 2000).astype(np.int64)]):
        key = w["queries"][qi]
        lo, hi = np.searchsorted(sk, key, "left"), np.searchsorted(sk, key, "right")
        seg = np.sort(o[off[qi]:off[qi + 1]])
        assert np.array_equal(seg, sv[lo:hi]), "segment disagrees"
    t_all = statistics.mean(cnt_ms) + statistics.mean(wr_ms)
    res["multi_zipf_grouped"] = {"insert_ms": round(statistics.mean(ins), 4),
                                 "count_scan_ms": round(statistics.mean(cnt_ms), 4),
                                 "write_ms": round(statistics.mean(wr_ms), 4),
                                 "insert_gops": round(n / statistics.mean(ins) / 1e6, 4),
                                 "retrieve_all_gops": round(n / t_all / 1e6, 4),
                                 "top_key_count": int(np.diff(off.astype(np.int64)).max())}
    del keys, vals, q, offs, out, w
    out = {
        "metric": "G ops/s of counting and multi-value tables (insert; count / prefix sum / retrieve-all)",
        "value": res["multi_uniform_r16"]["retrieve_all_gops"], "unit": "G ops/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "2^27-slot tables, 2^26 uint32 pairs; counting: Zipf(1.1) over 2^22 keys; "
                               "multi-value: keys uniform on 1..2^26/r, queries 1..2^26; "
                               "skewed multi-value: Zipf(1.1) over 2^22 keys, grouped insert",
                   "capacity": cap, "pairs": n},
        "modes": res,
    }
    print(json.dumps(out), flush=True)


def bench_bucket(args):
    """Bucket list tables (s0 = 1, growth 2) on the multi-value workloads: 2^26 pairs with keys uniform on
    1..2^26/r, and 2^26 pairs Zipf(1.1) over 2^22 keys.  Insert (per pair and grouped), count + prefix sum,
    retrieve-all of every key; storage density = 4 bytes per distinct key and per value over the table's key slots,
    per-slot records and used pool words (a multi-value table of 2^27 slots holding the same pairs has
    4 (keys + 2^26) / 2^30)."""
    import numpy as np
    import torch

    lib = os.path.join(ROOT, "paper_2009_07914_amd", "libhc.so")
    if not os.path.exists(lib):
        import __graft_entry__
        __graft_entry__.build()
    import gen
    import paper_2009_07914_amd as hc

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    s = torch.cuda.current_stream()
    n = 1 << 26
    reps = args.warmup + args.steps

    def ev_time(fn, count):
        ms = []
        for _ in range(count):
            if fn[0]:
                fn[0]()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            fn[1]()
            b.record(s)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        return ms

    def check(w, q, offs, out):
        off = offs.cpu().numpy().astype(np.int64)
        assert int(off[-1]) == n, "sum of counts must equal the number of stored pairs"
        order = np.lexsort((w["values"], w["keys"]))
        sk, sv = w["keys"][order], w["values"][order]
        o = out.cpu().numpy()
        qh = q.cpu().numpy()
        heavy = np.argsort(np.diff(off))[-4:]
        for qi in np.concatenate([heavy, np.linspace(0, qh.size - 1, 1000).astype(np.int64)]):
            lo, hi = np.searchsorted(sk, qh[qi], "left"), np.searchsorted(sk, qh[qi], "right")
            assert np.array_equal(np.sort(o[off[qi]:off[qi + 1]]), sv[lo:hi]), "segment disagrees"

    res = {}
    grow2 = dict(s0=1, growth=2.0, smax=1 << 16)
    cases = [(f"uniform_r{r}", r, grow2) for r in (1, 4, 16, 64)]
    cases.append(("zipf", 0, grow2))
    # the paper's two settings: its default (growth 1.1 from s0 = 1) and its best case (one bucket of
    # s0 = the values per key, growth 1)
    cases += [(f"paper_default_r{r}", r, dict(s0=1, growth=1.1, smax=1 << 16)) for r in (1, 4, 16, 64)]
    cases += [(f"paper_optimal_r{r}", r, dict(s0=r, growth=1.0, smax=r)) for r in (4, 16, 64)]
    for name, r, bparams in cases:
        if r:
            w, distinct = gen.multi_value_uniform_r_workload(n, r, gen.SEED_BASE + 20 + r), n // r
        else:
            w, distinct = gen.multi_value_zipf_workload(n, 1 << 22, 1.1, gen.SEED_BASE + 3), 1 << 22
        keys = torch.from_numpy(w["keys"]).to(dev)
        vals = torch.from_numpy(w["values"]).to(dev)
        q = torch.from_numpy(w["queries"]).to(dev)
        cap = int(distinct / 0.8)
        t = hc.Table("bucket", cap, scheme="double", window=16, group=4, device=dev,
                     bucket=dict(bparams, pool_values=3 * n))
        row = {}
        if name != "zipf":  # per pair: the Zipf batch's hottest key would take 8 M atomics on one slot
            ins = ev_time((t.clear, lambda: hc.hc_insert(t.handle, keys, vals, None, 4, s)), reps)[args.warmup:]
            row["insert_ms"] = round(statistics.mean(ins), 4)
        gins = ev_time((t.clear, lambda: hc.hc_insert_grouped(t.handle, keys, vals, s)), reps)[args.warmup:]
        row["insert_grouped_ms"] = round(statistics.mean(gins), 4)
        assert t.size() == n
        offs = torch.empty(q.numel() + 1, dtype=torch.uint64, device=dev)
        out = torch.empty(n, dtype=torch.uint32, device=dev)
        cnt = ev_time((None, lambda: hc.hc_count_values(t.handle, q, offs, None, False, 4, s)), reps)[args.warmup:]
        wr = ev_time((None, lambda: hc.hc_retrieve_all(t.handle, q, offs, out, 4, s)), reps)[args.warmup:]
        check(w, q, offs, out)
        u = t.bucket_usage()
        st = t.stats()
        # stored information (each distinct key once, each value once, 32 bits each) over everything the table
        # holds: key slots (8 B), per-slot records (16 B: last-bucket offset and insert bookkeeping) and used
        # pool words
        density = (4.0 * (int(st["live"]) + n)) / (8.0 * t.capacity + 16.0 * t.capacity + 4.0 * u["pool_used"])
        best_ins = min(row.get("insert_ms", 1e9), row["insert_grouped_ms"])
        row.update({"count_scan_ms": round(statistics.mean(cnt), 4), "write_ms": round(statistics.mean(wr), 4),
                    "insert_gops": round(n / best_ins / 1e6, 4),
                    "retrieve_all_gops": round(n / (statistics.mean(cnt) + statistics.mean(wr)) / 1e6, 4),
                    "keys": int(st["live"]), "pool_used_words": int(u["pool_used"]),
                    "storage_density": round(density, 4)})
        row["bucket"] = f"s0 {bparams['s0']}, growth {bparams['growth']}, smax {bparams['smax']}"
        res[name] = row
        print("# " + json.dumps({name: row}), flush=True)
        del t, keys, vals, q, offs, out, w
        torch.cuda.empty_cache()
    out = {
        "metric": "G pairs/s of bucket list tables (insert; count / prefix sum / retrieve-all) and storage density",
        "value": res["zipf"]["retrieve_all_gops"], "unit": "G ops/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "bucket list tables (s0 1, growth 2, cap 2^16; and the paper's default growth 1.1 "
                               "and its one-bucket setting) for 2^26 uint32 pairs: keys uniform on 1..2^26/r, and "
                               "Zipf(1.1) over 2^22 keys; key table at load 0.8 of the distinct keys",
                   "pairs": n},
        "modes": res,
    }
    print(json.dumps(out), flush=True)


def bench_wide(args):
    """Single-value table with 64-bit keys and values: 2^27 slots of 16 bytes (2 GiB, the memory of the
    2^28-slot 32-bit table), load 0.9, double hashing, in both layouts: array of structures (W = 8 is one
    128-byte line) and structure of arrays (W = 16 keys is one line).  Insert all, then retrieve 50% present /
    50% absent; every retrieved value checked against the inserted ones."""
    import numpy as np
    import torch

    lib = os.path.join(ROOT, "paper_2009_07914_amd", "libhc.so")
    if not os.path.exists(lib):
        import __graft_entry__
        __graft_entry__.build()
    import gen
    import paper_2009_07914_amd as hc

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    s = torch.cuda.current_stream()
    cap = 1 << 27
    n = int(0.9 * cap)
    low = gen.keys(gen.derive_seed(gen.SEED_BASE, 41), 1, 2 * n).astype(np.uint64)
    high = gen.values(gen.derive_seed(gen.SEED_BASE, 42), 2 * n).astype(np.uint64)
    allk = (high << np.uint64(32)) | low
    vals = (gen.values(gen.derive_seed(gen.SEED_BASE, 43), n).astype(np.uint64) << np.uint64(32)) | low[:n]
    src = gen.permutation(gen.derive_seed(gen.SEED_BASE, 44), 2 * n).astype(np.int64)
    keys = torch.from_numpy(allk[:n]).to(dev)
    dvals = torch.from_numpy(vals).to(dev)
    q = torch.from_numpy(allk[src]).to(dev)
    out = torch.empty(2 * n, dtype=torch.uint64, device=dev)
    fnd = torch.empty(2 * n, dtype=torch.uint8, device=dev)
    present = src < n
    cells = []
    for kind, W, G in (("single64", 8, 4), ("single64", 8, 2), ("single64_soa", 16, 4), ("single64_soa", 8, 4),
                       ("single64_soa", 16, 8)):
        t = hc.Table(kind, cap, scheme="double", window=W, group=G, device=dev)
        assert t.capacity == cap
        ins, ret = [], []
        for rep in range(args.warmup + args.steps):
            t.clear()
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record(s)
            hc.hc_insert64(t.handle, keys, dvals, None, G, s)
            e[1].record(s)
            hc.hc_retrieve64(t.handle, q, out, fnd, G, s)
            e[2].record(s)
            torch.cuda.synchronize()
            if rep >= args.warmup:
                ins.append(e[0].elapsed_time(e[1]))
                ret.append(e[1].elapsed_time(e[2]))
        assert t.size() == n
        assert np.array_equal(fnd.cpu().numpy(), present.astype(np.uint8)), "found flags"
        o = out.cpu().numpy()
        assert np.array_equal(o[present], vals[src[present]]), "values"
        ti, tr = statistics.mean(ins), statistics.mean(ret)
        cells.append({"layout": "soa" if kind.endswith("soa") else "aos", "window": W, "group": G,
                      "insert_ms": round(ti, 4), "retrieve_ms": round(tr, 4), "insert_gops": round(n / ti / 1e6, 4),
                      "retrieve_gops": round(2 * n / tr / 1e6, 4)})
        print(json.dumps(cells[-1]), file=sys.stderr, flush=True)
        t.close()
    best = min(cells, key=lambda c: c["insert_ms"] + c["retrieve_ms"])
    ms = best["insert_ms"] + best["retrieve_ms"]
    res = {"metric": "G inserts/s and G retrievals/s, 64-bit keys and values at load 0.9", "value": round(
        (n + 2 * n) / ms / 1e6, 4), "unit": "G ops/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "single-value table, 64-bit keys and values, 2^27 slots (2 GiB), load 0.9, "
                               "double hashing, AoS and SoA layouts; retrieve 50% present / 50% absent",
                   "capacity": cap, "n_insert": n, "n_retrieve": 2 * n, "best": best},
        "cells": cells}
    print(json.dumps(res), flush=True)


def bench_set(args):
    """HashSet of 2^28 four-byte slots (1 GiB) at load 0.9, double hashing: insert all keys, then test
    membership of as many present and absent ones (50/50), for a few (W, g) pairs; every cell checked
    (size = n, found flags equal to presence)."""
    import numpy as np
    import torch

    lib = os.path.join(ROOT, "paper_2009_07914_amd", "libhc.so")
    if not os.path.exists(lib):
        import __graft_entry__
        __graft_entry__.build()
    import gen
    import paper_2009_07914_amd as hc

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    s = torch.cuda.current_stream()
    w = gen.single_value_workload(1 << args.log2_capacity, args.load, gen.derive_seed(gen.SEED_BASE, 51))
    n = w["n"]
    keys = torch.from_numpy(w["keys"]).to(dev)
    q = torch.from_numpy(w["queries"]).to(dev)
    present = (w["query_src"] < n).astype(np.uint8)
    fnd = torch.empty(q.numel(), dtype=torch.uint8, device=dev)
    cells = []
    for W, G in ((16, 2), (16, 4), (32, 4), (32, 8)):
        t = hc.Table("set", 1 << args.log2_capacity, scheme="double", window=W, group=G, device=dev)
        ins, ret = [], []
        for rep in range(args.warmup + args.steps):
            t.clear()
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record(s)
            hc.hc_insert(t.handle, keys, None, None, G, s)
            e[1].record(s)
            hc.hc_retrieve(t.handle, q, None, fnd, G, s)
            e[2].record(s)
            torch.cuda.synchronize()
            if rep >= args.warmup:
                ins.append(e[0].elapsed_time(e[1]))
                ret.append(e[1].elapsed_time(e[2]))
        assert t.size() == n, "size"
        assert np.array_equal(fnd.cpu().numpy(), present), "found flags"
        ti, tr = statistics.mean(ins), statistics.mean(ret)
        cells.append({"window": W, "group": G, "insert_ms": round(ti, 4), "contains_ms": round(tr, 4),
                      "insert_gops": round(n / ti / 1e6, 4), "contains_gops": round(q.numel() / tr / 1e6, 4)})
        print(json.dumps(cells[-1]), file=sys.stderr, flush=True)
        t.close()
    best = min(cells, key=lambda c: c["insert_ms"] + c["contains_ms"])
    ms = best["insert_ms"] + best["contains_ms"]
    res = {"metric": "G inserts/s and G membership queries/s, HashSet of 32-bit keys at load %g" % args.load,
           "value": round((n + q.numel()) / ms / 1e6, 4), "unit": "G ops/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": f"HashSet, 2^{args.log2_capacity} four-byte slots, load {args.load}, double "
                                  "hashing; membership queries 50% present / 50% absent",
                      "n_insert": n, "n_contains": int(q.numel()), "best": best},
           "cells": cells}
    print(json.dumps(res), flush=True)


def bench_bloom(args):
    """Split-block Bloom filter of 2^32 bits (2^23 blocks of 16 words, 512 MiB) and 2^28 keys (16 bits per
    key): insert all, then test 2^27 present and 2^27 absent keys, for every group size.  Each cell checked:
    no false negatives, false-positive rate within 5% of the filter's closed form for distinct keys."""
    import math

    import numpy as np
    import torch

    lib = os.path.join(ROOT, "paper_2009_07914_amd", "libhc.so")
    if not os.path.exists(lib):
        import __graft_entry__
        __graft_entry__.build()
    import gen
    import paper_2009_07914_amd as hc

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    s = torch.cuda.current_stream()
    words, n = 16, 1 << 28
    keys_h = gen.keys(gen.derive_seed(gen.SEED_BASE, 61), 1, n + (1 << 27))
    keys = torch.from_numpy(keys_h[:n]).to(dev)
    src = gen.permutation(gen.derive_seed(gen.SEED_BASE, 62), 1 << 28).astype(np.int64)
    qsrc = np.where(src < (1 << 27), src, src - (1 << 27) + n)  # 2^27 present, 2^27 absent, shuffled
    q = torch.from_numpy(keys_h[qsrc]).to(dev)
    present = qsrc < n
    del keys_h
    fnd = torch.empty(q.numel(), dtype=torch.uint8, device=dev)
    cells = []
    for G in (1, 2, 4, 8, 16):
        f = hc.Bloom(1 << 32, block_words=words, group=G, device=dev)
        ins, qry = [], []
        for rep in range(args.warmup + args.steps):
            f.clear()
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record(s)
            hc.hc_bloom_insert(f.handle, keys, G, s)
            e[1].record(s)
            hc.hc_bloom_contains(f.handle, q, fnd, G, s)
            e[2].record(s)
            torch.cuda.synchronize()
            if rep >= args.warmup:
                ins.append(e[0].elapsed_time(e[1]))
                qry.append(e[1].elapsed_time(e[2]))
        got = fnd.cpu().numpy()
        assert got[present].all(), "false negative"
        # distinct keys: a block's key count is hypergeometric (2^32 / B hash values per block)
        M, K = 1 << 32, (1 << 32) // f.blocks
        lc = lambda a, b: math.lgamma(a + 1) - math.lgamma(b + 1) - math.lgamma(a - b + 1)  # noqa: E731
        expect = sum(math.exp(lc(K, j) + lc(M - K, n - j) - lc(M, n)) * (1 - (31 / 32) ** j) ** words
                     for j in range(0, K + 1) if lc(K, j) + lc(M - K, n - j) - lc(M, n) > -60)
        fpr = float(got[~present].mean())
        assert abs(fpr - expect) < 0.05 * expect, ("false-positive rate", fpr, expect)
        ti, tq = statistics.mean(ins), statistics.mean(qry)
        # algorithmic HBM bytes: insert reads the key and reads + writes its 64-byte block; a query reads
        # the key and the block and writes one byte
        cells.append({"group": G, "insert_ms": round(ti, 4), "contains_ms": round(tq, 4),
                      "insert_gops": round(n / ti / 1e6, 4), "contains_gops": round(q.numel() / tq / 1e6, 4),
                      "insert_tbs": round(n * (4 + 128) / ti / 1e9, 3),
                      "contains_tbs": round(q.numel() * (4 + 64 + 1) / tq / 1e9, 3), "fpr": round(fpr, 6),
                      "fpr_closed_form": round(expect, 6)})
        print(json.dumps(cells[-1]), file=sys.stderr, flush=True)
        f.close()
    # the group size never changes results, so each operation runs with its fastest one
    bi = min(cells, key=lambda c: c["insert_ms"])
    bq = min(cells, key=lambda c: c["contains_ms"])
    best = {"insert_group": bi["group"], "contains_group": bq["group"], "insert_ms": bi["insert_ms"],
            "contains_ms": bq["contains_ms"], "insert_gops": bi["insert_gops"], "contains_gops": bq["contains_gops"],
            "insert_tbs": bi["insert_tbs"], "contains_tbs": bq["contains_tbs"]}
    ms = best["insert_ms"] + best["contains_ms"]
    res = {"metric": "G inserts/s and G membership queries/s, split-block Bloom filter",
           "value": round((n + q.numel()) / ms / 1e6, 4), "unit": "G ops/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": "split-block Bloom filter, 2^32 bits in 2^23 blocks of 16 words, 2^28 keys "
                                  "(16 bits per key); queries 2^27 present + 2^27 absent",
                      "n_insert": n, "n_contains": int(q.numel()), "best": best},
           "cells": cells}
    print(json.dumps(res), flush=True)


def bench_sweep(args):
    """Single-value table of 2^log2 slots at each load: insert all keys, then retrieve them plus as many absent
    ones (50/50), for every probing scheme and group size at W = 16, and W = 32 / 64 for groups of 32 and 64.
    Each cell is checked: size = n, n queries found, and the values of a sample of present queries."""
    import numpy as np
    import torch

    lib = os.path.join(ROOT, "paper_2009_07914_amd", "libhc.so")
    if not os.path.exists(lib):
        import __graft_entry__
        __graft_entry__.build()
    import gen
    import paper_2009_07914_amd as hc

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    s = torch.cuda.current_stream()
    cap = 1 << args.log2_capacity
    cells = [(sc, 16, g) for sc in ("double", "quadratic", "linear") for g in (1, 2, 4, 8, 16, 32, 64)]
    cells += [(sc, w, g) for sc in ("double", "quadratic", "linear") for w in (32, 64) for g in (32, 64)]
    rows = []
    for load in [float(x) for x in args.loads.split(",")]:
        w = gen.single_value_workload(cap, load, gen.SEED_BASE + 1)
        n = w["n"]
        keys = torch.from_numpy(w["keys"]).to(dev)
        vals = torch.from_numpy(w["values"]).to(dev)
        q = torch.from_numpy(w["queries"]).to(dev)
        vout = torch.empty(q.numel(), dtype=torch.uint32, device=dev)
        fout = torch.empty(q.numel(), dtype=torch.uint8, device=dev)
        samp = np.linspace(0, q.numel() - 1, 1 << 16).astype(np.int64)
        src = w["query_src"][samp].astype(np.int64)
        exp_v = np.where(src < n, w["values"][np.minimum(src, n - 1)], 0).astype(np.uint32)
        exp_f = (src < n).astype(np.uint8)
        samp_t = torch.from_numpy(samp).to(dev)
        reps = 2 if load < 0.95 else 1
        tables = {}
        for scheme, W, G in cells:
            if (scheme, W) not in tables:
                tables.clear()
                torch.cuda.empty_cache()
                tables[(scheme, W)] = hc.Table("single", cap, scheme=scheme, window=W, group=4, device=dev)
            t = tables[(scheme, W)]
            ins, ret = [], []
            for rep in range(1 + reps):
                t.clear()
                e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
                e[0].record(s)
                hc.hc_insert(t.handle, keys, vals, None, G, s)
                e[1].record(s)
                hc.hc_retrieve(t.handle, q, vout, fout, G, s)
                e[2].record(s)
                torch.cuda.synchronize()
                if rep:
                    ins.append(e[0].elapsed_time(e[1]))
                    ret.append(e[1].elapsed_time(e[2]))
            ok = (t.size() == n and int(fout.sum(dtype=torch.int64).item()) == n
                  and np.array_equal(vout.view(torch.int32)[samp_t].cpu().numpy().view(np.uint32), exp_v)
                  and np.array_equal(fout[samp_t].cpu().numpy(), exp_f))
            ti, tr = statistics.mean(ins), statistics.mean(ret)
            row = {"load": load, "scheme": scheme, "W": W, "G": G, "insert_ms": round(ti, 3),
                   "retrieve_ms": round(tr, 3), "insert_gops": round(n / ti / 1e6, 3),
                   "retrieve_gops": round(q.numel() / tr / 1e6, 3), "ok": ok}
            rows.append(row)
            print("# " + json.dumps(row), flush=True)
            assert ok, f"sweep cell failed its check: {row}"
        tables.clear()
        del keys, vals, q, vout, fout, w
        torch.cuda.empty_cache()
    best = {}
    for r in rows:
        for kind in ("insert", "retrieve"):
            k = f"{r['load']}/{kind}"
            if k not in best or r[f"{kind}_gops"] > best[k][f"{kind}_gops"]:
                best[k] = r
    out = {
        "metric": "G inserts/s and G retrievals/s per (load, scheme, W, group size)", "value": None,
        "unit": "G ops/s", "n_gpus": 1, "steps": 2, "warmup": 1, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"single-value table, 2^{args.log2_capacity} slots, uniform distinct uint32 keys, "
                               "loads " + args.loads + "; retrieve 50% present / 50% absent"},
        "best": {k: {"scheme": v["scheme"], "W": v["W"], "G": v["G"],
                     "gops": v[k.split("/")[1] + "_gops"]} for k, v in best.items()},
        "cells": rows,
    }
    print(json.dumps(out), flush=True)


def bench_serving(args):
    """16 resident single-value tables (2^20..2^28 slots) prefilled to half of a 0.9-load key universe;
    requests of log-uniform size in [1, 2^max] (30% insert, 60% retrieve with 10% absent keys, 10% erase of
    prefilled keys) arrive as a Poisson process.  Uniform keys: inserts take fresh keys of the universe.
    Zipf keys (--zipf): inserts and retrieves draw Zipf(1.1) keys of the universe, so inserts update hot
    keys (upserts) and requests admitted together write the same keys; every insert writes the value
    fixed by its key, so results agree whichever write of an epoch wins.  The serial per-request path
    is measured first; the server then takes the same stream at 50%, 80% and 95% of that path's rate."""
    import threading

    import numpy as np
    import torch

    lib = os.path.join(ROOT, "paper_2009_07914_amd", "libhc.so")
    if not os.path.exists(lib):
        import __graft_entry__
        __graft_entry__.build()
    import gen
    import paper_2009_07914_amd as hc

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    caps = [1 << 20, 1 << 20, 1 << 21, 1 << 21, 1 << 22, 1 << 22, 1 << 23, 1 << 23,
            1 << 24, 1 << 24, 1 << 25, 1 << 25, 1 << 26, 1 << 26, 1 << 27, 1 << 28]
    seed = gen.SEED_BASE + 4
    uni = [gen.keys(gen.derive_seed(seed, 10 + j), 1, int(0.9 * c)) for j, c in enumerate(caps)]
    pre = [u.size // 2 for u in uni]
    rng = np.random.default_rng(seed & 0xFFFFFFFF)
    zipf_pool = {}
    reqs = []
    nxt_ins, nxt_er = list(pre), [0] * len(caps)

    def zipf_keys(t, n):
        """Zipf(1.1) over the table's universe (its first min(|U|, 2^22) keys, skipping the erase range):
        a wrapped slice of a per-table pool of 2^21 inverse-CDF draws."""
        if t not in zipf_pool:
            cdf = np.cumsum(gen.zipf_pmf(min(uni[t].size - pre[t] // 2, 1 << 22), 1.1))
            u = gen.values(gen.derive_seed(seed, 200000 + t), 1 << 21).astype(np.float64) / 2.0**32
            zipf_pool[t] = pre[t] // 2 + np.minimum(np.searchsorted(cdf, u * cdf[-1], side="right"), cdf.size - 1)
        pool = zipf_pool[t]
        start = int(rng.integers(pool.size))
        return uni[t][pool[(start + np.arange(n)) % pool.size]]

    def value_of(keys):  # the value an insert writes for a key (Zipf streams)
        return ((keys.astype(np.uint64) * np.uint64(0x9E3779B1)) >> np.uint64(7)).astype(np.uint32)

    for r in range(args.requests):
        t = int(rng.integers(len(caps)))
        n = max(1, int(2.0 ** (args.max_log2_request * rng.random())))
        kind = rng.choice(3, p=[0.3, 0.6, 0.1])
        if kind == 0 and args.zipf:
            keys = zipf_keys(t, n)
            reqs.append((t, hc.OP_INSERT, keys, value_of(keys)))
            continue
        if kind == 0 and uni[t].size - nxt_ins[t] >= n:
            keys = uni[t][nxt_ins[t]:nxt_ins[t] + n]
            nxt_ins[t] += n
            reqs.append((t, hc.OP_INSERT, keys, gen.values(gen.derive_seed(seed, 100000 + r), n)))
            continue
        if kind == 2 and pre[t] // 2 - nxt_er[t] >= n:  # erases take prefilled keys no other request uses
            keys = uni[t][nxt_er[t]:nxt_er[t] + n]
            nxt_er[t] += n
            reqs.append((t, hc.OP_ERASE, keys, None))
            continue
        if args.zipf:
            keys = zipf_keys(t, n)
        else:
            keys = uni[t][rng.integers(0, uni[t].size, n)]
        m = n // 10
        if m:
            keys[:m] = gen.keys(gen.derive_seed(seed, 300000 + r), 1, m)  # absent keys (another key family)
        reqs.append((t, hc.OP_RETRIEVE, keys, None))
    total_ops = sum(k.size for _, _, k, _ in reqs)

    def pinned(a):
        x = torch.empty(a.size, dtype=torch.uint32, pin_memory=True)
        x.numpy()[:] = a
        return x

    host = []
    for t, op, keys, vals in reqs:
        k = pinned(keys)
        v = pinned(vals) if vals is not None else None
        vo = torch.empty(keys.size, dtype=torch.uint32, pin_memory=True) if op == hc.OP_RETRIEVE else None
        fl = torch.empty(keys.size, dtype=torch.uint8, pin_memory=True)
        host.append((t, op, k, v, vo, fl))

    tables = [hc.Table("single", c, scheme="double", window=16, group=4, seed=gen.derive_seed(seed, 50 + j), device=dev)
              for j, c in enumerate(caps)]
    pre_d = [(torch.from_numpy(u[:p]).to(dev),
              torch.from_numpy(value_of(u[:p]) if args.zipf else gen.values(gen.derive_seed(seed, 60 + j), p)).to(dev))
             for j, (u, p) in enumerate(zip(uni, pre))]

    def reset():
        for t, (k, v) in zip(tables, pre_d):
            t.clear()
            t.insert(k, v)
        torch.cuda.synchronize()

    def run(serial, rate):
        """Submit the stream at Poisson times of `rate` requests/s (0: all at once)."""
        reset()
        srv = hc.Server(staging_bytes=4 << 30, serial=serial, max_group_ops=args.max_group_ops,
                        streams=args.server_streams)
        gaps = rng.exponential(1.0 / rate, len(host)) if rate > 0 else np.zeros(len(host))
        arrivals = np.cumsum(gaps)
        tickets = []
        t0 = time.perf_counter()
        for (t, op, k, v, vo, fl), at in zip(host, arrivals):
            while time.perf_counter() - t0 < at:
                pass
            tickets.append(srv.submit(tables[t], op, k, v, vo, fl))
        srv.drain()
        wall = time.perf_counter() - t0
        lat = np.array([srv.query(tk)[1] for tk in tickets]) / 1000.0
        st = srv.stats()
        srv.close()
        outs = [(None if vo is None else vo.numpy().copy(), fl.numpy().copy()) for _, _, _, _, vo, fl in host]
        return {"ops_per_s": total_ops / wall, "wall_s": wall, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
                "launch_groups": st["launch_groups"], "offered_rate": rate}, outs

    for _ in range(max(0, args.warmup)):
        run(False, 0)
    base, base_out = run(True, 0)  # serial path, saturated: its sustainable request rate
    base_rate = len(host) / base["wall_s"]
    res = {"serial_saturated": base}
    for frac in (0.5, 0.8, 0.95):
        r_serial, _ = run(True, frac * base_rate)
        r_server, out = run(False, frac * base_rate)
        res[f"serial_at_{frac}"] = r_serial
        res[f"server_at_{frac}"] = r_server
        ok_mix, ok_alone = [0] * len(caps), [0] * len(caps)
        for (t, op, _, _, _, _), (vm, fm), (vb, fb) in zip(host, out, base_out):  # alone and in the mix
            if op == hc.OP_INSERT and args.zipf:  # same-key inserts of one epoch: which one reports OK
                ok_mix[t] += int((fm == hc.S_OK).sum())  # is open, how many is not
                ok_alone[t] += int((fb == hc.S_OK).sum())
                continue
            assert np.array_equal(fm, fb), "flags differ between the serial path and the server"
            if vm is not None:
                assert np.array_equal(vm, vb), "values differ between the serial path and the server"
        assert ok_mix == ok_alone, "new keys inserted differ between the serial path and the server"
    sat, _ = run(False, 0)
    res["server_saturated"] = sat

    def fmt(d):
        return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}

    out = {
        "metric": "sustained G ops/s and p50/p99 request latency of the serving loop vs the per-request path",
        "value": round(sat["ops_per_s"] / 1e9, 4), "unit": "G ops/s", "n_gpus": 1, "steps": 1,
        "warmup": args.warmup, "ms_per_step": round(sat["wall_s"] * 1000, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "16 resident single-value tables (2^20..2^28 slots), prefilled to 45% of capacity; "
                               f"{len(host)} requests of log-uniform size in [1, 2^{args.max_log2_request}], "
                               "30% insert / 60% retrieve (10% absent keys) / 10% erase, "
                               + ("Zipf(1.1) insert and retrieve keys (over each table's first 2^22 keys)"
                                  if args.zipf else "uniform keys (inserts of fresh keys)")
                               + "; Poisson arrivals",
                   "requests": len(host), "ops": total_ops, "host_buffers": "pinned",
                   "max_group_ops": args.max_group_ops, "server_streams": args.server_streams},
        "modes": {k: fmt(v) for k, v in res.items()},
        "serial_rate_req_per_s": round(base_rate, 2),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
