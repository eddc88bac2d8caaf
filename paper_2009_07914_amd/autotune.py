"""Autotuner for per-table layout (probing scheme, window W) and group sizes.

The outer probing scheme and the window fix a table's layout, so they are chosen
when the table is created; the group size g is chosen per call (results never
depend on g).  ``tune()`` measures, on the GPU, batched builds and 50/50
retrievals of many same-sized tables for every candidate (scheme, W, g) at a grid
of capacities and loads, and keeps the fastest insert and query configuration per
grid point; ``choose()`` returns the entry of the nearest grid point.  The
measured table ships with the package as ``tuning.json``.

Each grid point is measured on enough elements (``elements``, spread over up to
``max_tables`` tables) that the launches run at steady throughput: with a few
million elements a launch is dominated by its start and its slowest groups, and
the winners there lose in large mixed batches.  The candidates cover the three
outer probing schemes and every group size with g <= W and at most 8 slots per
lane; the (g, W) pairs of the batched launcher's mixed-launch set let tables tuned
to different pairs share one launch per phase and operation kind.
"""
from __future__ import annotations

import json
import math
import os

TUNING_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
DEFAULT = {"scheme": "double", "window": 16, "group_insert": 4, "group_query": 4}

_cache = None


def _load():
    global _cache
    if _cache is None:
        try:
            _cache = json.load(open(TUNING_PATH))
        except (OSError, ValueError):
            _cache = {"points": []}
    return _cache


def choose(capacity: int, load: float) -> dict:
    """Best measured configuration for a table of `capacity` slots filled to `load`."""
    pts = _load().get("points", [])
    if not pts:
        return dict(DEFAULT)
    lc = math.log2(max(2, capacity))
    best = min(pts, key=lambda p: (abs(p["log2_capacity"] - lc), abs(p["load"] - load)))
    return {k: best[k] for k in ("scheme", "window", "group_insert", "group_query")}


def tune(log2_capacities=(10, 13, 16, 19, 22, 24), loads=(0.6, 0.8, 0.95), schemes=("linear", "quadratic", "double"),
         windows=(8, 16, 32, 64), groups=(1, 2, 4, 8, 16, 32, 64), elements=1 << 25, max_tables=1024, reps=3,
         out_path=TUNING_PATH, log=print):
    """Measure every candidate on the current GPU and write the winners to `out_path`.

    Candidates: every scheme x W x g with g <= W and at most 8 slots per lane (the register budget of
    the probing kernels), which includes the wide groups g = 32, 64 on W = 32, 64.  A pair outside the
    batched launcher's mixed-launch set still runs correctly but takes a launch of its own in a batch
    of differently tuned tables."""
    import torch

    import gen
    from . import OP_INSERT, OP_RETRIEVE, Batch, Table, hc_batch_op, hc_clear

    s = torch.cuda.current_stream()
    points = []
    for L in log2_capacities:
        cap = 1 << L
        m = max(1, min(max_tables, elements // cap))
        for load in loads:
            works = [gen.single_value_workload(cap, load, gen.SEED_BASE + 0x7000 + 97 * L + j) for j in range(m)]
            dev = [(torch.from_numpy(w["keys"]).cuda(), torch.from_numpy(w["values"]).cuda(),
                    torch.from_numpy(w["queries"]).cuda()) for w in works]
            outs = [(torch.empty(q.numel(), dtype=torch.uint32, device="cuda"),
                     torch.empty(q.numel(), dtype=torch.uint8, device="cuda")) for _, _, q in dev]
            n_ins = sum(w["n"] for w in works)
            n_ret = sum(w["queries"].size for w in works)
            per_layout = {}  # (scheme, W) -> [best insert (ms, g), best query (ms, g)]
            for scheme in schemes:
                for W in windows:
                    tabs = [Table("single", cap, scheme=scheme, window=W, group=4) for _ in range(m)]
                    rec = per_layout.setdefault((scheme, W), [(math.inf, 0), (math.inf, 0)])
                    for G in groups:
                        if W // G > 8 or G > W:  # 1 to 8 slots per lane
                            continue
                        ins = Batch([(hc_batch_op(t, OP_INSERT, k, v, group=G), [k, v])
                                     for t, (k, v, _) in zip(tabs, dev)])
                        ret = Batch([(hc_batch_op(t, OP_RETRIEVE, q, values_out=vo, flags=fo, group=G), [q, vo, fo])
                                     for t, (_, _, q), (vo, fo) in zip(tabs, dev, outs)])
                        ti, tr = [], []
                        for _ in range(reps):
                            for t in tabs:
                                hc_clear(t.handle, s)
                            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
                            e[0].record(s)
                            ins.launch(s)
                            e[1].record(s)
                            ret.launch(s)
                            e[2].record(s)
                            torch.cuda.synchronize()
                            ti.append(e[0].elapsed_time(e[1]))
                            tr.append(e[1].elapsed_time(e[2]))
                        ins.close()
                        ret.close()
                        ti, tr = min(ti), min(tr)
                        rec[0] = min(rec[0], (ti, G))
                        rec[1] = min(rec[1], (tr, G))
                        log(json.dumps({"log2_capacity": L, "load": load, "tables": m, "scheme": scheme, "window": W,
                                        "group": G, "insert_gops": round(n_ins / ti / 1e6, 3),
                                        "retrieve_gops": round(n_ret / tr / 1e6, 3)}))
                    for t in tabs:
                        t.close()
            (scheme, W), (bi, bq) = min(per_layout.items(), key=lambda kv: kv[1][0][0] + kv[1][1][0])
            points.append({"log2_capacity": L, "load": load, "tables": m, "scheme": scheme, "window": W,
                           "group_insert": bi[1], "group_query": bq[1],
                           "insert_ms": round(bi[0], 4), "retrieve_ms": round(bq[0], 4),
                           "insert_gops": round(n_ins / bi[0] / 1e6, 3), "retrieve_gops": round(n_ret / bq[0] / 1e6, 3)})
            log(json.dumps(points[-1]))
            del dev, outs, works
    res = {"device": torch.cuda.get_device_name(0), "points": points}
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1)
    global _cache
    _cache = res
    return res

