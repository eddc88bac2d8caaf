"""GPU parity of batched launches over many tables against the CPU oracle.

Every table's results are compared element by element with an oracle table that
replays the same operations one by one in list order.
"""
import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import check_layout, d, h

pytestmark = pytest.mark.gpu


def _tables(hc, n_tables, log2_lo, log2_hi, seed, kind="single"):
    spec = gen.batched_tables_spec(n_tables, log2_lo, log2_hi, 0.6, 0.95, 16, seed)
    out = []
    for j, sp in enumerate(spec):
        scheme = ["linear", "double", "quadratic"][j % 3]
        window = [8, 16, 32][(j // 3) % 3]
        group = [1, 2, 4, 8, 16][j % 5]
        t = hc.Table(kind, sp["capacity"], scheme=scheme, window=window, group=group, seed=sp["seed"])
        w = gen.single_value_workload(t.capacity, sp["load"], sp["seed"])
        out.append((t, w))
    return out


# (group size, window) pairs that share one mixed launch when a phase's operations of one
# kind use several pairs; other pairs get launches of their own
MIXED = {(1, 8), (2, 8), (4, 8), (8, 8), (2, 16), (4, 16), (8, 16), (16, 16), (4, 32), (8, 32), (16, 32)}


def _expected_launches(groups):
    """groups: per (phase, kind), the list of (G, W) pairs of its non-empty operations."""
    n = 0
    for pairs in groups:
        p = set(pairs)
        if len(p) == 1:
            n += 1
        else:
            n += int(any(x in MIXED for x in p)) + sum(x not in MIXED for x in p)
    return n


def test_many_tables_build_then_query(hc):
    tabs = _tables(hc, 40, 10, 16, 123)
    ins, ret, keep = [], [], []
    outs = []
    for j, (t, w) in enumerate(tabs):
        k, v, q = d(w["keys"]), d(w["values"]), d(w["queries"])
        st = torch.empty(k.numel(), dtype=torch.uint8, device="cuda")
        vo = torch.empty(q.numel(), dtype=torch.uint32, device="cuda")
        fo = torch.empty(q.numel(), dtype=torch.uint8, device="cuda")
        ins.append((hc.hc_batch_op(t, hc.OP_INSERT, k, v, flags=st, group=[1, 2, 4, 8, 16][(j + 1) % 5]), [k, v, st]))
        ret.append((hc.hc_batch_op(t, hc.OP_RETRIEVE, q, values_out=vo, flags=fo), [q, vo, fo]))
        outs.append((st, vo, fo))
    b = hc.Batch(ins + ret)
    assert b.phases == 2
    gi = [([1, 2, 4, 8, 16][(j + 1) % 5], t.window) for j, (t, _) in enumerate(tabs)]
    gr = [(t.group, t.window) for t, _ in tabs]
    assert b.launches == _expected_launches([gi, gr])
    b.launch()
    torch.cuda.synchronize()
    for (t, w), (st, vo, fo) in zip(tabs, outs):
        orc = oracle.OracleTable(oracle.SINGLE, t.capacity)
        assert np.array_equal(h(st), orc.insert(w["keys"], w["values"]))
        vv, ff = orc.retrieve(w["queries"])
        assert np.array_equal(h(vo), vv) and np.array_equal(h(fo), ff)
        assert t.size() == orc.size()
    for t, _ in tabs[:6]:
        check_layout(t, oracle.SINGLE)
    b.close()


def test_mixed_phases_follow_list_order(hc):
    t1 = hc.Table("single", 1 << 14, scheme="double", window=16, group=4)
    t2 = hc.Table("single", 1 << 13, scheme="linear", window=8, group=2)
    o1, o2 = oracle.OracleTable(oracle.SINGLE, t1.capacity), oracle.OracleTable(oracle.SINGLE, t2.capacity)
    k1, v1 = gen.keys(70, 1, 9000), gen.values(71, 9000)
    k2, v2 = gen.keys(72, 1, 5000), gen.values(73, 5000)
    er = k1[:3000]
    k2b, v2b = gen.keys(72, 5001, 1000), gen.values(74, 1000)
    q1 = np.concatenate([k1, gen.keys(70, 9001, 2000)])
    q2 = np.concatenate([k2, k2b, gen.keys(72, 7000, 500)])
    T = {}
    def buf(name, a):
        T[name] = d(a)
        return T[name]
    def out(name, n, dt):
        T[name] = torch.zeros(n, dtype=dt, device="cuda")
        return T[name]
    ops = [
        (hc.hc_batch_op(t1, hc.OP_INSERT, buf("k1", k1), buf("v1", v1), flags=out("s1", k1.size, torch.uint8)), []),
        (hc.hc_batch_op(t2, hc.OP_INSERT, buf("k2", k2), buf("v2", v2)), []),
        (hc.hc_batch_op(t2, hc.OP_RETRIEVE, buf("q2a", q2), values_out=out("r2a", q2.size, torch.uint32),
                        flags=out("f2a", q2.size, torch.uint8)), []),
        (hc.hc_batch_op(t1, hc.OP_ERASE, buf("e1", er), flags=out("se", er.size, torch.uint8), group=16), []),
        (hc.hc_batch_op(t1, hc.OP_RETRIEVE, buf("q1", q1), values_out=out("r1", q1.size, torch.uint32),
                        flags=out("f1", q1.size, torch.uint8), group=1), []),
        (hc.hc_batch_op(t2, hc.OP_INSERT, buf("k2b", k2b), buf("v2b", v2b)), []),
        (hc.hc_batch_op(t2, hc.OP_RETRIEVE, buf("q2b", q2), values_out=out("r2b", q2.size, torch.uint32),
                        flags=out("f2b", q2.size, torch.uint8), group=8), []),
    ]
    b = hc.Batch([(o, list(T.values())) for o, _ in ops])
    assert b.phases == 4
    b.launch()
    torch.cuda.synchronize()
    # oracle replay in list order
    assert np.array_equal(h(T["s1"]), o1.insert(k1, v1))
    o2.insert(k2, v2)
    vv, ff = o2.retrieve(q2)
    assert np.array_equal(h(T["r2a"]), vv) and np.array_equal(h(T["f2a"]), ff)
    assert np.array_equal(h(T["se"]), o1.erase(er))
    vv, ff = o1.retrieve(q1)
    assert np.array_equal(h(T["r1"]), vv) and np.array_equal(h(T["f1"]), ff)
    o2.insert(k2b, v2b)
    vv, ff = o2.retrieve(q2)
    assert np.array_equal(h(T["r2b"]), vv) and np.array_equal(h(T["f2b"]), ff)
    assert t1.size() == o1.size() and t2.size() == o2.size()
    b.close()


def test_graph_replays_match_eager(hc):
    tabs = _tables(hc, 12, 10, 15, 7)
    ops, outs = [], []
    for t, w in tabs:
        t.insert(d(w["keys"]), d(w["values"]))
        q = d(w["queries"])
        vo = torch.empty(q.numel(), dtype=torch.uint32, device="cuda")
        fo = torch.empty(q.numel(), dtype=torch.uint8, device="cuda")
        ops.append((hc.hc_batch_op(t, hc.OP_RETRIEVE, q, values_out=vo, flags=fo), [q, vo, fo]))
        outs.append((vo, fo))
    b = hc.Batch(ops)
    b.launch()
    torch.cuda.synchronize()
    eager = [(h(vo).copy(), h(fo).copy()) for vo, fo in outs]
    for rep in range(3):
        for vo, fo in outs:  # scribble over the outputs between replays
            vo.view(torch.int32).fill_(0xABCD)
            fo.fill_(7)
        torch.cuda.synchronize()
        b.replay()
        torch.cuda.synchronize()
        for (vo, fo), (ve, fe) in zip(outs, eager):
            assert np.array_equal(h(vo), ve) and np.array_equal(h(fo), fe), rep
    b.close()


def test_counting_tables_in_a_batch(hc):
    tabs = []
    ops = []
    for j in range(6):
        t = hc.Table("counting", 1 << (11 + j), scheme="double", window=16, group=[2, 4, 8][j % 3])
        w = gen.multi_value_zipf_workload(3 << (10 + j), 1 << (9 + j), 1.1, 200 + j)
        k = d(w["keys"])
        ops.append((hc.hc_batch_op(t, hc.OP_INSERT, k), [k]))
        tabs.append((t, w))
    hc.Batch(ops).launch()
    torch.cuda.synchronize()
    for t, w in tabs:
        o = oracle.OracleTable(oracle.COUNT, t.capacity)
        o.insert(w["keys"])
        v, f = t.retrieve(d(w["queries"]))
        vv, ff = o.retrieve(w["queries"])
        assert np.array_equal(h(v), vv) and np.array_equal(h(f), ff)
        assert t.size() == o.size()


def test_batch_argument_errors(hc):
    mv = hc.Table("multi", 1024)
    sv = hc.Table("single", 1024)
    k = torch.zeros(4, dtype=torch.uint32, device="cuda")
    with pytest.raises(hc.HcError) as e:
        hc.hc_batch_create([hc.hc_batch_op(mv, hc.OP_RETRIEVE, k)])
    assert e.value.code == hc.E_KIND
    with pytest.raises(hc.HcError) as e:
        hc.hc_batch_create([hc.HcBatchOp(sv.handle, hc.OP_INSERT, 0, None, None, None, None, 4)])
    assert e.value.code == hc.E_ARG
    with pytest.raises(hc.HcError) as e:
        hc.hc_batch_create([hc.hc_batch_op(sv, 9, k)])
    assert e.value.code == hc.E_ARG
    b = hc.hc_batch_create([])  # an empty plan launches nothing
    hc.hc_batch_launch(b)
    hc.hc_batch_destroy(b)


@pytest.mark.parametrize("kind", ["single", "counting"])
def test_every_mixed_pair_in_one_launch(hc, kind):
    """One table per (g, W) pair of the mixed set plus pairs outside it: every mixed pair runs in the
    phase's single mixed launch, the others in launches of their own, and every result matches the
    oracle replaying the list; a captured graph replays it to the same results."""
    pairs = sorted(MIXED) + [(1, 16), (2, 32), (16, 8), (32, 64)]
    tabs, ins, ret, outs = [], [], [], []
    for j, (g, w) in enumerate(pairs):
        t = hc.Table(kind, 3000 + 517 * j, scheme=["linear", "double", "quadratic"][j % 3], window=w, group=g,
                     seed=900 + j)
        n = int(0.85 * t.capacity)
        keys = gen.keys(800 + j, 1, n)
        vals = gen.values(850 + j, n)
        q = np.concatenate([keys, gen.keys(800 + j, n + 1, n // 3)])
        k_d, q_d = d(keys), d(q)
        v_d = d(vals) if kind == "single" else None
        st = torch.empty(n, dtype=torch.uint8, device="cuda")
        vo = torch.empty(q.size, dtype=torch.uint32, device="cuda")
        fo = torch.empty(q.size, dtype=torch.uint8, device="cuda")
        ins.append((hc.hc_batch_op(t, hc.OP_INSERT, k_d, v_d, flags=st, group=g), [k_d, v_d, st]))
        ret.append((hc.hc_batch_op(t, hc.OP_RETRIEVE, q_d, values_out=vo, flags=fo, group=g), [q_d, vo, fo]))
        tabs.append((t, keys, vals, q))
        outs.append((st, vo, fo))
    b = hc.Batch(ins + ret)
    assert b.phases == 2
    assert b.launches == _expected_launches([pairs, pairs]) == 2 * (1 + 4)
    okind = oracle.SINGLE if kind == "single" else oracle.COUNT

    def check():
        for (t, keys, vals, q), (st, vo, fo) in zip(tabs, outs):
            orc = oracle.OracleTable(okind, t.capacity)
            assert np.array_equal(h(st), orc.insert(keys, vals if kind == "single" else None))
            vv, ff = orc.retrieve(q)
            assert np.array_equal(h(vo), vv) and np.array_equal(h(fo), ff)
            assert t.size() == orc.size()

    b.launch()
    torch.cuda.synchronize()
    check()
    b.capture()
    for _ in range(2):
        for t, *_ in tabs:
            t.clear()
        b.replay()
        torch.cuda.synchronize()
        check()
    b.close()


def test_graph_replay_beside_eager_launches(hc):
    """A captured plan keeps its own work counters: after more eager launches than the device's
    launch-slot ring holds, replays of the graph on one stream run beside eager launches on another
    and both stay exact."""
    t1 = hc.Table("single", 1 << 17, scheme="double", window=16, group=4)
    t2 = hc.Table("single", 1 << 16, scheme="linear", window=8, group=2)
    w1 = gen.single_value_workload(t1.capacity, 0.9, 401)
    w2 = gen.single_value_workload(t2.capacity, 0.8, 402)
    k1, v1, q1 = d(w1["keys"]), d(w1["values"]), d(w1["queries"])
    st = torch.empty(k1.numel(), dtype=torch.uint8, device="cuda")
    vo = torch.empty(q1.numel(), dtype=torch.uint32, device="cuda")
    fo = torch.empty(q1.numel(), dtype=torch.uint8, device="cuda")
    b = hc.Batch([(hc.hc_batch_op(t1, hc.OP_INSERT, k1, v1, flags=st), [k1, v1, st]),
                  (hc.hc_batch_op(t1, hc.OP_RETRIEVE, q1, values_out=vo, flags=fo), [q1, vo, fo])])
    b.capture()
    k2, v2, q2 = d(w2["keys"]), d(w2["values"]), d(w2["queries"])
    t2.insert(k2, v2)
    small = q2[:64]
    for j in range(1100):  # wrap the launch-slot ring
        hc.hc_retrieve(t2.handle, small, None, None, 0)
    torch.cuda.synchronize()
    o1 = oracle.OracleTable(oracle.SINGLE, t1.capacity)
    st_o = o1.insert(w1["keys"], w1["values"])
    vv1, ff1 = o1.retrieve(w1["queries"])
    o2 = oracle.OracleTable(oracle.SINGLE, t2.capacity)
    o2.insert(w2["keys"], w2["values"])
    vv2, ff2 = o2.retrieve(w2["queries"])
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for rep in range(4):
        t1.clear(stream=s1)
        b.replay(s1)
        outs = []
        for j in range(300):
            v = torch.empty(q2.numel(), dtype=torch.uint32, device="cuda")
            f = torch.empty(q2.numel(), dtype=torch.uint8, device="cuda")
            if j % 100 == 0:
                hc.hc_retrieve(t2.handle, q2, v, f, 0, s2)
                outs.append((v, f))
            else:
                hc.hc_retrieve(t2.handle, small, None, None, 0, s2)
        torch.cuda.synchronize()
        assert np.array_equal(h(st), st_o)
        assert np.array_equal(h(vo), vv1) and np.array_equal(h(fo), ff1)
        for v, f in outs:
            assert np.array_equal(h(v), vv2) and np.array_equal(h(f), ff2)
    b.close()


@pytest.mark.parametrize("one_launch", [False, True])
def test_full_size_256_tables(hc, one_launch):
    """The 256-table workload at its full size (capacities log-uniform in [2^10, 2^24], loads in
    [0.6, 0.95], about 4.4e8 slots): tuned layouts in a phased plan, or one layout (double hashing,
    W = 16, g = 4) in a one-launch plan; launched and its graph replayed; every found flag, value and
    status against the inputs (keys are distinct, so a present query returns the value inserted with
    its key), sizes exact, and the smallest tables against the oracle."""
    from paper_2009_07914_amd import autotune
    spec = gen.batched_tables_spec(256, 10, 24, 0.6, 0.95, 16, gen.SEED_BASE + 3)
    tabs, data, ops = [], [], []
    for sp in spec:
        cfg = (dict(scheme="double", window=16, group_insert=4, group_query=4) if one_launch
               else autotune.choose(sp["capacity"], sp["load"]))
        t = hc.Table("single", sp["capacity"], scheme=cfg["scheme"], window=cfg["window"],
                     group=cfg["group_insert"], seed=sp["seed"])
        w = gen.single_value_workload(sp["capacity"], sp["load"], sp["seed"])
        k, v, q = d(w["keys"]), d(w["values"]), d(w["queries"])
        st = torch.empty(k.numel(), dtype=torch.uint8, device="cuda")
        vo = torch.empty(q.numel(), dtype=torch.uint32, device="cuda")
        fo = torch.empty(q.numel(), dtype=torch.uint8, device="cuda")
        ops.append((hc.hc_batch_op(t, hc.OP_INSERT, k, v, flags=st, group=cfg["group_insert"]), [k, v, st]))
        data.append((t, w, st, vo, fo, [q]))
        tabs.append((t, cfg))
    ops += [(hc.hc_batch_op(t, hc.OP_RETRIEVE, x[5][0], values_out=x[3], flags=x[4], group=cfg["group_query"]),
             [x[5][0], x[3], x[4]]) for (t, cfg), x in zip(tabs, data)]
    b = hc.Batch(ops, one_launch=one_launch)
    assert b.launches == 1 or not one_launch
    assert sum(x[1]["n"] for x in data) > 3e8

    def check():
        for t, w, st, vo, fo, _ in data:
            assert (h(st) == hc.S_OK).all()
            f, v = h(fo), h(vo)
            present = w["query_src"] < w["n"]
            assert np.array_equal(f.astype(bool), present)
            assert np.array_equal(v[present], w["values"][w["query_src"][present].astype(np.int64)])
            assert (v[~present] == 0).all()
            assert t.size() == w["n"]

    b.launch()
    torch.cuda.synchronize()
    check()
    b.capture()
    for rep in range(2):
        for t, _ in tabs:
            t.clear()
        for _, _, st, vo, fo, _ in data:
            st.fill_(77)
            vo.view(torch.int32).fill_(12345)
            fo.fill_(77)
        b.replay()
        torch.cuda.synchronize()
        check()
    small = sorted(range(len(data)), key=lambda j: data[j][0].capacity)[:8]
    for j in small:
        t, w, st, vo, fo, _ = data[j]
        orc = oracle.OracleTable(oracle.SINGLE, t.capacity)
        assert np.array_equal(h(st), orc.insert(w["keys"], w["values"]))
        vv, ff = orc.retrieve(w["queries"])
        assert np.array_equal(h(vo), vv) and np.array_equal(h(fo), ff)
        check_layout(t, oracle.SINGLE)
    assert b.abandoned_waits() == 0
    b.close()


def test_one_launch_phases_follow_list_order(hc):
    """HC_BATCH_ONE_LAUNCH: the four phases of a list over two tables (with an empty operation
    between two of them) run in one gated launch and give the oracle's list-order results; no
    completion wait is abandoned, and graph replays give the same results."""
    t1 = hc.Table("single", 1 << 15, scheme="double", window=16, group=4)
    t2 = hc.Table("single", 1 << 12, scheme="quadratic", window=16, group=4)
    k1, v1 = gen.keys(90, 1, 24000), gen.values(91, 24000)
    k2, v2 = gen.keys(92, 1, 2500), gen.values(93, 2500)
    er = k1[:9000]
    k2b, v2b = gen.keys(92, 2501, 900), gen.values(94, 900)
    q1 = np.concatenate([k1, gen.keys(90, 24001, 4000)])
    q2 = np.concatenate([k2, k2b, gen.keys(92, 4000, 500)])
    T = {}

    def buf(name, a):
        T[name] = d(a)
        return T[name]

    def out(name, n, dt):
        T[name] = torch.zeros(n, dtype=dt, device="cuda")
        return T[name]

    ops = [
        hc.hc_batch_op(t1, hc.OP_INSERT, buf("k1", k1), buf("v1", v1), flags=out("s1", k1.size, torch.uint8)),
        hc.hc_batch_op(t2, hc.OP_INSERT, buf("k2", k2), buf("v2", v2)),
        hc.hc_batch_op(t2, hc.OP_RETRIEVE, buf("q2a", q2), values_out=out("r2a", q2.size, torch.uint32),
                       flags=out("f2a", q2.size, torch.uint8)),
        hc.hc_batch_op(t1, hc.OP_RETRIEVE, buf("empty", np.zeros(0, np.uint32))),  # a phase with no chunks
        hc.hc_batch_op(t1, hc.OP_ERASE, buf("e1", er), flags=out("se", er.size, torch.uint8)),
        hc.hc_batch_op(t1, hc.OP_RETRIEVE, buf("q1", q1), values_out=out("r1", q1.size, torch.uint32),
                       flags=out("f1", q1.size, torch.uint8)),
        hc.hc_batch_op(t2, hc.OP_INSERT, buf("k2b", k2b), buf("v2b", v2b)),
        hc.hc_batch_op(t2, hc.OP_RETRIEVE, buf("q2b", q2), values_out=out("r2b", q2.size, torch.uint32),
                       flags=out("f2b", q2.size, torch.uint8)),
    ]
    b = hc.Batch([(o, list(T.values())) for o in ops], one_launch=True)
    assert b.phases == 4 and b.launches == 1

    def check():
        o1, o2 = oracle.OracleTable(oracle.SINGLE, t1.capacity), oracle.OracleTable(oracle.SINGLE, t2.capacity)
        assert np.array_equal(h(T["s1"]), o1.insert(k1, v1))
        o2.insert(k2, v2)
        vv, ff = o2.retrieve(q2)
        assert np.array_equal(h(T["r2a"]), vv) and np.array_equal(h(T["f2a"]), ff)
        assert np.array_equal(h(T["se"]), o1.erase(er))
        vv, ff = o1.retrieve(q1)
        assert np.array_equal(h(T["r1"]), vv) and np.array_equal(h(T["f1"]), ff)
        o2.insert(k2b, v2b)
        vv, ff = o2.retrieve(q2)
        assert np.array_equal(h(T["r2b"]), vv) and np.array_equal(h(T["f2b"]), ff)
        assert t1.size() == o1.size() and t2.size() == o2.size()

    b.launch()
    torch.cuda.synchronize()
    check()
    b.capture()
    for _ in range(2):
        t1.clear()
        t2.clear()
        for name in ("s1", "r2a", "f2a", "se", "r1", "f1", "r2b", "f2b"):
            T[name].fill_(0x5A)
        torch.cuda.synchronize()
        b.replay()
        torch.cuda.synchronize()
        check()
    assert b.abandoned_waits() == 0
    check_layout(t1, oracle.SINGLE)
    b.close()


def test_one_launch_many_tables_build_then_query(hc):
    """40 single-value and 8 counting tables of every probing scheme (one group size and window),
    built then queried in one gated launch, against the oracle per table."""
    spec = gen.batched_tables_spec(48, 10, 17, 0.6, 0.95, 16, 321)
    tabs, ops = [], []
    for j, sp in enumerate(spec):
        kind = "counting" if j % 6 == 5 else "single"
        t = hc.Table(kind, sp["capacity"], scheme=["linear", "double", "quadratic"][j % 3], window=16, group=8,
                     seed=sp["seed"])
        w = gen.single_value_workload(t.capacity, sp["load"], sp["seed"])
        k, q = d(w["keys"]), d(w["queries"])
        v = d(w["values"]) if kind == "single" else None
        st = torch.empty(k.numel(), dtype=torch.uint8, device="cuda")
        vo = torch.empty(q.numel(), dtype=torch.uint32, device="cuda")
        fo = torch.empty(q.numel(), dtype=torch.uint8, device="cuda")
        ops.append((hc.hc_batch_op(t, hc.OP_INSERT, k, v, flags=st), [k, v, st]))
        ops.append((hc.hc_batch_op(t, hc.OP_RETRIEVE, q, values_out=vo, flags=fo), [q, vo, fo]))
        tabs.append((t, kind, w, st, vo, fo))
    b = hc.Batch(ops, one_launch=True)
    assert b.phases == 2 and b.launches == 1
    b.launch()
    torch.cuda.synchronize()
    assert b.abandoned_waits() == 0
    for t, kind, w, st, vo, fo in tabs:
        orc = oracle.OracleTable(oracle.SINGLE if kind == "single" else oracle.COUNT, t.capacity)
        assert np.array_equal(h(st), orc.insert(w["keys"], w["values"] if kind == "single" else None))
        vv, ff = orc.retrieve(w["queries"])
        assert np.array_equal(h(vo), vv) and np.array_equal(h(fo), ff)
        assert t.size() == orc.size()
    b.close()


def test_one_launch_argument_errors(hc):
    t1 = hc.Table("single", 1024, window=16, group=4)
    t2 = hc.Table("single", 1024, window=8, group=4)
    k = torch.ones(4, dtype=torch.uint32, device="cuda")
    with pytest.raises(hc.HcError) as e:  # two windows
        hc.hc_batch_create_flags([hc.hc_batch_op(t1, hc.OP_RETRIEVE, k), hc.hc_batch_op(t2, hc.OP_RETRIEVE, k)],
                                 hc.HC_BATCH_ONE_LAUNCH)
    assert e.value.code == hc.E_ARG
    with pytest.raises(hc.HcError) as e:  # two group sizes
        hc.hc_batch_create_flags([hc.hc_batch_op(t1, hc.OP_RETRIEVE, k),
                                  hc.hc_batch_op(t1, hc.OP_RETRIEVE, k, group=8)], hc.HC_BATCH_ONE_LAUNCH)
    assert e.value.code == hc.E_ARG
    with pytest.raises(hc.HcError) as e:
        hc.hc_batch_create_flags([hc.hc_batch_op(t1, hc.OP_RETRIEVE, k)], 6)
    assert e.value.code == hc.E_ARG
    b = hc.hc_batch_create_flags([], hc.HC_BATCH_ONE_LAUNCH)
    hc.hc_batch_launch(b)
    assert hc.hc_batch_abandoned_waits(b) == 0
    hc.hc_batch_destroy(b)


def test_one_launch_single_phase(hc):
    """A one-launch plan with one phase has no completion counters to wait on: inserts into two
    tables, then the same plan relaunched after a clear, against the oracle."""
    tabs, ops = [], []
    for j in range(2):
        t = hc.Table("single", 1 << 13, scheme="double", window=16, group=4)
        w = gen.single_value_workload(t.capacity, 0.9, 700 + j)
        k, v = d(w["keys"]), d(w["values"])
        st = torch.empty(k.numel(), dtype=torch.uint8, device="cuda")
        ops.append((hc.hc_batch_op(t, hc.OP_INSERT, k, v, flags=st), [k, v, st]))
        tabs.append((t, w, st))
    b = hc.Batch(ops, one_launch=True)
    assert b.phases == 1 and b.launches == 1
    for rep in range(2):
        for t, _, _ in tabs:
            t.clear()
        b.launch()
        torch.cuda.synchronize()
        assert b.abandoned_waits() == 0
        for t, w, st in tabs:
            orc = oracle.OracleTable(oracle.SINGLE, t.capacity)
            assert np.array_equal(h(st), orc.insert(w["keys"], w["values"]))
            v, f = t.retrieve(d(w["queries"]))
            vo, fo = orc.retrieve(w["queries"])
            assert np.array_equal(h(v), vo) and np.array_equal(h(f), fo)
    b.close()
