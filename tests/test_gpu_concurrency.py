"""Same-kind calls overlapping on one table from two streams (Sec. IV-D), against the oracle.

Calls that need scratch memory (multi-value count and write passes, grouped inserts, bucket
list passes) take a workspace of their own per call, so two of them issued back to back on
two streams run concurrently without sharing any state; grouped inserts and bucket list
inserts of one table are ordered by the library on the device.  Every case enqueues both
calls before synchronising and then compares the results with the oracle.  Also here: the
failed-claim counter of hc_stats.
"""
import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import check_layout, d, h

pytestmark = pytest.mark.gpu


def _two_streams():
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    return s1, s2


def _count(hc, t, q, s):
    counts = torch.empty(q.numel(), dtype=torch.uint32, device="cuda")
    offsets = torch.empty(q.numel() + 1, dtype=torch.uint64, device="cuda")
    hc.hc_count_values(t.handle, q, offsets, counts, False, 0, s)
    return counts, offsets


def _check_segments(orc, queries, counts, offsets, vals):
    co, oo = orc.count_values(queries)
    assert np.array_equal(h(counts), co) and np.array_equal(h(offsets), oo)
    _, vo = orc.retrieve_all(queries, oo)
    v = h(vals)[: int(oo[-1])]
    seg = np.repeat(np.arange(queries.size), co.astype(np.int64))
    assert np.array_equal(v[np.lexsort((v, seg))], vo)


@pytest.mark.parametrize("kind", ["multi", "bucket"])
def test_count_and_retrieve_all_on_two_streams(hc, kind):
    """Zipf(1.1) pairs (keys with tens of thousands of values, so both passes hand queries to the
    long rounds); two query batches counted, then written, concurrently on two streams."""
    w = gen.multi_value_zipf_workload(1 << 18, 1 << 11, 1.1, 301)
    t = hc.Table(kind, 1 << 19, scheme="double", window=16, group=4)
    hc.hc_insert_grouped(t.handle, d(w["keys"]), d(w["values"]))
    orc = oracle.OracleTable(oracle.MULTI, 1 << 20)
    orc.insert(w["keys"], w["values"])
    qa = w["queries"]
    qb = qa[gen.permutation(302, qa.size).astype(np.int64)][: qa.size // 2]
    s1, s2 = _two_streams()
    qad, qbd = d(qa), d(qb)
    torch.cuda.synchronize()
    ca, oa = _count(hc, t, qad, s1)
    cb, ob = _count(hc, t, qbd, s2)
    torch.cuda.synchronize()
    va = torch.empty(max(int(h(oa)[-1]), 1), dtype=torch.uint32, device="cuda")
    vb = torch.empty(max(int(h(ob)[-1]), 1), dtype=torch.uint32, device="cuda")
    hc.hc_retrieve_all(t.handle, qad, oa, va, 0, s1)
    hc.hc_retrieve_all(t.handle, qbd, ob, vb, 0, s2)
    torch.cuda.synchronize()
    _check_segments(orc, qa, ca, oa, va)
    _check_segments(orc, qb, cb, ob, vb)
    # several concurrent calls per stream, the second stream's batches interleaved with the first's
    outs = []
    for j in range(3):
        for s, q in ((s1, qad), (s2, qbd)):
            outs.append((q, *_count(hc, t, q, s)))
    torch.cuda.synchronize()
    for q, c, o in outs:
        co, oo = orc.count_values(h(q))
        assert np.array_equal(h(c), co) and np.array_equal(h(o), oo)


@pytest.mark.parametrize("kind", ["multi", "counting", "bucket"])
def test_grouped_inserts_on_two_streams(hc, kind):
    """Two grouped inserts of overlapping Zipf batches into one table from two streams: the table
    holds both batches (the library runs them one after the other on the device)."""
    wa = gen.multi_value_zipf_workload(1 << 17, 1 << 10, 1.1, 311)
    wb = gen.multi_value_zipf_workload(1 << 17, 1 << 10, 1.1, 312)
    t = hc.Table(kind, 1 << 19, scheme="double", window=16, group=4)
    okind = oracle.COUNT if kind == "counting" else oracle.MULTI
    orc = oracle.OracleTable(okind, 1 << 20)
    ka, kb = d(wa["keys"]), d(wb["keys"])
    va, vb = (None, None) if kind == "counting" else (d(wa["values"]), d(wb["values"]))
    s1, s2 = _two_streams()
    hc.hc_insert_grouped(t.handle, ka, va, s1)
    hc.hc_insert_grouped(t.handle, kb, vb, s2)
    torch.cuda.synchronize()
    orc.insert(wa["keys"], None if kind == "counting" else wa["values"])
    orc.insert(wb["keys"], None if kind == "counting" else wb["values"])
    assert t.size() == orc.size()
    q = np.union1d(wa["queries"], wb["queries"]).astype(np.uint32)
    if kind == "counting":
        v, f = t.retrieve(d(q))
        vo, fo = orc.retrieve(q)
        assert np.array_equal(h(v), vo) and np.array_equal(h(f), fo)
        check_layout(t, oracle.COUNT)
    else:
        c, o, _ = t.count_values(d(q))
        _, vals = t.retrieve_all(d(q))
        _check_segments(orc, q, c, o, vals)
        if kind == "multi":
            check_layout(t, oracle.MULTI)


def test_bucket_list_per_pair_inserts_on_two_streams(hc):
    """hc_insert on a bucket list table from two streams (ordered by the library), then a third on
    the first stream: every key's list holds all its values."""
    w = gen.multi_value_uniform_r_workload(1 << 16, 4, 321)
    k, v = w["keys"], w["values"]
    n3 = k.size // 3
    t = hc.Table("bucket", 1 << 15, scheme="double", window=16, group=4, bucket={"pool_values": 1 << 20})
    orc = oracle.OracleTable(oracle.MULTI, 1 << 20)
    kd, vd = d(k), d(v)
    s1, s2 = _two_streams()
    st = torch.empty(k.size, dtype=torch.uint8, device="cuda")
    hc.hc_insert(t.handle, kd[:n3], vd[:n3], st[:n3], 0, s1)
    hc.hc_insert(t.handle, kd[n3:2 * n3], vd[n3:2 * n3], st[n3:2 * n3], 0, s2)
    hc.hc_insert(t.handle, kd[2 * n3:], vd[2 * n3:], st[2 * n3:], 0, s1)
    torch.cuda.synchronize()
    assert (h(st) == hc.S_OK).all()
    orc.insert(k, v)
    assert t.size() == orc.size() == k.size
    q = w["queries"]
    c, o, _ = t.count_values(d(q))
    _, vals = t.retrieve_all(d(q))
    _check_segments(orc, q, c, o, vals)


def test_cas_fails_counter(hc):
    """hc_stats' failed-claim count: zero for a lone insert, positive under heavy same-key contention,
    reset by hc_clear."""
    t = hc.Table("single", 1 << 16, scheme="double", window=16, group=4)
    t.insert(d(np.array([12345], np.uint32)), d(np.array([1], np.uint32)))
    assert t.stats()["cas_fails"] == 0
    base = gen.keys(330, 1, 16)
    keys = base[gen.uniform(331, 0, 15, 1 << 22).astype(np.int64)]
    st = h(t.insert(d(keys), d(gen.values(332, keys.size)), status=True))
    assert (st == hc.S_OK).sum() == 16
    fails = t.stats()["cas_fails"]
    # every failed claim is one of the 2^22 elements' attempts; a group fails at most once per
    # claimable slot it tries, and under this contention many do
    assert 0 < fails
    t.clear()
    assert t.stats()["cas_fails"] == 0 and t.size() == 0


def test_many_launches_beside_a_long_one(hc):
    """Each stream has work counters of its own: while long retrieves run on one stream, more small
    launches than the device has counter pairs run on another, and both stay exact."""
    big = hc.Table("single", 1 << 25, scheme="double", window=16, group=4)
    w = gen.single_value_workload(big.capacity, 0.9, 61)
    big.insert(d(w["keys"]), d(w["values"]))
    small = hc.Table("single", 1 << 12, scheme="linear", window=8, group=2)
    ws = gen.single_value_workload(small.capacity, 0.8, 62)
    small.insert(d(ws["keys"]), d(ws["values"]))
    torch.cuda.synchronize()
    q = d(np.concatenate([w["queries"]] * 4))
    qs = d(ws["queries"])
    a, b = torch.cuda.Stream(), torch.cuda.Stream()
    outs_a, outs_b = [], []
    for rep in range(3):
        v = torch.empty(q.numel(), dtype=torch.uint32, device="cuda")
        f = torch.empty(q.numel(), dtype=torch.uint8, device="cuda")
        hc.hc_retrieve(big.handle, q, v, f, 0, a)
        outs_a.append((v, f))
    for j in range(1200):
        v = torch.empty(qs.numel(), dtype=torch.uint32, device="cuda")
        f = torch.empty(qs.numel(), dtype=torch.uint8, device="cuda")
        hc.hc_retrieve(small.handle, qs, v, f, 0, b)
        if j % 200 == 199:
            outs_b.append((v, f))
    torch.cuda.synchronize()
    src = w["query_src"]
    present = src < w["n"]
    for v, f in outs_a:
        v, f = h(v).reshape(4, -1), h(f).reshape(4, -1)
        for r in range(4):
            assert np.array_equal(f[r].astype(bool), present)
            assert np.array_equal(v[r][present], w["values"][src[present].astype(np.int64)])
    o = oracle.OracleTable(oracle.SINGLE, small.capacity)
    o.insert(ws["keys"], ws["values"])
    vo, fo = o.retrieve(ws["queries"])
    for v, f in outs_b:
        assert np.array_equal(h(v), vo) and np.array_equal(h(f), fo)
