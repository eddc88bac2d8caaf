"""Parity at the benchmark's full sizes, in the launch configurations bench.py times.

The oracle cannot replay hundreds of millions of operations in a test's time, so these check every
output against what the map semantics fix for distinct keys (a present key returns the value inserted
with it, an absent key is not found, the size is the number of distinct keys), and the multi-value
outputs against a sort of the input pairs (every key's count for all keys; every value of a sample of
keys, the heaviest included).
"""
import numpy as np
import pytest
import torch

import gen
from tests.gpu_util import d, h

pytestmark = pytest.mark.gpu


def test_single_value_2e28_load_0_9_double_w16_g4(hc):
    cap = 1 << 28
    t = hc.Table("single", cap, scheme="double", window=16, group=4)
    assert t.capacity == cap
    w = gen.single_value_workload(cap, 0.9, gen.SEED_BASE + 1)
    n = w["n"]
    keys, vals, q = d(w["keys"]), d(w["values"]), d(w["queries"])
    st = t.insert(keys, vals, status=True, group=4)
    assert np.all(h(st) == hc.S_OK)
    assert t.size() == n
    v, f = t.retrieve(q, group=4)
    f, v = h(f).astype(bool), h(v)
    present = w["query_src"] < n
    assert np.array_equal(f, present)
    assert np.array_equal(v[present], w["values"][w["query_src"][present].astype(np.int64)])
    assert not v[~present].any()
    # erase a tenth of the keys, then query again: erased keys are gone, absent ones still absent,
    # and every other present key is still found with its value (each present key is queried once)
    er = w["erase"]
    assert np.all(h(t.erase(d(er), status=True, group=4)) == hc.S_OK)
    assert t.size() == n - er.size
    _, fe = t.retrieve(d(er), group=4)
    assert not h(fe).any()
    v, f = t.retrieve(q, group=4)
    f, v = h(f).astype(bool), h(v)
    erased = np.isin(w["keys"], er)  # per present key
    src = w["query_src"]
    live = present.copy()
    live[present] = ~erased[src[present].astype(np.int64)]
    assert np.array_equal(f, live) and int(f.sum()) == n - er.size
    assert np.array_equal(v[live], w["values"][src[live].astype(np.int64)])
    assert not v[~live].any()


def test_multi_value_and_counting_2e26_zipf_into_2e27(hc):
    n, ranks = 1 << 26, 1 << 22
    w = gen.multi_value_zipf_workload(n, ranks, 1.1, gen.SEED_BASE + 3)
    keys, vals, q = d(w["keys"]), d(w["values"]), d(w["queries"])
    u, c = np.unique(w["keys"], return_counts=True)
    expect = np.zeros(q.numel(), np.int64)
    pos = np.minimum(np.searchsorted(u, w["queries"]), u.size - 1)
    hit = u[pos] == w["queries"]
    expect[hit] = c[pos[hit]]
    # counting table, grouped insert: every key's multiplicity
    ct = hc.Table("counting", 1 << 27, scheme="double", window=16, group=4)
    hc.hc_insert_grouped(ct.handle, keys, None)
    assert ct.size() == u.size
    cv, cf = ct.retrieve(q)
    assert np.array_equal(h(cv).astype(np.int64), expect) and np.array_equal(h(cf).astype(bool), hit)
    # the per-element counting insert (equal keys of each tile combined): the same counts, one OK
    # status per distinct key and DUPLICATE for every other occurrence
    ct.clear()
    st = h(ct.insert(keys, None, status=True, group=4))
    assert ct.size() == u.size
    assert int((st == hc.S_OK).sum()) == u.size and int((st == hc.S_DUPLICATE).sum()) == n - u.size
    cv, cf = ct.retrieve(q)
    assert np.array_equal(h(cv).astype(np.int64), expect) and np.array_equal(h(cf).astype(bool), hit)
    ct.close()
    # multi-value table, grouped insert: counts of every key, values of a sample
    mv = hc.Table("multi", 1 << 27, scheme="double", window=16, group=4)
    hc.hc_insert_grouped(mv.handle, keys, vals)
    assert mv.size() == n
    counts, offsets, total = mv.count_values(q)
    assert np.array_equal(h(counts).astype(np.int64), expect) and total == n
    _, out = mv.retrieve_all(q)
    out, off = h(out), h(offsets).astype(np.int64)
    order = np.lexsort((w["values"], w["keys"]))
    sk, sv = w["keys"][order], w["values"][order]
    sample = np.concatenate([np.argsort(expect)[-8:], np.linspace(0, q.numel() - 1, 2000).astype(np.int64)])
    for i in sample:
        lo, hi = np.searchsorted(sk, w["queries"][i], "left"), np.searchsorted(sk, w["queries"][i], "right")
        assert np.array_equal(np.sort(out[off[i]:off[i + 1]]), sv[lo:hi])
    assert int(expect.max()) > 7_000_000  # the hottest key's millions of copies
