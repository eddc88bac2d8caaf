"""GPU parity of the counting and multi-value tables against the CPU oracle.

Counting: counts and statuses exact per element.  Multi-value: counts and
offsets exact, each value segment compared after sorting (the order inside a
segment is not specified), erase removes every pair of a key.
"""
import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import check_layout, d, h

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("group", [1, 4, 16, 64])
@pytest.mark.parametrize("scheme", ["linear", "double"])
def test_counting_zipf(hc, group, scheme):
    w = gen.multi_value_zipf_workload(1 << 18, 1 << 14, 1.1, 21)
    t = hc.Table("counting", 1 << 15, scheme=scheme, window=16, group=group)
    orc = oracle.OracleTable(oracle.COUNT, t.capacity)
    st = h(t.insert(d(w["keys"]), None, status=True))
    st_o = orc.insert(w["keys"])
    # per key: one OK (the first to claim) and the rest DUPLICATE; which occurrence is OK is unspecified
    assert (st == hc.S_OK).sum() == (st_o == oracle.ST_OK).sum()
    assert (st == hc.S_DUPLICATE).sum() == (st_o == oracle.ST_DUPLICATE).sum()
    assert t.size() == orc.size()
    v, f = t.retrieve(d(w["queries"]))
    vo, fo = orc.retrieve(w["queries"])
    assert np.array_equal(h(v), vo) and np.array_equal(h(f), fo)
    check_layout(t, oracle.COUNT)
    # erase a quarter of the universe, count again
    er = w["queries"][: w["queries"].size // 4]
    assert np.array_equal(h(t.erase(d(er), status=True)), orc.erase(er))
    t.insert(d(w["keys"][:5000]), None)
    orc.insert(w["keys"][:5000])
    v, f = t.retrieve(d(w["queries"]))
    vo, fo = orc.retrieve(w["queries"])
    assert np.array_equal(h(v), vo) and np.array_equal(h(f), fo)
    assert t.size() == orc.size()
    check_layout(t, oracle.COUNT)


def _mv_parity(t, orc, queries, group=0):
    counts, offsets, total = t.count_values(d(queries), group=group)
    co, oo = orc.count_values(queries)
    assert np.array_equal(h(counts), co)
    assert np.array_equal(h(offsets), oo) and total == int(oo[-1])
    off2, vals = t.retrieve_all(d(queries), group=group)
    _, vo = orc.retrieve_all(queries, oo)
    vals = h(vals)
    assert vals.size == vo.size
    # compare every segment after sorting
    seg_id = np.repeat(np.arange(queries.size), co.astype(np.int64))
    order = np.lexsort((vals, seg_id))
    assert np.array_equal(vals[order], vo)


@pytest.mark.parametrize("group", [1, 2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("r", [1, 4, 32])
def test_multivalue_uniform_r(hc, group, r):
    """Keys uniform on 1..n/r, queries 1..n (Sec. V-B workload shape): sum of counts = n."""
    n = 40000
    w = gen.multi_value_uniform_r_workload(n, r, 31 + r)
    t = hc.Table("multi", 1 << 16, scheme="double", window=16, group=group)
    orc = oracle.OracleTable(oracle.MULTI, t.capacity)
    st = h(t.insert(d(w["keys"]), d(w["values"]), status=True))
    assert np.array_equal(st, orc.insert(w["keys"], w["values"]))
    assert t.size() == n
    _mv_parity(t, orc, w["queries"], group)
    v, f = t.retrieve(d(w["queries"]))  # per-key counts through retrieve
    vo, fo = orc.retrieve(w["queries"])
    assert np.array_equal(h(v), vo) and np.array_equal(h(f), fo)
    check_layout(t, oracle.MULTI)


@pytest.mark.parametrize("scheme", ["linear", "quadratic", "double"])
def test_multivalue_zipf_small_and_erase(hc, scheme):
    w = gen.multi_value_zipf_workload(1 << 16, 1 << 12, 1.1, 41)
    t = hc.Table("multi", 1 << 17, scheme=scheme, window=16, group=8)
    orc = oracle.OracleTable(oracle.MULTI, t.capacity)
    st = h(t.insert(d(w["keys"]), d(w["values"]), status=True))
    assert np.array_equal(st, orc.insert(w["keys"], w["values"]))
    _mv_parity(t, orc, w["queries"], 4)
    assert int(h(t.count_values(d(w["queries"]))[1])[-1]) == 1 << 16  # every pair comes back
    # erase 10% of the universe (distinct keys), re-query; then re-insert some pairs
    er = w["queries"][: w["queries"].size // 10]
    assert np.array_equal(h(t.erase(d(er), status=True)), orc.erase(er))
    assert t.size() == orc.size()
    _mv_parity(t, orc, w["queries"], 16)
    t.insert(d(w["keys"][:3000]), d(w["values"][:3000]))
    orc.insert(w["keys"][:3000], w["values"][:3000])
    _mv_parity(t, orc, w["queries"], 1)
    check_layout(t, oracle.MULTI)


def test_multivalue_full_and_reserved(hc):
    t = hc.Table("multi", 64, scheme="linear", window=16, group=4)
    keys = np.array([7] * 70 + [0, 0xFFFFFFFF], dtype=np.uint32)
    vals = np.arange(72, dtype=np.uint32)
    st = h(t.insert(d(keys), d(vals), status=True))
    assert (st[:70] == hc.S_OK).sum() == 64 and (st[:70] == hc.S_FULL).sum() == 6
    assert list(st[70:]) == [hc.S_INVALID_KEY, hc.S_INVALID_KEY]
    counts, offsets, total = t.count_values(d(np.array([7, 8, 0], dtype=np.uint32)))
    assert list(h(counts)) == [64, 0, 0] and total == 64
    _, v = t.retrieve_all(d(np.array([7], dtype=np.uint32)))
    assert np.array_equal(np.sort(h(v)), np.sort(vals[:70][st[:70] == hc.S_OK]))
    # empty query batch still yields offsets[0] = 0
    _, off, tot = t.count_values(torch.empty(0, dtype=torch.uint32, device="cuda"))
    assert tot == 0 and int(h(off)[0]) == 0
