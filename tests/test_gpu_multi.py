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


# ---- grouped insert and long queries (keys with thousands of values) -------------------

@pytest.mark.parametrize("scheme", ["linear", "quadratic", "double"])
@pytest.mark.parametrize("window", [8, 16, 32, 64])
def test_grouped_insert_zipf_matches_oracle(hc, scheme, window):
    """Zipf(1.1) over 2^10 keys, 2^18 pairs: the top keys have tens of thousands of copies, so runs are
    claimed by whole blocks and count / retrieve-all hand them to the long-query kernels."""
    w = gen.multi_value_zipf_workload(1 << 18, 1 << 10, 1.1, 51 + window)
    t = hc.Table("multi", 1 << 19, scheme=scheme, window=window, group=4)
    hc.hc_insert_grouped(t.handle, d(w["keys"]), d(w["values"]))
    orc = oracle.OracleTable(oracle.MULTI, t.capacity)
    orc.insert(w["keys"], w["values"])
    assert t.size() == orc.size() == w["keys"].size
    _mv_parity(t, orc, w["queries"], 4)
    _mv_parity(t, orc, w["queries"], 64)
    check_layout(t, oracle.MULTI)


def test_grouped_then_per_pair_then_erase(hc):
    w = gen.multi_value_zipf_workload(1 << 17, 1 << 9, 1.1, 77)
    t = hc.Table("multi", 1 << 18, scheme="double", window=16, group=8)
    orc = oracle.OracleTable(oracle.MULTI, t.capacity)
    half = w["keys"].size // 2
    hc.hc_insert_grouped(t.handle, d(w["keys"][:half]), d(w["values"][:half]))
    orc.insert(w["keys"][:half], w["values"][:half])
    t.insert(d(w["keys"][half:]), d(w["values"][half:]))
    orc.insert(w["keys"][half:], w["values"][half:])
    _mv_parity(t, orc, w["queries"], 4)
    er = w["queries"][:40]  # includes heavy keys
    assert np.array_equal(h(t.erase(d(er), status=True)), orc.erase(er))
    hc.hc_insert_grouped(t.handle, d(w["keys"][:5000]), d(w["values"][:5000]))  # reuses tombstones
    orc.insert(w["keys"][:5000], w["values"][:5000])
    assert t.size() == orc.size()
    _mv_parity(t, orc, w["queries"], 16)
    check_layout(t, oracle.MULTI)


def test_grouped_insert_reserved_and_overfull(hc):
    keys = np.concatenate([np.full(3000, 5, np.uint32), np.arange(1, 2000, dtype=np.uint32),
                           np.array([0, 0xFFFFFFFF, 0], np.uint32)])
    vals = gen.values(9, keys.size)
    t = hc.Table("multi", 1 << 13, scheme="double", window=16)
    hc.hc_insert_grouped(t.handle, d(keys), d(vals))
    orc = oracle.OracleTable(oracle.MULTI, t.capacity)
    orc.insert(keys, vals)
    assert t.size() == orc.size() == keys.size - 3
    _mv_parity(t, orc, np.arange(0, 2001, dtype=np.uint32), 4)
    # over-full: 600 pairs into 512 slots -> exactly 512 stored, each an input pair, layout valid
    k2 = np.repeat(np.arange(1, 61, dtype=np.uint32), 10)
    v2 = gen.values(10, k2.size)
    t2 = hc.Table("multi", 512, scheme="linear", window=16)
    hc.hc_insert_grouped(t2.handle, d(k2), d(v2))
    assert t2.size() == 512
    slots = h(t2.dump_slots())
    stored = {(int(s & 0xFFFFFFFF), int(s >> 32)) for s in slots if s != 0}
    assert len(stored) == 512 and stored <= set(zip(k2.tolist(), v2.tolist()))
    check_layout(t2, oracle.MULTI)


def test_grouped_insert_needs_multi_value_or_counting(hc):
    t = hc.Table("single", 1024)
    k = d(np.arange(1, 10, dtype=np.uint32))
    with pytest.raises(hc.HcError) as e:
        hc.hc_insert_grouped(t.handle, k, k)
    assert e.value.code == hc.E_KIND
    c = hc.Table("counting", 1024)
    with pytest.raises(hc.HcError) as e:
        hc.hc_insert_grouped(c.handle, k, k)
    assert e.value.code == hc.E_ARG


@pytest.mark.parametrize("group", [1, 4, 16])
@pytest.mark.parametrize("scheme,window", [("linear", 16), ("quadratic", 8), ("double", 16), ("double", 64)])
def test_grouped_counting_matches_oracle(hc, group, scheme, window):
    """Zipf(1.1) keys (2^18 over 2^12): one insert per distinct key with its multiplicity as increment;
    then per-key inserts, erases and a second grouped batch on top, against the oracle's per-key counts."""
    w = gen.multi_value_zipf_workload(1 << 18, 1 << 12, 1.1, 61 + window + group)
    t = hc.Table("counting", 1 << 14, scheme=scheme, window=window, group=group)
    orc = oracle.OracleTable(oracle.COUNT, t.capacity)
    hc.hc_insert_grouped(t.handle, d(w["keys"]))
    orc.insert(w["keys"])
    assert t.size() == orc.size()
    v, f = t.retrieve(d(w["queries"]))
    vo, fo = orc.retrieve(w["queries"])
    assert np.array_equal(h(v), vo) and np.array_equal(h(f), fo)
    check_layout(t, oracle.COUNT)
    t.insert(d(w["keys"][:3000]), None)  # per-key path on top: counts go on from the grouped ones
    orc.insert(w["keys"][:3000])
    er = w["queries"][::7]
    assert np.array_equal(h(t.erase(d(er), status=True)), orc.erase(er))
    hc.hc_insert_grouped(t.handle, d(w["keys"][: 1 << 16]))  # present keys add, erased ones reuse tombstones
    orc.insert(w["keys"][: 1 << 16])
    assert t.size() == orc.size()
    v, f = t.retrieve(d(w["queries"]))
    vo, fo = orc.retrieve(w["queries"])
    assert np.array_equal(h(v), vo) and np.array_equal(h(f), fo)
    check_layout(t, oracle.COUNT)


def test_grouped_counting_reserved_and_full(hc):
    keys = np.concatenate([np.full(70000, 9, np.uint32), np.array([0, 0xFFFFFFFF] * 5, np.uint32),
                           np.repeat(np.arange(100, 2100, dtype=np.uint32), 3)])
    keys = keys[gen.permutation(5, keys.size).astype(np.int64)]
    t = hc.Table("counting", 1 << 13, scheme="double", window=16)
    hc.hc_insert_grouped(t.handle, d(keys))
    orc = oracle.OracleTable(oracle.COUNT, t.capacity)
    orc.insert(keys)
    q = np.concatenate([np.array([9, 0, 0xFFFFFFFF, 5], np.uint32), np.arange(100, 2100, dtype=np.uint32)])
    v, f = t.retrieve(d(q))
    vo, fo = orc.retrieve(q)
    assert np.array_equal(h(v), vo) and np.array_equal(h(f), fo)
    assert int(h(v)[0]) == 70000 and t.size() == 2001
    # full: 3000 distinct keys into 1024 slots -> 1024 stored, each with its exact multiplicity
    k2 = np.repeat(np.arange(1, 3001, dtype=np.uint32), 4)
    k2 = k2[gen.permutation(6, k2.size).astype(np.int64)]
    t2 = hc.Table("counting", 1024, scheme="linear", window=16)
    hc.hc_insert_grouped(t2.handle, d(k2))
    assert t2.size() == 1024
    slots = h(t2.dump_slots())
    assert np.all(slots != 0) and np.all((slots >> 32) == 4)
    assert np.unique(slots & 0xFFFFFFFF).size == 1024
    check_layout(t2, oracle.COUNT)


@pytest.mark.parametrize("window", [8, 16, 32, 64])
def test_grouped_many_rounds_against_grouping(hc, window):
    """A hot key with ~430 K copies (2^21 pairs, Zipf(1.1) over 2^8 keys, table 2^22 slots): heavy runs go
    through several claim rounds and the long queries through several segment rounds.  The per-pair
    oracle is quadratic here, so counts and segments are checked against a sort of the input pairs."""
    w = gen.multi_value_zipf_workload(1 << 21, 1 << 8, 1.1, 97)
    t = hc.Table("multi", 1 << 22, scheme="double", window=window, group=8)
    hc.hc_insert_grouped(t.handle, d(w["keys"]), d(w["values"]))
    assert t.size() == w["keys"].size
    q = w["queries"]
    counts, offsets, total = t.count_values(d(q))
    u, c = np.unique(w["keys"], return_counts=True)
    expect = np.zeros(q.size, np.int64)
    pos = np.searchsorted(u, q)
    expect[pos < u.size] = np.where(u[np.minimum(pos, u.size - 1)] == q, c[np.minimum(pos, u.size - 1)], 0)[pos < u.size]
    assert np.array_equal(h(counts).astype(np.int64), expect) and total == w["keys"].size
    assert int(expect.max()) > 400000
    _, vals = t.retrieve_all(d(q))
    vals, off = h(vals), h(offsets).astype(np.int64)
    order = np.lexsort((w["values"], w["keys"]))
    sk, sv = w["keys"][order], w["values"][order]
    for i in range(q.size):
        lo, hi = np.searchsorted(sk, q[i], "left"), np.searchsorted(sk, q[i], "right")
        assert np.array_equal(np.sort(vals[off[i]:off[i + 1]]), sv[lo:hi])
    check_layout(t, oracle.MULTI)


@pytest.mark.parametrize("group", [1, 4, 64])
def test_counting_statuses_per_key(hc, group):
    """Counting inserts combine equal keys of a tile before the table: per key, exactly one occurrence
    of a new key reports OK and the rest DUPLICATE, every occurrence of a present key DUPLICATE;
    reserved keys INVALID_KEY; a ragged batch spanning many tiles; then an over-full batch where
    each key either fits (counted exactly) or reports FULL at every occurrence."""
    t = hc.Table("counting", 1 << 16, scheme="double", window=16, group=group)
    orc = oracle.OracleTable(oracle.COUNT, t.capacity)
    first = gen.multi_value_zipf_workload(50001, 1 << 10, 1.1, 71)["keys"]
    t.insert(d(first), None)
    orc.insert(first)
    w = gen.multi_value_zipf_workload(100003, 1 << 12, 1.1, 72)
    keys = w["keys"].copy()
    keys[::997] = 0
    keys[5::1499] = 0xFFFFFFFF
    st = h(t.insert(d(keys), None, status=True))
    st_o = orc.insert(keys)
    assert np.array_equal(st == hc.S_INVALID_KEY, st_o == oracle.ST_INVALID_KEY)
    present_before = set(first.tolist())
    for k in np.unique(keys[(keys != 0) & (keys != 0xFFFFFFFF)])[:400]:
        s = st[keys == k]
        if int(k) in present_before:
            assert (s == hc.S_DUPLICATE).all()
        else:
            assert (s == hc.S_OK).sum() == 1 and (s == hc.S_DUPLICATE).sum() == s.size - 1
    assert (st == hc.S_OK).sum() == (st_o == oracle.ST_OK).sum()
    v, f = t.retrieve(d(w["queries"]))
    vo, fo = orc.retrieve(w["queries"])
    assert np.array_equal(h(v), vo) and np.array_equal(h(f), fo) and t.size() == orc.size()
    check_layout(t, oracle.COUNT)
    # over-full: 3000 distinct keys (1-5 copies each, shuffled) into 1024 slots
    t2 = hc.Table("counting", 1024, scheme="linear", window=16, group=group)
    ks = gen.keys(73, 1, 3000)
    mult = 1 + (np.arange(3000) % 5)
    k2 = np.repeat(ks, mult)
    k2 = k2[gen.permutation(74, k2.size).astype(np.int64)]
    st2 = h(t2.insert(d(k2), None, status=True))
    assert t2.size() == 1024
    v2, f2 = t2.retrieve(d(ks))
    v2, f2 = h(v2), h(f2).astype(bool)
    assert f2.sum() == 1024 and np.array_equal(v2[f2], mult[f2].astype(np.uint32))
    for i, k in enumerate(ks[:500]):
        s = st2[k2 == k]
        if f2[i]:
            assert (s == hc.S_OK).sum() == 1 and (s == hc.S_DUPLICATE).sum() == s.size - 1
        else:
            assert (s == hc.S_FULL).all()
    check_layout(t2, oracle.COUNT)
