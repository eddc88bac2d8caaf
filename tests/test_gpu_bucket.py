"""GPU parity of the bucket list table (Sec. IV-C) against the CPU oracle's multimap.

The bucket list table stores the same multiset as a multi-value table (each key's values,
count per key), so the oracle's multi-value table is the reference: counts, offsets and each
key's sorted values must match.  The list structure is checked on the host, independently
of the device code: bucket sizes follow the paper's growth rule s_0, s_i = ceil(lambda s_{i-1})
(capped), bucket 0 of the key in slot p is the pool range [p s_0, (p + 1) s_0), every bucket but
the first links to the one before it, and walking a key's list from its last bucket yields
exactly its values.
"""
import math

import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import check_layout, d, h

pytestmark = pytest.mark.gpu


def _sizes(s0, growth, smax, count):
    """Bucket sizes covering `count` values under the growth rule (written from the paper's formula)."""
    out, s, total = [], s0, 0
    while total < count:
        out.append(s)
        total += s
        s = min(math.ceil(growth * s), smax)
    return out


def _check_lists(t, orc, keys):
    """Walk every key's list on the host and compare with the oracle's values of the key."""
    slots = h(t.dump_slots())
    pool, last = (h(x) for x in t.dump_buckets())
    bp = t.bucket
    live = (slots & 0xFFFFFFFF) != 0
    live &= (slots & 0xFFFFFFFF) != 0xFFFFFFFF
    idx = np.nonzero(live)[0]
    by_key = {int(slots[i] & 0xFFFFFFFF): (int(i), int(slots[i] >> 32)) for i in idx}
    assert len(by_key) == idx.size, "a key stored twice"
    for k in np.unique(keys):
        k = int(k)
        c_o, _ = orc.count_values(np.array([k], np.uint32))
        if c_o[0] == 0:
            assert k not in by_key
            continue
        p, c = by_key[k]
        assert c == int(c_o[0])
        sizes = _sizes(bp["s0"], bp["growth"], bp["smax"], c)
        # bucket 0 is the slot's own range [p * s0, (p + 1) * s0); the last-bucket word is kept for
        # keys with more than one bucket
        bucket0 = p * bp["s0"]
        vals, o = [], (bucket0 if len(sizes) == 1 else int(last[p]))
        for i in range(len(sizes) - 1, -1, -1):
            lo = sum(sizes[:i])
            nv = min(sizes[i], c - lo)
            base = o + (1 if i >= 1 else 0)
            vals.append(pool[base:base + nv])
            if i >= 1:
                o = int(pool[o])
                if i == 1:
                    assert o == bucket0, f"key {k}: bucket 1 links to {o}, not to bucket 0 at {bucket0}"
        got = np.sort(np.concatenate(vals[::-1]))
        _, exp = orc.retrieve_all(np.array([k], np.uint32))
        assert np.array_equal(got, np.sort(exp)), f"values of key {k}"


def _parity(t, orc, queries):
    v, f = t.retrieve(d(queries))
    co, oo = orc.count_values(queries)
    assert np.array_equal(h(v), co.astype(np.uint32)) and np.array_equal(h(f), (co > 0).astype(np.uint8))
    counts, offsets, total = t.count_values(d(queries))
    assert np.array_equal(h(counts), co) and np.array_equal(h(offsets), oo) and total == int(oo[-1])
    _, vals = t.retrieve_all(d(queries))
    _, vo = orc.retrieve_all(queries, oo)
    seg = np.repeat(np.arange(queries.size), co.astype(np.int64))
    vals = h(vals)
    order = np.lexsort((vals, seg))
    assert np.array_equal(vals[order], vo)


@pytest.mark.parametrize("bucket", [dict(s0=1, growth=2.0, smax=1 << 16), dict(s0=4, growth=1.5, smax=64),
                                    dict(s0=8, growth=1.0, smax=8), dict(s0=2, growth=3.0, smax=1000),
                                    dict(s0=1, growth=1.1, smax=1 << 16)])
@pytest.mark.parametrize("group", [1, 4, 16])
def test_bucket_list_batches_match_oracle(hc, bucket, group):
    """Zipf(1.1) pairs in four batches (lists grow across batches and within one)."""
    w = gen.multi_value_zipf_workload(1 << 16, 1 << 11, 1.1, 71 + group)
    t = hc.Table("bucket", 1 << 12, scheme="double", window=16, group=group, bucket=dict(bucket, pool_values=1 << 18))
    orc = oracle.OracleTable(oracle.MULTI, 1 << 20)
    for part in np.array_split(np.arange(w["keys"].size), 4):
        st = h(t.insert(d(w["keys"][part]), d(w["values"][part]), status=True))
        assert np.all(st == hc.S_OK)
        orc.insert(w["keys"][part], w["values"][part])
    assert t.size() == w["keys"].size
    _parity(t, orc, w["queries"])
    _check_lists(t, orc, w["keys"])
    check_layout(t, oracle.SINGLE)  # the key table: each key once, at its place


@pytest.mark.parametrize("r", [1, 4, 32])
def test_bucket_list_uniform_multiplicity(hc, r):
    w = gen.multi_value_uniform_r_workload(30000, r, 81 + r)
    t = hc.Table("bucket", 1 << 15, scheme="linear", window=8, group=4)
    orc = oracle.OracleTable(oracle.MULTI, 1 << 20)
    t.insert(d(w["keys"]), d(w["values"]))
    orc.insert(w["keys"], w["values"])
    _parity(t, orc, w["queries"])
    _check_lists(t, orc, w["keys"])


def test_bucket_list_erase_and_reinsert(hc):
    w = gen.multi_value_zipf_workload(20000, 500, 1.1, 91)
    t = hc.Table("bucket", 2048, scheme="double", window=16, bucket=dict(pool_values=1 << 17))
    orc = oracle.OracleTable(oracle.MULTI, 1 << 20)
    assert np.all(h(t.insert(d(w["keys"]), d(w["values"]), status=True)) == hc.S_OK)
    orc.insert(w["keys"], w["values"])
    er = w["queries"][:150]
    st = h(t.erase(d(er), status=True))
    assert np.array_equal(st, orc.erase(er))
    assert t.size() == orc.size()
    # erased keys start new lists (in tombstone slots); their old buckets stay allocated
    assert np.all(h(t.insert(d(w["keys"][:5000]), d(w["values"][:5000]), status=True)) == hc.S_OK)
    orc.insert(w["keys"][:5000], w["values"][:5000])
    assert t.size() == orc.size()
    _parity(t, orc, w["queries"])
    _check_lists(t, orc, w["keys"])


def test_bucket_list_reserved_keys_and_full(hc):
    # reserved keys are skipped; a tiny pool fills up: the count of a key is cut back to what its
    # buckets hold, the rest report FULL, and what is stored is exactly a prefix-free subset
    keys = np.concatenate([np.array([0, 0xFFFFFFFF], np.uint32), np.repeat(np.arange(1, 41, dtype=np.uint32), 20)])
    vals = gen.values(5, keys.size)
    t = hc.Table("bucket", 64, scheme="double", window=16, bucket=dict(s0=2, growth=2.0, smax=8, pool_values=300))
    st = h(t.insert(d(keys), d(vals), status=True))
    assert np.all(st[:2] == hc.S_INVALID_KEY)
    stored = int((st == hc.S_OK).sum())
    assert np.all((st[2:] == hc.S_OK) | (st[2:] == hc.S_FULL)) and 0 < stored < keys.size - 2
    assert t.size() == stored
    u = t.bucket_usage()
    assert u["values"] == stored and u["pool_words"] == 300
    q = np.arange(1, 41, dtype=np.uint32)
    counts, offsets, total = t.count_values(d(q))
    assert total == stored
    _, got = t.retrieve_all(d(q))
    got, counts, offsets = h(got), h(counts), h(offsets)
    for i, k in enumerate(q):  # every stored value belongs to its key and appears at most as often as inserted
        mine = np.sort(got[offsets[i]:offsets[i + 1]])
        exp = np.sort(vals[2:][keys[2:] == k])
        assert np.all(np.isin(mine, exp)) and np.unique(mine).size == mine.size
    # the key table itself: 64 slots, more distinct keys than that -> FULL for keys that found no slot
    t2 = hc.Table("bucket", 16, scheme="linear", window=16)
    k2 = np.arange(1, 40, dtype=np.uint32)
    st2 = h(t2.insert(d(k2), d(k2), status=True))
    assert int((st2 == hc.S_OK).sum()) == t2.capacity and t2.size() == t2.capacity


@pytest.mark.parametrize("window,group", [(16, 4), (8, 1), (64, 16)])
def test_bucket_list_grouped_insert(hc, window, group):
    """Grouped batches (one ticket per run) mixed with per-pair batches: same lists, same multiset."""
    w = gen.multi_value_zipf_workload(1 << 17, 1 << 10, 1.1, 101 + window)
    t = hc.Table("bucket", 1 << 11, scheme="double", window=window, group=group,
                 bucket=dict(s0=2, growth=1.5, smax=4096, pool_values=1 << 19))
    orc = oracle.OracleTable(oracle.MULTI, 1 << 20)
    parts = np.array_split(np.arange(w["keys"].size), 3)
    hc.hc_insert_grouped(t.handle, d(w["keys"][parts[0]]), d(w["values"][parts[0]]))
    orc.insert(w["keys"][parts[0]], w["values"][parts[0]])
    assert np.all(h(t.insert(d(w["keys"][parts[1]]), d(w["values"][parts[1]]), status=True)) == hc.S_OK)
    orc.insert(w["keys"][parts[1]], w["values"][parts[1]])
    hc.hc_insert_grouped(t.handle, d(w["keys"][parts[2]]), d(w["values"][parts[2]]))
    orc.insert(w["keys"][parts[2]], w["values"][parts[2]])
    assert t.size() == w["keys"].size
    _parity(t, orc, w["queries"])
    _check_lists(t, orc, w["keys"])
    # reserved keys in a grouped batch are skipped
    k = np.array([0, 0xFFFFFFFF, 0, 7], np.uint32)
    hc.hc_insert_grouped(t.handle, d(k), d(k))
    assert t.size() == w["keys"].size + 1


def test_bucket_list_rejects_other_calls(hc):
    t = hc.Table("bucket", 1024)
    k = d(np.arange(1, 10, dtype=np.uint32))
    with pytest.raises(hc.HcError) as e:
        t.insert(k, None)
    assert e.value.code == hc.E_ARG
    single = hc.Table("single", 1024)
    with pytest.raises(hc.HcError) as e:
        single.bucket_usage()
    assert e.value.code == hc.E_KIND
