"""GPU parity of the HashSet (a set of 32-bit keys, Sec. IV) against the CPU oracle.

A set has the observable semantics of a single-value table whose values are all zero, so the
oracle's single-value table (values 0) is the reference: per-element statuses, found flags and
sizes are compared element by element.  The set's window sequence is the 32-bit tables', so its
dumped 4-byte keys, widened to 8-byte slots with value 0, must pass the oracle's layout checker
for single-value tables (every key once, reachable, no empty slot before it).
"""
import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import d, h

pytestmark = pytest.mark.gpu


def _layout(t):
    keys = h(t.dump_slots())
    assert keys.dtype == np.uint32 and keys.size == t.capacity
    rc, st = oracle.check_layout(keys.astype(np.uint64), t.windows, t.window, t.scheme, t.seed, oracle.SINGLE)
    assert rc == 0, f"layout: {oracle.LAYOUT_ERRORS[rc]} at slot {st['first_bad_slot']}"
    return st


def _zeros(n):
    return np.zeros(n, np.uint32)


@pytest.mark.parametrize("scheme", ["linear", "quadratic", "double"])
@pytest.mark.parametrize("window,group", [(8, 1), (8, 8), (16, 2), (16, 4), (32, 8), (64, 16), (64, 64)])
def test_set_roundtrip(hc, scheme, window, group):
    t = hc.Table("set", 1 << 16, scheme=scheme, window=window, group=group, seed=0xC0FFEE)
    w = gen.single_value_workload(t.capacity, 0.9, 301 + window + group)
    orc = oracle.OracleTable(oracle.SINGLE, t.capacity)
    st = h(t.insert(d(w["keys"]), status=True))
    assert np.array_equal(st, orc.insert(w["keys"], _zeros(w["n"])))
    assert t.size() == orc.size() == w["n"]
    _, f = t.retrieve(d(w["queries"]))
    assert np.array_equal(h(f), orc.retrieve(w["queries"])[1])
    _layout(t)
    # erase a tenth, then query and re-insert into the tombstones
    er = w["keys"][: w["n"] // 10]
    assert np.array_equal(h(t.erase(d(er), status=True)), orc.erase(er))
    _, f = t.retrieve(d(w["queries"]))
    assert np.array_equal(h(f), orc.retrieve(w["queries"])[1])
    assert np.array_equal(h(t.insert(d(er), status=True)), orc.insert(er, _zeros(er.size)))
    assert t.size() == orc.size()
    _, f = t.retrieve(d(w["queries"]))
    assert np.array_equal(h(f), orc.retrieve(w["queries"])[1])
    _layout(t)


def test_set_duplicates_in_one_launch(hc):
    # Zipf keys: each distinct key gets exactly one OK in the launch, every other copy DUPLICATE
    # (which copy wins is unspecified); keys present before the launch get DUPLICATE only
    keys = gen.multi_value_zipf_workload(1 << 18, 1 << 14, 1.1, 311)["keys"]
    t = hc.Table("set", 1 << 15, scheme="double", window=16, group=4)
    pre = np.unique(keys)[:100]
    assert np.all(h(t.insert(d(pre), status=True)) == hc.S_OK)
    st = h(t.insert(d(keys), status=True))
    assert np.all((st == hc.S_OK) | (st == hc.S_DUPLICATE))
    u, inv = np.unique(keys, return_inverse=True)
    ok_per_key = np.bincount(inv, weights=(st == hc.S_OK), minlength=u.size)
    expect = np.where(np.isin(u, pre), 0, 1)
    assert np.array_equal(ok_per_key.astype(np.int64), expect)
    assert t.size() == u.size
    _layout(t)


def test_set_full_and_reserved(hc):
    t = hc.Table("set", 256, scheme="linear", window=16, group=4)
    keys = np.concatenate([np.array([0, 0xFFFFFFFF], np.uint32), np.arange(1, 400, dtype=np.uint32)])
    orc = oracle.OracleTable(oracle.SINGLE, t.capacity)
    st = h(t.insert(d(keys), status=True))
    assert np.all(st[:2] == hc.S_INVALID_KEY)
    # a full set: exactly C keys stored, the rest FULL; which keys win is unspecified
    assert int((st == hc.S_OK).sum()) == t.capacity and int((st == hc.S_FULL).sum()) == keys.size - 2 - t.capacity
    assert t.size() == t.capacity
    stored = keys[st == hc.S_OK]
    _, f = t.retrieve(d(keys))
    assert np.array_equal(h(f).astype(bool), st == hc.S_OK)
    # sequential oracle on the stored keys: same set, same layout rules
    orc.insert(stored, _zeros(stored.size))
    assert orc.size() == t.capacity
    _layout(t)
    _, f = t.retrieve(d(np.array([0, 0xFFFFFFFF], np.uint32)))
    assert not h(f).any()


def test_set_clear_and_large(hc):
    # a set of 2^24 slots at load 0.95: every present key found, every absent one not
    t = hc.Table("set", 1 << 24, scheme="double", window=16, group=4)
    w = gen.single_value_workload(t.capacity, 0.95, 321)
    assert np.all(h(t.insert(d(w["keys"]), status=True)) == hc.S_OK)
    assert t.size() == w["n"]
    _, f = t.retrieve(d(w["queries"]))
    assert np.array_equal(h(f).astype(bool), w["query_src"] < w["n"])
    t.clear()
    assert t.size() == 0
    _, f = t.retrieve(d(w["queries"][:1000]))
    assert not h(f).any()


def test_set_rejects_table_calls(hc):
    t = hc.Table("set", 1024)
    k = d(np.arange(1, 10, dtype=np.uint32))
    for call in (lambda: hc.hc_insert(t.handle, k, k), lambda: hc.hc_retrieve(t.handle, k, k, None)):
        with pytest.raises(hc.HcError) as e:
            call()
        assert e.value.code == hc.E_ARG
    with pytest.raises(hc.HcError) as e:
        t.count_values(k)
    assert e.value.code == hc.E_KIND
    with pytest.raises(hc.HcError) as e:
        t.stats()
    assert e.value.code == hc.E_KIND
    with pytest.raises(hc.HcError) as e:
        hc.Batch([(hc.hc_batch_op(t, hc.OP_RETRIEVE, k, flags=torch.empty(9, dtype=torch.uint8, device="cuda")), [k])])
    assert e.value.code == hc.E_KIND
    with pytest.raises(hc.HcError) as e:
        hc.Table("set", 1024, window=8, group=16)
    assert e.value.code == hc.E_ARG


def test_set_empty_batches_and_info(hc):
    t = hc.Table("set", 4096, scheme="quadratic", window=32, group=8)
    info = hc.hc_info(t.handle)
    assert info.kind == hc.HASH_SET and info.capacity == t.capacity and t.capacity % 32 == 0
    empty = d(np.zeros(0, np.uint32))
    assert h(t.insert(empty, status=True)).size == 0
    assert h(t.retrieve(empty)[1]).size == 0
    assert h(t.erase(empty, status=True)).size == 0
    assert t.size() == 0
    # a ragged batch (not a multiple of any tile) into a fresh set
    keys = gen.keys(77, 1, 1001)
    orc = oracle.OracleTable(oracle.SINGLE, t.capacity)
    assert np.array_equal(h(t.insert(d(keys), status=True)), orc.insert(keys, _zeros(keys.size)))
    _layout(t)
