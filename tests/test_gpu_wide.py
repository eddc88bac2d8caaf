"""GPU parity of the single-value table with 64-bit keys and values against the 64-bit oracle.

Keys are (high word, low word) with the low words a seeded bijection of 1..n (so keys are
distinct and never reserved) and random high words; absent keys take low words n+1..2n.
Statuses, sizes and every retrieved value are compared element by element; the dumped
16-byte slots are checked by the oracle's independent layout checker.
"""
import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import d, h

pytestmark = pytest.mark.gpu

SCHEMES = {"linear": oracle.LINEAR, "quadratic": oracle.QUADRATIC, "double": oracle.DOUBLE}


def _keys64(seed, lo, n):
    low = gen.keys(seed, lo, n).astype(np.uint64)
    high = gen.values(seed + 1, n).astype(np.uint64)
    return (high << np.uint64(32)) | low


def _vals64(seed, n):
    return (gen.values(seed, n).astype(np.uint64) << np.uint64(32)) | gen.values(seed + 7, n).astype(np.uint64)


def _layout(t):
    raw = h(t.dump_slots())
    if t.kind == 6:  # structure of arrays: C keys, then C values -> interleave for the checker
        pairs = np.empty(2 * t.capacity, dtype=np.uint64)
        pairs[0::2], pairs[1::2] = raw[: t.capacity], raw[t.capacity:]
        raw = pairs
    rc, st = oracle.check_layout64(raw, t.windows, t.window, t.scheme, t.seed)
    assert rc == 0, f"layout code {rc} at slot {st['first_bad_slot']}"
    return st


@pytest.mark.parametrize("kind", ["single64", "single64_soa"])
@pytest.mark.parametrize("scheme", list(SCHEMES))
@pytest.mark.parametrize("window,group", [(8, 1), (8, 2), (8, 4), (8, 8), (16, 4), (16, 1), (32, 16)])
def test_wide_roundtrip(hc, kind, scheme, window, group):
    cap = 1 << 15
    t = hc.Table(kind, cap, scheme=scheme, window=window, group=group, seed=0x5EED)
    n = int(0.85 * t.capacity)
    keys, vals = _keys64(11, 1, n), _vals64(12, n)
    absent = _keys64(11, n + 1, n)
    orc = oracle.OracleTable64(t.capacity)
    st = h(t.insert(d(keys), d(vals), status=True))
    assert np.array_equal(st, orc.insert(keys, vals))
    assert t.size() == orc.size() == n
    q = np.concatenate([keys, absent])[gen.permutation(13, 2 * n).astype(np.int64)]
    v, f = t.retrieve(d(q))
    vo, fo = orc.retrieve(q)
    assert np.array_equal(h(v), vo) and np.array_equal(h(f), fo)
    er = keys[: n // 10]
    assert np.array_equal(h(t.erase(d(er), status=True)), orc.erase(er))
    v, f = t.retrieve(d(q))
    vo, fo = orc.retrieve(q)
    assert np.array_equal(h(v), vo) and np.array_equal(h(f), fo)
    # re-insert into tombstones with new values
    st = h(t.insert(d(er), d(vals[: er.size] ^ np.uint64(0xFFFF)), status=True))
    assert np.array_equal(st, orc.insert(er, vals[: er.size] ^ np.uint64(0xFFFF)))
    v, f = t.retrieve(d(keys))
    vo, fo = orc.retrieve(keys)
    assert np.array_equal(h(v), vo) and np.all(h(f) == 1)
    lay = _layout(t)
    assert lay["live"] == n


@pytest.mark.parametrize("kind", ["single64", "single64_soa"])
def test_wide_duplicates_reserved_full(hc, kind):
    t = hc.Table(kind, 64, scheme="double", window=8, group=4)
    M = np.uint64(2**64 - 1)
    k = np.array([0, 2**64 - 1, 5, 5, 2**63, 2**63], dtype=np.uint64)
    v = np.array([1, 2, 3, 4, 5, 5], dtype=np.uint64)
    st = h(t.insert(d(k), d(v), status=True))
    assert list(st[:2]) == [hc.S_INVALID_KEY] * 2
    assert sorted(st[2:4]) == [hc.S_OK, hc.S_DUPLICATE] and sorted(st[4:]) == [hc.S_OK, hc.S_DUPLICATE]
    out, f = t.retrieve(d(np.array([5, 2**63, 0, 2**64 - 1, 6], dtype=np.uint64)))
    assert int(h(out)[0]) in (3, 4) and int(h(out)[1]) == 5 and list(h(f)) == [1, 1, 0, 0, 0]
    # over-full: exactly capacity - size new keys succeed
    more = _keys64(21, 1, 200)
    st = h(t.insert(d(more), d(_vals64(22, 200)), status=True))
    assert int((st == hc.S_OK).sum()) == t.capacity - 2 and int((st == hc.S_FULL).sum()) == 200 - (t.capacity - 2)
    assert t.size() == t.capacity
    _layout(t)
    # 32-bit entry points are refused on a 64-bit table
    with pytest.raises(hc.HcError) as e:
        hc.hc_retrieve(t.handle, d(np.array([1], np.uint32)), torch.empty(1, dtype=torch.uint32, device="cuda"))
    assert e.value.code == hc.E_KIND
    with pytest.raises(hc.HcError) as e:
        hc.Table(kind, 64, window=8, group=16)
    assert e.value.code == hc.E_ARG


def test_wide_soa_layout_is_keys_then_values(hc):
    """The structure-of-arrays dump holds key i at word i and its value at word C + i."""
    t = hc.Table("single64_soa", 1 << 12, scheme="linear", window=16, group=4)
    n = 3000
    keys, vals = _keys64(51, 1, n), _vals64(52, n)
    assert np.all(h(t.insert(d(keys), d(vals), status=True)) == hc.S_OK)
    raw = h(t.dump_slots())
    ks, vs = raw[: t.capacity], raw[t.capacity:]
    live = (ks != 0) & (ks != np.uint64(2**64 - 1))
    assert live.sum() == n
    got = dict(zip(ks[live].tolist(), vs[live].tolist()))
    assert got == dict(zip(keys.tolist(), vals.tolist()))
    assert np.all(vs[~live] == 0)


@pytest.mark.parametrize("kind", ["single64", "single64_soa"])
def test_wide_empty_and_ragged(hc, kind):
    t = hc.Table(kind, 1000, scheme="double", window=8, group=2)  # P not a power of two: rounded up to a prime
    empty = d(np.zeros(0, np.uint64))
    assert h(t.insert(empty, empty, status=True)).size == 0
    assert h(t.retrieve(empty)[1]).size == 0
    assert t.size() == 0
    keys, vals = _keys64(61, 1, 777), _vals64(62, 777)
    orc = oracle.OracleTable64(t.capacity)
    assert np.array_equal(h(t.insert(d(keys), d(vals), status=True)), orc.insert(keys, vals))
    v, f = t.retrieve(d(keys))
    vo, fo = orc.retrieve(keys)
    assert np.array_equal(h(v), vo) and np.array_equal(h(f), fo)
    _layout(t)
