"""GPU parity of the single-value table against the CPU oracle (bit-exact).

Inputs are seeded synthetic keys (distinct, uniform over [1, 2^32-2]) and
SplitMix64 values; queries mix present and absent keys 50/50.  Every output
element, status and the size are compared with the oracle; the dumped slot
array is checked against the layout invariants (a key sits before any empty
position of its own window sequence, no key twice, exact encodings).
"""
import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import check_layout, d, h

pytestmark = pytest.mark.gpu

GROUPS = [1, 2, 4, 8, 16, 32, 64]
WINDOWS = [8, 16, 32, 64]
SCHEMES = ["linear", "quadratic", "double"]


def _roundtrip(hc, cap, load, scheme, window, group, seed, group_query=None):
    t = hc.Table("single", cap, scheme=scheme, window=window, group=group, seed=seed)
    assert t.capacity == window * oracle.round_windows(cap, window, hc.SCHEMES[scheme])
    w = gen.single_value_workload(t.capacity, load, seed)
    orc = oracle.OracleTable(oracle.SINGLE, t.capacity)
    st = t.insert(d(w["keys"]), d(w["values"]), status=True)
    assert np.array_equal(h(st), orc.insert(w["keys"], w["values"]))
    assert t.size() == orc.size()
    gq = group_query or group
    v, f = t.retrieve(d(w["queries"]), group=gq)
    vo, fo = orc.retrieve(w["queries"])
    assert np.array_equal(h(v), vo) and np.array_equal(h(f), fo)
    check_layout(t, oracle.SINGLE)
    st = t.erase(d(w["erase"]), status=True, group=gq)
    assert np.array_equal(h(st), orc.erase(w["erase"]))
    v, f = t.retrieve(d(w["queries"]), group=gq)
    vo, fo = orc.retrieve(w["queries"])
    assert np.array_equal(h(v), vo) and np.array_equal(h(f), fo)
    assert t.size() == orc.size()
    # re-insert the erased keys with new values: tombstones are reused (Sec. IV-B5)
    nv = gen.values(seed + 1, w["erase"].size)
    st = t.insert(d(w["erase"]), d(nv), status=True)
    assert np.array_equal(h(st), orc.insert(w["erase"], nv))
    v, f = t.retrieve(d(w["queries"]), group=gq)
    vo, fo = orc.retrieve(w["queries"])
    assert np.array_equal(h(v), vo) and np.array_equal(h(f), fo)
    assert t.size() == orc.size()
    check_layout(t, oracle.SINGLE)
    t.close()


def test_small_config_linear_g4(hc):
    """2^20 slots, 0.8 load, linear probing, g=4: insert, query 50/50, erase 10%, re-query."""
    cap = 1 << 20
    t = hc.Table("single", cap, scheme="linear", window=16, group=4, seed=gen.SEED_BASE)
    w = gen.single_value_workload(cap, 0.8, gen.SEED_BASE)
    assert w["n"] == 838860 and w["queries"].size == 1677720 and w["erase"].size == 83886
    orc = oracle.OracleTable(oracle.SINGLE, t.capacity)
    st = t.insert(d(w["keys"]), d(w["values"]), status=True)
    assert np.array_equal(h(st), orc.insert(w["keys"], w["values"]))
    assert t.size() == w["n"]
    v, f = t.retrieve(d(w["queries"]))
    vo, fo = orc.retrieve(w["queries"])
    assert np.array_equal(h(v), vo) and np.array_equal(h(f), fo)
    assert int(h(f).sum()) == w["n"]
    st = t.erase(d(w["erase"]), status=True)
    assert np.array_equal(h(st), orc.erase(w["erase"]))
    v, f = t.retrieve(d(w["queries"]))
    vo, fo = orc.retrieve(w["queries"])
    assert np.array_equal(h(v), vo) and np.array_equal(h(f), fo)
    assert t.size() == orc.size() == w["n"] - w["erase"].size
    assert abs(t.load_factor() - orc.size() / t.capacity) < 1e-12
    stats = check_layout(t, oracle.SINGLE)
    assert stats["tombstones"] == w["erase"].size and stats["live"] == orc.size()


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("window", WINDOWS)
@pytest.mark.parametrize("group", GROUPS)
def test_all_group_window_scheme(hc, scheme, window, group):
    # 3000 windows-ish, ragged capacity (not a multiple of the window for linear), load 0.9
    cap = 20011 if scheme == "linear" else 1 << 14
    _roundtrip(hc, cap, 0.9, scheme, window, group, seed=1000 + group * 7 + window)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_high_load_and_prime_windows(hc, scheme):
    cap = 3001 * 16 if scheme != "quadratic" else 1 << 15
    _roundtrip(hc, cap, 0.99, scheme, 16, 4, seed=77)


@pytest.mark.parametrize("ga,gb", [(1, 64), (4, 16), (64, 2), (8, 1)])
def test_group_size_independence(hc, ga, gb):
    """Build with g_a, query/erase with g_b: identical results (Sec. IV-B2)."""
    _roundtrip(hc, 1 << 15, 0.95, "double", 16, ga, seed=5, group_query=gb)


def test_in_batch_duplicates_and_upsert(hc):
    """A repeated key: one OK, the rest DUPLICATE; the survivor is one of the batch's values."""
    t = hc.Table("single", 1 << 12, scheme="double", window=16, group=4)
    base = gen.keys(3, 1, 500)
    reps = np.repeat(base, 8)
    perm = gen.permutation(4, reps.size)
    keys = reps[perm.astype(np.int64)]
    vals = gen.values(5, keys.size)
    st = h(t.insert(d(keys), d(vals), status=True))
    for k in base[:50]:
        s = st[keys == k]
        assert (s == hc.S_OK).sum() == 1 and (s == hc.S_DUPLICATE).sum() == 7
    assert t.size() == base.size
    v, f = t.retrieve(d(base))
    v, f = h(v), h(f)
    assert f.all()
    for i, k in enumerate(base):
        assert v[i] in set(vals[keys == k].tolist())
    # a later single-occurrence upsert is exact
    nv = gen.values(6, base.size)
    st = h(t.insert(d(base), d(nv), status=True))
    assert (st == hc.S_DUPLICATE).all()
    assert np.array_equal(h(t.retrieve(d(base))[0]), nv) and t.size() == base.size
    check_layout(t, oracle.SINGLE)


@pytest.mark.parametrize("group", [1, 4, 16])
def test_upsert_of_the_stored_value(hc, group):
    """Upserts that rewrite a key's stored value leave it (no write needed), the others replace it:
    re-inserting every pair with half the values changed gives exactly the new values, all DUPLICATE;
    2^21 copies of hot keys rewriting their own values beside a few copies with new values end on one
    of the call's values per key (any order of one call's writes is valid), with exact statuses."""
    t = hc.Table("single", 1 << 15, scheme="double", window=16, group=group)
    w = gen.single_value_workload(t.capacity, 0.8, 31)
    keys, vals = w["keys"], w["values"]
    orc = oracle.OracleTable(oracle.SINGLE, t.capacity)
    assert np.array_equal(h(t.insert(d(keys), d(vals), status=True)), orc.insert(keys, vals))
    nv = vals.copy()
    nv[::2] = gen.values(32, nv[::2].size)
    st = h(t.insert(d(keys), d(nv), status=True))
    assert np.array_equal(st, orc.insert(keys, nv)) and (st == hc.S_DUPLICATE).all()
    q = w["queries"]
    vo, fo = orc.retrieve(q)
    v, f = t.retrieve(d(q))
    assert np.array_equal(h(v), vo) and np.array_equal(h(f), fo)
    # hot keys: 2^21 copies of 8 stored keys with their own values, 64 copies with new values
    hot, hot_v = keys[:8], nv[:8]
    pick = gen.uniform(33, 0, 7, 1 << 21).astype(np.int64)
    hk, hv = hot[pick], hot_v[pick].copy()
    fresh = gen.values(34, 64)
    hv[:64] = fresh
    perm = gen.permutation(35, hk.size).astype(np.int64)
    hk, hv = hk[perm], hv[perm]
    st = h(t.insert(d(hk), d(hv), status=True))
    assert (st == hc.S_DUPLICATE).all() and t.size() == orc.size()
    v, f = t.retrieve(d(hot))
    assert h(f).all()
    for i, k in enumerate(hot):
        assert h(v)[i] in set(hv[hk == k].tolist())
    check_layout(t, oracle.SINGLE)


def test_reserved_keys_and_empty_batch(hc):
    t = hc.Table("single", 1024, window=16)
    keys = np.array([0, 5, 0xFFFFFFFF, 6], dtype=np.uint32)
    st = h(t.insert(d(keys), d(np.array([1, 2, 3, 4], dtype=np.uint32)), status=True))
    assert list(st) == [hc.S_INVALID_KEY, hc.S_OK, hc.S_INVALID_KEY, hc.S_OK]
    v, f = t.retrieve(d(keys))
    assert list(h(f)) == [0, 1, 0, 1] and list(h(v)) == [0, 2, 0, 4]
    assert list(h(t.erase(d(keys), status=True))) == [hc.S_INVALID_KEY, hc.S_OK, hc.S_INVALID_KEY, hc.S_OK]
    e = torch.empty(0, dtype=torch.uint32, device="cuda")
    t.insert(e, e)
    t.retrieve(e)
    t.erase(e)
    assert t.size() == 0


@pytest.mark.parametrize("group", [1, 4, 64])
def test_overfull_batch(hc, group):
    """More distinct new keys than free slots: exactly C - size succeed, the rest report FULL."""
    t = hc.Table("single", 256, scheme="double", window=16, group=group)
    keys = gen.keys(8, 1, 400)
    vals = gen.values(8, 400)
    st = h(t.insert(d(keys), d(vals), status=True))
    assert (st == hc.S_OK).sum() == t.capacity and (st == hc.S_FULL).sum() == 400 - t.capacity
    assert t.size() == t.capacity
    v, f = t.retrieve(d(keys))
    v, f = h(v), h(f)
    assert np.array_equal(f.astype(bool), st == hc.S_OK)
    assert np.array_equal(v[st == hc.S_OK], vals[st == hc.S_OK])
    # present keys still update in a full table; new ones still fail
    st2 = h(t.insert(d(keys), d(vals), status=True))
    assert np.array_equal(st2 == hc.S_DUPLICATE, st == hc.S_OK) and np.array_equal(st2 == hc.S_FULL, st == hc.S_FULL)
    # erase one, then exactly one new key fits into the tombstone
    ok_keys = keys[st == hc.S_OK]
    assert list(h(t.erase(d(ok_keys[:1]), status=True))) == [hc.S_OK]
    new = gen.keys(9, 1, 5)
    st3 = h(t.insert(d(new), d(gen.values(9, 5)), status=True))
    assert (st3 == hc.S_OK).sum() == 1 and (st3 == hc.S_FULL).sum() == 4
    check_layout(t, oracle.SINGLE)


def test_cas_contention_few_keys(hc):
    """2^22 inserts of only 16 distinct keys from every CU: each key ends in exactly one slot."""
    t = hc.Table("single", 1 << 16, scheme="double", window=16, group=4)
    base = gen.keys(10, 1, 16)
    keys = base[(gen.uniform(11, 0, 15, 1 << 22)).astype(np.int64)]
    vals = gen.values(12, keys.size)
    st = h(t.insert(d(keys), d(vals), status=True))
    assert (st == hc.S_OK).sum() == 16 and (st == hc.S_DUPLICATE).sum() == keys.size - 16
    assert t.size() == 16
    st = check_layout(t, oracle.SINGLE)
    assert st["live"] == 16


def test_many_small_launches_reuse_work_counters(hc):
    """3000 launches of 1..97 keys: every launch sees fresh work counters (launch-slot ring wraps)."""
    t = hc.Table("single", 1 << 20, scheme="double", window=16, group=4)
    orc = oracle.OracleTable(oracle.SINGLE, t.capacity)
    allk = gen.keys(50, 1, 150000)
    vals = gen.values(51, allk.size)
    pos = 0
    sizes = (gen.uniform(52, 1, 97, 3000)).astype(np.int64)
    kd, vd = d(allk), d(vals)
    for j, m in enumerate(sizes):
        g = [1, 2, 4, 8, 16, 32, 64][j % 7]
        hc.hc_insert(t.handle, kd[pos:pos + m], vd[pos:pos + m], None, g)
        pos += m
    orc.insert(allk[:pos], vals[:pos])
    assert t.size() == pos
    v, f = t.retrieve(d(allk))
    vo, fo = orc.retrieve(allk)
    assert np.array_equal(h(v), vo) and np.array_equal(h(f), fo)


def test_same_kind_overlap_on_two_streams(hc):
    """Inserts of disjoint key sets on two streams, then retrieves on two streams (Sec. IV-D)."""
    t = hc.Table("single", 1 << 18, scheme="double", window=16, group=4)
    ka, kb = gen.keys(60, 1, 100000), gen.keys(60, 100001, 100000)
    va, vb = gen.values(61, 100000), gen.values(62, 100000)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    kad, kbd, vad, vbd = d(ka), d(kb), d(va), d(vb)
    torch.cuda.synchronize()
    hc.hc_insert(t.handle, kad, vad, None, 2, s1)
    hc.hc_insert(t.handle, kbd, vbd, None, 8, s2)
    torch.cuda.synchronize()
    assert t.size() == 200000
    outa = torch.empty(100000, dtype=torch.uint32, device="cuda")
    outb = torch.empty(100000, dtype=torch.uint32, device="cuda")
    fa = torch.empty(100000, dtype=torch.uint8, device="cuda")
    fb = torch.empty(100000, dtype=torch.uint8, device="cuda")
    hc.hc_retrieve(t.handle, kad, outa, fa, 4, s1)
    hc.hc_retrieve(t.handle, kbd, outb, fb, 1, s2)
    torch.cuda.synchronize()
    assert np.array_equal(h(outa), va) and np.array_equal(h(outb), vb)
    assert h(fa).all() and h(fb).all()
    check_layout(t, oracle.SINGLE)


def _walk_probe_lengths(slots, P, W, scheme, seed):
    """Windows a retrieval visits to reach each live slot, by walking the oracle's window sequence."""
    out = []
    for i in np.nonzero((slots & 0xFFFFFFFF) != 0)[0]:
        k = int(slots[i] & 0xFFFFFFFF)
        if k == 0xFFFFFFFF:
            continue
        seq = oracle.window_sequence(k, P, P, scheme, seed)
        out.append(int(np.nonzero(seq == i // W)[0][0]) + 1)
    return np.array(out, dtype=np.int64)


@pytest.mark.parametrize("scheme,cap", [("linear", 3000), ("quadratic", 3000), ("double", 4096), ("double", 3000)])
@pytest.mark.parametrize("window", [8, 16, 64])
def test_stats_full_scan(hc, scheme, cap, window):
    """hc_stats against a walk of every live key's window sequence (power-of-two and prime P)."""
    t = hc.Table("single", cap, scheme=scheme, window=window, group=4, seed=11)
    w = gen.single_value_workload(t.capacity, 0.93, 12)
    t.insert(d(w["keys"]), d(w["values"]))
    t.erase(d(w["keys"][::9]))
    st = t.stats()
    slots = h(t.dump_slots())
    probes = _walk_probe_lengths(slots, t.windows, t.window, t.scheme, t.seed)
    assert st["live"] == probes.size == t.size()
    assert st["tombstones"] == int(((slots & 0xFFFFFFFF) == 0xFFFFFFFF).sum())
    assert st["empty"] == t.capacity - st["live"] - st["tombstones"]
    assert st["max_probe"] == probes.max() and st["probe_sum"] == probes.sum()
    hist = np.bincount(np.minimum(np.floor(np.log2(probes)).astype(np.int64), hc.PROBE_BUCKETS - 1),
                       minlength=hc.PROBE_BUCKETS)
    assert st["probe_hist"] == hist.tolist()


def test_stats_multi_value_long_sequences(hc):
    """A multi-value table with a key of ~20 K copies: probe lengths in the hundreds of windows."""
    w = gen.multi_value_zipf_workload(1 << 16, 1 << 6, 1.1, 14)
    for scheme in ("linear", "quadratic", "double"):
        t = hc.Table("multi", 1 << 17, scheme=scheme, window=16)
        hc.hc_insert_grouped(t.handle, d(w["keys"]), d(w["values"]))
        st = t.stats()
        rc, lay = oracle.check_layout(h(t.dump_slots()), t.windows, t.window, t.scheme, t.seed, oracle.MULTI)
        assert rc == 0
        assert st["live"] == lay["live"] == w["keys"].size
        assert st["max_probe"] == lay["max_windows"] and st["probe_sum"] == lay["sum_windows"]
        assert st["max_probe"] > 500 and sum(st["probe_hist"]) == st["live"]


def test_create_in_caller_memory(hc):
    p = hc.hc_default_params()
    p.scheme, p.window = hc.SCHEMES["double"], 16
    nbytes = hc.hc_table_bytes(5000, p)
    assert nbytes == 8 * 16 * oracle.round_windows(5000, 16, hc.SCHEMES["double"])
    mem = torch.full((nbytes // 8 + 3,), 0x1234, dtype=torch.uint64, device="cuda")
    t = hc.Table("single", 5000, scheme="double", window=16, slots=mem)
    assert t.capacity * 8 == nbytes and int((mem[: t.capacity] != 0).sum()) == 0  # cleared
    assert int(mem[-1]) == 0x1234  # nothing written past the table
    w = gen.single_value_workload(t.capacity, 0.9, 15)
    orc = oracle.OracleTable(oracle.SINGLE, t.capacity)
    assert np.array_equal(h(t.insert(d(w["keys"]), d(w["values"]), status=True)), orc.insert(w["keys"], w["values"]))
    v, f = t.retrieve(d(w["queries"]))
    vo, fo = orc.retrieve(w["queries"])
    assert np.array_equal(h(v), vo) and np.array_equal(h(f), fo)
    assert torch.equal(t.dump_slots(), mem[: t.capacity])  # the table lives in the caller's tensor
    t.close()
    assert int((mem[: t.capacity] != 0).sum()) == w["keys"].size  # still allocated and intact after destroy
    small = torch.zeros(nbytes // 8 - 1, dtype=torch.uint64, device="cuda")
    with pytest.raises(hc.HcError) as e:
        hc.Table("single", 5000, scheme="double", window=16, slots=small)
    assert e.value.code == hc.E_ARG
