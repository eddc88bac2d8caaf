"""Forced collisions: keys built to share one home window (GPU vs the CPU oracle).

The paper's worked insertion figure (Sec. IV-B2) lost its values, so these cases
play its part.  Keys are chosen with the oracle's own window sequence so that
many of them start in one window, runs of one home window spill over window
boundaries, windows on the way are filled by other keys first, and tables are
filled to their last slot.  Every status, value, found flag and the size are
compared with the oracle; the dumped slots are checked against the layout
invariants; where every key of a pile-up shares one window sequence (linear and
quadratic probing), the first-fit placement is checked window by window.
"""
import numpy as np
import pytest

import gen
import oracle
from tests.gpu_util import check_layout, d, h

pytestmark = pytest.mark.gpu

GROUPS = [1, 4, 16, 64]
SCHEMES = ["linear", "quadratic", "double"]


def homed_at(t, window, count, start=1, skip=()):
    """The first `count` keys >= start whose first window is `window` in table t."""
    out, k, skip = [], start, set(int(x) for x in skip)
    while len(out) < count:
        if k not in skip and oracle.window_at(k, 0, t.windows, t.scheme, t.seed) == window:
            out.append(k)
        k += 1
    return np.array(out, dtype=np.uint32)


def occupancy(t, windows):
    """Live keys per window for the listed windows."""
    s = h(t.dump_slots()).reshape(t.windows, t.window) & 0xFFFFFFFF
    live = (s != 0) & (s != 0xFFFFFFFF)
    return [int(live[w].sum()) for w in windows]


def _parity(t, orc, keys):
    v, f = t.retrieve(d(keys))
    vo, fo = orc.retrieve(keys)
    assert np.array_equal(h(v), vo) and np.array_equal(h(f), fo)
    assert t.size() == orc.size()


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("group", GROUPS)
@pytest.mark.parametrize("window", [8, 16, 32])
def test_pileup_one_home_window(hc, scheme, group, window):
    """3W+5 keys with one home window inserted in one launch: every claim contends on one line."""
    t = hc.Table("single", 256 * window, scheme=scheme, window=window, group=group, seed=0xC0111DE)
    home = 17
    keys = homed_at(t, home, 3 * window + 5)
    absent = homed_at(t, home, 24, start=int(keys[-1]) + 1)
    keys = keys[gen.permutation(3, keys.size).astype(np.int64)]
    vals = gen.values(4, keys.size)
    orc = oracle.OracleTable(oracle.SINGLE, t.capacity)
    assert np.array_equal(h(t.insert(d(keys), d(vals), status=True)), orc.insert(keys, vals))
    check_layout(t, oracle.SINGLE)
    q = np.concatenate([keys, absent])
    _parity(t, orc, q)
    if scheme != "double":  # one shared sequence: three windows full, the fourth holds the rest
        seq = oracle.window_sequence(int(keys[0]), 4, t.windows, t.scheme, t.seed)
        assert occupancy(t, seq) == [window, window, window, 5]
    er = keys[::2]
    assert np.array_equal(h(t.erase(d(er), status=True)), orc.erase(er))
    _parity(t, orc, q)
    nv = gen.values(5, er.size)
    assert np.array_equal(h(t.insert(d(er), d(nv), status=True)), orc.insert(er, nv))
    _parity(t, orc, q)
    check_layout(t, oracle.SINGLE)
    t.close()


@pytest.mark.parametrize("scheme", ["linear", "quadratic"])
@pytest.mark.parametrize("group", GROUPS)
def test_run_skips_a_window_filled_by_others(hc, scheme, group):
    """The second window of a pile-up's sequence is filled first by keys homed there; the run skips
    it, and after those keys are erased, new keys take its tombstones in sequence order."""
    W = 16
    t = hc.Table("single", 256 * W, scheme=scheme, window=W, group=group, seed=0xB10C)
    home = 40
    seq = oracle.window_sequence(int(homed_at(t, home, 1)[0]), 4, t.windows, t.scheme, t.seed)
    blockers = homed_at(t, int(seq[1]), W)
    run = homed_at(t, home, 2 * W + 3, skip=blockers)
    orc = oracle.OracleTable(oracle.SINGLE, t.capacity)
    bv, rv = gen.values(6, blockers.size), gen.values(7, run.size)
    assert np.array_equal(h(t.insert(d(blockers), d(bv), status=True)), orc.insert(blockers, bv))
    assert occupancy(t, [seq[1]]) == [W]
    assert np.array_equal(h(t.insert(d(run), d(rv), status=True)), orc.insert(run, rv))
    assert occupancy(t, seq) == [W, W, W, 3]
    check_layout(t, oracle.SINGLE)
    q = np.concatenate([blockers, run])
    _parity(t, orc, q)
    # tombstones in seq[1]: the run's keys further on are still found
    assert np.array_equal(h(t.erase(d(blockers), status=True)), orc.erase(blockers))
    assert occupancy(t, seq) == [W, 0, W, 3]
    _parity(t, orc, q)
    # new keys of the same home window take seq[1]'s tombstones first (first reusable position)
    more = homed_at(t, home, 5, start=int(run.max()) + 1, skip=blockers)
    mv = gen.values(8, more.size)
    assert np.array_equal(h(t.insert(d(more), d(mv), status=True)), orc.insert(more, mv))
    assert occupancy(t, seq) == [W, 5, W, 3]
    _parity(t, orc, np.concatenate([q, more]))
    check_layout(t, oracle.SINGLE)
    t.close()


@pytest.mark.parametrize("kind", ["single", "counting"])
@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("group", GROUPS)
def test_fill_to_last_slot(hc, kind, scheme, group):
    """C - 1 keys in one launch, the last slot by a launch of one key, then a full table: new keys
    report FULL, absent keys walk all P windows and are not found, a tombstone is reused once."""
    W = 16
    okind = oracle.SINGLE if kind == "single" else oracle.COUNT
    t = hc.Table(kind, 64 * W, scheme=scheme, window=W, group=group, seed=0xF111)
    C = t.capacity
    keys = gen.keys(20 + group, 1, C + 8)
    vals = gen.values(21, keys.size) if kind == "single" else None
    orc = oracle.OracleTable(okind, C)

    def ins(k, v):
        st = h(t.insert(d(k), None if v is None else d(v), status=True))
        assert np.array_equal(st, orc.insert(k, v))
        return st

    ins(keys[: C - 1], None if vals is None else vals[: C - 1])
    assert ins(keys[C - 1:C], None if vals is None else vals[C - 1:C])[0] == hc.S_OK
    assert t.size() == C
    stats = check_layout(t, okind)
    assert stats["live"] == C
    assert ins(keys[C:C + 1], None if vals is None else vals[C:C + 1])[0] == hc.S_FULL
    _parity(t, orc, keys)  # C present, 8 absent: the absent ones scan every window
    # present keys still update in a full table
    st = ins(keys[:5], None if vals is None else gen.values(22, 5))
    assert (st == hc.S_DUPLICATE).all()
    er = np.array([keys[C + 2], keys[7]], dtype=np.uint32)  # absent, present
    assert list(h(t.erase(d(er), status=True))) == list(orc.erase(er)) == [hc.S_NOT_FOUND, hc.S_OK]
    _parity(t, orc, keys)  # one tombstone, no empty slot anywhere
    # three new keys race for the one tombstone in one launch: exactly one wins (which is unspecified)
    new = keys[C + 3:C + 6]
    nv = None if vals is None else vals[C + 3:C + 6]
    st = h(t.insert(d(new), None if nv is None else d(nv), status=True))
    assert sorted(st.tolist()) == [hc.S_OK, hc.S_FULL, hc.S_FULL]
    win = int(np.nonzero(st == hc.S_OK)[0][0])
    assert orc.insert(new[win:win + 1], None if nv is None else nv[win:win + 1])[0] == oracle.ST_OK
    _parity(t, orc, keys)
    check_layout(t, okind)
    t.close()


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("group", GROUPS)
def test_multi_value_pileup(hc, scheme, group):
    """Four keys sharing a home window, 20 copies each (five windows' worth of pairs), inserted pair by
    pair in one launch and by the grouped insert; then a multi-value table filled to its last slot."""
    W = 16
    for grouped in (False, True):
        t = hc.Table("multi", 128 * W, scheme=scheme, window=W, group=group, seed=0x3A1)
        ks = homed_at(t, 9, 4)
        keys = np.repeat(ks, 20)[gen.permutation(30, 80).astype(np.int64)]
        vals = gen.values(31, keys.size)
        orc = oracle.OracleTable(oracle.MULTI, t.capacity)
        if grouped:
            hc.hc_insert_grouped(t.handle, d(keys), d(vals))
            orc.insert(keys, vals)
        else:
            assert np.array_equal(h(t.insert(d(keys), d(vals), status=True)), orc.insert(keys, vals))
        check_layout(t, oracle.MULTI)
        q = np.concatenate([ks, homed_at(t, 9, 3, start=int(ks[-1]) + 1)])
        _mv_check(t, orc, q, group)
        assert np.array_equal(h(t.erase(d(ks[1:2]), status=True)), orc.erase(ks[1:2]))
        _mv_check(t, orc, q, group)
        t.close()
    # a full multi-value table: C pairs of 3 keys, then one more pair is FULL
    t = hc.Table("multi", 32 * W, scheme=scheme, window=W, group=group, seed=0x3A2)
    C = t.capacity
    ks = gen.keys(32, 1, 3)
    keys = ks[(np.arange(C + 1) % 3)]
    vals = gen.values(33, C + 1)
    orc = oracle.OracleTable(oracle.MULTI, C)
    st = h(t.insert(d(keys[:C]), d(vals[:C]), status=True))
    assert np.array_equal(st, orc.insert(keys[:C], vals[:C])) and t.size() == C
    assert np.array_equal(h(t.insert(d(keys[C:]), d(vals[C:]), status=True)), orc.insert(keys[C:], vals[C:]))
    _mv_check(t, orc, np.concatenate([ks, gen.keys(34, 1, 2)]), group)
    check_layout(t, oracle.MULTI)
    t.close()


def _mv_check(t, orc, queries, group):
    counts, offsets, total = t.count_values(d(queries), group=group)
    co, oo = orc.count_values(queries)
    assert np.array_equal(h(counts), co) and np.array_equal(h(offsets), oo) and total == int(oo[-1])
    _, vals = t.retrieve_all(d(queries), group=group)
    _, vo = orc.retrieve_all(queries, oo)
    vals = h(vals)
    seg = np.repeat(np.arange(queries.size), co.astype(np.int64))
    assert np.array_equal(vals[np.lexsort((vals, seg))], vo)
    assert t.size() == orc.size()


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("group", GROUPS)
def test_counting_pileup(hc, scheme, group):
    """3W+5 keys of one home window, each repeated 1-7 times in one launch: exact counts."""
    W = 16
    t = hc.Table("counting", 256 * W, scheme=scheme, window=W, group=group, seed=0xC0C0)
    ks = homed_at(t, 100, 3 * W + 5)
    reps = 1 + (np.arange(ks.size) % 7)
    keys = np.repeat(ks, reps)
    keys = keys[gen.permutation(40, keys.size).astype(np.int64)]
    orc = oracle.OracleTable(oracle.COUNT, t.capacity)
    st = h(t.insert(d(keys), None, status=True))
    st_o = orc.insert(keys)
    for k in ks[:10]:  # one OK per key (which occurrence is unspecified), the rest DUPLICATE
        assert (st[keys == k] == hc.S_OK).sum() == 1
    assert (st == hc.S_OK).sum() == (st_o == oracle.ST_OK).sum() == ks.size
    _parity(t, orc, np.concatenate([ks, homed_at(t, 100, 5, start=int(ks[-1]) + 1)]))
    check_layout(t, oracle.COUNT)
    t.close()
