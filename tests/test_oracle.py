"""Pins of the CPU oracle against things other than itself.

* brute force: a linear-scan list model (tests/brute.py) on random op sequences
  with tiny capacities and key ranges, every kind and op, reserved keys, full
  tables, erase then re-insert -- exact agreement of every result, the size, the
  number of distinct keys and the full sorted content after every operation;
* library routines on larger inputs: counting = numpy.unique counts,
  multi-value segments = lexsort grouping, offsets = cumsum;
* invariants: every inserted key found with its last-written value, absent keys
  not found, size = distinct live keys, sum of counts = offsets[n];
* probe geometry: closed-form coverage (every window exactly once, Sec. II /
  Sec. IV-B2), hash-mixer bijectivity via its algebraic inverse, and the layout
  checker catching planted mistakes in layouts built by the scalar model.
"""
import random

import numpy as np
import pytest

import gen
import oracle
from oracle import COUNT, DOUBLE, LINEAR, MULTI, QUADRATIC, SINGLE, OracleTable
from tests.brute import BruteTable

RES = [0, 0xFFFFFFFF]


def _random_ops(rng, n_ops, key_hi):
    ops = []
    for _ in range(n_ops):
        kind = rng.choice(["insert", "insert", "insert", "retrieve", "erase", "retrieve_all"])
        batch = [rng.choice(RES) if rng.random() < 0.05 else rng.randint(1, key_hi)
                 for _ in range(rng.randint(0, 12))]
        vals = [rng.choice([0, 1, 7, 0xFFFFFFFF, rng.getrandbits(32)]) for _ in batch]
        ops.append((kind, batch, vals))
    return ops


@pytest.mark.parametrize("kind", [SINGLE, MULTI, COUNT])
@pytest.mark.parametrize("seed", range(40))
def test_oracle_equals_brute_force(kind, seed):
    rng = random.Random(seed * 31 + kind)
    cap = rng.choice([1, 2, 3, 5, 8, 16, 64])
    o, b = OracleTable(kind, cap), BruteTable(kind, cap)
    for op, batch, vals in _random_ops(rng, 30, rng.choice([3, 10, 100])):
        if op == "insert":
            st_o = o.insert(batch, vals if kind != COUNT else None)
            st_b = b.insert(batch, vals)
            assert list(st_o) == st_b
        elif op == "retrieve":
            v_o, f_o = o.retrieve(batch)
            v_b, f_b = b.retrieve(batch)
            assert list(v_o) == v_b and list(f_o) == f_b
        elif op == "erase":
            assert list(o.erase(batch)) == b.erase(batch)
        else:
            off_o, val_o = o.retrieve_all(batch)
            off_b, val_b = b.retrieve_all(batch)
            assert list(off_o) == off_b and list(val_o) == val_b
        assert o.size() == b.size()
        assert o.num_keys() == b.num_keys()
        k_o, v_o = o.dump()
        assert list(zip(k_o.tolist(), v_o.tolist())) == b.contents()


def test_counting_equals_numpy_unique():
    keys = gen.multi_value_zipf_workload(1 << 18, 1 << 12, 1.1, 3)["keys"]
    o = OracleTable(COUNT, 1 << 20)
    st = o.insert(keys)
    u, c = np.unique(keys, return_counts=True)
    cnt, found = o.retrieve(u)
    assert np.array_equal(cnt, c.astype(np.uint32)) and found.all()
    assert o.size() == u.size
    # exactly one OK (first occurrence) per distinct key; the rest DUPLICATE
    assert (st == oracle.ST_OK).sum() == u.size and (st == oracle.ST_DUPLICATE).sum() == keys.size - u.size


def test_multivalue_equals_lexsort_grouping():
    w = gen.multi_value_uniform_r_workload(1 << 15, 8, 4)
    o = OracleTable(MULTI, 1 << 16)
    assert (o.insert(w["keys"], w["values"]) == oracle.ST_OK).all()
    counts, offsets = o.count_values(w["queries"])
    order = np.lexsort((w["values"], w["keys"]))
    sk, sv = w["keys"][order], w["values"][order]
    lo = np.searchsorted(sk, w["queries"], side="left")
    hi = np.searchsorted(sk, w["queries"], side="right")
    assert np.array_equal(counts, (hi - lo).astype(np.uint32))
    assert np.array_equal(offsets, np.concatenate([[0], np.cumsum(hi - lo)]).astype(np.uint64))
    # every stored value comes back: queries cover 1..n, so sum of counts = n (Sec. V-B design)
    assert int(offsets[-1]) == w["keys"].size
    _, vals = o.retrieve_all(w["queries"], offsets)
    expect = np.concatenate([sv[a:b] for a, b in zip(lo, hi)])
    assert np.array_equal(vals, expect)


def test_single_value_invariants_and_last_write():
    w = gen.single_value_workload(1 << 14, 0.9, 5)
    o = OracleTable(SINGLE, 1 << 14)
    assert (o.insert(w["keys"], w["values"]) == oracle.ST_OK).all()
    assert o.size() == w["n"]
    v, f = o.retrieve(w["keys"])
    assert np.array_equal(v, w["values"]) and f.all()
    v, f = o.retrieve(w["absent"])
    assert not f.any() and not v.any()
    # upsert with new values: last write wins, status DUPLICATE, size unchanged
    nv = gen.values(99, w["n"])
    assert (o.insert(w["keys"], nv) == oracle.ST_DUPLICATE).all()
    assert np.array_equal(o.retrieve(w["keys"])[0], nv) and o.size() == w["n"]
    # in-batch duplicates: last occurrence's value survives (numpy: last index of each key)
    k2 = np.concatenate([w["keys"][:100], w["keys"][:100]])
    v2 = gen.values(100, 200)
    o.insert(k2, v2)
    assert np.array_equal(o.retrieve(w["keys"][:100])[0], v2[100:])
    # erase 10%, re-query
    st = o.erase(w["erase"])
    assert (st == oracle.ST_OK).all() and o.size() == w["n"] - w["erase"].size
    assert (o.erase(w["erase"]) == oracle.ST_NOT_FOUND).all()
    _, f = o.retrieve(w["erase"])
    assert not f.any()


def test_full_table_and_reserved():
    o = OracleTable(SINGLE, 4)
    st = o.insert([5, 6, 7, 8, 9, 5, 0, 0xFFFFFFFF], [1, 2, 3, 4, 5, 6, 7, 8])
    assert list(st) == [0, 0, 0, 0, 2, 1, 3, 3]
    assert list(o.erase([5, 0])) == [0, 3]
    assert list(o.insert([9], [1])) == [0]
    # counting: one stored key, count = number of occurrences
    c = OracleTable(COUNT, 2)
    c.insert(np.full(1000, 42, dtype=np.uint32))
    assert c.retrieve([42])[0][0] == 1000


# ------------------------------ probe geometry ----------------------------------

def _is_prime(p):
    return p >= 2 and all(p % d for d in range(2, int(p ** 0.5) + 1))


@pytest.mark.parametrize("scheme", [LINEAR, QUADRATIC, DOUBLE])
def test_window_sequence_covers_every_window_once(scheme):
    Ps = [1, 2, 4, 8, 64, 256, 1024, 4096]
    if scheme == LINEAR:
        Ps += [3, 5, 6, 100, 1000]
    if scheme == DOUBLE:
        Ps += [p for p in (3, 5, 7, 31, 101, 127, 1009, 4093) if _is_prime(p)]
    rng = random.Random(scheme)
    for P in Ps:
        for _ in range(6):
            k = rng.randint(1, 0xFFFFFFFE)
            seed = rng.getrandbits(64)
            seq = oracle.window_sequence(k, P, P, scheme, seed)
            assert np.array_equal(np.sort(seq), np.arange(P, dtype=np.uint64)), (scheme, P)


def test_window_sequence_closed_forms():
    # the k-th step of each scheme against its textbook form (Sec. II): LP h+l, QP h+l(l+1)/2, DH h+l*s
    P, seed, k = 1024, 0x1234_5678_9ABC_DEF0, 0xDEADBEEF
    h = oracle.window_at(k, 0, P, LINEAR, seed)
    assert h == oracle.window_at(k, 0, P, QUADRATIC, seed) == oracle.window_at(k, 0, P, DOUBLE, seed)
    for l in range(1, 50):
        assert oracle.window_at(k, l, P, LINEAR, seed) == (h + l) % P
        assert oracle.window_at(k, l, P, QUADRATIC, seed) == (h + l * (l + 1) // 2) % P
    s = (oracle.window_at(k, 1, P, DOUBLE, seed) - h) % P
    assert s % 2 == 1  # odd step => coprime with a power-of-two P
    for l in range(1, 50):
        assert oracle.window_at(k, l, P, DOUBLE, seed) == (h + l * s) % P


def test_plain_square_quadratic_probing_does_not_cover():
    # Why the triangular-number reading: (h + l^2) mod P reaches only (P+1)/2 residues for prime P
    for P in (31, 101, 1009):
        assert len({(l * l) % P for l in range(P)}) == (P + 1) // 2


def test_round_windows():
    assert oracle.round_windows(1 << 20, 16, LINEAR) == 1 << 16
    assert oracle.round_windows(1 << 20, 16, DOUBLE) == 1 << 16
    assert oracle.round_windows(1000, 16, LINEAR) == 63
    assert oracle.round_windows(1000, 16, QUADRATIC) == 64
    assert oracle.round_windows(1000, 16, DOUBLE) == 67  # next prime >= 63
    assert oracle.round_windows(1, 16, DOUBLE) == 1


def _fmix32_inverse(h):
    # algebraic inverse of the MurmurHash3 finaliser: undo xorshifts and odd multiplies
    M = 0xFFFFFFFF

    def unxorshift(x, s):
        y = x
        for _ in range(32 // s + 1):
            y = x ^ (y >> s)
        return y & M

    h = unxorshift(h, 16)
    h = (h * pow(0xc2b2ae35, -1, 1 << 32)) & M
    h = unxorshift(h, 13)
    h = (h * pow(0x85ebca6b, -1, 1 << 32)) & M
    return unxorshift(h, 16)


def test_hash_mixer_is_bijective():
    rng = random.Random(3)
    xs = [0, 1, 2, 0xFFFFFFFF, 0x80000000] + [rng.getrandbits(32) for _ in range(20000)]
    for x in xs:
        assert _fmix32_inverse(oracle.fmix32(x)) == x
    assert oracle.fmix32(0) == 0


def test_home_windows_are_uniform():
    P, seed = 256, 99
    ks = gen.keys(1, 1, 1 << 16)
    homes = np.array([oracle.window_at(int(k), 0, P, LINEAR, seed) for k in ks])
    obs = np.bincount(homes, minlength=P)
    exp = ks.size / P
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert chi2 < (P - 1) + 6 * np.sqrt(2 * (P - 1))


# ------------------------------ layout checker ----------------------------------

@pytest.mark.parametrize("scheme", [LINEAR, QUADRATIC, DOUBLE])
@pytest.mark.parametrize("W", [1, 4, 16])
def test_model_layouts_pass_and_planted_mistakes_fail(scheme, W):
    P = oracle.round_windows(4096 // W, 1, scheme) if scheme != LINEAR else 4096 // W
    C, seed = P * W, 0xABCDEF
    slots = np.zeros(C, dtype=np.uint64)
    n = int(0.9 * C)
    ks, vs = gen.keys(2, 1, n), gen.values(3, n)
    failed, win = oracle.model_insert(slots, P, W, scheme, seed, ks, vs)
    assert failed == 0
    rc, st = oracle.check_layout(slots, P, W, scheme, seed, SINGLE)
    assert rc == 0 and st["live"] == n and st["tombstones"] == 0
    assert st["sum_windows"] == int(win.sum())
    # scalar-model lookups of present keys reach them; of absent keys they stop at an empty window
    lw = oracle.model_lookup_windows(slots, P, W, scheme, seed, ks)
    assert np.array_equal(lw, win)

    # planted 1: a key moved behind an empty position of its own sequence
    bad = slots.copy()
    occupied = np.nonzero(bad)[0]
    for i in occupied[:200]:
        k = int(bad[i] & 0xFFFFFFFF)
        seq = oracle.window_sequence(k, P, P, scheme, seed)
        # find an empty slot strictly later in k's sequence than slot i
        pos = {int(w) * W + j: (l, j) for l, w in enumerate(seq) for j in range(W)}
        later = [s for s in np.nonzero(bad == 0)[0] if pos[int(s)] > pos[int(i)]]
        if later:
            # keep an empty position before the new one: move the key, leaving slot i empty
            bad[later[-1]] = bad[i]
            bad[i] = 0
            break
    assert oracle.check_layout(bad, P, W, scheme, seed, SINGLE)[0] == 2

    # planted 2: a key stored twice (single-value forbids; multi-value allows)
    bad = slots.copy()
    i0, i1 = occupied[0], np.nonzero(bad == 0)[0]
    k0 = int(bad[i0] & 0xFFFFFFFF)
    seq = oracle.window_sequence(k0, P, P, scheme, seed)
    target = None
    for l, w in enumerate(seq):  # first empty position of k0's sequence: a legal spot for a copy
        for j in range(W):
            if bad[int(w) * W + j] == 0:
                target = int(w) * W + j
                break
        if target is not None:
            break
    bad[target] = bad[i0]
    assert oracle.check_layout(bad, P, W, scheme, seed, SINGLE)[0] == 3
    assert oracle.check_layout(bad, P, W, scheme, seed, MULTI)[0] == 0

    # planted 3: a tombstone with a non-zero value half, or an empty key with a value
    bad = slots.copy()
    bad[occupied[1]] = 0xFFFFFFFF | (5 << 32)
    assert oracle.check_layout(bad, P, W, scheme, seed, SINGLE)[0] == 1
    bad = slots.copy()
    bad[i1[0]] = 7 << 32
    assert oracle.check_layout(bad, P, W, scheme, seed, SINGLE)[0] == 1

    # a proper tombstone keeps the layout valid (retrieval treats it as occupied, Sec. IV-B5)
    ok = slots.copy()
    ok[occupied[2]] = 0xFFFFFFFF
    rc, st = oracle.check_layout(ok, P, W, scheme, seed, SINGLE)
    assert rc == 0 and st["tombstones"] == 1 and st["live"] == n - 1


def test_model_windows_grow_with_load():
    # longer probing at higher load (Sec. II): mean windows per insert increase with alpha
    P, W, seed = 1 << 12, 16, 5
    means = []
    for a in (0.5, 0.8, 0.9, 0.95):
        slots = np.zeros(P * W, dtype=np.uint64)
        n = int(a * P * W)
        _, win = oracle.model_insert(slots, P, W, DOUBLE, seed, gen.keys(4, 1, n), gen.values(4, n))
        means.append(win.mean())
    assert all(x < y for x, y in zip(means, means[1:]))
    assert 1.0 <= means[0] < 1.05
