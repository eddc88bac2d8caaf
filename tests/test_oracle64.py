"""Pins of the 64-bit single-value oracle against things other than itself.

* brute force: a linear-scan list of (key, value) pairs on random op sequences with tiny
  capacities and key ranges, reserved keys (0 and 2^64 - 1), full tables, erase then re-insert;
* probe geometry: MurmurHash3's 64-bit finaliser checked through its algebraic inverse, every
  scheme's window sequence visiting every window exactly once;
* the layout checker: layouts built by first-fit insertion along each key's sequence pass, and
  planted mistakes (a key behind an empty slot, a key twice, bad encodings, a key off its
  sequence) are caught with their codes.
"""
import random

import numpy as np
import pytest

import oracle
from oracle import DOUBLE, LINEAR, QUADRATIC

M64 = 2**64 - 1
RES = [0, M64]
OK, DUP, FULL, INVALID, NOT_FOUND = 0, 1, 2, 3, 4


class Brute64:
    def __init__(self, cap):
        self.cap, self.pairs = cap, []

    def _find(self, k):
        for j, (kk, _) in enumerate(self.pairs):
            if kk == k:
                return j
        return -1

    def insert(self, keys, vals):
        out = []
        for k, v in zip(keys, vals):
            if k in RES:
                out.append(INVALID)
                continue
            j = self._find(k)
            if j >= 0:
                self.pairs[j] = (k, v)
                out.append(DUP)
            elif len(self.pairs) < self.cap:
                self.pairs.append((k, v))
                out.append(OK)
            else:
                out.append(FULL)
        return out

    def retrieve(self, keys):
        vals, found = [], []
        for k in keys:
            j = -1 if k in RES else self._find(k)
            vals.append(self.pairs[j][1] if j >= 0 else 0)
            found.append(1 if j >= 0 else 0)
        return vals, found

    def erase(self, keys):
        out = []
        for k in keys:
            j = -1 if k in RES else self._find(k)
            if k in RES:
                out.append(INVALID)
            elif j >= 0:
                self.pairs.pop(j)
                out.append(OK)
            else:
                out.append(NOT_FOUND)
        return out


@pytest.mark.parametrize("seed", range(30))
def test_oracle64_equals_brute_force(seed):
    rng = random.Random(seed)
    cap = rng.choice([1, 2, 5, 16, 64])
    hi = rng.choice([4, 20, 2**40])
    o, b = oracle.OracleTable64(cap), Brute64(cap)
    for _ in range(30):
        op = rng.choice(["insert", "insert", "retrieve", "erase"])
        batch = [rng.choice(RES) if rng.random() < 0.05 else rng.randint(1, hi) for _ in range(rng.randint(0, 10))]
        if op == "insert":
            vals = [rng.choice([0, 1, M64, rng.getrandbits(64)]) for _ in batch]
            assert list(o.insert(batch, vals)) == b.insert(batch, vals)
        elif op == "retrieve":
            v, f = o.retrieve(batch)
            vb, fb = b.retrieve(batch)
            assert [int(x) for x in v] == vb and list(f) == fb
        else:
            assert list(o.erase(batch)) == b.erase(batch)
        assert o.size() == len(b.pairs)


def _fmix64_inverse(y):
    def unshift(x):  # inverse of x ^= x >> 33 (one step suffices: 2 * 33 > 64)
        return x ^ (x >> 33)
    y = unshift(y)
    y = (y * pow(0xc4ceb9fe1a85ec53, -1, 2**64)) & M64
    y = unshift(y)
    y = (y * pow(0xff51afd7ed558ccd, -1, 2**64)) & M64
    return unshift(y)


def test_fmix64_is_bijective():
    rng = random.Random(5)
    for x in [0, 1, 2, M64, 2**63] + [rng.getrandbits(64) for _ in range(20000)]:
        assert _fmix64_inverse(oracle.fmix64(x)) == x
    assert oracle.fmix64(0) == 0


@pytest.mark.parametrize("scheme", [LINEAR, QUADRATIC, DOUBLE])
def test_window_sequence64_covers_every_window_once(scheme):
    Ps = [1, 2, 8, 64, 512]
    if scheme == LINEAR:
        Ps += [3, 100]
    if scheme == DOUBLE:
        Ps += [3, 31, 101, 1009]
    rng = random.Random(scheme + 10)
    for P in Ps:
        for _ in range(5):
            k, seed = rng.randint(1, M64 - 1), rng.getrandbits(64)
            seq = sorted(oracle.window_at64(k, l, P, scheme, seed) for l in range(P))
            assert seq == list(range(P)), (scheme, P)


def _first_fit(keys, vals, P, W, scheme, seed):
    """A layout by sequential first-fit insertion: each key at the first empty slot of its sequence."""
    slots = np.zeros(2 * P * W, dtype=np.uint64)
    for k, v in zip(keys, vals):
        for l in range(P):
            w = oracle.window_at64(k, l, P, scheme, seed)
            free = [j for j in range(W) if slots[2 * (w * W + j)] == 0]
            if free:
                i = w * W + free[0]
                slots[2 * i], slots[2 * i + 1] = k, v
                break
    return slots


@pytest.mark.parametrize("scheme", [LINEAR, QUADRATIC, DOUBLE])
@pytest.mark.parametrize("W", [1, 4, 8])
def test_layout64_checker(scheme, W):
    P = 256 // W
    seed, rng = 0x1234, random.Random(scheme * 7 + W)
    keys = rng.sample(range(1, 2**62), int(0.85 * P * W))
    vals = [rng.getrandbits(64) for _ in keys]
    slots = _first_fit(keys, vals, P, W, scheme, seed)
    rc, st = oracle.check_layout64(slots, P, W, scheme, seed)
    assert rc == 0 and st["live"] == len(keys) and st["tombstones"] == 0
    live = [i for i in range(P * W) if slots[2 * i] not in (0, M64)]
    empty = [i for i in range(P * W) if slots[2 * i] == 0]
    # a key moved to a later empty slot of its own sequence, leaving an empty slot before it
    moved = False
    for i in live:
        k = int(slots[2 * i])
        order = [oracle.window_at64(k, l, P, scheme, seed) * W + j for l in range(P) for j in range(W)]
        pos = {s: r for r, s in enumerate(order)}
        later = [e for e in empty if pos[e] > pos[i]]
        if later:
            bad = slots.copy()
            bad[2 * later[-1]], bad[2 * later[-1] + 1] = bad[2 * i], bad[2 * i + 1]
            bad[2 * i] = bad[2 * i + 1] = 0
            assert oracle.check_layout64(bad, P, W, scheme, seed)[0] == 2
            moved = True
            break
    assert moved
    # a key twice
    bad = slots.copy()
    bad[2 * empty[0]], bad[2 * empty[0] + 1] = bad[2 * live[0]], 1
    assert oracle.check_layout64(bad, P, W, scheme, seed)[0] in (2, 3)
    # bad encodings: an empty slot with a value, a tombstone with a value
    bad = slots.copy()
    bad[2 * empty[0] + 1] = 9
    assert oracle.check_layout64(bad, P, W, scheme, seed)[0] == 1
    bad = slots.copy()
    bad[2 * live[1]], bad[2 * live[1] + 1] = M64, 3
    assert oracle.check_layout64(bad, P, W, scheme, seed)[0] == 1
    # a proper tombstone keeps the layout valid
    ok = slots.copy()
    ok[2 * live[2]], ok[2 * live[2] + 1] = M64, 0
    rc, st = oracle.check_layout64(ok, P, W, scheme, seed)
    assert rc == 0 and st["tombstones"] == 1 and st["live"] == len(keys) - 1
