"""GPU tests of the serving loop: each request's results are the same alone (serial
server) and in the continuous-batching mix, and equal the oracle replay in arrival order."""
import numpy as np
import pytest
import torch

import gen
import oracle

pytestmark = pytest.mark.gpu


def _pinned(a, dtype=torch.uint32):
    t = torch.empty(a.size, dtype=dtype, pin_memory=True)
    t.numpy()[:] = a
    return t


def _stream(n_req, caps, seed):
    """Requests over tables: inserts of fresh key slices, erases of disjoint prefilled slices,
    retrieves of any universe key plus absent keys (concurrent writes never share a key)."""
    rng = np.random.default_rng(seed)
    uni = [gen.keys(seed + j, 1, int(0.9 * c)) for j, c in enumerate(caps)]
    pre = [u.size // 2 for u in uni]
    nxt_ins = list(pre)
    nxt_er = [0] * len(caps)
    reqs = []
    for r in range(n_req):
        t = int(rng.integers(len(caps)))
        n = int(2 ** rng.uniform(0, 12))
        kind = rng.choice(["insert", "retrieve", "erase"], p=[0.3, 0.6, 0.1])
        if kind == "insert":
            n = min(n, uni[t].size - nxt_ins[t])
            if n <= 0:
                kind = "retrieve"
            else:
                keys = uni[t][nxt_ins[t]:nxt_ins[t] + n]
                nxt_ins[t] += n
                reqs.append((t, "insert", keys, gen.values(seed * 1000 + r, n)))
                continue
        if kind == "erase":
            n = min(n, pre[t] // 2 - nxt_er[t])
            if n > 0:
                keys = uni[t][nxt_er[t]:nxt_er[t] + n]
                nxt_er[t] += n
                reqs.append((t, "erase", keys, None))
                continue
        idx = rng.integers(0, uni[t].size, n)
        keys = uni[t][idx]
        keys[: max(1, n // 10)] = gen.keys(seed + 99, 1 + r * 64, max(1, n // 10))[: keys[: max(1, n // 10)].size]
        reqs.append((t, "retrieve", keys, None))
    return uni, pre, reqs


def _run(hc, caps, uni, pre, reqs, serial, staging=64 << 20):
    tabs = [hc.Table("single", c, scheme="double", window=16, group=4, seed=7 + j) for j, c in enumerate(caps)]
    for t, u, p in zip(tabs, uni, pre):
        t.insert(torch.from_numpy(u[:p]).cuda(), torch.from_numpy(gen.values(3, p)).cuda())
    torch.cuda.synchronize()
    srv = hc.Server(staging_bytes=staging, serial=serial)
    outs, tickets = [], []
    for j, (t, kind, keys, vals) in enumerate(reqs):
        k = _pinned(keys)
        if kind == "insert":
            fl = torch.empty(keys.size, dtype=torch.uint8, pin_memory=True)
            tickets.append(srv.submit(tabs[t], hc.OP_INSERT, k, _pinned(vals), flags=fl, group=[2, 4, 8][j % 3]))
            outs.append((None, fl))
        elif kind == "erase":
            fl = torch.empty(keys.size, dtype=torch.uint8, pin_memory=True)
            tickets.append(srv.submit(tabs[t], hc.OP_ERASE, k, flags=fl))
            outs.append((None, fl))
        else:
            vo = torch.empty(keys.size, dtype=torch.uint32, pin_memory=True)
            fl = torch.empty(keys.size, dtype=torch.uint8, pin_memory=True)
            tickets.append(srv.submit(tabs[t], hc.OP_RETRIEVE, k, values_out=vo, flags=fl, group=[1, 4, 16][j % 3]))
            outs.append((vo, fl))
    srv.drain()
    st = srv.stats()
    lat = [srv.query(tk)[1] for tk in tickets]
    srv.close()
    res = [(None if vo is None else vo.numpy().copy(), fl.numpy().copy()) for vo, fl in outs]
    sizes = [t.size() for t in tabs]
    for t in tabs:
        t.close()
    return res, sizes, st, lat


def test_same_alone_and_in_the_mix(hc):
    caps = [1 << 14, 1 << 16, 1 << 15, 1 << 17]
    uni, pre, reqs = _stream(300, caps, 11)
    mix, size_mix, st_mix, lat = _run(hc, caps, uni, pre, reqs, serial=False)
    alone, size_alone, st_alone, _ = _run(hc, caps, uni, pre, reqs, serial=True)
    assert st_mix["completed"] == len(reqs) and st_alone["completed"] == len(reqs)
    nonempty = sum(1 for r in reqs if r[2].size > 0)
    assert nonempty < len(reqs)  # the stream holds empty requests too: they complete at submission
    assert st_alone["launch_groups"] == nonempty
    assert st_mix["launch_groups"] < len(reqs)  # requests were coalesced
    assert all(x >= 0 for x in lat)
    for (vm, fm), (va, fa) in zip(mix, alone):
        assert np.array_equal(fm, fa)
        if vm is not None:
            assert np.array_equal(vm, va)
    assert size_mix == size_alone
    # oracle replay in arrival order
    orcs = [oracle.OracleTable(oracle.SINGLE, 1 << 30) for _ in caps]
    for o, u, p in zip(orcs, uni, pre):
        o.insert(u[:p], gen.values(3, p))
    for (t, kind, keys, vals), (vo, fl) in zip(reqs, mix):
        if kind == "insert":
            assert np.array_equal(fl, orcs[t].insert(keys, vals))
        elif kind == "erase":
            assert np.array_equal(fl, orcs[t].erase(keys))
        else:
            v, f = orcs[t].retrieve(keys)
            assert np.array_equal(vo, v) and np.array_equal(fl, f)
    assert size_mix == [o.size() for o in orcs]


def test_tight_staging_budget_admits_in_order(hc):
    caps = [1 << 16, 1 << 15]
    uni, pre, reqs = _stream(120, caps, 5)
    # 1 MiB of staging: large requests wait until earlier ones free the ring
    small, size_small, st, _ = _run(hc, caps, uni, pre, reqs, serial=False, staging=1 << 20)
    ref, size_ref, _, _ = _run(hc, caps, uni, pre, reqs, serial=True)
    for (vm, fm), (va, fa) in zip(small, ref):
        assert np.array_equal(fm, fa)
        if vm is not None:
            assert np.array_equal(vm, va)
    assert size_small == size_ref and st["completed"] == len(reqs)


def test_server_argument_errors(hc):
    srv = hc.Server(staging_bytes=1 << 20)
    mv = hc.Table("multi", 1024)
    sv = hc.Table("single", 1024)
    k = torch.zeros(4, dtype=torch.uint32, pin_memory=True)
    with pytest.raises(hc.HcError) as e:
        srv.submit(mv, hc.OP_RETRIEVE, k)
    assert e.value.code == hc.E_KIND
    with pytest.raises(hc.HcError) as e:
        srv.submit(sv, hc.OP_INSERT, k)  # values missing
    assert e.value.code == hc.E_ARG
    big = torch.zeros(1 << 20, dtype=torch.uint32)
    with pytest.raises(hc.HcError) as e:
        srv.submit(sv, hc.OP_RETRIEVE, big, values_out=torch.zeros(1 << 20, dtype=torch.uint32))
    assert e.value.code == hc.E_ARG  # can never fit 1 MiB of staging
    t = srv.submit(sv, hc.OP_RETRIEVE, torch.zeros(0, dtype=torch.uint32))
    assert srv.query(t)[0]
    srv.close()
