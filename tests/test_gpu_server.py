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


def _wait_all(srv, tickets, seconds=60.0):
    """Poll until every ticket is done (fails instead of blocking forever)."""
    import time
    end = time.time() + seconds
    while time.time() < end:
        if all(srv.query(t)[0] for t in tickets):
            return
        time.sleep(0.001)
    raise AssertionError("requests did not complete")


def test_conflicting_writes_allowed_set(hc):
    """Requests admitted together may write the same keys of one table (Sec. IV-D: concurrent
    same-kind writes are valid but order-dependent).  Whatever the grouping: a key's value after the
    inserts is one of the values written to it; of the inserts of a key absent before, exactly one
    reports OK and the rest DUPLICATE (all DUPLICATE for a present key); of the erases of a present
    key exactly one reports OK; counting tables count exactly; later retrieves see those results."""
    rng = np.random.default_rng(21)
    capA, capB = 1 << 14, 1 << 13
    A = hc.Table("single", capA, scheme="double", window=16, group=4, seed=5)
    B = hc.Table("counting", capB, scheme="linear", window=16, group=4, seed=6)
    U = gen.keys(600, 1, 6000)
    pre = U[:2000]
    pre_v = gen.values(601, pre.size)
    A.insert(torch.from_numpy(pre).cuda(), torch.from_numpy(pre_v).cuda())
    B.insert(torch.from_numpy(pre).cuda(), None)
    torch.cuda.synchronize()
    srv = hc.Server(staging_bytes=64 << 20)
    reqs = []  # (table, kind, keys, values, out tensors)
    def submit(tab, op, keys, vals=None, want_vals=False):
        k = _pinned(keys)
        fl = torch.empty(keys.size, dtype=torch.uint8, pin_memory=True)
        vo = torch.empty(keys.size, dtype=torch.uint32, pin_memory=True) if want_vals else None
        v = None if vals is None else _pinned(vals)
        tk = srv.submit(tab, op, k, v, values_out=vo, flags=fl, group=[1, 4, 16][len(reqs) % 3])
        reqs.append((tab, op, keys, vals, vo, fl, tk))
    for j in range(8):  # overlapping inserts (random subsets of U, so keys repeat across requests)
        keys = U[rng.choice(U.size, 1500, replace=False)]
        submit(A, hc.OP_INSERT, keys, gen.values(610 + j, keys.size))
        submit(B, hc.OP_INSERT, U[rng.choice(U.size, 1200, replace=False)])
    submit(A, hc.OP_RETRIEVE, U, want_vals=True)
    for j in range(4):  # overlapping erases
        submit(A, hc.OP_ERASE, U[rng.choice(U.size, 2500, replace=False)])
    submit(A, hc.OP_RETRIEVE, U, want_vals=True)
    submit(B, hc.OP_RETRIEVE, U, want_vals=True)
    _wait_all(srv, [r[6] for r in reqs])
    srv.close()
    ins_A = [r for r in reqs if r[0] is A and r[1] == hc.OP_INSERT]
    ins_B = [r for r in reqs if r[0] is B and r[1] == hc.OP_INSERT]
    er_A = [r for r in reqs if r[0] is A and r[1] == hc.OP_ERASE]
    ret_A = [r for r in reqs if r[0] is A and r[1] == hc.OP_RETRIEVE]
    pre_set = set(pre.tolist())
    written, ins_st = {}, {}
    for _, _, keys, vals, _, fl, _ in ins_A:
        for k, v, s in zip(keys.tolist(), vals.tolist(), fl.numpy().tolist()):
            written.setdefault(k, set()).add(v)
            ins_st.setdefault(k, []).append(s)
    # a written key holds one of the values written to it; an untouched one its prefilled value
    allowed = {int(k): {int(v)} for k, v in zip(pre, pre_v)}
    allowed.update(written)
    for k, sts in ins_st.items():
        ok = sum(s == hc.S_OK for s in sts)
        assert ok == (0 if k in pre_set else 1) and sum(s == hc.S_DUPLICATE for s in sts) == len(sts) - ok
    present = set(allowed)
    v1, f1 = ret_A[0][4].numpy(), ret_A[0][5].numpy()
    for i, k in enumerate(U.tolist()):
        assert bool(f1[i]) == (k in present)
        if f1[i]:
            assert int(v1[i]) in allowed[k]
    er_st = {}
    for _, _, keys, _, _, fl, _ in er_A:
        for k, s in zip(keys.tolist(), fl.numpy().tolist()):
            er_st.setdefault(k, []).append(s)
    for k, sts in er_st.items():
        ok = sum(s == hc.S_OK for s in sts)
        assert ok == (1 if k in present else 0) and sum(s == hc.S_NOT_FOUND for s in sts) == len(sts) - ok
    v2, f2 = ret_A[1][4].numpy(), ret_A[1][5].numpy()
    for i, k in enumerate(U.tolist()):
        assert bool(f2[i]) == (k in present and k not in er_st)
        if f2[i]:
            assert v2[i] == v1[i]  # no write in between: the epoch's value stays
    # counting: exact counts, one OK per key new to the table
    orc = oracle.OracleTable(oracle.COUNT, capB)
    orc.insert(pre)
    cst = {}
    for _, _, keys, _, _, fl, _ in ins_B:
        orc.insert(keys)
        for k, s in zip(keys.tolist(), fl.numpy().tolist()):
            cst.setdefault(k, []).append(s)
    for k, sts in cst.items():
        assert sum(s == hc.S_OK for s in sts) == (0 if k in pre_set else 1)
    vb, fb = [r for r in reqs if r[0] is B and r[1] == hc.OP_RETRIEVE][0][4:6]
    vo, fo = orc.retrieve(U)
    assert np.array_equal(vb.numpy(), vo) and np.array_equal(fb.numpy(), fo)
    assert A.size() == len(present - set(er_st)) and B.size() == orc.size()


def test_ring_reuses_space_after_draining(hc):
    """An idle staging ring starts again at offset 0: a request of almost the whole ring is admitted
    after a smaller one left the ring's head in the middle."""
    t = hc.Table("single", 1 << 18, scheme="double", window=16, group=4)
    keys = gen.keys(620, 1, 200000)
    t.insert(torch.from_numpy(keys).cuda(), torch.from_numpy(gen.values(621, keys.size)).cuda())
    torch.cuda.synchronize()
    srv = hc.Server(staging_bytes=1 << 20)
    outs = []
    for n in (60000, 110000, 30000, 115000):  # 9 bytes of staging per retrieved key
        k = _pinned(keys[:n])
        vo = torch.empty(n, dtype=torch.uint32, pin_memory=True)
        fl = torch.empty(n, dtype=torch.uint8, pin_memory=True)
        tk = srv.submit(t, hc.OP_RETRIEVE, k, values_out=vo, flags=fl)
        _wait_all(srv, [tk], 30.0)
        outs.append((n, vo, fl))
    assert srv.stats()["staging_in_use"] == 0
    srv.close()
    vals = gen.values(621, keys.size)
    for n, vo, fl in outs:
        assert fl.numpy().all() and np.array_equal(vo.numpy(), vals[:n])


def test_groups_on_disjoint_tables_overlap(hc):
    """Two launch groups on different tables: the second does not wait for the first on the device,
    so a small request on table B completes while a long one on table A (absent keys in a linear
    probing table at load 0.99: hundreds of windows per query) is still running; both results equal
    the serial server's."""
    A = hc.Table("single", 1 << 22, scheme="linear", window=16, group=4, seed=9)
    B = hc.Table("single", 1 << 12, scheme="double", window=16, group=4, seed=10)
    ka = gen.keys(630, 1, int(0.99 * A.capacity))
    A.insert(torch.from_numpy(ka).cuda(), torch.from_numpy(gen.values(631, ka.size)).cuda())
    kb = gen.keys(632, 1, 2000)
    B.insert(torch.from_numpy(kb).cuda(), torch.from_numpy(gen.values(633, kb.size)).cuda())
    torch.cuda.synchronize()
    qa = gen.keys(630, ka.size + 1, 1 << 22)  # absent from A
    qb = kb[:64]

    def run(serial):
        srv = hc.Server(staging_bytes=256 << 20, max_group_requests=1, serial=serial)
        ra = (torch.empty(qa.size, dtype=torch.uint32, pin_memory=True),
              torch.empty(qa.size, dtype=torch.uint8, pin_memory=True))
        rb = (torch.empty(qb.size, dtype=torch.uint32, pin_memory=True),
              torch.empty(qb.size, dtype=torch.uint8, pin_memory=True))
        ta = srv.submit(A, hc.OP_RETRIEVE, _pinned(qa), values_out=ra[0], flags=ra[1])
        tb = srv.submit(B, hc.OP_RETRIEVE, _pinned(qb), values_out=rb[0], flags=rb[1])
        _wait_all(srv, [tb])
        a_done_first = srv.query(ta)[0]
        _wait_all(srv, [ta])
        lat = (srv.query(ta)[1], srv.query(tb)[1])
        srv.close()
        return ra, rb, a_done_first, lat

    ra, rb, a_first, lat = run(False)
    sa, sb, _, _ = run(True)
    assert not a_first and lat[1] < lat[0], (a_first, lat)
    assert np.array_equal(ra[1].numpy(), sa[1].numpy()) and not ra[1].numpy().any()
    assert np.array_equal(rb[0].numpy(), sb[0].numpy()) and rb[1].numpy().all()
    assert np.array_equal(rb[0].numpy(), gen.values(633, kb.size)[:64])


def test_staging_budget_bounded_by_free_memory(hc):
    free, _ = torch.cuda.mem_get_info()
    srv = hc.Server(staging_bytes=1 << 60)
    st = srv.stats()
    srv.close()
    assert (1 << 20) <= st["staging_bytes"] <= free // 2 + (1 << 20)
