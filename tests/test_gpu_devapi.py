"""The device-side API (hc_device_api.hpp) called from user kernels, against the oracle and numpy.

The kernels live in tests/devapi/devapi_kernels.hip (built by __graft_entry__.build()): a fused
k-mer counter that turns a DNA read into 2-bit k-mer codes and counts them in a counting table
from inside one kernel, a fused k-mer index that inserts (k-mer, position) pairs into a
multi-value table from one kernel (the paper's device-sided database build, Sec. V-C), group
lookups, group inserts, a per-key for_each collection of values and a for_all export.
"""
import ctypes
import os

import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import check_layout, d, h

pytestmark = pytest.mark.gpu

LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "devapi", "libhc_devapi.so")


@pytest.fixture(scope="module")
def dev():
    if not os.path.exists(LIB):
        raise RuntimeError("tests/devapi/libhc_devapi.so is not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB)
    lib.devapi_view_bytes.restype = ctypes.c_uint64
    P = ctypes.c_void_p
    lib.devapi_count_kmers.argtypes = [P, ctypes.c_uint32, P, ctypes.c_uint64, ctypes.c_uint32, P]
    lib.devapi_lookup.argtypes = [P, ctypes.c_uint32, P, ctypes.c_uint64, P, P, P]
    lib.devapi_insert.argtypes = [P, ctypes.c_uint32, P, P, ctypes.c_uint64, P, P]
    lib.devapi_export.argtypes = [P, ctypes.c_uint32, P, P, P, P]
    lib.devapi_index_kmers.argtypes = [P, ctypes.c_uint32, P, ctypes.c_uint64, ctypes.c_uint32, P, P]
    lib.devapi_collect.argtypes = [P, ctypes.c_uint32, P, ctypes.c_uint64, P, P, P, P]
    return lib


def _view(hc, dev, t):
    return hc.hc_device_view(t.handle, int(dev.devapi_view_bytes()))


@pytest.mark.parametrize("k", [5, 12, 15])
def test_fused_kmer_counting(hc, dev, k):
    n = 200000
    seq = (gen.values(300 + k, n) & 3).astype(np.uint8)  # a random read, bases 0..3
    t = hc.Table("counting", 1 << 18, scheme="double", window=16, group=4)
    s = torch.cuda.current_stream()
    dseq = d(seq)
    assert dev.devapi_count_kmers(_view(hc, dev, t), 16, dseq.data_ptr(), n, k, ctypes.c_void_p(s.cuda_stream)) == 0
    torch.cuda.synchronize()
    # numpy: codes of every window of the read, then counts per distinct code
    w = np.lib.stride_tricks.sliding_window_view(seq.astype(np.uint64), k)
    codes = (w * (4 ** np.arange(k - 1, -1, -1, dtype=np.uint64))).sum(axis=1).astype(np.uint64)
    u, c = np.unique(codes + 1, return_counts=True)
    assert t.size() == u.size
    v, f = t.retrieve(d(u.astype(np.uint32)))
    assert np.all(h(f) == 1) and np.array_equal(h(v), c.astype(np.uint32))
    check_layout(t, oracle.COUNT)


def test_device_insert_lookup_export(hc, dev):
    w = gen.single_value_workload(1 << 16, 0.85, 17)
    t = hc.Table("single", 1 << 16, scheme="quadratic", window=16, group=4)
    orc = oracle.OracleTable(oracle.SINGLE, t.capacity)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    keys = np.concatenate([w["keys"], w["keys"][:1000], np.array([0, 0xFFFFFFFF], np.uint32)])
    vals = np.concatenate([w["values"], w["values"][:1000], np.array([1, 2], np.uint32)])
    dk, dv = d(keys), d(vals)
    st = torch.empty(keys.size, dtype=torch.uint8, device="cuda")
    assert dev.devapi_insert(_view(hc, dev, t), 16, dk.data_ptr(), dv.data_ptr(), keys.size, st.data_ptr(), s) == 0
    torch.cuda.synchronize()
    # one copy of a repeated key reports OK, the other DUPLICATE; which one is unspecified within a launch
    st, st_o = h(st), orc.insert(keys, vals)
    order = np.lexsort((st, keys))
    order_o = np.lexsort((st_o, keys))
    assert np.array_equal(st[order], st_o[order_o])
    assert t.size() == orc.size()
    q = w["queries"]
    out = torch.empty(q.size, dtype=torch.uint32, device="cuda")
    fnd = torch.empty(q.size, dtype=torch.uint8, device="cuda")
    dq = d(q)
    assert dev.devapi_lookup(_view(hc, dev, t), 16, dq.data_ptr(), q.size, out.data_ptr(), fnd.data_ptr(), s) == 0
    torch.cuda.synchronize()
    vo, fo = orc.retrieve(q)
    assert np.array_equal(h(out), vo) and np.array_equal(h(fnd), fo)
    ek = torch.empty(t.capacity, dtype=torch.uint32, device="cuda")
    ev = torch.empty(t.capacity, dtype=torch.uint32, device="cuda")
    en = torch.zeros(1, dtype=torch.uint64, device="cuda")
    assert dev.devapi_export(_view(hc, dev, t), 16, ek.data_ptr(), ev.data_ptr(), en.data_ptr(), s) == 0
    torch.cuda.synchronize()
    m = int(en.item())
    assert m == orc.size()
    ek, ev = h(ek)[:m], h(ev)[:m]
    order = np.argsort(ek)
    vo2, fo2 = orc.retrieve(ek[order])
    assert np.all(fo2 == 1) and np.array_equal(vo2, ev[order])
    check_layout(t, oracle.SINGLE)


def _kmer_codes(seq, k):
    w = np.lib.stride_tricks.sliding_window_view(seq.astype(np.uint64), k)
    return (w * (4 ** np.arange(k - 1, -1, -1, dtype=np.uint64))).sum(axis=1).astype(np.uint32)


@pytest.mark.parametrize("k", [4, 9, 15])
def test_fused_kmer_index_multi_value(hc, dev, k):
    """One kernel turns a read into k-mer codes and inserts (code + 1, position) into a multi-value
    table through dev::insert; a second user kernel collects every k-mer's positions with
    dev::for_each.  Both against the oracle's multimap (segments compared sorted)."""
    n = 150000
    seq = (gen.values(500 + k, n) & 3).astype(np.uint8)
    t = hc.Table("multi", 1 << 18, scheme="double", window=16, group=4)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    dseq = d(seq)
    st = torch.empty(n - k + 1, dtype=torch.uint8, device="cuda")
    assert dev.devapi_index_kmers(_view(hc, dev, t), 16, dseq.data_ptr(), n, k, st.data_ptr(), s) == 0
    torch.cuda.synchronize()
    keys = _kmer_codes(seq, k) + 1
    pos = np.arange(keys.size, dtype=np.uint32)
    orc = oracle.OracleTable(oracle.MULTI, t.capacity)
    assert np.array_equal(h(st), orc.insert(keys, pos))
    assert t.size() == orc.size() == keys.size
    check_layout(t, oracle.MULTI)
    q = np.concatenate([np.unique(keys), np.array([0, 0xFFFFFFFF], np.uint32),
                        np.setdiff1d(np.arange(1, 4 ** min(k, 12) + 1, 97, dtype=np.uint32), keys)[:500]])
    co, oo = orc.count_values(q)
    _, vo = orc.retrieve_all(q, oo)
    seg = np.repeat(np.arange(q.size), co.astype(np.int64))
    # bulk two-pass retrieval of the same table
    counts, offsets, total = t.count_values(d(q))
    assert np.array_equal(h(counts), co) and np.array_equal(h(offsets), oo)
    _, vals = t.retrieve_all(d(q))
    vals = h(vals)
    assert np.array_equal(vals[np.lexsort((vals, seg))], vo)
    # one-pass for_each into the same segments
    out = torch.zeros(max(int(oo[-1]), 1), dtype=torch.uint32, device="cuda")
    cnt = torch.empty(q.size, dtype=torch.uint32, device="cuda")
    dq, doff = d(q), d(oo)
    assert dev.devapi_collect(_view(hc, dev, t), 16, dq.data_ptr(), q.size, doff.data_ptr(), out.data_ptr(),
                              cnt.data_ptr(), s) == 0
    torch.cuda.synchronize()
    assert np.array_equal(h(cnt), co)
    o = h(out)[: int(oo[-1])]
    assert np.array_equal(o[np.lexsort((o, seg))], vo)


def test_for_each_single_value(hc, dev):
    """for_each on a single-value table yields the key's one value (count 1) or nothing."""
    w = gen.single_value_workload(1 << 15, 0.9, 23)
    t = hc.Table("single", 1 << 15, scheme="linear", window=16, group=4)
    t.insert(d(w["keys"]), d(w["values"]))
    orc = oracle.OracleTable(oracle.SINGLE, t.capacity)
    orc.insert(w["keys"], w["values"])
    q = w["queries"]
    vo, fo = orc.retrieve(q)
    offsets = np.arange(q.size + 1, dtype=np.uint64)
    out = torch.zeros(q.size, dtype=torch.uint32, device="cuda")
    cnt = torch.empty(q.size, dtype=torch.uint32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    dq, doff = d(q), d(offsets)
    assert dev.devapi_collect(_view(hc, dev, t), 16, dq.data_ptr(), q.size, doff.data_ptr(), out.data_ptr(),
                              cnt.data_ptr(), s) == 0
    torch.cuda.synchronize()
    assert np.array_equal(h(cnt), fo.astype(np.uint32))
    assert np.array_equal(h(out)[fo == 1], vo[fo == 1])
