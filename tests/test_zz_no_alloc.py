"""hc_count_values_noalloc (no device allocation; scratch in a fixed per-GPU array) against
hc_count_values through the C ABI: two calls in a row, the second with a smaller input, on a
multi-value table whose heavy keys send queries to the long-query rounds, then a bucket list
table; and the size limit."""
import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import d, h

pytestmark = pytest.mark.gpu


def _both(hc, t, q, group):
    n = q.numel()
    ca = torch.empty(n, dtype=torch.uint32, device="cuda")
    oa = torch.empty(n + 1, dtype=torch.uint64, device="cuda")
    cb = torch.empty(n, dtype=torch.uint32, device="cuda")
    ob = torch.empty(n + 1, dtype=torch.uint64, device="cuda")
    ta = hc.hc_count_values(t.handle, q, oa, ca, True, group)
    tb = hc.hc_count_values_noalloc(t.handle, q, ob, cb, True, group)
    assert ta == tb
    assert torch.equal(ca, cb) and torch.equal(oa, ob)
    return h(cb), h(ob)


@pytest.mark.parametrize("kind", ["multi", "bucket"])
def test_noalloc_count_matches_allocating_call(hc, kind):
    w = gen.multi_value_zipf_workload(1 << 18, 1 << 11, 1.1, 700)
    t = hc.Table(kind, 1 << 19, scheme="double", window=16, group=4)
    hc.hc_insert_grouped(t.handle, d(w["keys"]), d(w["values"]))
    orc = oracle.OracleTable(oracle.MULTI, 1 << 20)
    orc.insert(w["keys"], w["values"])
    q = w["queries"]
    for qs, group in ((q, 4), (q[: q.size // 3 + 17], 16)):  # second call smaller (ragged)
        c, o = _both(hc, t, d(qs), group)
        co, oo = orc.count_values(qs)
        assert np.array_equal(c, co) and np.array_equal(o, oo)
    # an empty batch still writes offsets[0] = 0
    e = torch.empty(0, dtype=torch.uint32, device="cuda")
    c, o = _both(hc, t, e, 0)
    assert o.tolist() == [0]


def test_noalloc_size_limit(hc):
    t = hc.Table("multi", 1 << 12)
    keys = torch.ones(4, dtype=torch.uint32, device="cuda")
    off = torch.empty(5, dtype=torch.uint64, device="cuda")
    import ctypes
    rc = hc._lib.hc_count_values_noalloc(t.handle, keys.data_ptr(), (1 << 28) + 1, None, off.data_ptr(), None, 0,
                                         None)
    assert rc == hc.E_ARG
