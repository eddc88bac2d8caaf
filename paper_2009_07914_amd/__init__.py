"""Python binding of libhc.so, the MI355X cooperative-probing hash tables.

Argument marshalling only: every operation runs in the library's HIP kernels.
Device arrays are torch tensors on the table's GPU (PyTorch supplies device
memory and streams); the functions mirror the C ABI of ``include/hc.h`` one to
one, and ``Table`` wraps a handle for convenience.  There is no CPU fallback:
if ``libhc.so`` is missing this module raises on import.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loads the HIP runtime first, so libhc.so binds to the same one

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python paper_2009_07914_amd/build.py` "
                      "or `__graft_entry__.build()`")

_lib = ctypes.CDLL(LIB_PATH)

SINGLE_VALUE, MULTI_VALUE, COUNTING = 0, 1, 2
LINEAR, QUADRATIC, DOUBLE = 0, 1, 2
S_OK, S_DUPLICATE, S_FULL, S_INVALID_KEY, S_NOT_FOUND = 0, 1, 2, 3, 4
E_OK, E_ARG, E_NOMEM, E_KIND, E_DEVICE = 0, 1, 2, 3, 4

OP_INSERT, OP_RETRIEVE, OP_ERASE = 0, 1, 2

SCHEMES = {"linear": LINEAR, "quadratic": QUADRATIC, "double": DOUBLE}
BUCKET_LIST, SINGLE_VALUE_64, HASH_SET, SINGLE_VALUE_64_SOA = 3, 4, 5, 6
KINDS = {"single": SINGLE_VALUE, "multi": MULTI_VALUE, "counting": COUNTING, "bucket": BUCKET_LIST,
         "single64": SINGLE_VALUE_64, "set": HASH_SET, "single64_soa": SINGLE_VALUE_64_SOA}
WIDE_KINDS = (SINGLE_VALUE_64, SINGLE_VALUE_64_SOA)


class HcParams(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_uint32), ("window", ctypes.c_uint32), ("group", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("seed", ctypes.c_uint64)]


class HcTableInfo(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("scheme", ctypes.c_uint32), ("window", ctypes.c_uint32),
                ("group", ctypes.c_uint32), ("windows", ctypes.c_uint64), ("capacity", ctypes.c_uint64),
                ("seed", ctypes.c_uint64), ("d_slots", ctypes.c_void_p)]


PROBE_BUCKETS = 16


class HcBucketParams(ctypes.Structure):
    _fields_ = [("pool_values", ctypes.c_uint64), ("s0", ctypes.c_uint32), ("smax", ctypes.c_uint32),
                ("growth", ctypes.c_double)]


class HcBucketUsage(ctypes.Structure):
    _fields_ = [("values", ctypes.c_uint64), ("pool_used", ctypes.c_uint64), ("pool_words", ctypes.c_uint64),
                ("smax", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class HcBloomParams(ctypes.Structure):
    _fields_ = [("block_words", ctypes.c_uint32), ("group", ctypes.c_uint32), ("seed", ctypes.c_uint64)]


class HcBloomInfo(ctypes.Structure):
    _fields_ = [("blocks", ctypes.c_uint64), ("block_words", ctypes.c_uint32), ("group", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("d_bits", ctypes.c_void_p)]


class HcTableStats(ctypes.Structure):
    _fields_ = [("live", ctypes.c_uint64), ("tombstones", ctypes.c_uint64), ("empty", ctypes.c_uint64),
                ("max_probe", ctypes.c_uint64), ("probe_sum", ctypes.c_uint64),
                ("probe_hist", ctypes.c_uint64 * PROBE_BUCKETS), ("cas_fails", ctypes.c_uint64)]


class HcBatchOp(ctypes.Structure):
    _fields_ = [("table", ctypes.c_void_p), ("op", ctypes.c_uint32), ("group", ctypes.c_uint32),
                ("d_keys", ctypes.c_void_p), ("d_values", ctypes.c_void_p), ("d_values_out", ctypes.c_void_p),
                ("d_flags", ctypes.c_void_p), ("n", ctypes.c_uint64)]


class HcServerParams(ctypes.Structure):
    _fields_ = [("staging_bytes", ctypes.c_uint64), ("max_group_ops", ctypes.c_uint64),
                ("max_group_requests", ctypes.c_uint32), ("streams", ctypes.c_uint32),
                ("serial", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class HcRequest(ctypes.Structure):
    _fields_ = [("table", ctypes.c_void_p), ("op", ctypes.c_uint32), ("group", ctypes.c_uint32),
                ("h_keys", ctypes.c_void_p), ("h_values", ctypes.c_void_p), ("h_values_out", ctypes.c_void_p),
                ("h_flags", ctypes.c_void_p), ("n", ctypes.c_uint64)]


class HcServerCounts(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("launch_groups", ctypes.c_uint64),
                ("ops_completed", ctypes.c_uint64), ("staging_in_use", ctypes.c_uint64),
                ("staging_bytes", ctypes.c_uint64)]


_p, _u32, _u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
_SIGS = {
    "hc_default_params": ([ctypes.POINTER(HcParams)], None),
    "hc_create": ([ctypes.POINTER(_p), _u32, _u64, ctypes.POINTER(HcParams)], ctypes.c_int),
    "hc_create_in": ([ctypes.POINTER(_p), _u32, _p, _u64, _u64, ctypes.POINTER(HcParams)], ctypes.c_int),
    "hc_table_bytes": ([_u64, ctypes.POINTER(HcParams), ctypes.POINTER(_u64)], ctypes.c_int),
    "hc_stats": ([_p, ctypes.POINTER(HcTableStats), _p], ctypes.c_int),
    "hc_default_bucket_params": ([ctypes.POINTER(HcBucketParams)], None),
    "hc_create_bucket_list": ([ctypes.POINTER(_p), _u64, ctypes.POINTER(HcParams), ctypes.POINTER(HcBucketParams)],
                              ctypes.c_int),
    "hc_bucket_usage": ([_p, ctypes.POINTER(HcBucketUsage), _p], ctypes.c_int),
    "hc_dump_buckets": ([_p, _p, _p, _p], ctypes.c_int),
    "hc_device_view": ([_p, _p, _u64], ctypes.c_int),
    "hc_insert64": ([_p, _p, _p, _u64, _p, _u32, _p], ctypes.c_int),
    "hc_retrieve64": ([_p, _p, _u64, _p, _p, _u32, _p], ctypes.c_int),
    "hc_erase64": ([_p, _p, _u64, _p, _u32, _p], ctypes.c_int),
    "hc_diag_copy": ([_p, _p, _u64, _p], ctypes.c_int),
    "hc_diag_read": ([_p, _u64, _p, _p], ctypes.c_int),
    "hc_diag_atomic": ([_p, _u64, _u32, _u64, _u32, _p, _p], ctypes.c_int),
    "hc_diag_gather": ([_p, _u64, _u32, _u64, _u32, _p, _p], ctypes.c_int),
    "hc_default_bloom_params": ([ctypes.POINTER(HcBloomParams)], None),
    "hc_bloom_create": ([ctypes.POINTER(_p), _u64, ctypes.POINTER(HcBloomParams)], ctypes.c_int),
    "hc_bloom_destroy": ([_p], ctypes.c_int),
    "hc_bloom_clear": ([_p, _p], ctypes.c_int),
    "hc_bloom_insert": ([_p, _p, _u64, _u32, _p], ctypes.c_int),
    "hc_bloom_contains": ([_p, _p, _u64, _p, _u32, _p], ctypes.c_int),
    "hc_bloom_info": ([_p, ctypes.POINTER(HcBloomInfo)], ctypes.c_int),
    "hc_bloom_dump": ([_p, _p, _p], ctypes.c_int),
    "hc_destroy": ([_p], ctypes.c_int),
    "hc_clear": ([_p, _p], ctypes.c_int),
    "hc_insert": ([_p, _p, _p, _u64, _p, _u32, _p], ctypes.c_int),
    "hc_retrieve": ([_p, _p, _u64, _p, _p, _u32, _p], ctypes.c_int),
    "hc_erase": ([_p, _p, _u64, _p, _u32, _p], ctypes.c_int),
    "hc_count_values": ([_p, _p, _u64, _p, _p, ctypes.POINTER(_u64), _u32, _p], ctypes.c_int),
    "hc_count_values_noalloc": ([_p, _p, _u64, _p, _p, ctypes.POINTER(_u64), _u32, _p], ctypes.c_int),
    "hc_retrieve_all": ([_p, _p, _u64, _p, _p, _u32, _p], ctypes.c_int),
    "hc_insert_grouped": ([_p, _p, _p, _u64, _p], ctypes.c_int),
    "hc_size": ([_p, ctypes.POINTER(_u64), _p], ctypes.c_int),
    "hc_load_factor": ([_p, ctypes.POINTER(ctypes.c_double), _p], ctypes.c_int),
    "hc_capacity": ([_p, ctypes.POINTER(_u64)], ctypes.c_int),
    "hc_info": ([_p, ctypes.POINTER(HcTableInfo)], ctypes.c_int),
    "hc_dump_slots": ([_p, _p, _p], ctypes.c_int),
    "hc_batch_create": ([ctypes.POINTER(_p), ctypes.POINTER(HcBatchOp), _u32], ctypes.c_int),
    "hc_batch_create_flags": ([ctypes.POINTER(_p), ctypes.POINTER(HcBatchOp), _u32, _u32], ctypes.c_int),
    "hc_batch_abandoned_waits": ([_p, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "hc_batch_launch": ([_p, _p], ctypes.c_int),
    "hc_batch_info": ([_p, ctypes.POINTER(_u32), ctypes.POINTER(_u32)], ctypes.c_int),
    "hc_batch_destroy": ([_p], ctypes.c_int),
    "hc_batch_run": ([ctypes.POINTER(HcBatchOp), _u32, _p], ctypes.c_int),
    "hc_batch_capture": ([_p, ctypes.POINTER(_p)], ctypes.c_int),
    "hc_graph_launch": ([_p, _p], ctypes.c_int),
    "hc_graph_destroy": ([_p], ctypes.c_int),
    "hc_default_server_params": ([ctypes.POINTER(HcServerParams)], None),
    "hc_server_create": ([ctypes.POINTER(_p), ctypes.POINTER(HcServerParams)], ctypes.c_int),
    "hc_server_submit": ([_p, ctypes.POINTER(HcRequest), ctypes.POINTER(_u64)], ctypes.c_int),
    "hc_server_query": ([_p, _u64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "hc_server_wait": ([_p, _u64], ctypes.c_int),
    "hc_server_drain": ([_p], ctypes.c_int),
    "hc_server_stats": ([_p, ctypes.POINTER(HcServerCounts)], ctypes.c_int),
    "hc_server_destroy": ([_p], ctypes.c_int),
    "hc_error_string": ([ctypes.c_int], ctypes.c_char_p),
    "hc_last_error": ([], ctypes.c_char_p),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


class HcError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _lib.hc_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_lib.hc_error_string(code).decode()} ({msg})")


def _check(rc: int, where: str):
    if rc != E_OK:
        raise HcError(rc, where)


def _stream(stream) -> int | None:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _dptr(t, dtype, what, n=None):
    """Device pointer of a contiguous tensor of ``dtype`` on a GPU (or None)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if n is not None and t.numel() < n:
        raise ValueError(f"{what} has {t.numel()} elements, needs {n}")
    return t.data_ptr()


def _u32t(t, what, n=None):
    # uint32 data travels in int32 or uint32 tensors (same bits)
    if t is not None and t.dtype == torch.int32:
        t = t.view(torch.uint32)
    return _dptr(t, torch.uint32, what, n)


# ---- one-to-one mirrors of the C ABI -------------------------------------------------

def hc_default_params() -> HcParams:
    p = HcParams()
    _lib.hc_default_params(ctypes.byref(p))
    return p


def hc_create(kind: int, capacity: int, params: HcParams | None = None) -> int:
    h = ctypes.c_void_p()
    _check(_lib.hc_create(ctypes.byref(h), kind, capacity, ctypes.byref(params) if params else None), "hc_create")
    return h.value


def hc_table_bytes(capacity: int, params: HcParams | None = None) -> int:
    out = ctypes.c_uint64(0)
    _check(_lib.hc_table_bytes(capacity, ctypes.byref(params) if params else None, ctypes.byref(out)),
           "hc_table_bytes")
    return out.value


def hc_create_in(kind: int, slots, capacity: int, params: HcParams | None = None) -> int:
    """Table over caller-owned device memory ``slots`` (a tensor the caller keeps alive)."""
    h = ctypes.c_void_p()
    nbytes = slots.numel() * slots.element_size()
    _check(_lib.hc_create_in(ctypes.byref(h), kind, slots.data_ptr(), nbytes, capacity,
                             ctypes.byref(params) if params else None), "hc_create_in")
    return h.value


def hc_stats(h: int, stream=None) -> HcTableStats:
    out = HcTableStats()
    _check(_lib.hc_stats(h, ctypes.byref(out), _stream(stream)), "hc_stats")
    return out


def hc_default_bucket_params() -> HcBucketParams:
    p = HcBucketParams()
    _lib.hc_default_bucket_params(ctypes.byref(p))
    return p


def hc_create_bucket_list(key_capacity: int, params: HcParams | None = None,
                          bparams: HcBucketParams | None = None) -> int:
    h = ctypes.c_void_p()
    _check(_lib.hc_create_bucket_list(ctypes.byref(h), key_capacity, ctypes.byref(params) if params else None,
                                      ctypes.byref(bparams) if bparams else None), "hc_create_bucket_list")
    return h.value


def hc_bucket_usage(h: int, stream=None) -> HcBucketUsage:
    out = HcBucketUsage()
    _check(_lib.hc_bucket_usage(h, ctypes.byref(out), _stream(stream)), "hc_bucket_usage")
    return out


def hc_dump_buckets(h: int, pool, last, stream=None):
    _check(_lib.hc_dump_buckets(h, _u32t(pool, "pool"), _u32t(last, "last"), _stream(stream)), "hc_dump_buckets")


def hc_device_view(h: int, nbytes: int) -> ctypes.Array:
    """The table's device view (a hc::TableView, nbytes long) for kernels on the device-side API."""
    buf = (ctypes.c_ubyte * nbytes)()
    _check(_lib.hc_device_view(h, buf, nbytes), "hc_device_view")
    return buf


def _u64t(t, what, n=None):
    if t is not None and t.dtype == torch.int64:
        t = t.view(torch.uint64)
    return _dptr(t, torch.uint64, what, n)


def hc_insert64(h: int, keys, values, status=None, group: int = 0, stream=None):
    n = keys.numel()
    _check(_lib.hc_insert64(h, _u64t(keys, "keys"), _u64t(values, "values", n), n,
                            _dptr(status, torch.uint8, "status", n), group, _stream(stream)), "hc_insert64")


def hc_retrieve64(h: int, keys, values_out, found_out=None, group: int = 0, stream=None):
    n = keys.numel()
    _check(_lib.hc_retrieve64(h, _u64t(keys, "keys"), n, _u64t(values_out, "values_out", n),
                              _dptr(found_out, torch.uint8, "found_out", n), group, _stream(stream)), "hc_retrieve64")


def hc_erase64(h: int, keys, status=None, group: int = 0, stream=None):
    n = keys.numel()
    _check(_lib.hc_erase64(h, _u64t(keys, "keys"), n, _dptr(status, torch.uint8, "status", n), group,
                           _stream(stream)), "hc_erase64")


def hc_destroy(h: int):
    _check(_lib.hc_destroy(h), "hc_destroy")


def hc_clear(h: int, stream=None):
    _check(_lib.hc_clear(h, _stream(stream)), "hc_clear")


def hc_insert(h: int, keys, values=None, status=None, group: int = 0, stream=None):
    n = keys.numel()
    _check(_lib.hc_insert(h, _u32t(keys, "keys"), _u32t(values, "values", n), n,
                          _dptr(status, torch.uint8, "status", n), group, _stream(stream)), "hc_insert")


def hc_retrieve(h: int, keys, values_out=None, found_out=None, group: int = 0, stream=None):
    n = keys.numel()
    _check(_lib.hc_retrieve(h, _u32t(keys, "keys"), n, _u32t(values_out, "values_out", n),
                            _dptr(found_out, torch.uint8, "found_out", n), group, _stream(stream)), "hc_retrieve")


def hc_erase(h: int, keys, status=None, group: int = 0, stream=None):
    n = keys.numel()
    _check(_lib.hc_erase(h, _u32t(keys, "keys"), n, _dptr(status, torch.uint8, "status", n), group,
                         _stream(stream)), "hc_erase")


def hc_count_values(h: int, keys, offsets, counts=None, want_total: bool = False, group: int = 0,
                    stream=None):
    n = keys.numel()
    tot = ctypes.c_uint64(0)
    _check(_lib.hc_count_values(h, _u32t(keys, "keys"), n, _u32t(counts, "counts", n),
                                _dptr(offsets.view(torch.uint64) if offsets.dtype == torch.int64 else offsets,
                                      torch.uint64, "offsets", n + 1),
                                ctypes.byref(tot) if want_total else None, group, _stream(stream)),
           "hc_count_values")
    return int(tot.value) if want_total else None


def hc_count_values_noalloc(h: int, keys, offsets, counts=None, want_total: bool = False, group: int = 0,
                            stream=None):
    n = keys.numel()
    tot = ctypes.c_uint64(0)
    _check(_lib.hc_count_values_noalloc(h, _u32t(keys, "keys"), n, _u32t(counts, "counts", n),
                                        _dptr(offsets.view(torch.uint64) if offsets.dtype == torch.int64 else offsets,
                                              torch.uint64, "offsets", n + 1),
                                        ctypes.byref(tot) if want_total else None, group, _stream(stream)),
           "hc_count_values_noalloc")
    return int(tot.value) if want_total else None


def hc_retrieve_all(h: int, keys, offsets, values_out, group: int = 0, stream=None):
    n = keys.numel()
    off = offsets.view(torch.uint64) if offsets.dtype == torch.int64 else offsets
    _check(_lib.hc_retrieve_all(h, _u32t(keys, "keys"), n, _dptr(off, torch.uint64, "offsets", n + 1),
                                _u32t(values_out, "values_out"), group, _stream(stream)), "hc_retrieve_all")


def hc_insert_grouped(h: int, keys, values=None, stream=None):
    n = keys.numel()
    _check(_lib.hc_insert_grouped(h, _u32t(keys, "keys"), _u32t(values, "values", n), n, _stream(stream)),
           "hc_insert_grouped")


def hc_size(h: int, stream=None) -> int:
    out = ctypes.c_uint64(0)
    _check(_lib.hc_size(h, ctypes.byref(out), _stream(stream)), "hc_size")
    return int(out.value)


def hc_load_factor(h: int, stream=None) -> float:
    out = ctypes.c_double(0)
    _check(_lib.hc_load_factor(h, ctypes.byref(out), _stream(stream)), "hc_load_factor")
    return float(out.value)


def hc_capacity(h: int) -> int:
    out = ctypes.c_uint64(0)
    _check(_lib.hc_capacity(h, ctypes.byref(out)), "hc_capacity")
    return int(out.value)


def hc_info(h: int) -> HcTableInfo:
    out = HcTableInfo()
    _check(_lib.hc_info(h, ctypes.byref(out)), "hc_info")
    return out


def slot_words(h: int) -> int:
    """uint64 words of a table's slot array: C, 2C for 64-bit tables, C/2 for sets."""
    info = hc_info(h)
    return {SINGLE_VALUE_64: 2 * info.capacity, SINGLE_VALUE_64_SOA: 2 * info.capacity,
            HASH_SET: info.capacity // 2}.get(info.kind, info.capacity)


def hc_dump_slots(h: int, dst, stream=None):
    _check(_lib.hc_dump_slots(h, _dptr(dst, torch.uint64, "dst", slot_words(h)), _stream(stream)),
           "hc_dump_slots")


def _ops_array(ops):
    arr = (HcBatchOp * max(1, len(ops)))()
    for j, o in enumerate(ops):
        arr[j] = o
    return arr


def hc_batch_op(table, op: int, keys, values=None, values_out=None, flags=None, group: int = 0) -> HcBatchOp:
    """One batched operation; ``table`` is a handle or a ``Table``.  Tensors must outlive the plan."""
    h = table.handle if isinstance(table, Table) else table
    n = keys.numel()
    return HcBatchOp(h, op, group, _u32t(keys, "keys"), _u32t(values, "values", n),
                     _u32t(values_out, "values_out", n), _dptr(flags, torch.uint8, "flags", n), n)


HC_BATCH_ONE_LAUNCH = 1


def hc_batch_create(ops) -> int:
    h = ctypes.c_void_p()
    _check(_lib.hc_batch_create(ctypes.byref(h), _ops_array(ops), len(ops)), "hc_batch_create")
    return h.value


def hc_batch_create_flags(ops, flags: int) -> int:
    h = ctypes.c_void_p()
    _check(_lib.hc_batch_create_flags(ctypes.byref(h), _ops_array(ops), len(ops), flags), "hc_batch_create_flags")
    return h.value


def hc_batch_abandoned_waits(batch: int) -> int:
    c = ctypes.c_uint64(0)
    _check(_lib.hc_batch_abandoned_waits(batch, ctypes.byref(c)), "hc_batch_abandoned_waits")
    return int(c.value)


def hc_batch_launch(batch: int, stream=None):
    _check(_lib.hc_batch_launch(batch, _stream(stream)), "hc_batch_launch")


def hc_batch_info(batch: int):
    ph, la = ctypes.c_uint32(0), ctypes.c_uint32(0)
    _check(_lib.hc_batch_info(batch, ctypes.byref(ph), ctypes.byref(la)), "hc_batch_info")
    return int(ph.value), int(la.value)


def hc_batch_destroy(batch: int):
    _check(_lib.hc_batch_destroy(batch), "hc_batch_destroy")


def hc_batch_run(ops, stream=None):
    _check(_lib.hc_batch_run(_ops_array(ops), len(ops), _stream(stream)), "hc_batch_run")


def hc_batch_capture(batch: int) -> int:
    g = ctypes.c_void_p()
    _check(_lib.hc_batch_capture(batch, ctypes.byref(g)), "hc_batch_capture")
    return g.value


def hc_graph_launch(graph: int, stream=None):
    _check(_lib.hc_graph_launch(graph, _stream(stream)), "hc_graph_launch")


def hc_graph_destroy(graph: int):
    _check(_lib.hc_graph_destroy(graph), "hc_graph_destroy")


class Batch:
    """A launch plan over many tables; keeps the tensors of its operations alive."""

    def __init__(self, ops_with_tensors, one_launch: bool = False):
        # ops_with_tensors: list of (HcBatchOp, [tensors...]); one_launch: every phase in one
        # gated launch (HC_BATCH_ONE_LAUNCH)
        self._keep = [t for _, ts in ops_with_tensors for t in ts]
        self.handle = hc_batch_create_flags([o for o, _ in ops_with_tensors],
                                            HC_BATCH_ONE_LAUNCH if one_launch else 0)
        self.phases, self.launches = hc_batch_info(self.handle)
        self.graph = None

    def abandoned_waits(self) -> int:
        return hc_batch_abandoned_waits(self.handle)

    def launch(self, stream=None):
        hc_batch_launch(self.handle, stream)

    def capture(self):
        if self.graph is None:
            self.graph = hc_batch_capture(self.handle)
        return self.graph

    def replay(self, stream=None):
        hc_graph_launch(self.capture(), stream)

    def close(self):
        if getattr(self, "graph", None):
            hc_graph_destroy(self.graph)
            self.graph = None
        if getattr(self, "handle", None):
            hc_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _hptr(t, dtype, what, n=None):
    """Host pointer of a contiguous CPU tensor (pinned for asynchronous copies) or None."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.is_cuda:
        raise TypeError(f"{what} must be a CPU tensor")
    if t.dtype == torch.int32 and dtype == torch.uint32:
        t = t.view(torch.uint32)
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous {dtype} tensor")
    if n is not None and t.numel() < n:
        raise ValueError(f"{what} has {t.numel()} elements, needs {n}")
    return t.data_ptr()


def hc_default_server_params() -> HcServerParams:
    p = HcServerParams()
    _lib.hc_default_server_params(ctypes.byref(p))
    return p


def hc_server_create(params: HcServerParams | None = None) -> int:
    h = ctypes.c_void_p()
    _check(_lib.hc_server_create(ctypes.byref(h), ctypes.byref(params) if params else None), "hc_server_create")
    return h.value


def hc_request(table, op: int, keys, values=None, values_out=None, flags=None, group: int = 0) -> HcRequest:
    h = table.handle if isinstance(table, Table) else table
    n = keys.numel()
    return HcRequest(h, op, group, _hptr(keys, torch.uint32, "keys"), _hptr(values, torch.uint32, "values", n),
                     _hptr(values_out, torch.uint32, "values_out", n), _hptr(flags, torch.uint8, "flags", n), n)


def hc_server_submit(server: int, req: HcRequest) -> int:
    t = ctypes.c_uint64(0)
    _check(_lib.hc_server_submit(server, ctypes.byref(req), ctypes.byref(t)), "hc_server_submit")
    return int(t.value)


def hc_server_query(server: int, ticket: int):
    done, lat = ctypes.c_int(0), ctypes.c_double(0)
    _check(_lib.hc_server_query(server, ticket, ctypes.byref(done), ctypes.byref(lat)), "hc_server_query")
    return bool(done.value), float(lat.value)


def hc_server_wait(server: int, ticket: int):
    _check(_lib.hc_server_wait(server, ticket), "hc_server_wait")


def hc_server_drain(server: int):
    _check(_lib.hc_server_drain(server), "hc_server_drain")


def hc_server_stats(server: int) -> dict:
    c = HcServerCounts()
    _check(_lib.hc_server_stats(server, ctypes.byref(c)), "hc_server_stats")
    return {k: int(getattr(c, k)) for k, _ in HcServerCounts._fields_}


def hc_server_destroy(server: int):
    _check(_lib.hc_server_destroy(server), "hc_server_destroy")


class Server:
    """Continuous-batching server; keeps each request's host tensors alive until it completes."""

    def __init__(self, staging_bytes=1 << 30, max_group_ops=1 << 22, max_group_requests=1024, streams=3, serial=False):
        p = hc_default_server_params()
        p.staging_bytes, p.max_group_ops = staging_bytes, max_group_ops
        p.max_group_requests, p.streams, p.serial = max_group_requests, streams, int(serial)
        self.handle = hc_server_create(p)
        self._keep = {}

    def submit(self, table, op, keys, values=None, values_out=None, flags=None, group=0) -> int:
        t = hc_server_submit(self.handle, hc_request(table, op, keys, values, values_out, flags, group))
        self._keep[t] = (keys, values, values_out, flags)
        return t

    def query(self, ticket):
        return hc_server_query(self.handle, ticket)

    def wait(self, ticket):
        hc_server_wait(self.handle, ticket)

    def drain(self):
        hc_server_drain(self.handle)
        self._keep.clear()

    def stats(self):
        return hc_server_stats(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            hc_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- convenience wrapper ---------------------------------------------------------------

class Table:
    """A table handle with allocation of outputs.  ``kind``: 'single' | 'multi' | 'counting'."""

    def __init__(self, kind="single", capacity=1 << 20, scheme="double", window=16, group=4,
                 seed=None, device=None, slots=None, bucket=None):
        """``slots``: optional caller-owned uint8/uint64 device tensor holding the slot array
        (hc_create_in); the Table keeps a reference to it.  ``kind="bucket"``: a bucket list table
        for ``capacity`` keys; ``bucket`` = dict(pool_values=, s0=, smax=, growth=) overrides."""
        self.kind = KINDS[kind] if isinstance(kind, str) else int(kind)
        p = hc_default_params()
        p.scheme = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
        p.window, p.group = window, group
        if seed is not None:
            p.seed = seed & (2**64 - 1)
        if slots is not None:
            device = slots.device
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.slots = slots
        with torch.cuda.device(self.device):
            if self.kind == BUCKET_LIST:
                bp = hc_default_bucket_params()
                for key, val in (bucket or {}).items():
                    setattr(bp, key, val)
                self.handle = hc_create_bucket_list(capacity, p, bp)
                self.bucket = {"pool_values": bp.pool_values, "s0": bp.s0, "smax": bp.smax, "growth": bp.growth}
            else:
                self.handle = hc_create(self.kind, capacity, p) if slots is None else \
                    hc_create_in(self.kind, slots, capacity, p)
        info = hc_info(self.handle)
        self.capacity, self.windows, self.window = int(info.capacity), int(info.windows), int(info.window)
        self.scheme, self.seed, self.group = int(info.scheme), int(info.seed), int(info.group)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                hc_destroy(h)
            except Exception:
                pass
            self.handle = None

    def close(self):
        self.__del__()

    def clear(self, stream=None):
        hc_clear(self.handle, stream)

    def insert(self, keys, values=None, status=False, group=0, stream=None):
        st = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device) if status else None
        if self.kind in WIDE_KINDS:
            hc_insert64(self.handle, keys, values, st, group, stream)
        else:
            hc_insert(self.handle, keys, values, st, group, stream)
        return st

    def retrieve(self, keys, group=0, stream=None):
        """(values, found); a set returns (None, found)."""
        if self.kind == HASH_SET:
            found = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device)
            hc_retrieve(self.handle, keys, None, found, group, stream)
            return None, found
        wide = self.kind in WIDE_KINDS
        vals = torch.empty(keys.numel(), dtype=torch.uint64 if wide else torch.uint32, device=keys.device)
        found = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device)
        (hc_retrieve64 if wide else hc_retrieve)(self.handle, keys, vals, found, group, stream)
        return vals, found

    def erase(self, keys, status=False, group=0, stream=None):
        st = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device) if status else None
        (hc_erase64 if self.kind in WIDE_KINDS else hc_erase)(self.handle, keys, st, group, stream)
        return st

    def count_values(self, keys, group=0, stream=None):
        counts = torch.empty(keys.numel(), dtype=torch.uint32, device=keys.device)
        offsets = torch.empty(keys.numel() + 1, dtype=torch.uint64, device=keys.device)
        total = hc_count_values(self.handle, keys, offsets, counts, True, group, stream)
        return counts, offsets, total

    def retrieve_all(self, keys, group=0, stream=None):
        """Two passes (count + prefix sum, then write): returns (offsets, values)."""
        _, offsets, total = self.count_values(keys, group, stream)
        vals = torch.empty(max(total, 1), dtype=torch.uint32, device=keys.device)
        hc_retrieve_all(self.handle, keys, offsets, vals, group, stream)
        return offsets, vals[:total]

    def size(self, stream=None) -> int:
        return hc_size(self.handle, stream)

    def load_factor(self, stream=None) -> float:
        return hc_load_factor(self.handle, stream)

    def bucket_usage(self, stream=None) -> dict:
        u = hc_bucket_usage(self.handle, stream)
        return {"values": u.values, "pool_used": u.pool_used, "pool_words": u.pool_words, "smax": u.smax}

    def dump_buckets(self, stream=None):
        u = hc_bucket_usage(self.handle, stream)
        pool = torch.empty(u.pool_words, dtype=torch.uint32, device=self.device)
        last = torch.empty(self.capacity, dtype=torch.uint32, device=self.device)
        hc_dump_buckets(self.handle, pool, last, stream)
        return pool, last

    def stats(self, stream=None) -> dict:
        st = hc_stats(self.handle, stream)
        return {"live": st.live, "tombstones": st.tombstones, "empty": st.empty, "max_probe": st.max_probe,
                "probe_sum": st.probe_sum, "probe_hist": list(st.probe_hist), "cas_fails": st.cas_fails}

    def dump_slots(self, stream=None):
        """The slot array: C uint64 words (2C for 64-bit tables: pairs, or C keys then C values in the
        structure-of-arrays layout); a set's C uint32 keys."""
        out = torch.empty(slot_words(self.handle), dtype=torch.uint64, device=self.device)
        hc_dump_slots(self.handle, out, stream)
        return out.view(torch.uint32) if self.kind == HASH_SET else out


# ---- Bloom filter ------------------------------------------------------------

def hc_default_bloom_params() -> HcBloomParams:
    p = HcBloomParams()
    _lib.hc_default_bloom_params(ctypes.byref(p))
    return p


def hc_bloom_create(bits: int, params: HcBloomParams | None = None) -> int:
    h = ctypes.c_void_p()
    _check(_lib.hc_bloom_create(ctypes.byref(h), bits, ctypes.byref(params) if params else None), "hc_bloom_create")
    return h.value


def hc_bloom_destroy(h: int):
    _check(_lib.hc_bloom_destroy(h), "hc_bloom_destroy")


def hc_bloom_clear(h: int, stream=None):
    _check(_lib.hc_bloom_clear(h, _stream(stream)), "hc_bloom_clear")


def hc_bloom_insert(h: int, keys, group: int = 0, stream=None):
    _check(_lib.hc_bloom_insert(h, _u32t(keys, "keys"), keys.numel(), group, _stream(stream)), "hc_bloom_insert")


def hc_bloom_contains(h: int, keys, found_out, group: int = 0, stream=None):
    n = keys.numel()
    _check(_lib.hc_bloom_contains(h, _u32t(keys, "keys"), n, _dptr(found_out, torch.uint8, "found_out", n), group,
                                  _stream(stream)), "hc_bloom_contains")


def hc_bloom_info(h: int) -> HcBloomInfo:
    out = HcBloomInfo()
    _check(_lib.hc_bloom_info(h, ctypes.byref(out)), "hc_bloom_info")
    return out


def hc_bloom_dump(h: int, dst, stream=None):
    info = hc_bloom_info(h)
    _check(_lib.hc_bloom_dump(h, _dptr(dst, torch.uint32, "dst", info.blocks * info.block_words), _stream(stream)),
           "hc_bloom_dump")


class Bloom:
    """Blocked Bloom filter handle (see ``hc_bloom_create``)."""

    def __init__(self, bits, block_words=16, group=0, seed=None, device=None):
        p = hc_default_bloom_params()
        p.block_words, p.group = block_words, group
        if seed is not None:
            p.seed = seed & (2**64 - 1)
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        with torch.cuda.device(self.device):
            self.handle = hc_bloom_create(bits, p)
        info = hc_bloom_info(self.handle)
        self.blocks, self.block_words, self.group, self.seed = (
            int(info.blocks), int(info.block_words), int(info.group), int(info.seed))

    def close(self):
        if getattr(self, "handle", None):
            with torch.cuda.device(self.device):
                hc_bloom_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def clear(self, stream=None):
        hc_bloom_clear(self.handle, stream)

    def insert(self, keys, group=0, stream=None):
        hc_bloom_insert(self.handle, keys, group, stream)

    def contains(self, keys, group=0, stream=None):
        found = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device)
        hc_bloom_contains(self.handle, keys, found, group, stream)
        return found

    def dump(self, stream=None):
        out = torch.empty(self.blocks * self.block_words, dtype=torch.uint32, device=self.device)
        hc_bloom_dump(self.handle, out, stream)
        return out


# ---- bandwidth diagnostics ------------------------------------------------------

def hc_diag_copy(dst, src, stream=None):
    """Copy src into dst (same byte size, a multiple of 16) with the library's streaming kernel."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst is smaller than src")
    _check(_lib.hc_diag_copy(dst.data_ptr(), src.data_ptr(), nbytes, _stream(stream)), "hc_diag_copy")


def hc_diag_read(src, sink, stream=None):
    """Read all of src (a multiple of 16 bytes) with the library's streaming kernel."""
    _check(_lib.hc_diag_read(src.data_ptr(), src.numel() * src.element_size(), _dptr(sink, torch.uint32, "sink", 1),
                             _stream(stream)), "hc_diag_read")


def hc_diag_atomic(region, cas: bool, n_ops: int, sink, seed: int = 1, stream=None):
    """n_ops random 8-byte atomics (OR, or CAS of 0) inside the device tensor ``region``."""
    _check(_lib.hc_diag_atomic(region.data_ptr(), region.numel() * region.element_size(), int(cas), n_ops, seed,
                               _dptr(sink, torch.uint32, "sink", 1), _stream(stream)), "hc_diag_atomic")


def hc_diag_gather(base_ptr: int, nbytes: int, line_bytes: int, n_lines: int, sink, seed: int = 1, stream=None):
    """Read n_lines random lines of line_bytes inside [base_ptr, base_ptr + nbytes) (device memory)."""
    _check(_lib.hc_diag_gather(base_ptr, nbytes, line_bytes, n_lines, seed, _dptr(sink, torch.uint32, "sink", 1),
                               _stream(stream)), "hc_diag_gather")
