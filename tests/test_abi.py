"""The C ABI library loads on a CPU-only host and exports every symbol include/hc.h declares."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hc.h")
LIB = os.path.join(ROOT, "paper_2009_07914_amd", "libhc.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hc_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["hc_create", "hc_destroy", "hc_clear", "hc_insert", "hc_retrieve", "hc_erase",
                 "hc_count_values", "hc_retrieve_all", "hc_size", "hc_load_factor", "hc_capacity"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (hc_[a-z_]+)$", out, flags=re.M))
    assert set(_declared()) <= exported


def test_host_side_argument_errors_need_no_gpu(lib):
    # argument validation happens before any device call
    lib.hc_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p]
    lib.hc_last_error.restype = ctypes.c_char_p
    lib.hc_error_string.restype = ctypes.c_char_p
    h = ctypes.c_void_p()
    assert lib.hc_create(ctypes.byref(h), 7, 1024, None) == 1  # bad kind -> HC_E_ARG
    assert b"kind" in lib.hc_last_error()
    assert lib.hc_create(ctypes.byref(h), 0, 0, None) == 1     # capacity 0
    assert lib.hc_create(None, 0, 1024, None) == 1
    assert lib.hc_insert(None, None, None, 0, None, 0, None) == 1  # NULL handle
    assert lib.hc_error_string(2) == b"device allocation failed"


def test_no_oracle_in_product_path():
    # the product package never imports or links the oracle
    pkg = os.path.join(ROOT, "paper_2009_07914_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f), errors="replace").read()
                assert "import oracle" not in src and "from oracle" not in src and "liboracle" not in src, f
    deps = subprocess.run(["objdump", "-p", LIB], capture_output=True, text=True).stdout
    assert "liboracle" not in deps


class _Params(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_uint32), ("window", ctypes.c_uint32), ("group", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("seed", ctypes.c_uint64)]


def test_table_bytes_and_create_in_arguments(lib):
    import oracle
    lib.hc_default_params.argtypes = [ctypes.POINTER(_Params)]
    lib.hc_table_bytes.argtypes = [ctypes.c_uint64, ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_uint64)]
    lib.hc_create_in.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint64,
                                 ctypes.c_uint64, ctypes.POINTER(_Params)]
    p = _Params()
    lib.hc_default_params(ctypes.byref(p))
    out = ctypes.c_uint64()
    for scheme in (0, 1, 2):
        for w in (8, 16, 32, 64):
            for cap in (1, 1000, 4096, 100003):
                p.scheme, p.window = scheme, w
                assert lib.hc_table_bytes(cap, ctypes.byref(p), ctypes.byref(out)) == 0
                assert out.value == 8 * w * oracle.round_windows(cap, w, scheme)
    p.scheme, p.window = 2, 16
    lib.hc_table_bytes(1000, ctypes.byref(p), ctypes.byref(out))
    h = ctypes.c_void_p()
    assert lib.hc_create_in(ctypes.byref(h), 0, None, 1 << 20, 1000, ctypes.byref(p)) == 1         # NULL array
    assert lib.hc_create_in(ctypes.byref(h), 0, 0x10010, 1 << 20, 1000, ctypes.byref(p)) == 1      # misaligned
    assert lib.hc_create_in(ctypes.byref(h), 0, 0x10000, out.value - 8, 1000, ctypes.byref(p)) == 1  # too small
    assert h.value is None


class _BucketParams(ctypes.Structure):
    _fields_ = [("pool_values", ctypes.c_uint64), ("s0", ctypes.c_uint32), ("smax", ctypes.c_uint32),
                ("growth", ctypes.c_double)]


def test_bucket_list_arguments(lib):
    lib.hc_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p]
    lib.hc_create_bucket_list.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint64, ctypes.c_void_p,
                                          ctypes.POINTER(_BucketParams)]
    lib.hc_default_bucket_params.argtypes = [ctypes.POINTER(_BucketParams)]
    h = ctypes.c_void_p()
    assert lib.hc_create(ctypes.byref(h), 3, 1024, None) == 1  # bucket lists have their own constructor
    bp = _BucketParams()
    lib.hc_default_bucket_params(ctypes.byref(bp))
    assert (bp.s0, bp.smax, bp.growth, bp.pool_values) == (1, 1 << 16, 2.0, 0)
    for s0, smax, growth in [(0, 8, 2.0), (9, 8, 2.0), (1, 1 << 25, 2.0), (1, 8, 0.5), (1, 8, 100.0),
                             (1, 1 << 20, 1.0)]:  # the last never reaches smax: ramp too long
        bad = _BucketParams(0, s0, smax, growth)
        assert lib.hc_create_bucket_list(ctypes.byref(h), 1024, None, ctypes.byref(bad)) == 1, (s0, smax, growth)


class _BloomParams(ctypes.Structure):
    _fields_ = [("block_words", ctypes.c_uint32), ("group", ctypes.c_uint32), ("seed", ctypes.c_uint64)]


def test_bloom_and_diagnostic_arguments(lib):
    # every check below happens before any device call
    lib.hc_bloom_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint64, ctypes.POINTER(_BloomParams)]
    lib.hc_default_bloom_params.argtypes = [ctypes.POINTER(_BloomParams)]
    lib.hc_bloom_info.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.hc_diag_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
    lib.hc_diag_gather.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32,
                                   ctypes.c_void_p, ctypes.c_void_p]
    lib.hc_diag_atomic.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32,
                                   ctypes.c_void_p, ctypes.c_void_p]
    p = _BloomParams()
    lib.hc_default_bloom_params(ctypes.byref(p))
    assert (p.block_words, p.group) == (16, 0)
    h = ctypes.c_void_p()
    for words, group in [(12, 0), (16, 3), (8, 16), (64, 0)]:
        bad = _BloomParams(words, group, 1)
        assert lib.hc_bloom_create(ctypes.byref(h), 1 << 20, ctypes.byref(bad)) == 1, (words, group)
    assert lib.hc_bloom_create(ctypes.byref(h), 0, ctypes.byref(p)) == 1          # no bits
    assert lib.hc_bloom_create(ctypes.byref(h), 1 << 50, ctypes.byref(p)) == 1    # more than 2^32 blocks
    assert lib.hc_bloom_create(None, 1 << 20, ctypes.byref(p)) == 1
    assert h.value is None
    assert lib.hc_bloom_info(None, None) == 1
    fake, sink = 0x100000, 0x200000  # never dereferenced: the checks fail first
    assert lib.hc_diag_copy(None, fake, 64, None) == 1
    assert lib.hc_diag_copy(fake, fake, 17, None) == 1
    assert lib.hc_diag_gather(fake, 1 << 20, 48, 16, 1, sink, None) == 1           # line size
    assert lib.hc_diag_gather(fake + 4, 1 << 20, 64, 16, 1, sink, None) == 1       # alignment
    assert lib.hc_diag_atomic(fake + 4, 1 << 20, 1, 16, 1, sink, None) == 1        # alignment
    assert lib.hc_diag_atomic(fake, 4, 0, 16, 1, sink, None) == 1                  # no whole word
