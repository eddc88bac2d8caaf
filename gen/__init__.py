"""Seeded synthetic input generators (inputs only; no hash-table arithmetic).

Both sides of every parity check draw their inputs from here: the HIP path's
tests and benchmark, and the CPU oracle's tests.  Nothing in this package
hashes, probes or encodes table slots.  See ``gen.c`` for the published
definitions (SplitMix64, cycle-walked Feistel bijection, inverse-CDF Zipf).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libgen.so")

KEY_EMPTY = 0
KEY_TOMBSTONE = 0xFFFFFFFF
MAX_KEY_INDEX = 0xFFFFFFFE


def build(force: bool = True) -> str:
    """Compile gen.c into libgen.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        u64, u32, p = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
        lib.gen_keys.argtypes = [u64, u64, u64, p]
        lib.gen_keys.restype = ctypes.c_int
        lib.gen_values.argtypes = [u64, u64, p]
        lib.gen_uniform.argtypes = [u64, u32, u32, u64, p]
        lib.gen_permutation.argtypes = [u64, u64, p]
        lib.gen_gather_u32.argtypes = [p, p, u64, p]
        lib.gen_zipf_ranks.argtypes = [u64, u32, ctypes.c_double, u64, p]
        lib.gen_zipf_ranks.restype = ctypes.c_int
        lib.gen_zipf_pmf.argtypes = [u32, ctypes.c_double, p]
        lib.gen_splitmix64_at.argtypes = [u64, u64]
        lib.gen_splitmix64_at.restype = u64
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def splitmix64_at(seed: int, i: int) -> int:
    """i-th (0-based) output of the SplitMix64 stream seeded with ``seed``."""
    return int(_load().gen_splitmix64_at(seed & (2**64 - 1), i))


def keys(seed: int, start: int, count: int) -> np.ndarray:
    """Distinct keys perm_seed(start .. start+count-1), never 0 or 2^32-1."""
    out = np.empty(count, dtype=np.uint32)
    if count and _load().gen_keys(seed & (2**64 - 1), start, count, _ptr(out)) != 0:
        raise ValueError("key index range must lie in [1, 2^32-2]")
    return out


def values(seed: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint32)
    if count:
        _load().gen_values(seed & (2**64 - 1), count, _ptr(out))
    return out


def uniform(seed: int, lo: int, hi: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint32)
    if count:
        _load().gen_uniform(seed & (2**64 - 1), lo, hi, count, _ptr(out))
    return out


def permutation(seed: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    if n:
        _load().gen_permutation(seed & (2**64 - 1), n, _ptr(out))
    return out


def shuffle(seed: int, a: np.ndarray) -> np.ndarray:
    """Return ``a`` reordered by the seeded bijection ``permutation(seed, len(a))``."""
    a = np.ascontiguousarray(a, dtype=np.uint32)
    idx = permutation(seed, a.size)
    out = np.empty_like(a)
    if a.size:
        _load().gen_gather_u32(_ptr(a), _ptr(idx), a.size, _ptr(out))
    return out


def zipf_ranks(seed: int, n_ranks: int, s: float, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint32)
    if count and _load().gen_zipf_ranks(seed & (2**64 - 1), n_ranks, s, count, _ptr(out)) != 0:
        raise MemoryError("zipf CDF table allocation failed")
    return out


def zipf_pmf(n_ranks: int, s: float) -> np.ndarray:
    out = np.empty(n_ranks, dtype=np.float64)
    _load().gen_zipf_pmf(n_ranks, s, _ptr(out))
    return out


from .workloads import *  # noqa: E402,F401,F403
