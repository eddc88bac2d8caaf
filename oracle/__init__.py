"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP library and its Python binding
never import it, and it shares no code with them.

The oracle is a plain single-threaded C++ implementation (``oracle.cpp``) of
what the hash tables of WarpCore (arXiv 2009.07914) compute, applied op by op
in batch order over ``std::unordered_map``:

* single-value table: bounded map K -> V, upsert, duplicate warning
  (Sec. IV-B3), tombstone deletion (Sec. IV-B5);
* multi-value table: bounded multimap, count pass + exclusive prefix sum into
  n+1 offsets + value pass (Sec. IV-B4);
* counting table: K -> occurrences mod 2^32 (Sec. IV, CountingHashTable).

It also carries an independent re-derivation of the probe geometry (Sec. II
probing schemes, Sec. IV-B2 windows) with a layout checker for dumped GPU slot
arrays and a sequential scalar probing model.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

SINGLE, MULTI, COUNT = 0, 1, 2
LINEAR, QUADRATIC, DOUBLE = 0, 1, 2
ST_OK, ST_DUPLICATE, ST_FULL, ST_INVALID_KEY, ST_NOT_FOUND = 0, 1, 2, 3, 4
LAYOUT_ERRORS = {0: "ok", 1: "bad empty/tombstone encoding", 2: "key stored past an empty position",
                 3: "key stored twice", 4: "key stored off its sequence"}


def build(force: bool = True) -> str:
    """Compile oracle.cpp into liboracle.so (g++, -O2, single-threaded)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        u64, u32, p, i = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int
        lib.orc_create.argtypes = [i, u64]
        lib.orc_create.restype = p
        lib.orc_destroy.argtypes = [p]
        lib.orc_clear.argtypes = [p]
        lib.orc_size.argtypes = [p]
        lib.orc_size.restype = u64
        lib.orc_num_keys.argtypes = [p]
        lib.orc_num_keys.restype = u64
        lib.orc_insert.argtypes = [p, p, p, u64, p]
        lib.orc_retrieve.argtypes = [p, p, u64, p, p]
        lib.orc_erase.argtypes = [p, p, u64, p]
        lib.orc_count_values.argtypes = [p, p, u64, p, p]
        lib.orc_retrieve_all.argtypes = [p, p, u64, p, p]
        lib.orc_dump.argtypes = [p, p, p, u64]
        lib.orc_dump.restype = u64
        lib.orc_fmix32.argtypes = [u32]
        lib.orc_fmix32.restype = u32
        lib.orc_round_windows.argtypes = [u64, u32, i]
        lib.orc_round_windows.restype = u64
        lib.orc_window_at.argtypes = [u32, u64, u64, i, u64]
        lib.orc_window_at.restype = u64
        lib.orc_window_sequence.argtypes = [u32, u64, u64, i, u64, p]
        lib.orc_check_layout.argtypes = [p, u64, u32, i, u64, i, p]
        lib.orc_check_layout.restype = i
        lib.orc_model_insert.argtypes = [p, u64, u32, i, u64, p, p, u64, p]
        lib.orc_model_insert.restype = u64
        lib.orc_model_lookup_windows.argtypes = [p, u64, u32, i, u64, p, u64, p]
        lib.orc64_create.argtypes = [u64]
        lib.orc64_create.restype = p
        lib.orc64_destroy.argtypes = [p]
        lib.orc64_size.argtypes = [p]
        lib.orc64_size.restype = u64
        lib.orc64_insert.argtypes = [p, p, p, u64, p]
        lib.orc64_retrieve.argtypes = [p, p, u64, p, p]
        lib.orc64_erase.argtypes = [p, p, u64, p]
        lib.orc_fmix64.argtypes = [u64]
        lib.orc_fmix64.restype = u64
        lib.orc64_window_at.argtypes = [u64, u64, u64, i, u64]
        lib.orc64_window_at.restype = u64
        lib.orc64_check_layout.argtypes = [p, u64, u32, i, u64, p]
        lib.orc_bloom_insert.argtypes = [p, u64, u32, u64, p, u64]
        lib.orc_bloom_insert.restype = None
        lib.orc_bloom_query.argtypes = [p, u64, u32, u64, p, u64, p]
        lib.orc_bloom_query.restype = None
        lib.orc_bloom_positions.argtypes = [u32, u64, u32, u64, p, p]
        lib.orc_bloom_blocks.argtypes = [p, u64, u64, u64, p]
        lib.orc_bloom_blocks.restype = None
        lib.orc_bloom_positions.restype = None
        lib.orc64_check_layout.restype = i
        _lib = lib
    return _lib


def _u32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint32)


def _ptr(a):
    return None if a is None else a.ctypes.data


class OracleTable:
    """Bounded map / multimap / counter with the hash tables' observable semantics."""

    def __init__(self, kind: int, capacity: int):
        self._lib = _load()
        self.kind = kind
        self.capacity = int(capacity)
        self._h = self._lib.orc_create(kind, self.capacity)
        if not self._h:
            raise ValueError("bad table kind")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    def clear(self):
        self._lib.orc_clear(self._h)

    def size(self) -> int:
        return int(self._lib.orc_size(self._h))

    def num_keys(self) -> int:
        return int(self._lib.orc_num_keys(self._h))

    def insert(self, keys, values=None) -> np.ndarray:
        keys = _u32(keys)
        vals = None if values is None else _u32(values)
        if vals is None and self.kind != COUNT:
            raise ValueError("values required")
        status = np.empty(keys.size, dtype=np.uint8)
        self._lib.orc_insert(self._h, _ptr(keys), _ptr(vals), keys.size, _ptr(status))
        return status

    def retrieve(self, keys):
        keys = _u32(keys)
        out = np.empty(keys.size, dtype=np.uint32)
        found = np.empty(keys.size, dtype=np.uint8)
        self._lib.orc_retrieve(self._h, _ptr(keys), keys.size, _ptr(out), _ptr(found))
        return out, found

    def erase(self, keys) -> np.ndarray:
        keys = _u32(keys)
        status = np.empty(keys.size, dtype=np.uint8)
        self._lib.orc_erase(self._h, _ptr(keys), keys.size, _ptr(status))
        return status

    def count_values(self, keys):
        keys = _u32(keys)
        counts = np.empty(keys.size, dtype=np.uint32)
        offsets = np.empty(keys.size + 1, dtype=np.uint64)
        self._lib.orc_count_values(self._h, _ptr(keys), keys.size, _ptr(counts), _ptr(offsets))
        return counts, offsets

    def retrieve_all(self, keys, offsets=None):
        """Returns (offsets, values); each segment sorted ascending."""
        keys = _u32(keys)
        if offsets is None:
            _, offsets = self.count_values(keys)
        out = np.zeros(int(offsets[-1]), dtype=np.uint32)
        self._lib.orc_retrieve_all(self._h, _ptr(keys), keys.size, _ptr(offsets), _ptr(out))
        return offsets, out

    def dump(self):
        n = self.size()
        k = np.empty(n, dtype=np.uint32)
        v = np.empty(n, dtype=np.uint32)
        m = self._lib.orc_dump(self._h, _ptr(k), _ptr(v), n)
        return k[:m], v[:m]


# ---- probe geometry (independent re-derivation) ---------------------------------

def fmix32(x: int) -> int:
    return int(_load().orc_fmix32(x & 0xFFFFFFFF))


def round_windows(capacity: int, window: int, scheme: int) -> int:
    return int(_load().orc_round_windows(capacity, window, scheme))


def window_at(key: int, l: int, P: int, scheme: int, seed: int) -> int:
    return int(_load().orc_window_at(key, l, P, scheme, seed & (2**64 - 1)))


def window_sequence(key: int, count: int, P: int, scheme: int, seed: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _load().orc_window_sequence(key, count, P, scheme, seed & (2**64 - 1), _ptr(out))
    return out


def check_layout(slots: np.ndarray, P: int, W: int, scheme: int, seed: int, kind: int):
    """Returns (error_code, stats dict).  error_code 0 means every invariant holds."""
    slots = np.ascontiguousarray(slots, dtype=np.uint64)
    assert slots.size == P * W
    st = np.zeros(5, dtype=np.uint64)
    rc = _load().orc_check_layout(_ptr(slots), P, W, scheme, seed & (2**64 - 1), kind, _ptr(st))
    return int(rc), {"live": int(st[0]), "tombstones": int(st[1]), "max_windows": int(st[2]),
                     "sum_windows": int(st[3]), "first_bad_slot": int(st[4])}


def model_insert(slots: np.ndarray, P: int, W: int, scheme: int, seed: int, keys, values):
    """Sequential scalar probing model; mutates ``slots``; returns (failed, windows per insert)."""
    keys, values = _u32(keys), _u32(values)
    win = np.empty(keys.size, dtype=np.uint32)
    failed = _load().orc_model_insert(_ptr(slots), P, W, scheme, seed & (2**64 - 1), _ptr(keys),
                                      _ptr(values), keys.size, _ptr(win))
    return int(failed), win


def model_lookup_windows(slots: np.ndarray, P: int, W: int, scheme: int, seed: int, keys) -> np.ndarray:
    keys = _u32(keys)
    win = np.empty(keys.size, dtype=np.uint32)
    _load().orc_model_lookup_windows(_ptr(slots), P, W, scheme, seed & (2**64 - 1), _ptr(keys), keys.size,
                                     _ptr(win))
    return win


# ---- single-value table with 64-bit keys and values ----------------------------

class OracleTable64:
    """Bounded map uint64 -> uint64 with the single-value table's observable semantics."""

    def __init__(self, capacity: int):
        self._lib = _load()
        self.capacity = int(capacity)
        self._h = self._lib.orc64_create(self.capacity)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc64_destroy(h)
            self._h = None

    def size(self) -> int:
        return int(self._lib.orc64_size(self._h))

    def insert(self, keys, values) -> np.ndarray:
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        vals = np.ascontiguousarray(values, dtype=np.uint64)
        status = np.empty(keys.size, dtype=np.uint8)
        self._lib.orc64_insert(self._h, _ptr(keys), _ptr(vals), keys.size, _ptr(status))
        return status

    def retrieve(self, keys):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        out = np.empty(keys.size, dtype=np.uint64)
        found = np.empty(keys.size, dtype=np.uint8)
        self._lib.orc64_retrieve(self._h, _ptr(keys), keys.size, _ptr(out), _ptr(found))
        return out, found

    def erase(self, keys) -> np.ndarray:
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        status = np.empty(keys.size, dtype=np.uint8)
        self._lib.orc64_erase(self._h, _ptr(keys), keys.size, _ptr(status))
        return status


def fmix64(x: int) -> int:
    return int(_load().orc_fmix64(x & (2**64 - 1)))


def window_at64(key: int, l: int, P: int, scheme: int, seed: int) -> int:
    return int(_load().orc64_window_at(key & (2**64 - 1), l, P, scheme, seed & (2**64 - 1)))


def check_layout64(slots: np.ndarray, P: int, W: int, scheme: int, seed: int):
    """slots: 2 * P * W uint64 words (key, value per slot).  Returns (error_code, stats dict)."""
    slots = np.ascontiguousarray(slots, dtype=np.uint64)
    assert slots.size == 2 * P * W
    st = np.zeros(5, dtype=np.uint64)
    rc = _load().orc64_check_layout(_ptr(slots), P, W, scheme, seed & (2**64 - 1), _ptr(st))
    return int(rc), {"live": int(st[0]), "tombstones": int(st[1]), "max_windows": int(st[2]),
                     "sum_windows": int(st[3]), "first_bad_slot": int(st[4])}



# ---- Bloom filter (blocked) --------------------------------------------------

class OracleBloom:
    """Split-block Bloom filter: ``blocks`` blocks of ``words`` 32-bit words; each key sets one bit
    in every word of one block (k = words).  ``bits`` is the word array (blocks * words uint32)."""

    def __init__(self, blocks: int, words: int, seed: int):
        assert words in (8, 16, 32) and blocks >= 1
        self.blocks, self.words, self.seed = blocks, words, seed & (2**64 - 1)
        self.bits = np.zeros(blocks * words, dtype=np.uint32)

    def insert(self, keys):
        keys = _u32(keys)
        _load().orc_bloom_insert(_ptr(self.bits), self.blocks, self.words, self.seed, _ptr(keys), keys.size)

    def query(self, keys) -> np.ndarray:
        keys = _u32(keys)
        out = np.empty(keys.size, dtype=np.uint8)
        _load().orc_bloom_query(_ptr(self.bits), self.blocks, self.words, self.seed, _ptr(keys), keys.size,
                                _ptr(out))
        return out

    def blocks_of(self, keys) -> np.ndarray:
        """Block index of every key."""
        keys = _u32(keys)
        out = np.empty(keys.size, dtype=np.uint64)
        _load().orc_bloom_blocks(_ptr(keys), keys.size, self.blocks, self.seed, _ptr(out))
        return out

    def positions(self, key: int):
        """(block, bit of each word) of one key."""
        blk = np.zeros(1, dtype=np.uint64)
        bit = np.zeros(self.words, dtype=np.uint32)
        _load().orc_bloom_positions(key & 0xFFFFFFFF, self.blocks, self.words, self.seed, _ptr(blk), _ptr(bit))
        return int(blk[0]), bit
