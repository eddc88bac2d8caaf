"""Workload recipes: the synthetic inputs of each benchmarked configuration.

Every array is a deterministic function of (recipe, sizes, seed).  The recipes
state shapes and distributions only; they never touch table arithmetic.
"""
from __future__ import annotations

import math

import numpy as np

from . import keys, permutation, shuffle, uniform, values, zipf_ranks, splitmix64_at

SEED_BASE = 0x20090791

__all__ = [
    "SEED_BASE", "single_value_workload", "multi_value_zipf_workload",
    "multi_value_uniform_r_workload", "batched_tables_spec", "derive_seed",
]


def derive_seed(seed: int, tag: int) -> int:
    """Independent sub-stream seed for component ``tag`` of a workload."""
    return splitmix64_at(seed, 0x1000 + tag)


def single_value_workload(capacity: int, load: float, seed: int, erase_frac: float = 0.1,
                          n_keys: int | None = None) -> dict:
    """Distinct uniform keys at a target load, with a 50/50 present/absent query mix.

    present = perm(1..n), absent = perm(n+1..2n) (same keyed bijection, disjoint index
    ranges, so the sets are distinct and disjoint); values are SplitMix64 words;
    queries = seeded shuffle of present ∪ absent; ``erase`` = the first
    floor(erase_frac * n) keys of an independent shuffle of the present keys.
    """
    n = int(math.floor(load * capacity)) if n_keys is None else int(n_keys)
    kseed = derive_seed(seed, 1)
    present = keys(kseed, 1, n)
    absent = keys(kseed, n + 1, n)
    vals = values(derive_seed(seed, 2), n)
    src = permutation(derive_seed(seed, 3), 2 * n)   # query j is (present ++ absent)[src[j]]
    both = np.concatenate([present, absent])
    queries = both[src.astype(np.int64)] if n else both
    del both
    n_erase = int(math.floor(erase_frac * n))
    erase = shuffle(derive_seed(seed, 4), present)[:n_erase].copy()
    return {"n": n, "keys": present, "values": vals, "absent": absent,
            "queries": queries, "query_src": src, "erase": erase}


def multi_value_zipf_workload(n_pairs: int, n_ranks: int, s: float, seed: int) -> dict:
    """k-mer-like keys with heavy duplication: key = perm(rank), rank ~ Zipf(s) on 1..n_ranks.

    Queries are every rank's key (perm(1..n_ranks)), shuffled, so the total
    number of stored values over all queries equals n_pairs.
    """
    kseed = derive_seed(seed, 1)
    ranks = zipf_ranks(derive_seed(seed, 5), n_ranks, s, n_pairs)
    universe = keys(kseed, 1, n_ranks)
    pair_keys = universe[ranks.astype(np.int64) - 1]
    vals = values(derive_seed(seed, 2), n_pairs)
    queries = shuffle(derive_seed(seed, 3), universe)
    return {"keys": pair_keys, "values": vals, "queries": queries, "universe": universe}


def multi_value_uniform_r_workload(n_pairs: int, r: int, seed: int) -> dict:
    """Average multiplicity r: keys uniform on 1..n/r; queries are 1..n (shuffled)."""
    hi = max(1, n_pairs // r)
    pair_keys = uniform(derive_seed(seed, 6), 1, hi, n_pairs)
    vals = values(derive_seed(seed, 2), n_pairs)
    queries = shuffle(derive_seed(seed, 3), np.arange(1, n_pairs + 1, dtype=np.uint32))
    return {"keys": pair_keys, "values": vals, "queries": queries}


def batched_tables_spec(n_tables: int, log2_lo: float, log2_hi: float, load_lo: float,
                        load_hi: float, window: int, seed: int) -> list[dict]:
    """Per-table capacity (log-uniform, rounded down to a multiple of ``window``) and load."""
    out = []
    for t in range(n_tables):
        u1 = (splitmix64_at(derive_seed(seed, 7), t) >> 11) / float(1 << 53)
        u2 = (splitmix64_at(derive_seed(seed, 8), t) >> 11) / float(1 << 53)
        cap = int(2.0 ** (log2_lo + (log2_hi - log2_lo) * u1))
        cap = max(window, cap - cap % window)
        out.append({"capacity": cap, "load": load_lo + (load_hi - load_lo) * u2,
                    "seed": derive_seed(seed, 0x100 + t)})
    return out
