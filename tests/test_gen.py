"""Input generators: distinctness, reserved words, disjointness, determinism, Zipf fit."""
import numpy as np
import pytest

import gen


def test_keys_distinct_and_never_reserved():
    k = gen.keys(123, 1, 1 << 22)
    assert np.unique(k).size == k.size
    assert not np.any(k == 0) and not np.any(k == 0xFFFFFFFF)


def test_present_absent_disjoint():
    w = gen.single_value_workload(1 << 16, 0.9, 7)
    assert np.intersect1d(w["keys"], w["absent"]).size == 0
    assert w["queries"].size == 2 * w["n"]
    assert np.array_equal(np.sort(w["queries"]), np.sort(np.concatenate([w["keys"], w["absent"]])))
    assert np.isin(w["erase"], w["keys"]).all() and np.unique(w["erase"]).size == w["erase"].size


def test_key_range_edges():
    top = gen.keys(9, 0xFFFFFFFE - 9, 10)
    assert np.unique(top).size == 10 and not np.any(top == 0xFFFFFFFF) and not np.any(top == 0)
    with pytest.raises(ValueError):
        gen.keys(9, 0xFFFFFFFE, 2)
    with pytest.raises(ValueError):
        gen.keys(9, 0, 1)


def test_bijection_on_a_small_full_domain_image():
    # keys of indices 1..2^20 under two seeds: distinct within each; different orders
    a, b = gen.keys(1, 1, 1 << 20), gen.keys(2, 1, 1 << 20)
    assert np.unique(a).size == a.size and np.unique(b).size == b.size
    assert not np.array_equal(a, b)


def test_deterministic():
    assert np.array_equal(gen.keys(5, 10, 1000), gen.keys(5, 10, 1000))
    assert np.array_equal(gen.values(5, 1000), gen.values(5, 1000))
    assert np.array_equal(gen.permutation(5, 1001), gen.permutation(5, 1001))


def test_permutation_is_bijection():
    for n in (1, 2, 3, 17, 1000, 65537):
        p = gen.permutation(11, n)
        assert np.array_equal(np.sort(p), np.arange(n, dtype=np.uint64))


def test_splitmix64_reference_stream():
    # SplitMix64 seeded with 0: the published algorithm's first outputs are the
    # finaliser applied to gamma, 2*gamma, ...; recompute them with Python ints.
    g = 0x9E3779B97F4A7C15
    M = (1 << 64) - 1

    def mix(z):
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return z ^ (z >> 31)

    for i in range(8):
        assert gen.splitmix64_at(0, i) == mix(((i + 1) * g) & M)


def test_uniform_range():
    u = gen.uniform(3, 1, 100, 200000)
    assert u.min() == 1 and u.max() == 100
    counts = np.bincount(u, minlength=101)[1:]
    assert abs(counts.mean() - 2000) < 1e-9 and counts.min() > 1700 and counts.max() < 2300


def test_zipf_chi_square():
    N, s, m = 1 << 10, 1.1, 1 << 20
    r = gen.zipf_ranks(77, N, s, m)
    assert r.min() >= 1 and r.max() <= N
    pmf = gen.zipf_pmf(N, s)
    assert abs(pmf.sum() - 1.0) < 1e-12
    obs = np.bincount(r, minlength=N + 1)[1:].astype(np.float64)
    exp = pmf * m
    # pool the tail so every cell expects >= 5
    keep = exp >= 5
    chi2 = (((obs[keep] - exp[keep]) ** 2) / exp[keep]).sum()
    tail_o, tail_e = obs[~keep].sum(), exp[~keep].sum()
    if tail_e > 0:
        chi2 += (tail_o - tail_e) ** 2 / tail_e
    dof = keep.sum()  # (cells - 1) + pooled tail
    # mean dof, sd sqrt(2 dof): accept within 6 sd
    assert chi2 < dof + 6 * np.sqrt(2 * dof)


def test_zipf_top_rank_mass_at_headline_size():
    # Zipf(1.1) over 2^22 ranks: p(1) = 1 / H_{2^22,1.1}
    pmf = gen.zipf_pmf(1 << 22, 1.1)
    H = (np.arange(1, (1 << 22) + 1, dtype=np.float64) ** -1.1).sum()
    assert abs(pmf[0] - 1.0 / H) < 1e-12
    assert 0.11 < pmf[0] < 0.13
