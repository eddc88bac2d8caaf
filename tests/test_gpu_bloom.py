"""GPU parity of the split-block Bloom filter against the CPU oracle's filter.

Bit-exact: after the same inserts the dumped bit array equals the oracle's word for word, and
every membership answer equals the oracle's (integer work, no tolerance).  Cases span every
block size and group size, power-of-two and other block counts, repeated keys, several insert
launches, clear, and a filter of 2^32 bits with 2^28 keys (the benchmark's configuration),
where 4096 sampled blocks are rebuilt by the oracle from the keys that map to them and the
false-positive rate is checked against the filter's closed form.
"""
import math

import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import d, h

pytestmark = pytest.mark.gpu


def _fpr_distinct_keys(n, blocks, words):
    """False-positive rate after n distinct keys.  h1 is a bijection of the 32-bit keys and a
    power-of-two block count takes its low bits, so every block owns 2^32 / B hash values and a
    block's key count j is hypergeometric (not binomial: drawing 2^28 of 2^32 values without
    replacement narrows it); each of the words of the queried block then holds the query's bit
    with probability 1 - (31/32)^j, independently."""
    M = 1 << 32
    K = M // blocks

    def lc(a, b):
        return math.lgamma(a + 1) - math.lgamma(b + 1) - math.lgamma(a - b + 1)

    base, total = lc(M, n), 0.0
    for j in range(0, min(K, n) + 1):
        lp = lc(K, j) + lc(M - K, n - j) - base
        if lp > -60:
            total += math.exp(lp) * (1 - (31 / 32) ** j) ** words
    return total


def _pairs():
    for words in (8, 16, 32):
        for g in (1, 2, 4, 8, 16, 32):
            if g <= words:
                yield words, g


@pytest.mark.parametrize("words,group", list(_pairs()))
@pytest.mark.parametrize("blocks", [4096, 3001])
def test_bloom_bits_and_answers_match_oracle(hc, words, group, blocks):
    seed = 0xB100 + words * 7 + group
    f = hc.Bloom(blocks * words * 32, block_words=words, group=group, seed=seed)
    assert f.blocks == blocks
    orc = oracle.OracleBloom(blocks, words, seed)
    n = blocks * words * 32 // 12
    keys = gen.keys(seed, 1, n)
    keys[::97] = keys[::89][: keys[::97].size]  # repeated keys
    for part in np.array_split(keys, 3):  # three launches
        f.insert(d(part))
        orc.insert(part)
    assert np.array_equal(h(f.dump()), orc.bits)
    q = np.concatenate([keys[: n // 2], gen.keys(seed, n + 1, n // 2), np.array([0, 0xFFFFFFFF], np.uint32)])
    got = h(f.contains(d(q)))
    assert np.array_equal(got, orc.query(q))
    assert got[: n // 2].all()  # no false negatives
    # another group size on the same filter gives the same answers
    other = 1 if group != 1 else 2
    assert np.array_equal(h(f.contains(d(q), group=other)), got)


def test_bloom_default_group_per_operation(hc):
    # group 0: inserts one lane per word, queries one lane per key; same bits and answers as any explicit group
    keys = gen.keys(9, 1, 200000)
    q = np.concatenate([keys[:1000], gen.keys(9, 200001, 100000)])
    a = hc.Bloom(1 << 22, block_words=32, seed=3)
    assert a.group == 0
    b = hc.Bloom(1 << 22, block_words=32, group=2, seed=3)
    a.insert(d(keys))
    b.insert(d(keys))
    assert np.array_equal(h(a.dump()), h(b.dump()))
    assert np.array_equal(h(a.contains(d(q))), h(b.contains(d(q))))


def test_bloom_clear_and_empty(hc):
    f = hc.Bloom(1 << 20, block_words=16, group=4)
    keys = gen.keys(3, 1, 50000)
    assert not h(f.contains(d(keys))).any()
    f.insert(d(keys))
    assert h(f.contains(d(keys))).all()
    f.clear()
    assert not h(f.dump()).any()
    assert not h(f.contains(d(keys))).any()
    f.insert(d(keys[:0]))  # empty launch


def test_bloom_full_size_sampled_blocks_and_closed_form(hc):
    # 2^32 bits (2^23 blocks of 16 words), 2^28 keys: the oracle rebuilds 4096 sampled blocks
    # from exactly the keys that map to them, and answers the queries that fall into them
    words, log2_bits, log2_n = 16, 32, 28
    f = hc.Bloom(1 << log2_bits, block_words=words, seed=0x5EED)  # per-operation default groups
    n = 1 << log2_n
    keys = gen.keys(41, 1, n)
    f.insert(d(keys))
    orc = oracle.OracleBloom(f.blocks, words, 0x5EED)
    sample = np.unique(gen.uniform(43, 0, f.blocks - 1, 4096).astype(np.uint64))
    mine = np.isin(orc.blocks_of(keys), sample)
    orc.insert(keys[mine])
    words_idx = (sample[:, None] * words + np.arange(words, dtype=np.uint64)[None, :]).ravel().astype(np.int64)
    dump = h(f.dump())
    assert np.array_equal(dump[words_idx], orc.bits[words_idx])
    absent = gen.keys(41, n + 1, 1 << 22)
    fp = h(f.contains(d(absent)))
    inq = np.isin(orc.blocks_of(absent), sample)
    assert inq.sum() > 100 and np.array_equal(fp[inq], orc.query(absent[inq]))
    assert h(f.contains(d(keys[: 1 << 22]))).all()  # no false negatives
    expect = _fpr_distinct_keys(n, f.blocks, words)
    # about 7000 false positives expected: sampling error near 1.2%
    assert abs(fp.mean() - expect) < 0.05 * expect, (fp.mean(), expect)


def test_bloom_argument_errors(hc):
    for kw in (dict(block_words=12), dict(block_words=8, group=16), dict(group=3)):
        with pytest.raises(hc.HcError) as e:
            hc.Bloom(1 << 12, **kw)
        assert e.value.code == hc.E_ARG
    with pytest.raises(hc.HcError) as e:
        hc.Bloom(0)
    assert e.value.code == hc.E_ARG
    f = hc.Bloom(1 << 12, block_words=8)
    k = d(np.arange(1, 10, dtype=np.uint32))
    with pytest.raises(hc.HcError) as e:
        f.contains(k, group=16)
    assert e.value.code == hc.E_ARG
