"""Pins of the oracle's Bloom filter (Sec. IV lists a BloomFilter for set membership).

The filter's layout is a reading (the paper gives none): a split-block filter, B blocks of
`words` 32-bit words, each key setting one bit in every word of one block (k = words).  The
pins check what that reading and probability fix, not the oracle's own formula:
  * one key sets exactly one bit in each word of exactly one block (a dropped term, a wrong
    word or bit index breaks this);
  * no false negatives;
  * given j keys in a block, a word's bit is set with probability 1 - (31/32)^j, independently
    across words, so the expected fraction of set bits is 1 - (1 - 1/(32 B))^n and the
    false-positive rate is sum_j Binom(j; n, 1/B) (1 - (31/32)^j)^k (the keys here are a few
    hundred thousand distinct values of 2^32, where the exact hypergeometric block count is
    binomial to well within the tolerance);
  * block choice and the bits inside words are uniform (chi-square), for power-of-two and
    other block counts;
  * an empty filter answers no and a full one yes.
"""
import math

import numpy as np
import pytest

import gen
import oracle


def _keys(seed, n):
    return gen.keys(seed, 1, n)


def _popcount(a):
    return int(np.unpackbits(np.ascontiguousarray(a).view(np.uint8)).sum())


@pytest.mark.parametrize("words", [8, 16, 32])
def test_one_key_sets_one_bit_per_word_of_one_block(words):
    for key in (1, 2, 0xDEADBEEF, 0xFFFFFFFF, 0):
        f = oracle.OracleBloom(37, words, 0x1234)
        f.insert(np.array([key], np.uint32))
        bits = f.bits.reshape(37, words)
        touched = np.nonzero(bits.any(axis=1))[0]
        assert touched.size == 1
        row = bits[touched[0]]
        assert all(_popcount(np.array([w], np.uint32)) == 1 for w in row)
        blk, bit = f.positions(key)
        assert blk == touched[0] and np.array_equal(row, (np.uint32(1) << bit.astype(np.uint32)))
        assert f.query(np.array([key], np.uint32))[0] == 1


@pytest.mark.parametrize("blocks,words", [(4096, 16), (1000, 8), (3001, 32)])
def test_no_false_negatives_and_set_fraction(blocks, words):
    n = 200_000
    f = oracle.OracleBloom(blocks, words, 77)
    keys = _keys(5, n)
    f.insert(keys)
    assert f.query(keys).all()
    total = blocks * words * 32
    frac = _popcount(f.bits) / total
    expect = 1.0 - (1.0 - 1.0 / (32 * blocks)) ** n
    sd = math.sqrt(expect * (1 - expect) / total)
    assert abs(frac - expect) < 8 * sd + 1e-4, (frac, expect, sd)


@pytest.mark.parametrize("blocks", [1024, 1000])
def test_block_choice_and_bits_uniform(blocks):
    words, n = 16, 60_000
    f = oracle.OracleBloom(blocks, words, 99)
    keys = _keys(11, n)
    blk = np.empty(n, np.int64)
    bit = np.empty((n, words), np.int64)
    for i, x in enumerate(keys):
        blk[i], bit[i] = f.positions(int(x))
    assert blk.min() >= 0 and blk.max() < blocks and bit.max() < 32
    cnt = np.bincount(blk, minlength=blocks)
    e = n / blocks
    chi2 = ((cnt - e) ** 2 / e).sum()
    assert abs(chi2 - (blocks - 1)) < 6 * math.sqrt(2 * (blocks - 1))
    for i in (0, 5, words - 1):  # each word's bit uniform on 0..31
        pc = np.bincount(bit[:, i], minlength=32)
        e = n / 32
        chi2 = ((pc - e) ** 2 / e).sum()
        assert abs(chi2 - 31) < 6 * math.sqrt(62)
    # bits of different words of one key are not tied together (pairs uniform on 32 x 32)
    pair = np.bincount(bit[:, 0] * 32 + bit[:, 1], minlength=1024)
    e = n / 1024
    chi2 = ((pair - e) ** 2 / e).sum()
    assert abs(chi2 - 1023) < 6 * math.sqrt(2 * 1023)


def _fpr_closed_form(n, blocks, words):
    """sum over j ~ Binomial(n, 1/B) of (1 - (31/32)^j)^k, k = words."""
    p = 1.0 / blocks
    logc = math.lgamma(n + 1)
    total = 0.0
    mean = n * p
    hi = int(mean + 12 * math.sqrt(mean) + 50)
    for j in range(0, min(n, hi) + 1):
        lp = logc - math.lgamma(j + 1) - math.lgamma(n - j + 1) + j * math.log(p) + (n - j) * math.log1p(-p)
        total += math.exp(lp) * (1 - (31 / 32) ** j) ** words
    return total


@pytest.mark.parametrize("words,bits_per_key", [(16, 12), (8, 8), (32, 16)])
def test_false_positive_rate_closed_form(words, bits_per_key):
    blocks = 2048
    n = blocks * words * 32 // bits_per_key
    f = oracle.OracleBloom(blocks, words, 5)
    f.insert(_keys(21, n))
    absent = gen.keys(21, n + 1, 600_000)  # disjoint from the inserted keys
    fpr = f.query(absent).mean()
    expect = _fpr_closed_form(n, blocks, words)
    assert 0.001 < expect < 0.2, expect
    # binomial sampling error of 600k queries is under 3% of the rate here
    assert abs(fpr - expect) < 0.08 * expect, (fpr, expect)


def test_empty_and_full_filters():
    f = oracle.OracleBloom(64, 16, 3)
    q = _keys(31, 5000)
    assert not f.query(q).any()
    f.bits[:] = 0xFFFFFFFF
    assert f.query(q).all()
