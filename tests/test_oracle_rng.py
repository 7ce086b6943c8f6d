"""Pins for the oracle's random bits (CPU only).

* Philox4x64-10 against numpy's independent implementation.
* The geometric-gap thresholds against exact rational arithmetic.
* ZRAND / noise draws against numpy's Philox through the counter layout.
* Hit statistics: Binomial(64, p) hit counts per word and uniform Pauli choice.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle

MASK = (1 << 64) - 1


def numpy_philox_block(counter, key):
    """numpy's Philox increments its counter before producing a block, so the
    block for counter c is what it emits after being set to c - 1."""
    c = list(counter)
    # subtract one with borrow across the 256-bit counter
    for i in range(4):
        if c[i] > 0:
            c[i] -= 1
            break
        c[i] = MASK
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(c, dtype=np.uint64))
    return [int(v) for v in g.random_raw(4)]


@pytest.mark.parametrize("counter,key", [
    ([0, 0, 0, 0], [0, 0]),
    ([1, 2, 3, 4], [5, 6]),
    ([MASK, MASK, MASK, MASK], [MASK, MASK]),
    ([0x0123456789ABCDEF, 17, 1 << 40, (3 << 32) | 5], [42, 0x5354494D5F465241]),
])
def test_philox_matches_numpy(counter, key):
    assert oracle.philox(counter, key) == numpy_philox_block(counter, key)


def test_philox_random_counters_match_numpy():
    rng = np.random.Generator(np.random.PCG64(1))
    for _ in range(200):
        ctr = [int(v) for v in rng.integers(0, 2**63, size=4, dtype=np.int64)]
        key = [int(v) for v in rng.integers(0, 2**63, size=2, dtype=np.int64)]
        assert oracle.philox(ctr, key) == numpy_philox_block(ctr, key)


def exact_thresholds(p):
    a = math.floor((1 - Fraction(p)) * 2**64)
    t = [a]
    for _ in range(63):
        t.append((t[-1] * a) >> 64)
    return t


@pytest.mark.parametrize("p", [1e-4, 1e-3, 1e-2, 0.3, 0.5, 0.999, 1.0, 5e-324, 1e-300, 2**-60, 2**-64, 2**-70])
def test_thresholds_exact(p):
    assert oracle.thresholds(p) == exact_thresholds(p)


def test_thresholds_track_geometric_probability():
    for p in (1e-4, 1e-3, 1e-2, 0.2):
        t = oracle.thresholds(p)
        for g in (1, 10, 64):
            assert abs(t[g - 1] / 2**64 - (1 - p) ** g) < 1e-12


def test_zrand_counter_layout():
    seed, key_hi = 7, oracle.key_hi()
    for instr, slot, word in [(0, 0, 0), (5, 3, 9), (12, 6, 1 << 33), (MASK, 17, 4)]:
        block = numpy_philox_block([instr, slot >> 2, word, 1 << 32], [seed, key_hi])
        assert oracle.zrand(seed, instr, slot, word) == block[slot & 3]


def python_hits(seed, instr, slot, word, p, K):
    """The noise draw sequence and gap sampling, restated with numpy Philox
    blocks and exact thresholds."""
    key = [seed, oracle.key_hi()]
    t = exact_thresholds(p)
    pre = numpy_philox_block([instr, slot >> 5, word, 2 << 32], key)
    k = slot & 31
    v = (pre[k >> 3] >> (8 * (k & 7))) & 0xFF
    draws = []
    j = 0

    def draw():
        nonlocal j
        blk = numpy_philox_block([instr, slot, word, (3 << 32) | (j >> 2)], key)
        d = blk[j & 3]
        if j == 0:
            d = (v << 56) | (d & ((1 << 56) - 1))
        j += 1
        return d

    hits = []
    pos = 0
    while True:
        u = draw()
        G = sum(1 for g in range(64) if u < t[g])
        pos += G
        if pos >= 64:
            break
        c = (draw() * K) >> 64 if K else 0
        hits.append((pos, c))
        pos += 1
        if pos >= 64:
            break
    return hits


@pytest.mark.parametrize("p,K", [(0.05, 0), (0.3, 3), (0.2, 15), (1.0, 0), (1.0, 15)])
def test_hits_match_restatement(p, K):
    for (instr, slot, word) in [(3, 0, 0), (7, 21, 5), (100, 1, 77), (9, 16, 2), (4, 63, 1), (5, 32, 9)]:
        assert oracle.hits(11, instr, slot, word, p, K) == python_hits(11, instr, slot, word, p, K)


def test_p_one_hits_every_shot():
    h = oracle.hits(1, 2, 3, 4, 1.0, 0)
    assert [x for x, _ in h] == list(range(64))


@pytest.mark.parametrize("p", [0.02, 0.2])
def test_hit_counts_are_binomial(p):
    counts = np.zeros(65, dtype=np.int64)
    n = 20000
    for w in range(n):
        counts[len(oracle.hits(3, 1, w % 7, w, p, 0))] += 1
    expected = np.array([stats.binom.pmf(k, 64, p) for k in range(65)]) * n
    keep = expected > 5
    obs = np.append(counts[keep], counts[~keep].sum())
    exp = np.append(expected[keep], expected[~keep].sum())
    exp *= obs.sum() / exp.sum()
    assert stats.chisquare(obs, exp).pvalue > 1e-4


def test_hit_positions_uniform_and_choice_uniform():
    pos = np.zeros(64)
    ch = np.zeros(15)
    for w in range(5000):
        for x, c in oracle.hits(5, 9, 0, w, 0.1, 15):
            pos[x] += 1
            ch[c] += 1
    assert stats.chisquare(pos).pvalue > 1e-4
    assert stats.chisquare(ch).pvalue > 1e-4


def test_zrand_bits_balanced():
    words = [oracle.zrand(2, 10, s, w) for s in range(8) for w in range(256)]
    ones = sum(bin(v).count("1") for v in words)
    n = 64 * len(words)
    assert abs(ones - n / 2) < 5 * math.sqrt(n / 4)
