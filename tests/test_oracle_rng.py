"""Pins of the oracle's random stream: Philox4x64-10 against numpy's
independent implementation, and the bounded draw against properties that
a correct multiply-and-reject (Lemire 2019) must have."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def numpy_block(ctr, key):
    """numpy's Philox advances its counter before producing a block, so the
    first block of a generator started at counter c is the block of c + 1."""
    c = np.array(ctr, dtype=np.uint64)
    prev = c.copy()
    # subtract one with borrow over the four 64-bit words
    for i in range(4):
        if prev[i] != 0:
            prev[i] -= np.uint64(1)
            break
        prev[i] = np.uint64(0xFFFFFFFFFFFFFFFF)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=prev)
    return bg.random_raw(4)


def test_philox_known_answer():
    g = GOLD["philox4x64_10_zero"]
    out = O.philox4x64_10(g["counter"], g["key"])
    assert [int(h, 16) for h in g["out_hex"]] == [int(x) for x in out]


@pytest.mark.parametrize("trial", range(40))
def test_philox_matches_numpy(trial):
    rng = np.random.default_rng(1000 + trial)
    ctr = [int(x) for x in rng.integers(0, 2 ** 63, size=4, dtype=np.int64)]
    if trial % 4 == 0:
        ctr = [int(rng.integers(0, 10 ** 6)), trial % 3, 0, 0]
    key = [int(x) for x in rng.integers(0, 2 ** 63, size=2, dtype=np.int64)]
    if trial == 1:
        ctr, key = [2 ** 64 - 1] * 4, [2 ** 64 - 1] * 2
    assert [int(x) for x in O.philox4x64_10(ctr, key)] == [int(x) for x in numpy_block(ctr, key)]


def test_stream_layout():
    """word(seed, phase, idx, variate, attempt) is word 0 of the block with
    counter (idx, variate, attempt, 0) and key (seed, phase)."""
    for seed, phase, idx, var, att in [(1, 0, 0, 0, 0), (7, 2, 12345, 2, 3), (2 ** 63, 1, 2 ** 40, 1, 0)]:
        assert O.word(seed, phase, idx, var, att) == int(numpy_block([idx, var, att, 0], [seed, phase])[0])


def test_bounded_power_of_two_never_rejects():
    for b in [0, 1, 5, 17, 32, 63]:
        N = 1 << b
        for idx in range(200):
            v, used = O.bounded(3, 0, idx, 1, N)
            assert used == 1
            assert v == O.word(3, 0, idx, 1, 0) >> (64 - b) if b else v == 0


def test_bounded_range_and_uniformity_small():
    for N in [3, 7, 10]:
        counts = np.zeros(N, np.int64)
        draws = 30000
        for idx in range(draws):
            v, _ = O.bounded(11, 0, idx, 0, N)
            assert 0 <= v < N
            counts[v] += 1
        exp = draws / N
        chi2 = float(((counts - exp) ** 2 / exp).sum())
        # 99.9% quantile of chi-square with N-1 <= 9 dof is below 28
        assert chi2 < 28.0, (N, counts)


def test_bounded_removes_multiply_shift_bias():
    """For N = floor(2^64 * 2/3), multiply-shift alone gives even outputs
    twice the preimages of odd ones (P(even) = 2/3); rejection makes the
    parity fair and accepts with probability N / 2^64 = 2/3."""
    N = (2 ** 64 * 2) // 3
    even = 0
    attempts = 0
    draws = 20000
    for idx in range(draws):
        v, used = O.bounded(5, 1, idx, 2, N)
        assert v < N
        even += (v % 2 == 0)
        attempts += used
    p = even / draws
    assert abs(p - 0.5) < 4.5 * np.sqrt(0.25 / draws), p
    mean_att = attempts / draws
    assert abs(mean_att - 1.5) < 0.05, mean_att


def test_bounded_is_high_word_of_product_when_accepted():
    """When the first attempt is accepted, the result is floor(x N / 2^64)."""
    N = 1_000_003
    for idx in range(500):
        v, used = O.bounded(9, 0, idx, 0, N)
        if used == 1:
            x = O.word(9, 0, idx, 0, 0)
            assert v == (x * N) >> 64


def test_bounded128_powers_of_two_and_range():
    """Lemire at 128 bits: a power-of-two range never rejects and returns the
    top bits of the 128-bit word (word 1 high, word 0 low); every value is
    in range."""
    for e in (64, 65, 100, 127):
        N = 1 << e
        for idx in range(20):
            r, used = O.bounded128(3, 2, idx, 2, N)
            x = (O.word(3, 2, idx, 2, 0) | (_word1(3, 2, idx, 2, 0) << 64))
            assert used == 1 and r == x >> (128 - e)
    for N in ((1 << 64) + 1, 3 << 100, (1 << 128) - 3):
        for idx in range(200):
            r, _ = O.bounded128(5, 1, idx, 2, N)
            assert 0 <= r < N


def test_bounded128_rejection_is_exact():
    """N = floor(2^128 * 2/3) + 1: multiply-shift without rejection would make
    even values twice as likely as odd ones (P(even) = 2/3); the rejection
    zone is a third of the words, so the mean number of attempts is 1.5."""
    N = (1 << 128) * 2 // 3 + 1
    even, attempts, M = 0, 0, 4000
    for idx in range(M):
        r, used = O.bounded128(11, 0, idx, 2, N)
        even += (r % 2 == 0)
        attempts += used
    p = even / M
    assert abs(p - 0.5) < 4 * math.sqrt(0.25 / M)
    assert abs(attempts / M - 1.5) < 0.08


def _word1(seed, phase, idx, variate, attempt):
    ctr = np.array([idx, variate, attempt, 0], dtype=np.uint64)
    key = np.array([seed, phase], dtype=np.uint64)
    return int(O.philox4x64_10(ctr, key)[1])
