"""Pins of the oracle's random streams and function selection.

Philox4x32-10 is pinned by the published known-answer vectors (golden file);
selection by the exact closed form of equal-probability thresholds, an
exhaustive count over all 2^32 draws, and the integer identity
min{i : u < ceil((i+1) 2^32 / n)} = floor(u n / 2^32).
"""
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(orc):
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, expect in rows:
        got = orc.philox4x32_10(ctr, key)
        assert [int(x) for x in got] == expect


def test_philox_many_matches_single(orc):
    rng = np.random.default_rng(5)
    ctrs = rng.integers(0, 2**32, size=(64, 4), dtype=np.uint64).astype(np.uint32)
    seed = 0x0123456789ABCDEF
    many = orc.philox_many(seed, ctrs)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for i in range(64):
        assert np.array_equal(many[i], orc.philox4x32_10(ctrs[i], key))


def test_philox_bits_uniform(orc):
    # 2^18 words from consecutive counters: every 4-bit nibble position is
    # uniform (chi-square, 15 dof, p > 1e-6 => statistic < 50).
    n = 1 << 16
    ctrs = np.zeros((n, 4), np.uint32)
    ctrs[:, 0] = np.arange(n, dtype=np.uint32)
    words = orc.philox_many(0, ctrs).reshape(-1)
    for shift in range(0, 32, 4):
        nib = (words >> np.uint32(shift)) & np.uint32(15)
        cnt = np.bincount(nib.astype(np.int64), minlength=16)
        exp = words.size / 16
        chi2 = float(((cnt - exp) ** 2 / exp).sum())
        assert chi2 < 50.0, (shift, chi2)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 16, 20, 64])
def test_equal_thresholds_closed_form(orc, n):
    th = orc.thresholds(None, n)
    expect = [-(-((i + 1) << 32) // n) for i in range(n)]  # exact ceil
    assert [int(x) for x in th] == expect
    assert int(th[-1]) == 1 << 32


@pytest.mark.parametrize("n", [3, 4, 20])
def test_equal_selection_is_mulhi(orc, n):
    th = orc.thresholds(None, n)
    rng = np.random.default_rng(n)
    us = list(rng.integers(0, 2**32, size=2000, dtype=np.uint64))
    # every boundary and its neighbours
    for t in th[:-1]:
        us += [int(t) - 1, int(t), int(t) + 1]
    us += [0, 2**32 - 1]
    for u in us:
        u = int(u) & 0xFFFFFFFF
        assert orc.select(u, th) == (u * n) >> 32


def test_probability_thresholds(orc):
    rng = np.random.default_rng(3)
    for n in (2, 5, 16):
        p = rng.dirichlet(np.ones(n))
        th = orc.thresholds(p, n)
        cum = np.cumsum(p)
        for i in range(n - 1):
            assert int(th[i]) == math.ceil(math.ldexp(cum[i], 32))
        assert int(th[-1]) == 1 << 32
        assert np.all(np.diff(th.astype(np.int64)) >= 0)
        widths = np.diff(np.concatenate([[0], th.astype(np.float64)])) / 2.0**32
        assert np.max(np.abs(widths - p)) < 2.0**-31


def test_probability_rejects_bad_tables(orc):
    with pytest.raises(ValueError):
        orc.thresholds(np.array([0.5, 0.6]), 2)
    with pytest.raises(ValueError):
        orc.thresholds(np.array([1.5, -0.5]), 2)


@pytest.mark.slow
def test_selection_exhaustive_unequal(orc):
    # Every u in [0, 2^32) is drawn once: index i must be drawn exactly
    # thresh[i] - thresh[i-1] times (inverse CDF over integer thresholds).
    p = np.array([0.2, 0.5, 0.3])
    th = orc.thresholds(p, 3)
    counts = orc.select_histogram(th)
    widths = np.diff(np.concatenate([[0], th.astype(np.int64)]))
    assert [int(c) for c in counts] == [int(w) for w in widths]
    assert int(counts.sum()) == 1 << 32


def test_selection_boundaries_unequal(orc):
    rng = np.random.default_rng(11)
    p = rng.dirichlet(np.ones(16))
    th = orc.thresholds(p, 16)
    lo = 0
    for i in range(16):
        hi = int(th[i])
        if hi > lo:
            assert orc.select(lo, th) == i
            assert orc.select(hi - 1, th) == i
        lo = hi
