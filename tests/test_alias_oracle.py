"""Pins of the oracle's sampler: the alias table of p_i = |c_i| / sum_j |c_j|
(paper, section II.B, sampling-probability equation; alias method) and the
seeded SplitMix64 draws.  CPU only.

The pins do not re-type the oracle's construction:
  - SplitMix64 against published output sequences of the generator;
  - the alias table against its defining property: every item's mass is split
    exactly over its own bucket and the buckets that alias it (integers);
  - the sampler's exact output distribution (every bucket and threshold
    enumerated in rational arithmetic) against p_i = |c_i| / sum |c|;
  - draw frequencies against p_i by a chi-square test.
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

from oracle import ref


def test_splitmix64_published_outputs():
    # SplitMix64 (Steele, Lea and Flood 2014; Vigna's reference splitmix64.c):
    # the first outputs for seed 1234567 as listed by the Rosetta Code task
    # "Pseudo-random numbers/Splitmix64", and the first two for seed 0.
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    assert [ref.splitmix64(1234567, m) for m in range(1, 6)] == want
    assert ref.splitmix64(0, 1) == 0xE220A8397B1DCDAF
    assert ref.splitmix64(0, 2) == 0x6E789E6AA1B965F4


def _coefficients(rng, n, zeros=0):
    c = rng.normal(size=n) * np.exp(rng.uniform(-12, 0, size=n))
    c[0] = 0.9
    if zeros:
        c[rng.choice(np.arange(1, n), size=zeros, replace=False)] = 0.0
    return c


def _check_masses(t: ref.AliasTable):
    n = len(t.alias)
    got = list(t.own)
    for k in range(n):
        a = int(t.alias[k])
        assert 0 <= a < n
        if a != k:
            got[a] += t.capacity - t.own[k]
        else:
            assert t.own[k] == t.capacity
        assert 0 <= t.own[k] <= t.capacity
    assert got == t.mass
    assert sum(t.mass) == n * t.capacity


def _exact_distribution(t: ref.AliasTable):
    """Probability of each item under the sampler: bucket b = floor(r1 n / 2^64),
    item b when r2 < threshold[b], else alias[b]; r1, r2 uniform on 64 bits."""
    n = len(t.alias)
    two64 = 1 << 64
    p = [Fraction(0)] * n
    for b in range(n):
        lo = -((-b * two64) // n)          # ceil(b 2^64 / n)
        hi = -((-(b + 1) * two64) // n)
        pb = Fraction(hi - lo, two64)
        keep = Fraction(int(t.threshold[b]), two64)
        p[b] += pb * keep
        p[int(t.alias[b])] += pb * (1 - keep)
    return p


@pytest.mark.parametrize("n,zeros,seed", [(1, 0, 0), (2, 0, 1), (7, 0, 2), (37, 3, 3), (200, 10, 4), (3000, 900, 5)])
def test_alias_table_masses_and_distribution(n, zeros, seed):
    c = _coefficients(np.random.default_rng(seed), n, zeros)
    t = ref.alias_table(c)
    _check_masses(t)
    # every sum of masses or bucket deficits fits 128 bits (a device
    # construction by prefix sums forms them)
    assert n * t.capacity < 2**127
    # sampled distribution against p_i = |c_i| / sum |c| in exact rationals
    exact = _exact_distribution(t)
    tot = sum(Fraction(abs(float(v))) for v in c)
    for i in range(n):
        p = Fraction(abs(float(c[i]))) / tot
        touching = 1 + int((t.alias == i).sum())
        assert abs(exact[i] - p) <= Fraction(touching + 2, 1 << 62) + p * Fraction(1, 1 << 60), i
        if c[i] == 0.0:
            assert exact[i] == 0


def test_alias_table_invariances():
    rng = np.random.default_rng(7)
    c = _coefficients(rng, 300, 5)
    t = ref.alias_table(c)
    for other in (-c, np.ldexp(c, 17), np.ldexp(c, -40), np.where(rng.random(300) < 0.5, c, -c)):
        u = ref.alias_table(other)
        assert np.array_equal(u.threshold, t.threshold)
        assert np.array_equal(u.alias, t.alias)


def test_alias_degenerate_inputs():
    # equal weights: every bucket keeps itself
    t = ref.alias_table(np.full(64, -0.125))
    assert (t.threshold == np.uint64(2**64 - 1)).all()
    assert np.array_equal(t.alias, np.arange(64, dtype=np.uint32))
    # a single non-zero coefficient takes every draw
    c = np.zeros(50)
    c[17] = 3e-200
    d = ref.alias_draws(c, 3, 1000, 5)
    assert (d == 17).all()
    with pytest.raises(ref.OracleError):
        ref.alias_table(np.zeros(4))
    with pytest.raises(ref.OracleError):
        ref.alias_table(np.array([1.0, np.nan]))


def test_draw_frequencies_chi_square():
    rng = np.random.default_rng(11)
    c = _coefficients(rng, 40, 4)
    c = np.abs(c) ** 0.25 * np.sign(c)  # flatter, so every cell is well populated
    p = np.abs(c) / np.abs(c).sum()
    d = ref.alias_draws(c, 50, 8000, 2024)
    assert d.shape == (50, 8000)
    counts = np.bincount(d.ravel(), minlength=len(c))
    assert (counts[p == 0] == 0).all()
    keep = p > 0
    chi2, pval = stats.chisquare(counts[keep], d.size * p[keep])
    assert pval > 1e-4, (chi2, pval)


def test_draws_are_counter_based():
    # draw k of sample s depends only on (seed, s, k): a prefix of the samples
    # and draws is the same array cut
    c = _coefficients(np.random.default_rng(3), 500, 0)
    big = ref.alias_draws(c, 6, 300, 99)
    small = ref.alias_draws(c, 4, 300, 99)
    assert np.array_equal(big[:4], small)
    other = ref.alias_draws(c, 6, 300, 100)
    assert not np.array_equal(big, other)
