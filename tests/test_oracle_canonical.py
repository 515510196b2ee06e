"""Pins of the oracle's binomial convolution R_L(p) (not GPU).

Closed forms: the grid ends; a single-spike histogram gives the upper binomial
tail, the regularised incomplete beta I_p(m, N-m+1) (scipy.special.betainc); the
exact L = 2 spanning polynomial sum_n S_n p^n (1-p)^(32-n) from exhaustive
counting; a 50-digit mpmath evaluation; monotonicity in p.
"""
from fractions import Fraction
from math import comb

import mpmath
import numpy as np
import pytest
from scipy.special import betainc

from test_oracle_sweep import l2_spanning_counts

P101 = np.linspace(0.0, 1.0, 101)


def test_grid_ends(nzo):
    h = np.zeros(1025, dtype=np.uint64)
    h[100] = 3
    h[700] = 5
    h[0] = 2
    R = nzo.canonical(h, [0.0, 1.0])
    assert R[0] == 0.0
    assert R[1] == pytest.approx(8 / 10, abs=1e-15)


@pytest.mark.parametrize("N,m", [(1024, 1), (1024, 150), (1024, 1024), (32768, 4600), (1048576, 147000)])
def test_single_spike_is_incomplete_beta(nzo, N, m):
    h = np.zeros(N + 1, dtype=np.uint64)
    h[m] = 7
    p = np.linspace(0.0, 1.0, 201) if N < 100000 else np.concatenate([[0.0, 0.5, 1.0], np.linspace(0.135, 0.145, 9)])
    R = nzo.canonical(h, p)
    want = betainc(m, N - m + 1, p)
    assert np.max(np.abs(R - want)) < 1e-12


def test_l2_exact_polynomial(nzo):
    S = l2_spanning_counts(1)
    cdf = [Fraction(S[n], comb(32, n)) for n in range(33)]
    scale = 2**52
    h = np.array([0] + [round((cdf[n] - cdf[n - 1]) * scale) for n in range(1, 33)], dtype=np.uint64)
    R = nzo.canonical(h, P101)
    for p, r in zip(P101, R):
        q = Fraction(p)
        exact = sum(S[n] * q**n * (1 - q) ** (32 - n) for n in range(33))
        assert abs(r - float(exact)) < 1e-12


def test_mpmath_50_digits(nzo):
    rng = np.random.default_rng(11)
    N = 1024
    h = np.zeros(N + 1, dtype=np.uint64)
    np.add.at(h, rng.integers(100, 400, size=1000), 1)
    R = nzo.canonical(h, P101)
    mpmath.mp.dps = 50
    tot = int(h.sum())
    F = np.cumsum(h.astype(object))
    F[0] = 0
    for p, r in zip(P101[::5], R[::5]):
        mp = mpmath.mpf(p)
        s = mpmath.fsum(mpmath.binomial(N, n) * mp**n * (1 - mp) ** (N - n) * mpmath.mpf(int(F[n])) / tot
                        for n in range(N + 1))
        assert abs(r - float(s)) < 1e-14


def test_monotone_in_p(nzo):
    rng = np.random.default_rng(2)
    N = 32768
    h = np.zeros(N + 1, dtype=np.uint64)
    np.add.at(h, rng.integers(3000, 6000, size=5000), 1)
    R = nzo.canonical(h, np.linspace(0, 1, 1001))
    assert (np.diff(R) >= -1e-15).all()
