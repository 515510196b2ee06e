"""Pins of the oracle's largest-cluster track S_max(n) and of its binomial
convolution of a windowed observable (eqs. (5)-(6)), not GPU."""
import numpy as np
import pytest
from scipy import stats

import lattice_np


def _smax_bruteforce(L, mask, order, n):
    """Largest cluster of the first n sites of the order, from the labels that
    scipy's connected_components gives (tests/lattice_np.py)."""
    lab = lattice_np.components(L, mask, order[:n])
    return int(np.bincount(lab[lab >= 0]).max())


@pytest.mark.parametrize("L,mask,sample", [(3, 0x01, 0), (4, 0x01, 1), (4, 0x06, 2), (3, 0x7F, 3)])
def test_smax_matches_connected_components(nzo, L, mask, sample):
    N = L**5
    o = nzo.order(L, 77, sample)
    _, _, sm = nzo.sweep_order(L, mask, o, smax=True, run_to_end=True)
    for n in sorted({1, 2, N // 10, N // 5, N // 3, N // 2, (2 * N) // 3, N}):
        assert sm[n - 1] == _smax_bruteforce(L, mask, o, n), n


def test_smax_monotone_and_full_lattice(nzo):
    L = 4
    N = L**5
    o = nzo.order(L, 5, 0)
    _, _, sm = nzo.sweep_order(L, 0x01, o, smax=True, run_to_end=True)
    assert sm[0] == 1 and (np.diff(sm) >= 0).all() and sm[-1] == N


def test_smax_window_sums_samples(nzo):
    L, mask = 3, 0x03
    N = L**5
    acc = nzo.smax_window(L, mask, 9, 4, 3, 20, 60)
    want = np.zeros(40, dtype=np.int64)
    for s in (4, 5, 6):
        _, _, sm = nzo.sweep_order(L, mask, nzo.order(L, 9, s), smax=True, run_to_end=True)
        want += sm[19:59]
    assert (acc == want).all()
    assert N == 243


@pytest.mark.parametrize("N", [1, 7, 1000, 32768])
def test_convolution_closed_forms(nzo, N):
    p = np.array([0.0, 0.013, 0.1408, 0.5, 0.93, 1.0])
    n = np.arange(N + 1, dtype=np.float64)
    one, cov = nzo.convolve_window(np.ones(N + 1), 0, N, p)
    assert np.allclose(one, 1.0, atol=1e-13) and np.allclose(cov, 1.0, atol=1e-13)
    mean, _ = nzo.convolve_window(n, 0, N, p)
    assert np.allclose(mean, N * p, rtol=1e-12, atol=1e-9)
    second, _ = nzo.convolve_window(n * n, 0, N, p)
    assert np.allclose(second, N * p * (1 - p) + (N * p) ** 2, rtol=1e-12, atol=1e-9)


def test_window_coverage_is_binomial_mass(nzo):
    N = 100_000
    p = np.array([0.1, 0.1408, 0.2])
    lo, hi = 13_000, 15_500
    _, cov = nzo.convolve_window(np.zeros(hi - lo), lo, N, p)
    want = stats.binom.cdf(hi - 1, N, p) - stats.binom.cdf(lo - 1, N, p)
    assert np.allclose(cov, want, atol=1e-10)


@pytest.mark.parametrize("L,mask,sample", [(5, 0x01, 0), (5, 0x7F, 1), (6, 0x06, 2)])
def test_periodic_smax_matches_connected_components(nzo, L, mask, sample):
    N = L**5
    o = nzo.order(L, 31, sample)
    ns, ms, sm = nzo.sweep_order(L, mask, o, smax=True, run_to_end=True, periodic=True)
    # no borders: n* and mass refer to the first cluster wrapping around axis 0
    assert (ns, ms) == lattice_np.first_wrap(L, mask, o)
    for n in sorted({1, N // 20, N // 8, N // 4, N // 2, N}):
        lab = lattice_np.components(L, mask, o[:n], periodic=True)
        assert sm[n - 1] == int(np.bincount(lab[lab >= 0]).max()), n
    assert sm[-1] == N


def test_periodic_translation_invariance(nzo):
    """Translating every site by a fixed vector (mod L) maps a periodic lattice
    onto itself, so the largest-cluster track of the translated order is the
    same; with free boundaries it is not."""
    L, mask = 5, 0x03
    N = L**5
    o = nzo.order(L, 8, 3)
    x = lattice_np.coords(L, o)
    c = np.array([2, 0, 4, 1, 3])
    t = (np.mod(x + c, L) * (L ** np.arange(5))).sum(axis=1).astype(np.uint32)
    _, _, a = nzo.sweep_order(L, mask, o, smax=True, run_to_end=True, periodic=True)
    _, _, b = nzo.sweep_order(L, mask, t, smax=True, run_to_end=True, periodic=True)
    assert (a == b).all()
    _, _, fa = nzo.sweep_order(L, mask, o, smax=True, run_to_end=True)
    _, _, fb = nzo.sweep_order(L, mask, t, smax=True, run_to_end=True)
    assert not (fa == fb).all()
    # every site has its full neighbourhood: a sweep of all N sites merges to one cluster
    assert a[-1] == N
