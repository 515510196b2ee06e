"""Pins of the oracle's Newman-Ziff sweep (not GPU).

(i) exact law of n* at L = 2 by exhaustive counting over all 2^32 occupation
subsets, and brute-force first-spanning prefixes; (ii) snapshots re-labelled by a
library connected-components routine; (iii) conservation of cluster sizes; (iv)
special cases; (v) bounds; (vi) subset monotonicity under common random numbers.
"""
from math import comb

import numpy as np
import pytest
from scipy import stats

import lattice_np

SEED = 0x5EED


# ---------------------------------------------------------------- L = 2 exact law
def l2_crossing_neighbours(mask):
    """For each of the 16 sites with x0 = 0 at L = 2 (site index i = sum x_j 2^j, even
    i), the 16-bit set of x0 = 1 sites adjacent to it."""
    off = lattice_np.shell_offsets(mask)
    nb = np.zeros(16, dtype=np.int64)
    for a in range(16):
        s = 2 * a
        x = np.array([(s >> j) & 1 for j in range(5)])
        y = x + off
        inb = ((y >= 0) & (y < 2)).all(axis=1)
        for t in (y[inb] * (1 << np.arange(5))).sum(axis=1):
            if t & 1:
                nb[a] |= 1 << (t >> 1)
    return nb


def l2_spanning_counts(mask):
    """S_n = number of n-subsets of the 32 sites that span, n = 0..32.

    At L = 2 a cluster spans iff it joins an x0 = 0 site to an x0 = 1 site, i.e.
    iff the occupied set contains an adjacent pair with different x0 (any path
    between the two faces has such a step).  A non-spanning set is therefore a
    choice B of x0 = 0 sites plus any sites of x0 = 1 not adjacent to B.
    """
    nb = l2_crossing_neighbours(mask)
    N1 = np.zeros(1 << 16, dtype=np.int64)
    for b in range(16):
        N1[1 << b : 1 << (b + 1)] = N1[: 1 << b] | nb[b]
    popB = np.array([bin(b).count("1") for b in range(1 << 16)])
    free = 16 - np.array([bin(int(v)).count("1") for v in N1])
    ns = [0] * 33
    for a, f in zip(popB.tolist(), free.tolist()):
        for n in range(a, a + f + 1):
            ns[n] += comb(f, n - a)
    return [comb(32, n) - ns[n] for n in range(33)]


def test_l2_characterisation_against_connected_components():
    rng = np.random.default_rng(3)
    for mask in (1, 2, 3, 0x1F, 0x14, 0x7F):
        off = lattice_np.shell_offsets(mask)
        nb = l2_crossing_neighbours(mask)
        for _ in range(120):
            occ = np.nonzero(rng.random(32) < rng.random())[0]
            lab = lattice_np.components(2, mask, occ)
            sp = lattice_np.spans(2, lab)
            s = set(occ.tolist())
            cross = any((nb[a] >> b) & 1 for a in range(16) for b in range(16)
                        if 2 * a in s and 2 * b + 1 in s)
            assert sp == cross


@pytest.mark.parametrize("mask", [1, 2, 3, 4, 0x0F, 0x10, 0x1F])
def test_l2_nstar_is_first_spanning_prefix(nzo, mask):
    nb = l2_crossing_neighbours(mask)
    rng = np.random.default_rng(mask)
    for it in range(800):
        order = rng.permutation(32).astype(np.uint32)
        ns, ms = nzo.sweep_order(2, mask, order)
        # brute force: first prefix containing a crossing pair
        seen0, seen1, first = 0, 0, 0
        for k, s in enumerate(order.tolist()):
            if s & 1:
                seen1 |= 1 << (s >> 1)
            else:
                seen0 |= 1 << (s >> 1)
            if any((seen0 >> a) & 1 and nb[a] & seen1 for a in range(16)):
                first = k + 1
                break
        assert ns == first
        if it < 100:
            lab = lattice_np.components(2, mask, order[:ns])
            assert ms == int((lab == lab[order[ns - 1]]).sum())


@pytest.mark.parametrize("mask", [1, 3, 0x1F])
def test_l2_law_chi2(nzo, mask):
    S = l2_spanning_counts(mask)
    cdf = np.array([S[n] / comb(32, n) for n in range(33)])
    assert cdf[0] == 0 and cdf[32] == 1
    pmf = np.diff(cdf)                 # P(n* = n), n = 1..32
    count = 200_000
    ns, _ = nzo.sweep_many(2, mask, SEED, 0, count, nthreads=8)
    h = np.bincount(ns, minlength=33)[1:]
    exp = pmf * count
    keep = exp > 5
    obs = np.append(h[keep], h[~keep].sum())
    ex = np.append(exp[keep], exp[~keep].sum())
    if ex[-1] == 0:
        obs, ex = obs[:-1], ex[:-1]
    p = stats.chisquare(obs, ex).pvalue
    assert p > 1e-4, p


def test_l2_zones_6_7_vanish(nzo):
    for s in range(20):
        for m in range(1, 128):
            eff = m & 0x1F
            got = nzo.sweep(2, m, SEED, s)
            if eff == 0:
                assert got == (0, 0)
            else:
                assert got == nzo.sweep(2, eff, SEED, s)


# ---------------------------------------------------------------- snapshots
@pytest.mark.parametrize("L,masks", [(3, list(range(1, 128, 3))), (4, [1, 2, 5, 0x0F, 0x30, 0x7F]),
                                     (5, [1, 0x13, 0x7F])])
def test_snapshots_match_connected_components(nzo, L, masks):
    for mask in masks:
        order = nzo.order(L, SEED, mask)
        ns, ms = nzo.sweep_order(L, mask, order)
        assert ns > 0
        for n in sorted({1, max(1, ns // 2), ns - 1, ns}):
            lab = nzo.prefix_labels(L, mask, order, n)
            ref = lattice_np.components(L, mask, order[:n])
            assert (lab == ref).all(), (L, mask, n)
        ref_prev = lattice_np.components(L, mask, order[: ns - 1])
        ref_at = lattice_np.components(L, mask, order[:ns])
        assert not lattice_np.spans(L, ref_prev)
        assert lattice_np.spans(L, ref_at)
        assert ms == int((ref_at == ref_at[order[ns - 1]]).sum())


# ---------------------------------------------------------------- invariants
@pytest.mark.parametrize("L,mask", [(3, 1), (3, 0x7F), (4, 1), (4, 0x2A), (4, 0x7F), (5, 3)])
def test_conservation_every_step(nzo, L, mask):
    for s in range(3):
        order = nzo.order(L, SEED, s)
        nzo.sweep_order(L, mask, order, check=True, run_to_end=True)


def test_special_case_L1(nzo):
    for m in (1, 64, 127):
        assert nzo.sweep(1, m, SEED, 0) == (1, 1)


@pytest.mark.parametrize("L", [3, 4, 6])
def test_bounds(nzo, L):
    N = L**5
    for mask in (1, 2, 4, 8, 0x10, 0x20, 0x40, 0x7F, 0x41):
        reach = 2 if mask & 0x78 else 1
        ns, ms = nzo.sweep_many(L, mask, SEED, 0, 16, nthreads=8)
        lo = -(-(L - 1) // reach) + 1
        assert (ns >= ms).all() and (ms >= lo).all() and (ns <= N).all()


def test_subset_monotonicity(nzo):
    L = 5
    for s in range(3):
        order = nzo.order(L, SEED, 100 + s)
        res = {m: nzo.sweep_order(L, m, order)[0] for m in range(1, 128)}
        for a in range(1, 128):
            for b in range(1, 128):
                if a & b == a:
                    assert res[b] <= res[a], (a, b)


@pytest.mark.parametrize("L", [2, 3, 4, 5])
def test_full_lattice_spans(nzo, L):
    N = L**5
    order = np.arange(N, dtype=np.uint32)
    for m in range(1, 128):
        ns, _ = nzo.sweep_order(L, m, order)
        if L == 2 and (m & 0x1F) == 0:
            assert ns == 0
        else:
            assert ns > 0
