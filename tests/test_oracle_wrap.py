"""Pins of the oracle's first-wrapping sweep on the periodic lattice (Newman &
Ziff 2001, Sec. III: a cluster wraps around axis 0 when it holds a loop whose
unwrapped x0 displacement is a non-zero multiple of L).

The oracle tracks each site's x0 displacement from its parent inside the
union-find; these tests check it against loops of known winding built by hand
and against a breadth-first search that unwraps every cluster from scratch
(tests/lattice_np.py), which shares nothing with the union-find."""
import numpy as np
import pytest

import lattice_np


def site(L, x):
    return int(sum(int(c) % L * L**j for j, c in enumerate(x)))


def test_line_along_axis0_wraps_when_it_closes(nzo):
    L = 6
    line = [site(L, (k, 0, 0, 0, 0)) for k in range(L)]
    assert nzo.sweep_order(L, 0x01, line, periodic=True) == (L, L)
    # one site short: an open path, no loop
    assert nzo.sweep_order(L, 0x01, line[:-1], periodic=True) == (0, 0)
    # the same line built from both ends towards the middle
    mixed = [line[i] for i in (0, 5, 1, 4, 3, 2)]
    assert nzo.sweep_order(L, 0x01, mixed, periodic=True) == (L, L)


def test_line_along_other_axes_does_not_wrap_axis0(nzo):
    L = 5
    for ax in range(1, 5):
        line = []
        for k in range(L):
            x = [0] * 5
            x[ax] = k
            line.append(site(L, x))
        assert nzo.sweep_order(L, 0x01, line, periodic=True) == (0, 0), ax
        assert lattice_np.first_wrap(L, 0x01, line) == (0, 0)


def test_diagonal_helix_wraps(nzo):
    """(k, k, 0, 0, 0), k < L, linked by the zone-2 vector (1, 1, 0, 0, 0): the
    loop winds once around axes 0 and 1."""
    L = 7
    helix = [site(L, (k, k, 0, 0, 0)) for k in range(L)]
    assert nzo.sweep_order(L, 0x02, helix, periodic=True) == (L, L)
    # (k, -k): the same with the other diagonal
    anti = [site(L, (k, -k, 0, 0, 0)) for k in range(L)]
    assert nzo.sweep_order(L, 0x02, anti, periodic=True) == (L, L)


def test_double_winding(nzo):
    """Zone 4 holds (2, 0, 0, 0, 0).  On L = 5 the sites x0 = 0, 2, 4, 1, 3 close
    a loop of unwrapped length 10 = 2L (winding 2) at the fifth site; on L = 6
    the sites 0, 2, 4 close one of length 6 (winding 1) at the third."""
    assert nzo.sweep_order(5, 0x08, [site(5, (x, 0, 0, 0, 0)) for x in (0, 2, 4, 1, 3)],
                           periodic=True) == (5, 5)
    assert nzo.sweep_order(6, 0x08, [site(6, (x, 0, 0, 0, 0)) for x in (0, 2, 4)], periodic=True) == (3, 3)


def test_contractible_loop_does_not_wrap(nzo):
    L = 5
    square = [site(L, x) for x in ((0, 0, 0, 0, 0), (1, 0, 0, 0, 0), (1, 1, 0, 0, 0), (0, 1, 0, 0, 0))]
    assert nzo.sweep_order(L, 0x01, square, periodic=True) == (0, 0)
    # a ring that crosses the x0 = 0 face and comes back the way it went
    ring = [site(L, x) for x in ((4, 0, 0, 0, 0), (0, 0, 0, 0, 0), (0, 1, 0, 0, 0), (4, 1, 0, 0, 0))]
    assert nzo.sweep_order(L, 0x01, ring, periodic=True) == (0, 0)


def test_mass_counts_what_the_closing_site_joins(nzo):
    """A line along axis 0 missing one site, plus a side branch: the closing
    site merges both and the wrapping cluster's mass includes the branch."""
    L = 5
    line = [site(L, (k, 0, 0, 0, 0)) for k in range(L)]
    branch = [site(L, (2, 1, 0, 0, 0)), site(L, (2, 2, 0, 0, 0))]
    order = line[:2] + line[3:] + branch + [line[2]]
    assert nzo.sweep_order(L, 0x01, order, periodic=True) == (len(order), len(order))


@pytest.mark.parametrize("L,mask,sample", [(5, 0x01, 0), (5, 0x01, 1), (5, 0x02, 2), (5, 0x03, 3),
                                           (6, 0x01, 4), (5, 0x08, 5), (5, 0x05, 6), (6, 0x04, 7)])
def test_first_wrap_matches_bfs(nzo, L, mask, sample):
    o = nzo.order(L, 0xA11CE, sample)
    assert nzo.sweep_order(L, mask, o, periodic=True, check=True) == lattice_np.first_wrap(L, mask, o)


def test_wrap_translation_invariant(nzo):
    """The torus is translation invariant: shifting every site of the order by a
    fixed vector keeps n* and the mass."""
    L, mask = 8, 0x03
    o = nzo.order(L, 0xBEE, 0)
    x = lattice_np.coords(L, o)
    t = (np.mod(x + np.array([3, 5, 1, 7, 2]), L) * (L ** np.arange(5))).sum(axis=1)
    a = nzo.sweep_order(L, mask, o, periodic=True)
    b = nzo.sweep_order(L, mask, t.astype(np.uint32), periodic=True)
    assert a == b and a[0] > 0


def test_wrap_never_later_than_span_on_reflection(nzo):
    """Wrapping is defined on the torus and spanning between free faces, so no
    order can be compared site for site; but both thresholds are close to p_c
    for large L.  On L = 12, mask 0x01, the mean n*/N of either lies within a
    few percent of p_c = 0.1408 (Table I)."""
    L, mask = 12, 0x01
    N = L**5
    w, _ = nzo.sweep_many(L, mask, 0xC0DE, 0, 24, nthreads=8, periodic=True)
    f, _ = nzo.sweep_many(L, mask, 0xC0DE, 0, 24, nthreads=8)
    assert (w > 0).all() and (f > 0).all()
    assert abs(w.mean() / N - 0.1408) < 0.01 and abs(f.mean() / N - 0.1408) < 0.015


def test_periodic_rejects_small_L(nzo):
    with pytest.raises(Exception):
        nzo.sweep_order(4, 0x01, [0, 1, 2], periodic=True)
