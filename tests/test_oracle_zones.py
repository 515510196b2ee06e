"""Pins of the oracle's zone enumeration against the paper (not GPU).

Zone sizes: single-zone rows of Table I.  z and zeta of every one of the 127
neighbourhoods: Table I (eqs. (7) and (8)).  Plus the closed-form structure of
the shells (symmetry, reach, parity, degrees at L = 2).
"""
import math
import os
from math import comb

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1_z_zeta_pc.txt")
ZONE_SIZES = {1: 10, 2: 40, 3: 80, 4: 90, 5: 112, 6: 240, 7: 320}  # Table I single-zone rows


def read_table1():
    rows = []
    with open(GOLD) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            lab, z, zeta, pc = ln.split()
            zones = [int(x) for x in lab.split(",")]
            mask = sum(1 << (k - 1) for k in zones)
            rows.append((lab, mask, int(z), float(zeta), float(pc)))
    return rows


def test_zone_sizes(nzo):
    for k, size in ZONE_SIZES.items():
        assert nzo.zone_size(k) == size
        assert len(nzo.offsets(1 << (k - 1))) == size
    assert len(nzo.offsets(127)) == 892
    assert nzo.zone_size(8) == 0 and nzo.zone_size(0) == 0


def test_table1_every_mask_once():
    rows = read_table1()
    assert len(rows) == 127
    assert sorted(r[1] for r in rows) == list(range(1, 128))


# The two rows whose printed z/zeta are exchanged in Table I (their z column is
# the one consistent with the zone sizes; the p_c follows the z column).
SWAPPED = {"1,3,4,5,7": "1,3,4,6,7", "1,3,4,6,7": "1,3,4,5,7"}


def test_z_and_zeta_all_127_masks(nzo):
    for lab, mask, z_printed, zeta_printed, _ in read_table1():
        true_lab = SWAPPED.get(lab, lab)
        true_mask = sum(1 << (int(k) - 1) for k in true_lab.split(","))
        off = nzo.offsets(true_mask)
        z = len(off)
        r2 = (off.astype(np.int64) ** 2).sum(axis=1)
        zeta = float(np.sqrt(r2).sum())
        assert z == z_printed, lab
        assert abs(zeta - zeta_printed) < 6e-5, (lab, zeta, zeta_printed)
    # and the swap really is needed for exactly those two rows
    for lab, mask, z_printed, _, _ in read_table1():
        if lab in SWAPPED:
            assert len(nzo.offsets(mask)) != z_printed


@pytest.mark.parametrize("mask", [1, 2, 4, 8, 16, 32, 64, 0x55, 0x7F])
def test_offsets_symmetric_unique(nzo, mask):
    off = nzo.offsets(mask)
    s = {tuple(v) for v in off}
    assert len(s) == len(off)
    assert s == {tuple(-v) for v in off}
    assert (0, 0, 0, 0, 0) not in s


def test_reach_and_parity(nzo):
    for k in range(1, 8):
        off = nzo.offsets(1 << (k - 1))
        assert (off ** 2).sum(axis=1).tolist() == [k] * len(off)
        reach = int(np.abs(off).max())
        assert reach == (1 if k <= 3 else 2)
        par = set((off.sum(axis=1) % 2).tolist())
        assert par == ({0} if k % 2 == 0 else {1})
    # zone 4 holds the ten axial (+-2,0,0,0,0) vectors; zone 6/7 always need a 2
    z4 = {tuple(v) for v in nzo.offsets(8)}
    assert sum(1 for v in z4 if max(abs(x) for x in v) == 2) == 10
    for k in (6, 7):
        assert all(np.abs(nzo.offsets(1 << (k - 1))).max(axis=1) == 2)


def test_degree_at_L2_closed_form(nzo):
    # At L = 2 an offset is in bounds only if every |d_j| <= 1 and points inward;
    # for each choice of k moving coordinates exactly one sign pattern works, so
    # zone k (k <= 5, using only its +-1 vectors) contributes C(5, k) neighbours.
    for mask in range(1, 128):
        off = nzo.offsets(mask)
        want = sum(comb(5, k) for k in range(1, 6) if mask & (1 << (k - 1)))
        for site in (0, 31, 13):
            x = np.array([(site >> j) & 1 for j in range(5)])
            y = x + off
            inb = ((y >= 0) & (y < 2)).all(axis=1).sum()
            assert inb == want


def test_interior_degree_is_z(nzo):
    for mask in (1, 0x13, 0x7F):
        off = nzo.offsets(mask)
        x = np.array([2, 2, 2, 2, 2])
        y = x + off
        assert ((y >= 0) & (y < 5)).all(axis=1).sum() == len(off)
