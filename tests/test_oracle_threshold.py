"""Statistical pin of the oracle against the known nearest-neighbour threshold of
the 5D simple cubic lattice, p_c = 0.14079633 (Table I footnote for sc(5)-1).

The median of n*/N at size L approaches p_c with a finite-size correction
proportional to L^(-1/nu), nu_5 = 0.5720 (Sec. II.A.3).  A least-squares fit over
L = 6, 8, 10 must land within 0.003 of p_c.  Loose by design: the paper's own
estimate needs R = 10^6 samples per L.
"""
import numpy as np
import pytest

PC_SC5_1 = 0.14079633
NU5 = 0.5720


@pytest.mark.slow
def test_zone1_threshold_extrapolates_to_pc(nzo):
    xs, ys = [], []
    for L, count in ((6, 4000), (8, 3000), (10, 2000)):
        ns, _ = nzo.sweep_many(L, 1, 0x5EED, 0, count, nthreads=8)
        xs.append(L ** (-1.0 / NU5))
        ys.append(np.median(ns) / L**5)
    a, pc = np.polyfit(xs, ys, 1)
    assert abs(pc - PC_SC5_1) < 0.003, (pc, ys)
    assert a > 0          # free boundaries delay spanning at small L
