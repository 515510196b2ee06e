"""The threshold and fractal-dimension estimators end to end on the GPU
(Sec. II.A.1 eqs. (5)-(6); Sec. II.A.3 eq. (9) with Sec. III.C, Table II).

The windows they consume are checked against the oracle sum by sum in
test_gpu_smax.py; here the estimates themselves are checked against the values
the paper reports for sc(5)-1, with bars that the statistical error of these
short runs (a few thousand samples at L <= 24) stays well inside.  With
periodic boundaries the crossing of P_max L^(beta/nu) lands on the quoted
p_c = 0.14079633 and the slope of ln <S_max(p_c)> against ln L on Table II's
d_f = 3.5453; free boundaries give a smaller slope at these sizes, since the
largest cluster loses mass at the faces.
"""
import pytest

pytestmark = pytest.mark.gpu

PC_SC5_1 = 0.14079633  # Table I / Table II, sc(5)-1
DF_SC5_1 = 3.5453  # Table II, sc(5)-1


def test_fss_crossing_periodic_sc5_1():
    import numpy as np

    from paper_2607_18991_amd import fss, nz

    p = np.arange(0.1390, 0.1425, 0.0001)
    res = fss.estimate(0x01, [8, 12, 16], [4000, 4000, 2000], p, boundary=nz.NZ_PERIODIC)
    found = [c["p"] for c in res["crossings"]]
    assert all(x is not None for x in found), res["crossings"]
    assert abs(res["p_c"] - PC_SC5_1) < 4e-4, res["crossings"]


def test_df_periodic_and_free_sc5_1():
    from paper_2607_18991_amd import fss, nz

    Ls, S = [12, 16, 20, 24], [2000, 2000, 1000, 1000]
    per = fss.df_estimate(0x01, PC_SC5_1, Ls, S, boundary=nz.NZ_PERIODIC)
    free = fss.df_estimate(0x01, PC_SC5_1, Ls, S, boundary=nz.NZ_FREE)
    assert abs(per["d_f"] - DF_SC5_1) < 0.2, per["d_f"]
    assert free["d_f"] < per["d_f"] - 0.1, (free["d_f"], per["d_f"])
    for a, b in zip(per["runs"], free["runs"]):
        assert a["smax"] > b["smax"], (a["L"], a["smax"], b["smax"])
