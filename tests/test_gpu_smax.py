"""S_max(n) windows (the observable of eqs. (5)-(6)) on the GPU against the
oracle's serial sweep run past n*, sample sums compared exactly (GPU)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,mask,seed,s0,ns,lo,hi,n0", [
    (3, 0x01, 4, 0, 40, 1, 243, -1),          # the whole lattice, n_hi = N
    (4, 0x01, 7, 3, 50, 100, 400, -1),
    (5, 0x03, 8, 0, 30, 50, 400, -1),
    (6, 0x7F, 9, 0, 20, 5, 200, -1),
    (6, 0x01, 10, 0, 16, 800, 1600, 500),     # prefilled below the window
    (8, 0x01, 11, 0, 8, 3500, 5500, 3000),
    (7, 0x0C, 12, 5, 12, 100, 900, 60),
])
def test_smax_window_matches_oracle(L, mask, seed, s0, ns, lo, hi, n0):
    import oracle
    from paper_2607_18991_amd import nz

    got = nz.nz_smax_window(L, mask, seed, s0, ns, lo, hi, n0=n0)
    want = oracle.smax_window(L, mask, seed, s0, ns, lo, hi)
    assert got.dtype == np.uint64 and (got.astype(np.int64) == want).all()
    assert (np.diff(want) >= 0).all()


def test_prefill_reaching_the_window_is_redone():
    """n0 just below the window: the count of keys below its threshold exceeds
    n_lo for about half the samples, which are redone with a halved n0."""
    import oracle
    from paper_2607_18991_amd import nz

    got = nz.nz_smax_window(6, 0x01, 13, 0, 24, 1000, 1300, n0=999)
    want = oracle.smax_window(6, 0x01, 13, 0, 24, 1000, 1300)
    assert (got.astype(np.int64) == want).all()


def test_pmax_convolution_on_gpu_sums():
    """P_max(p) of the GPU sums equals the oracle's convolution of the oracle's
    sums, and the window holds the binomial mass in the middle of the grid."""
    import oracle
    from paper_2607_18991_amd import nz

    L, mask, ns, lo, hi = 5, 0x01, 64, 300, 700
    N = L**5
    got = nz.nz_smax_window(L, mask, 21, 0, ns, lo, hi).astype(np.float64) / (ns * N)
    want = oracle.smax_window(L, mask, 21, 0, ns, lo, hi).astype(np.float64) / (ns * N)
    p = np.linspace(0.12, 0.18, 7)
    a, ca = nz.nz_convolve_window(got, lo, N, p)
    b, cb = oracle.convolve_window(want, lo, N, p)
    assert np.allclose(a, b, rtol=1e-12) and np.allclose(ca, cb, atol=1e-12)
    assert (ca[2:5] > 0.999).all()


@pytest.mark.parametrize("L,mask,seed,ns,lo,hi,n0", [
    (5, 0x01, 31, 24, 200, 700, -1),
    (6, 0x7F, 32, 16, 5, 300, -1),
    (6, 0x01, 33, 16, 900, 1500, 600),
    (8, 0x03, 34, 8, 900, 1600, 700),
    (7, 0x1C, 35, 12, 60, 500, 30),
])
def test_periodic_smax_window_matches_oracle(L, mask, seed, ns, lo, hi, n0):
    import oracle
    from paper_2607_18991_amd import nz

    got = nz.nz_smax_window(L, mask, seed, 0, ns, lo, hi, n0=n0, boundary=nz.NZ_PERIODIC)
    want = oracle.smax_window(L, mask, seed, 0, ns, lo, hi, periodic=True)
    assert (got.astype(np.int64) == want).all()
    free = oracle.smax_window(L, mask, seed, 0, ns, lo, hi)
    assert not (free == want).all()   # the boundaries do matter here


@pytest.mark.parametrize("L,mask,p", [(28, 0x01, 0.14079633), (32, 0x7F, 0.001934)])
def test_large_lattice_window_matches_oracle(L, mask, p):
    """The d_f runs' largest lattices (L = 28 and 32: 17.2 M and 33.6 M sites),
    periodic, with a bulk prefill below the window as fss.py runs them: the
    window sums of two samples equal the oracle's serial sweep run past n*."""
    import oracle
    from paper_2607_18991_amd import nz

    N = L**5
    centre = int(p * N)
    lo, hi = centre - 400, centre + 400
    n0 = int(0.9 * lo)
    got = nz.nz_smax_window(L, mask, 0xDF5 + L, 0, 2, lo, hi, n0=n0, boundary=nz.NZ_PERIODIC)
    want = oracle.smax_window(L, mask, 0xDF5 + L, 0, 2, lo, hi, periodic=True)
    assert (got.astype(np.int64) == want).all()
    assert want[-1] >= want[0] > 0
