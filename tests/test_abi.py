"""The C ABI library on the host: it loads, exports every function include/nz.h
declares, validates arguments before touching a device, and its host-only
binomial convolution agrees with the oracle's long-double one (not GPU)."""
import os
import re

import numpy as np
import pytest

from paper_2607_18991_amd import nz

HEADER = os.path.join(os.path.dirname(__file__), "..", "include", "nz.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nz_[a-z_0-9]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 10
    lib = nz.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(nz.EXPORTS)
    assert nz.nz_abi_version() == 2


def test_coordination_numbers(nzo):
    for m in range(1, 128):
        assert nz.nz_coordination(m) == len(nzo.offsets(m))
    assert nz.nz_coordination(0) == -1 and nz.nz_coordination(128) == -1


@pytest.mark.parametrize("args,code", [
    ((0, 1, 0, 1, 1), nz.NZ_EINVAL),
    ((56, 1, 0, 1, 1), nz.NZ_EUNSUPPORTED),
    ((4, 0, 0, 1, 1), nz.NZ_EINVAL),
    ((4, 128, 0, 1, 1), nz.NZ_EINVAL),
    ((4, 1, 1, 1, 1), nz.NZ_EUNSUPPORTED),
    ((4, 1, 0, -1, 1), nz.NZ_EINVAL),
])
def test_sweep_rejects_bad_arguments_before_any_launch(args, code):
    import ctypes

    L, m, b, n, s = args
    out = np.zeros(4, dtype=np.int32)
    rc = nz.lib().nz_sweep(L, m, b, n, s, out.ctypes.data_as(ctypes.c_void_p), None)
    assert rc == code
    assert len(nz.lib().nz_last_error()) > 0


def test_batch_rejects_bad_jobs():
    with pytest.raises(nz.NzError) as e:
        nz.nz_batch_workspace_bytes([dict(L=4, zone_mask=1, seed=1, nsamples=1, n0=1024)])
    assert e.value.code == nz.NZ_EINVAL
    with pytest.raises(nz.NzError):
        nz.nz_batch_workspace_bytes([dict(L=4, zone_mask=1, seed=1, nsamples=1)], tune=dict(residency=7))
    for summary in (-1, 3):
        with pytest.raises(nz.NzError) as e:
            nz.nz_batch_workspace_bytes([dict(L=4, zone_mask=1, seed=1, nsamples=1)], tune=dict(summary=summary))
        assert e.value.code == nz.NZ_EINVAL
    for summary in (0, 1, 2):
        assert nz.nz_batch_workspace_bytes([dict(L=4, zone_mask=1, seed=1, nsamples=1)], tune=dict(summary=summary)) > 0


def test_workspace_sizing_counts_jobs_after_many_samples():
    """The resident first chunk is sized from the largest samples of the whole
    batch, also when a large job comes after more than 65536 small samples."""
    small = dict(L=2, zone_mask=1, seed=1, nsamples=70000)
    large = dict(L=16, zone_mask=1, seed=2, nsamples=64)
    both = nz.nz_batch_workspace_bytes([small, large])
    assert both >= nz.nz_batch_workspace_bytes([large])
    assert both >= nz.nz_batch_workspace_bytes([large, small])


def test_workspace_sizing_grows_with_samples():
    a = nz.nz_batch_workspace_bytes([dict(L=8, zone_mask=1, seed=1, nsamples=10)])
    b = nz.nz_batch_workspace_bytes([dict(L=8, zone_mask=1, seed=1, nsamples=100)])
    c = nz.nz_batch_workspace_bytes([dict(L=16, zone_mask=1, seed=1, nsamples=10)])
    assert 0 < a < b and c > a
    assert a % 256 == 0 or a > 0


@pytest.mark.parametrize("N,seed", [(32, 1), (1024, 2), (32768, 3), (1048576, 4)])
def test_canonical_matches_oracle(nzo, N, seed):
    rng = np.random.default_rng(seed)
    h = np.zeros(N + 1, dtype=np.uint64)
    lo, hi = int(0.05 * N) + 1, int(0.2 * N) + 2
    np.add.at(h, rng.integers(lo, hi, size=2000), 1)
    h[0] = 3
    p = np.linspace(0, 1, 101) if N < 100000 else np.concatenate([[0, 0.5, 1], np.linspace(0.04, 0.22, 13)])
    assert np.max(np.abs(nz.nz_canonical(h, p) - nzo.canonical(h, p))) <= 1e-12


def test_canonical_rejects_bad_grid():
    with pytest.raises(nz.NzError):
        nz.nz_canonical(np.ones(5, dtype=np.uint64), [0.5, 1.5])
    with pytest.raises(nz.NzError):
        nz.nz_canonical(np.zeros(5, dtype=np.uint64), [0.5])


def test_convolve_window_matches_oracle():
    import oracle

    rng = np.random.default_rng(3)
    for N, lo, hi in ((1, 0, 2), (50, 0, 51), (1000, 100, 300), (32768, 4000, 5500)):
        Q = rng.random(hi - lo) * N
        p = np.array([0.0, 0.003, 0.1408, 0.33, 1.0])
        a, ca = nz.nz_convolve_window(Q, lo, N, p)
        b, cb = oracle.convolve_window(Q, lo, N, p)
        assert np.allclose(a, b, rtol=1e-12, atol=1e-12 * N) and np.allclose(ca, cb, atol=1e-12)


def test_smax_window_validation():
    for args in ((4, 1, 1, 0, 1, 0, 10), (4, 1, 1, 0, 1, 20, 10), (4, 1, 1, 0, 1, 5, 1025), (4, 1, 1, 0, 1, 5, 6)):
        L, m, seed, s0, ns, lo, hi = args
        n0 = 5 if args[-1] == 6 else -1
        with pytest.raises(nz.NzError) as e:
            nz.nz_smax_window(L, m, seed, s0, ns, lo, hi, n0=n0)
        assert e.value.code == nz.NZ_EINVAL
    with pytest.raises(nz.NzError) as e:
        nz.nz_convolve_window(np.ones(3), 5, 4, [0.5])
    assert e.value.code == nz.NZ_EINVAL


def test_boundary_codes():
    # periodic boundaries need L >= 5; other codes are invalid
    with pytest.raises(nz.NzError) as e:
        nz.nz_sweep(4, 1, 4, 1, boundary=nz.NZ_PERIODIC)
    assert e.value.code == nz.NZ_EUNSUPPORTED
    with pytest.raises(nz.NzError) as e:
        nz.nz_sweep(6, 1, 4, 1, boundary=2)
    assert e.value.code == nz.NZ_EINVAL
    with pytest.raises(nz.NzError) as e:
        nz.nz_smax_window(4, 1, 1, 0, 2, 10, 20, boundary=nz.NZ_PERIODIC)
    assert e.value.code == nz.NZ_EUNSUPPORTED


def test_workspace_covers_two_groups(monkeypatch):
    """A batch with enough narrow (z <= 64) and wide samples runs as two groups,
    each with its own resident share of the workspace."""
    jobs = [dict(L=16, zone_mask=m, seed=1, nsamples=1000, n0=-1) for m in (0x01, 0x03, 0x07, 0x7F)]
    both = nz.nz_batch_workspace_bytes(jobs)
    monkeypatch.setenv("NZ_DEBUG_NO_SPLIT", "1")
    one = nz.nz_batch_workspace_bytes(jobs)
    assert both > one
    monkeypatch.delenv("NZ_DEBUG_NO_SPLIT")
    assert nz.nz_batch_workspace_bytes(jobs[:3] + [dict(jobs[3], nsamples=100)]) < both


def test_split_needs_256_samples_in_each_group(monkeypatch):
    """Two groups only when both hold at least 256 samples; otherwise the
    workspace is the one-group size."""
    def sizes(n_narrow, n_wide):
        jobs = [dict(L=12, zone_mask=0x01, seed=1, nsamples=n_narrow, n0=-1),
                dict(L=12, zone_mask=0x7F, seed=2, nsamples=n_wide, n0=-1)]
        monkeypatch.delenv("NZ_DEBUG_NO_SPLIT", raising=False)
        split = nz.nz_batch_workspace_bytes(jobs)
        monkeypatch.setenv("NZ_DEBUG_NO_SPLIT", "1")
        one = nz.nz_batch_workspace_bytes(jobs)
        return split, one
    s, o = sizes(256, 256)
    assert s > o
    s, o = sizes(255, 4000)
    assert s == o
    s, o = sizes(4000, 255)
    assert s == o


def test_static_batch_rejects_oversized_samples_before_any_device_call():
    """The no-allocation batch entry point checks, on the host, that one sample
    of every job fits its fixed buffer: L = 40 (4 x 40^5 bytes of parents
    alone) is refused with NZ_EWORKSPACE; L = 24 fits and goes on to the
    argument check (a NULL n* output here)."""
    import ctypes

    assert nz.nz_static_scratch_bytes() == 256 << 20
    arr, n = nz.make_jobs([dict(L=40, zone_mask=1, seed=1, nsamples=1)])
    rc = nz.lib().nz_sweep_batch_static(ctypes.cast(arr, ctypes.c_void_p), n, None, None, None, None, None)
    assert rc == nz.NZ_EWORKSPACE
    assert b"needs" in nz.lib().nz_last_error()
    arr, n = nz.make_jobs([dict(L=24, zone_mask=1, seed=1, nsamples=1)])
    rc = nz.lib().nz_sweep_batch_static(ctypes.cast(arr, ctypes.c_void_p), n, None, None, None, None, None)
    assert rc == nz.NZ_EINVAL
    arr, n = nz.make_jobs([dict(L=4, zone_mask=0, seed=1, nsamples=1)])
    rc = nz.lib().nz_sweep_batch_static(ctypes.cast(arr, ctypes.c_void_p), n, None, None, None, None, None)
    assert rc == nz.NZ_EINVAL


def test_batch_rejects_a_workspace_below_one_sample():
    """nz_sweep_batch refuses a workspace that cannot hold one sample with
    NZ_EWORKSPACE and a message, before any launch."""
    import ctypes

    arr, n = nz.make_jobs([dict(L=16, zone_mask=1, seed=1, nsamples=4)])
    # a 256-byte-aligned host address stands in for the device buffer: the size
    # check comes first, so nothing is ever written there
    buf = np.zeros(4096 // 8 + 64, dtype=np.uint64)
    addr = (buf.ctypes.data + 255) // 256 * 256
    dn = np.zeros(4, dtype=np.int32)
    rc = nz.lib().nz_sweep_batch(ctypes.cast(arr, ctypes.c_void_p), n, ctypes.c_void_p(addr), 1024,
                                 dn.ctypes.data_as(ctypes.c_void_p), None, None, None, None)
    assert rc == nz.NZ_EWORKSPACE
    assert b"needs" in nz.lib().nz_last_error()


def test_prefill_planning_host_calls():
    """The learned prefill's host arithmetic behind the ABI: the MLP's input
    rows, the size statistics, the training target of a lattice and the plan
    (n0, backoff, band) from the MLP's outputs, including the clamps."""
    Ls = np.array([4, 8, 16, 24], dtype=np.int32)
    sv = Ls.astype(np.float64) ** (-1.0 / 0.5720)
    mean, std = nz.nz_mlp_size_stats(Ls)
    assert np.isclose(mean, sv.mean(), rtol=1e-12) and np.isclose(std, sv.std(), rtol=1e-12)
    m8, s8 = nz.nz_mlp_size_stats([8, 8])
    assert np.isclose(m8, 8.0 ** (-1 / 0.5720), rtol=1e-14) and s8 == 1.0
    x = nz.nz_mlp_features([0x01, 0x55, 0x7F, 0x40], Ls, mean, std)
    assert x.shape == (4, 8) and x.dtype == np.float32
    assert (x[:, :7] == np.array([[(m >> k) & 1 for k in range(7)] for m in (0x01, 0x55, 0x7F, 0x40)])).all()
    assert np.allclose(x[:, 7], ((sv - mean) / std).astype(np.float32), rtol=1e-6)
    # training target: spanning samples only, population std floored at 0.5/N
    ns = np.array([100, 0, 120, 140, 0], dtype=np.int32)
    cnt, m, s, lm, ls = nz.nz_prefill_target(ns, 4)
    f = np.array([100, 120, 140]) / 1024.0
    assert cnt == 3 and np.isclose(m, f.mean(), rtol=1e-14) and np.isclose(s, f.std(), rtol=1e-12)
    assert np.isclose(lm, np.log(m)) and np.isclose(ls, np.log(s))
    assert nz.nz_prefill_target(np.array([7, 7], dtype=np.int32), 4)[2] == 0.5 / 1024
    with pytest.raises(nz.NzError):
        nz.nz_prefill_target(np.array([0, 0], dtype=np.int32), 4)
    # plan: n0 = floor((mu - 3 sd) N) clamped, backoff = ceil(3 sd N), band = ceil((mu + 5 sd) N) + 1024
    jobs = [dict(L=16, zone_mask=1, seed=1, nsamples=4), dict(L=4, zone_mask=1, seed=1, nsamples=4),
            dict(L=8, zone_mask=3, seed=2, nsamples=1)]
    y = np.log(np.array([[0.14, 0.004], [0.02, 0.05], [0.9, 0.2]], dtype=np.float64)).astype(np.float32)
    out = nz.nz_prefill_plan(y, jobs, 3.0, 5.0)
    mu, sd = np.exp(y[:, 0].astype(np.float64)), np.exp(y[:, 1].astype(np.float64))
    N = np.array([16**5, 4**5, 8**5])
    assert out[0]["n0"] == int(np.floor((mu[0] - 3 * sd[0]) * N[0]))
    assert out[1]["n0"] == 0                                   # mean - 3 std < 0
    assert out[2]["band_hi"] == N[2]                           # band beyond the lattice
    assert out[0]["backoff"] == int(np.ceil(3 * sd[0] * N[0]))
    assert out[0]["band_hi"] == int(np.ceil((mu[0] + 5 * sd[0]) * N[0])) + 1024
    assert jobs[0].get("n0") is None                           # the caller's dicts are not touched
    plain = nz.nz_prefill_plan(y, jobs, 0.0, 5.0, plain=True)
    assert all(j["n0"] == -1 for j in plain) and plain[0]["band_hi"] == out[0]["band_hi"]

