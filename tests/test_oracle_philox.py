"""Pins of the oracle's Philox4x32-10 keys and its sort (not GPU).

The Philox block is pinned to rocRAND's implementation of the same bijection
(built on the host from ROCm's header by tests/philox_rocrand_ref.hip) and to
a second implementation written for the tests from the SC'11 definition
(tests/philox_np.py); the keys' uniformity is tested statistically and the
order's defining invariants are checked against NumPy's own lexsort.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import philox_np

_ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
_ROCRAND_HEADER = os.path.join(_ROCM, "include", "rocrand", "rocrand_philox4x32_10.h")


def _hipcc():
    return shutil.which("hipcc") or (os.path.join(_ROCM, "bin", "hipcc")
                                     if os.path.exists(os.path.join(_ROCM, "bin", "hipcc")) else None)


@pytest.mark.skipif(_hipcc() is None or not os.path.exists(_ROCRAND_HEADER), reason="hipcc or rocRAND missing")
def test_philox_block_matches_rocrand(nzo, tmp_path):
    exe = str(tmp_path / "philox_ref")
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "philox_rocrand_ref.hip")
    subprocess.run([_hipcc(), "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-O1", src, "-o", exe], check=True, capture_output=True, timeout=300)
    rng = np.random.default_rng(7)
    blocks = [np.zeros(6, dtype=np.uint64), np.full(6, 2**32 - 1, dtype=np.uint64)]
    blocks += [rng.integers(0, 2**32, size=6, dtype=np.uint64) for _ in range(500)]
    text = "".join(" ".join(f"{int(w):x}" for w in b) + "\n" for b in blocks)
    out = subprocess.run([exe], input=text, check=True, capture_output=True, text=True, timeout=60).stdout.split()
    want = np.array([int(w, 16) for w in out], dtype=np.uint64).reshape(len(blocks), 4)
    for b, w in zip(blocks, want):
        got = nzo.philox4x32_10(b[:4].astype(np.uint32), b[4:].astype(np.uint32))
        assert [int(x) for x in got] == [int(x) for x in w], b


def test_philox_block_matches_independent_numpy(nzo):
    rng = np.random.default_rng(1)
    for _ in range(200):
        ctr = rng.integers(0, 2**32, size=4, dtype=np.uint64)
        key = rng.integers(0, 2**32, size=2, dtype=np.uint64)
        got = nzo.philox4x32_10(ctr.astype(np.uint32), key.astype(np.uint32))
        want = philox_np.philox4x32_10(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1])
        assert [int(x) for x in got] == [int(w) for w in want]


@pytest.mark.parametrize("seed,sample", [(0, 0), (1, 2), (0xDEADBEEFCAFEF00D, 2**40 + 7)])
def test_site_key_layout(nzo, seed, sample):
    sites = np.arange(0, 5000, 37, dtype=np.uint64)
    want = philox_np.site_keys(seed, sample, sites)
    got = np.array([nzo.key(seed, sample, int(s)) for s in sites], dtype=np.uint64)
    assert (got == want).all()
    # the tag word is part of the counter
    assert nzo.key(seed, sample, 5, 1) != nzo.key(seed, sample, 5, 0)


def test_site_pair_shares_one_block(nzo):
    """Sites 2j and 2j+1 take words (1, 0) and (3, 2) of the block of counter j."""
    for seed, sample, j in ((3, 4, 0), (2**63 + 5, 2**33 + 1, 12345), (7, 0, 2**27 - 1)):
        w = philox_np.philox4x32_10(j, sample & 0xFFFFFFFF, sample >> 32, 0, seed & 0xFFFFFFFF, seed >> 32)
        w = [int(x) for x in w]
        assert nzo.key(seed, sample, 2 * j) == (w[1] << 32) | w[0]
        assert nzo.key(seed, sample, 2 * j + 1) == (w[3] << 32) | w[2]


def test_keys_uniform_chi2():
    k = philox_np.site_keys(1234, 0, np.arange(1 << 18, dtype=np.uint64))
    # even and odd sites (different words of the blocks) are each uniform
    for part in (k, k[0::2], k[1::2]):
        b = (part >> np.uint64(60)).astype(np.int64)
        assert stats.chisquare(np.bincount(b, minlength=16)).pvalue > 1e-4
    for shift in (60, 32, 0):
        b = ((k >> np.uint64(shift)) & np.uint64(15)).astype(np.int64)
        cnt = np.bincount(b, minlength=16)
        p = stats.chisquare(cnt).pvalue
        assert p > 1e-4, (shift, p)


def test_keys_distinct_across_samples_and_seeds():
    s = np.arange(4096, dtype=np.uint64)
    a = philox_np.site_keys(1, 0, s)
    b = philox_np.site_keys(1, 1, s)
    c = philox_np.site_keys(2, 0, s)
    assert len(set(a.tolist()) | set(b.tolist()) | set(c.tolist())) == 3 * 4096


@pytest.mark.parametrize("L,seed,sample", [(3, 5, 0), (4, 77, 9), (5, 1, 123)])
def test_order_is_lexsort_of_keys(nzo, L, seed, sample):
    N = L**5
    k = philox_np.site_keys(seed, sample, np.arange(N, dtype=np.uint64))
    want = np.lexsort((np.arange(N), k)).astype(np.uint32)
    got = nzo.order(L, seed, sample)
    assert (got == want).all()
    assert sorted(got.tolist()) == list(range(N))
    assert (np.diff(k[got].astype(np.float64)) >= 0).all() or (k[got][1:] >= k[got][:-1]).all()


def test_sort_ties_break_by_index(nzo):
    keys = np.array([7, 3, 7, 3, 0, 7, 2**64 - 1, 0], dtype=np.uint64)
    got = nzo.sort_keyed(keys)
    assert got.tolist() == [4, 7, 1, 3, 0, 2, 5, 6]
    rng = np.random.default_rng(5)
    keys = rng.integers(0, 4, size=1000).astype(np.uint64)
    got = nzo.sort_keyed(keys)
    assert (got == np.lexsort((np.arange(1000), keys))).all()
