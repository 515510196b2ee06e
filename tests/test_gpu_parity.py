"""Bit-exact parity of the HIP path with the oracle, sample by sample (GPU).

Every case runs the C ABI on cuda:0 and the oracle on the host with the same
(seed, sample) keys.  n* and mass are integers: the bar is equality.
"""
import numpy as np
import pytest

from gpu_util import assert_same, oracle_batch, run_batch

pytestmark = pytest.mark.gpu

COMPACT = [0x01, 0x03, 0x07, 0x0F, 0x1F, 0x3F, 0x7F]


def test_plain_sweep_entry_point_L4():
    from paper_2607_18991_amd import nz
    import oracle

    ns, ms = nz.nz_sweep(4, 1, 1000, 2607)
    ons, oms = oracle.sweep_many(4, 1, 2607, 0, 1000, nthreads=8)
    assert (ns == ons).all() and (ms == oms).all()


def test_L1_and_L2_every_mask():
    jobs = [dict(L=1, zone_mask=m, seed=5, nsamples=2) for m in (1, 64, 127)]
    jobs += [dict(L=2, zone_mask=m, seed=5, nsamples=40) for m in range(1, 128)]
    gn, gm, _, _ = run_batch(jobs)
    wn, wm = oracle_batch(jobs)
    assert_same(jobs, gn, gm, wn, wm)
    # zones 6 and 7 alone never span at L = 2
    off = 6
    for m in range(1, 128):
        if m & 0x1F == 0:
            assert (gn[off:off + 40] == 0).all()
        off += 40


def test_L3_every_mask():
    jobs = [dict(L=3, zone_mask=m, seed=11, nsamples=12) for m in range(1, 128)]
    gn, gm, _, _ = run_batch(jobs)
    assert_same(jobs, gn, gm, *oracle_batch(jobs))


def test_L4_W1_shape():
    jobs = [dict(L=4, zone_mask=1, seed=2607, nsamples=1000)]
    gn, gm, _, _ = run_batch(jobs)
    assert_same(jobs, gn, gm, *oracle_batch(jobs))


@pytest.mark.parametrize("L,count", [(5, 64), (7, 24), (8, 60)])
def test_compact_masks(L, count):
    jobs = [dict(L=L, zone_mask=m, seed=0xC0FFEE + L, nsamples=count) for m in COMPACT]
    gn, gm, _, _ = run_batch(jobs)
    assert_same(jobs, gn, gm, *oracle_batch(jobs))


def test_L6_random_masks_mixed_batch():
    rng = np.random.default_rng(6)
    masks = rng.choice(np.arange(1, 128), size=24, replace=False)
    jobs = [dict(L=int(L), zone_mask=int(m), seed=77, sample0=int(1000 * k), nsamples=8)
            for k, (L, m) in enumerate(zip(rng.choice([3, 5, 6], size=24), masks))]
    gn, gm, _, _ = run_batch(jobs)
    assert_same(jobs, gn, gm, *oracle_batch(jobs))


def test_L16_sampled():
    jobs = [dict(L=16, zone_mask=m, seed=0x5EED3, sample0=0, nsamples=3) for m in COMPACT]
    gn, gm, _, _ = run_batch(jobs)
    assert_same(jobs, gn, gm, *oracle_batch(jobs))
