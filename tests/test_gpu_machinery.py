"""The machinery around the sweep, on the GPU, against the oracle: the learned
prefill (bulk connected components then the sequential sweep) including forced
backoff, the redo of samples whose key band, sort bucket or prefill list ran
short, every tuning knob, chunking through a small workspace, and run-to-run
determinism.  None of these may change any n* or mass."""
import os

import numpy as np
import pytest

from gpu_util import assert_same, oracle_batch, run_batch

pytestmark = pytest.mark.gpu

COMPACT = [0x01, 0x03, 0x07, 0x0F, 0x1F, 0x3F, 0x7F]


class env:
    def __init__(self, **kv):
        self.kv = kv

    def __enter__(self):
        for k, v in self.kv.items():
            os.environ[k] = str(v)

    def __exit__(self, *a):
        for k in self.kv:
            os.environ.pop(k, None)


def typical_nstar(L, mask, samples=16):
    import oracle

    ns, _ = oracle.sweep_many(L, mask, 999, 0, samples, nthreads=8)
    return int(np.median(ns)), int(max(1, ns.std()))


@pytest.mark.parametrize("L", [6, 8])
def test_prefill_exact(L):
    jobs = []
    for m in COMPACT:
        med, sd = typical_nstar(L, m)
        jobs.append(dict(L=L, zone_mask=m, seed=4242 + L, nsamples=48, n0=max(1, med - 2 * sd), backoff=2 * sd))
    gn, gm, back, stats = run_batch(jobs)
    assert_same(jobs, gn, gm, *oracle_batch(jobs))
    assert stats["backoffs"] == int(back.sum())


@pytest.mark.parametrize("tune", [dict(residency=1), dict(residency=3), dict(sweep_mode=1),
                                  dict(sweep_mode=2, residency=3), dict(sweep_mode=1, residency=3)])
def test_prefill_every_residency(tune):
    """Prefilled sites enter the sweep as list nodes of the bulk labelling's
    forest: with the bitset, or bitset and parents, in LDS and with either
    step shape, results equal the oracle's."""
    L = 6
    jobs = []
    for m in (0x01, 0x07, 0x7F):
        med, sd = typical_nstar(L, m)
        jobs.append(dict(L=L, zone_mask=m, seed=5150, nsamples=24, n0=max(1, med - 2 * sd), backoff=2 * sd))
    gn, gm, _, _ = run_batch(jobs, tune=tune)
    assert_same(jobs, gn, gm, *oracle_batch(jobs))


def test_prefill_exact_thresholds():
    """With the prefill thresholds left unrounded (test hook), the keys kernel
    classifies sites by full 64-bit compares; results equal the oracle's."""
    L = 8
    jobs = []
    for m in (0x01, 0x0F, 0x7F):
        med, sd = typical_nstar(L, m)
        jobs.append(dict(L=L, zone_mask=m, seed=6161, nsamples=24, n0=max(1, med - 2 * sd), backoff=2 * sd))
    with env(NZ_DEBUG_EXACT_T0=1):
        gn, gm, back, stats = run_batch(jobs)
    assert_same(jobs, gn, gm, *oracle_batch(jobs))
    assert stats["prefilled_sites"] > 0


def test_forced_backoff():
    L = 6
    N = L**5
    jobs = [dict(L=L, zone_mask=m, seed=17, nsamples=24, n0=N - 1, backoff=N // 2) for m in (1, 0x0F, 0x7F)]
    gn, gm, back, stats = run_batch(jobs)
    assert_same(jobs, gn, gm, *oracle_batch(jobs))
    # every sample spans at N-1, so each backs off at least once
    assert (back >= 24).all()


def test_band_redo():
    jobs = [dict(L=7, zone_mask=m, seed=5, nsamples=16, band_hi=2) for m in (1, 0x3F)]
    gn, gm, _, stats = run_batch(jobs)
    assert_same(jobs, gn, gm, *oracle_batch(jobs))
    # a 2-site band still rounds up to one bucket of ~256 keys: only the
    # zone-1 samples (n* in the thousands) outrun it
    assert stats["band_redo"] >= 16


def test_bucket_redo():
    from paper_2607_18991_amd import nz

    jobs = [dict(L=5, zone_mask=m, seed=6, nsamples=12) for m in (1, 0x7F)]
    with env(NZ_DEBUG_BUCKET_CAP=8):
        # a pinned capacity makes every redo double the bucket count, so give
        # the redone samples room (with the default capacity memory stays flat)
        gn, gm, _, stats = run_batch(jobs, ws_bytes=64 * nz.nz_batch_workspace_bytes(jobs))
    assert_same(jobs, gn, gm, *oracle_batch(jobs))
    assert stats["bucket_redo"] > 0


def test_prefix_list_redo():
    jobs = [dict(L=6, zone_mask=0x03, seed=8, nsamples=12, n0=300, backoff=100)]
    with env(NZ_DEBUG_PREFIX_CAP=4):
        gn, gm, _, _ = run_batch(jobs)
    assert_same(jobs, gn, gm, *oracle_batch(jobs))


@pytest.mark.parametrize("tune", [
    dict(residency=1), dict(residency=3), dict(residency=2, wg_waves=1), dict(wg_waves=2, waves_per_simd=2),
    dict(wg_waves=3), dict(bucket_log2=4), dict(bucket_log2=10), dict(residency=1, wg_waves=2),
    dict(sweep_mode=1), dict(sweep_mode=2), dict(sweep_mode=1, residency=1), dict(sweep_mode=1, residency=3),
    dict(sweep_mode=2, residency=3), dict(sweep_mode=2, residency=1, wg_waves=4),
    dict(summary=1), dict(summary=2), dict(summary=1, sweep_mode=1), dict(summary=1, sweep_mode=2, wg_waves=4),
    dict(summary=2, sweep_mode=2),
])
def test_tuning_never_changes_results(tune):
    jobs = [dict(L=L, zone_mask=m, seed=99, nsamples=10) for L in (4, 6, 8) for m in (1, 0x07, 0x7F)]
    gn, gm, _, _ = run_batch(jobs, tune=tune)
    assert_same(jobs, gn, gm, *oracle_batch(jobs))


def test_early_merge_path():
    jobs = [dict(L=L, zone_mask=m, seed=31, nsamples=12) for L in (5, 8) for m in (0x7F, 0x3C, 0x61)]
    with env(NZ_DEBUG_DCAP=2):
        gn, gm, _, _ = run_batch(jobs)
    assert_same(jobs, gn, gm, *oracle_batch(jobs))


@pytest.mark.parametrize("cap", [0, 3])
@pytest.mark.parametrize("residency", [0, 1])
def test_block_fallback_path(cap, residency):
    """Blocks that touch more earlier roots than allowed are redone one site at
    a time; plain and prefilled samples, sparse and dense neighbourhoods."""
    jobs = [dict(L=L, zone_mask=m, seed=47, nsamples=10) for L in (5, 8) for m in (1, 0x0C, 0x7F)]
    jobs += [dict(L=8, zone_mask=m, seed=48, nsamples=10, n0=n0, backoff=200) for m, n0 in ((1, 3000), (0x03, 900))]
    with env(NZ_DEBUG_BLOCK_OLD=cap):
        gn, gm, _, _ = run_batch(jobs, tune=dict(sweep_mode=2, residency=residency))
    assert_same(jobs, gn, gm, *oracle_batch(jobs))


@pytest.mark.parametrize("tune", [dict(), dict(sweep_mode=1), dict(residency=1), dict(sweep_mode=2, residency=1)])
def test_workspace_bytes_written_before_read(tune):
    """Every workspace byte a kernel reads was written earlier in the same
    batch: with the workspace set to 0xFF bytes first (a parent entry of -1
    would read as a spanning root, a list position of 2^32 - 1 would leave the
    forest), results still equal the oracle's.  L = 9 gives each sample eight
    ranges of the keys kernel, so the sparse prefills of the wide
    neighbourhoods leave whole ranges without a prefilled site; plain,
    prefilled and periodic first-wrap samples run together."""
    import oracle
    from paper_2607_18991_amd import nz

    L = 9
    jobs = []
    for m in (0x01, 0x07, 0x7F, 0x48):
        med, sd = typical_nstar(L, m)
        jobs.append(dict(L=L, zone_mask=m, seed=777, nsamples=16, n0=max(1, med - 2 * sd), backoff=2 * sd))
    jobs.append(dict(L=L, zone_mask=0x03, seed=778, nsamples=16))
    ns, _ = oracle.sweep_many(L, 0x03, 999, 0, 16, nthreads=8, periodic=True)
    med, sd = int(np.median(ns)), int(max(1, ns.std()))
    jobs.append(dict(L=L, zone_mask=0x03, seed=779, nsamples=16, n0=max(1, med - 2 * sd), backoff=2 * sd,
                     boundary=nz.NZ_PERIODIC))
    gn, gm, _, _ = run_batch(jobs, tune=tune, fill=0xFF)
    assert_same(jobs, gn, gm, *oracle_batch(jobs))


@pytest.mark.parametrize("L", [9, 12])
def test_block_matches_single_site(L):
    """The 64-site block sweep and the one-site sweep agree sample by sample on
    prefilled runs of every compact neighbourhood (no oracle: too large)."""
    from paper_2607_18991_amd import learned

    model = learned.PrefillModel.load()
    jobs = [dict(L=L, zone_mask=m, seed=1200 + L, nsamples=24) for m in COMPACT]
    jobs = model.plan(jobs)
    a = run_batch(jobs, tune=dict(sweep_mode=1))
    b = run_batch(jobs, tune=dict(sweep_mode=2))
    assert (a[0] == b[0]).all() and (a[1] == b[1]).all()
    assert (a[0] > 0).all()


def test_sized_workspace_holds_prefilled_batch_in_one_chunk():
    """The workspace size reported for jobs with a prefill and a backoff step
    also holds the backed-off key band, so the batch needs no second chunk."""
    jobs = [dict(L=8, zone_mask=m, seed=61, nsamples=40, n0=n0, backoff=bo, band_hi=8**5)
            for m, n0, bo in ((1, 1000, 500), (0x07, 150, 60), (0x7F, 15, 10))]
    gn, gm, _, stats = run_batch(jobs)
    assert_same(jobs, gn, gm, *oracle_batch(jobs))
    assert stats["backoffs"] == 0 and stats["band_redo"] == 0 and stats["bucket_redo"] == 0
    assert stats["chunks"] == 1


def test_small_workspace_chunks():
    from paper_2607_18991_amd import nz

    jobs = [dict(L=6, zone_mask=m, seed=3, nsamples=20) for m in COMPACT]
    one = nz.nz_batch_workspace_bytes([dict(L=6, zone_mask=0x7F, seed=3, nsamples=1)])
    gn, gm, _, stats = run_batch(jobs, ws_bytes=3 * one)
    assert stats["chunks"] > 3
    assert_same(jobs, gn, gm, *oracle_batch(jobs))


def test_deterministic_across_runs():
    jobs = [dict(L=8, zone_mask=m, seed=12, nsamples=32) for m in (1, 0x7F)]
    a = run_batch(jobs)
    b = run_batch(jobs, tune=dict(residency=1))
    assert (a[0] == b[0]).all() and (a[1] == b[1]).all()


def test_sample_offsets_resume():
    # a range split in two (sample0) equals the whole range: the unit of recovery
    whole = [dict(L=6, zone_mask=0x05, seed=77, nsamples=40)]
    parts = [dict(L=6, zone_mask=0x05, seed=77, nsamples=15), dict(L=6, zone_mask=0x05, seed=77, sample0=15, nsamples=25)]
    a = run_batch(whole)
    b = run_batch(parts)
    assert (a[0] == b[0]).all() and (a[1] == b[1]).all()


def test_L24_sampled():
    jobs = [dict(L=24, zone_mask=m, seed=0x5EED5, nsamples=1) for m in (0x7F, 0x1F)]
    gn, gm, _, _ = run_batch(jobs)
    assert_same(jobs, gn, gm, *oracle_batch(jobs))


def test_autotune_class_keeps_outputs():
    """Timing every candidate of a class checks each against the default's
    outputs (tune_class raises on a difference) and keeps the fastest."""
    from paper_2607_18991_amd import autotune

    e = autotune.tune_class(5, 64, 16)
    assert e["ms"] <= e["default_ms"]
    assert any("ms" in t for t in e["tried"])


def test_shipped_tuning_reproduces_oracle():
    from paper_2607_18991_amd import autotune

    for L in (4, 8):
        for m in (0x01, 0x04, 0x07, 0x1F, 0x7F):
            jobs = [dict(L=L, zone_mask=m, seed=515, nsamples=8)]
            gn, gm, _, _ = run_batch(jobs, tune=autotune.lookup(L, m) or None)
            assert_same(jobs, gn, gm, *oracle_batch(jobs))


@pytest.mark.parametrize("count", [20, 300])
def test_zero_sample_job_between_others(count):
    # 300 samples a side take the two-group path (narrow and wide masks side
    # by side); outputs stay in job order across the empty job
    jobs = [dict(L=6, zone_mask=0x01, seed=71, nsamples=count),
            dict(L=8, zone_mask=0x03, seed=72, nsamples=0),
            dict(L=6, zone_mask=0x7F, seed=73, nsamples=count // 2 + 150)]
    gn, gm, back, _ = run_batch(jobs)
    assert len(gn) == sum(j["nsamples"] for j in jobs) and len(back) == 3
    assert back[1] == 0
    assert_same(jobs, gn, gm, *oracle_batch(jobs))


def test_empty_inputs():
    import torch

    from paper_2607_18991_amd import nz

    ns, ms = nz.nz_sweep(8, 0x01, 0, 5)
    assert ns.size == 0 and ms.size == 0
    gn, gm, back, _ = run_batch([])
    assert gn.size == 0 and back.size == 0
    # a batch with no samples leaves the outputs as they were
    jobs = [dict(L=8, zone_mask=0x01, seed=1, nsamples=0), dict(L=6, zone_mask=0x7F, seed=2, nsamples=0)]
    ws = torch.empty(nz.nz_batch_workspace_bytes(jobs), dtype=torch.uint8, device="cuda")
    dn = torch.full((4,), -7, dtype=torch.int32, device="cuda")
    dm = torch.full((4,), -7, dtype=torch.int32, device="cuda")
    back = nz.nz_sweep_batch(jobs, ws, dn, dm)
    torch.cuda.synchronize()
    assert (back == 0).all()
    assert (dn.cpu() == -7).all() and (dm.cpu() == -7).all()


def test_shared_seed_jobs_mixed_members():
    """Jobs that share seed, sample indices and L (the same occupation orders):
    different prefill depths, a plain job, the same job twice, a job whose
    prefill spans and backs off, sample ranges that only partly overlap, in a
    chunked workspace and whole; every output equals the oracle's."""
    from paper_2607_18991_amd import nz

    L = 8
    jobs = [dict(L=L, zone_mask=0x01, seed=91, nsamples=40, n0=4000, backoff=800),
            dict(L=L, zone_mask=0x01, seed=91, nsamples=40),                          # plain, same keys
            dict(L=L, zone_mask=0x01, seed=91, nsamples=40, n0=4000, backoff=800),   # the first job again
            dict(L=L, zone_mask=0x7F, seed=91, nsamples=40, n0=40, backoff=20),
            dict(L=L, zone_mask=0x7F, seed=91, nsamples=40, n0=L**5 - 1, backoff=L**5 // 2),  # spans: backs off
            dict(L=L, zone_mask=0x0C, seed=91, sample0=25, nsamples=30, n0=300, backoff=100),
            dict(L=6, zone_mask=0x01, seed=91, nsamples=20),                         # other size: its own groups
            dict(L=L, zone_mask=0x03, seed=92, nsamples=20, n0=800, backoff=200)]    # other seed
    want = oracle_batch(jobs)
    gn, gm, back, _ = run_batch(jobs)
    assert_same(jobs, gn, gm, *want)
    assert back[4] >= 40
    one = nz.nz_batch_workspace_bytes([dict(L=L, zone_mask=0x7F, seed=91, nsamples=1)])
    gn, gm, _, stats = run_batch(jobs, ws_bytes=12 * one)
    assert stats["chunks"] > 2
    assert_same(jobs, gn, gm, *want)
