"""Periodic boundaries on the GPU: n* and mass of the first cluster wrapping
around axis 0 (Newman & Ziff 2001, Sec. III), against the oracle's serial
union-find with displacements, sample by sample.  Integers: the bar is
equality."""
import numpy as np
import pytest

from gpu_util import assert_same, oracle_batch, run_batch

pytestmark = pytest.mark.gpu

PERIODIC = 1


@pytest.mark.parametrize("L,mask,count", [(5, 0x01, 200), (5, 0x7F, 64), (6, 0x03, 100), (7, 0x0C, 64),
                                          (8, 0x01, 100), (8, 0x7F, 48), (10, 0x05, 40), (12, 0x01, 24),
                                          (16, 0x01, 6), (16, 0x40, 6)])
def test_plain_wrap_matches_oracle(L, mask, count):
    import oracle
    from paper_2607_18991_amd import nz

    ns, ms = nz.nz_sweep(L, mask, count, 0x3A9 + L, boundary=nz.NZ_PERIODIC)
    on, om = oracle.sweep_many(L, mask, 0x3A9 + L, 0, count, nthreads=16, periodic=True)
    assert (ns == on).all() and (ms == om).all(), (np.nonzero(ns != on)[0][:5], ns[:5], on[:5])
    assert (ns > 0).all()


def _jobs(n0_frac, L=8, masks=(0x01, 0x03, 0x7F), count=40, seed=0x77):
    import oracle

    out = []
    for m in masks:
        on, _ = oracle.sweep_many(L, m, seed, 0, count, nthreads=16, periodic=True)
        N = L**5
        n0 = int(n0_frac * on.mean())
        out.append(dict(L=L, zone_mask=m, boundary=PERIODIC, seed=seed, sample0=0, nsamples=count,
                        n0=n0, backoff=max(1, int(0.1 * n0))))
        assert n0 < N
    return out


def test_prefilled_wrap_matches_oracle():
    """Prefill at 80% of the mean n*: the displacement-carrying bulk labelling
    hands its state to the sweep."""
    jobs = _jobs(0.8)
    gn, gm, back, _ = run_batch(jobs)
    on, om = oracle_batch(jobs)
    assert_same(jobs, gn, gm, on, om)


def test_prefilled_wrap_backs_off():
    """Prefill past the mean n*: about half of the prefilled states already wrap,
    which the hook finds from the displacements, and those samples back off."""
    jobs = _jobs(1.3)
    gn, gm, back, _ = run_batch(jobs)
    on, om = oracle_batch(jobs)
    assert_same(jobs, gn, gm, on, om)
    assert back.sum() > 0


def test_wrap_early_merge(monkeypatch):
    """A distinct-root list of two forces the merge-and-refind path, whose
    re-found roots carry the displacement of the merged root."""
    monkeypatch.setenv("NZ_DEBUG_DCAP", "2")
    jobs = [dict(L=6, zone_mask=0x7F, boundary=PERIODIC, seed=0x99, nsamples=40, n0=-1),
            dict(L=8, zone_mask=0x3F, boundary=PERIODIC, seed=0x9A, nsamples=24, n0=-1)]
    gn, gm, _, _ = run_batch(jobs)
    on, om = oracle_batch(jobs)
    assert_same(jobs, gn, gm, on, om)


def test_mixed_boundaries_in_one_batch():
    """Free and periodic jobs in one batch land in separate chunks and each
    matches its own oracle."""
    jobs = [dict(L=8, zone_mask=0x01, boundary=0, seed=0x51, nsamples=30, n0=-1),
            dict(L=8, zone_mask=0x01, boundary=PERIODIC, seed=0x51, nsamples=30, n0=-1),
            dict(L=6, zone_mask=0x7F, boundary=PERIODIC, seed=0x52, nsamples=20, n0=-1),
            dict(L=6, zone_mask=0x7F, boundary=0, seed=0x52, nsamples=20, n0=-1)]
    gn, gm, _, _ = run_batch(jobs)
    on, om = oracle_batch(jobs)
    assert_same(jobs, gn, gm, on, om)
    # the two boundary conditions give different thresholds on the same orders
    assert (gn[:30] != gn[30:60]).any()


def test_learned_plan_on_periodic_jobs():
    """The prefill model (trained on free boundaries) plans periodic jobs too;
    its prediction only sets where the prefill stops, and the outputs equal the
    plain periodic sweep's."""
    from paper_2607_18991_amd import learned

    model = learned.PrefillModel.load()
    jobs = [dict(L=L, zone_mask=m, boundary=PERIODIC, seed=0x5EED, nsamples=64)
            for L in (8, 12) for m in (0x01, 0x07, 0x7F)]
    ln, lm, _, _ = run_batch(model.plan(jobs))
    pn, pm, _, _ = run_batch(learned.plan_band_only(model, jobs))
    assert (ln == pn).all() and (lm == pm).all()
    on, om = oracle_batch([dict(j, nsamples=4) for j in jobs])
    off = 0
    for k, j in enumerate(jobs):
        assert (ln[off:off + 4] == on[4 * k:4 * k + 4]).all() and (lm[off:off + 4] == om[4 * k:4 * k + 4]).all()
        off += j["nsamples"]
