"""Two groups of a batch side by side (GPU): narrow neighbourhoods (z <= 64)
and wide ones run concurrently on two host threads and streams.  The outputs
and per-job backoff counts must equal those of the single-group path sample by
sample, and sampled outputs the oracle's."""
import numpy as np
import pytest

from gpu_util import THREADS, run_batch

pytestmark = pytest.mark.gpu

COMPACT = [0x01, 0x03, 0x07, 0x0F, 0x1F, 0x3F, 0x7F]


def _both(jobs, monkeypatch):
    gn, gm, gb, st = run_batch(jobs)
    monkeypatch.setenv("NZ_DEBUG_NO_SPLIT", "1")
    sn, sm, sb, _ = run_batch(jobs)
    monkeypatch.delenv("NZ_DEBUG_NO_SPLIT")
    return (gn, gm, gb), (sn, sm, sb), st


def test_split_plain_equals_single_group(monkeypatch):
    import oracle

    jobs = [dict(L=8, zone_mask=m, seed=0x5B1, nsamples=600, n0=-1) for m in COMPACT]
    (gn, gm, _), (sn, sm, _), st = _both(jobs, monkeypatch)
    assert (gn == sn).all() and (gm == sm).all()
    assert st["chunks"] >= 2   # one chunk per group at least
    for k, m in enumerate(COMPACT):
        on, om = oracle.sweep_many(8, m, 0x5B1, 590, 10, nthreads=THREADS)
        assert (gn[k * 600 + 590:(k + 1) * 600] == on).all() and (gm[k * 600 + 590:(k + 1) * 600] == om).all()


def test_split_learned_with_backoffs(monkeypatch):
    """Learned plans (prefill, in-chunk backoffs) in both groups; the job order
    interleaves narrow and wide neighbourhoods so outputs map back by job."""
    from paper_2607_18991_amd import learned

    model = learned.PrefillModel.load()
    order = [0x7F, 0x01, 0x1F, 0x03, 0x07]
    jobs = model.plan([dict(L=10, zone_mask=m, seed=0x5B2, nsamples=400) for m in order], k_sigma=1.5)
    (gn, gm, gb), (sn, sm, sb), _ = _both(jobs, monkeypatch)
    assert (gn == sn).all() and (gm == sm).all()
    assert (np.asarray(gb) == np.asarray(sb)).all() and np.asarray(gb).sum() > 0
