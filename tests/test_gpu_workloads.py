"""Parity at the workloads' full sizes (GPU).

Every sample of each workload runs on the GPU in one batch, in the shape the
benchmark times; the oracle checks sampled outputs (the first and last samples
of every (L, mask) it can afford), and the learned-prefill path is compared
with the plain path sample by sample over the whole workload.  n* and mass are
integers: the bar is equality.
"""
import numpy as np
import pytest

from gpu_util import THREADS

pytestmark = pytest.mark.gpu

COMPACT = [0x01, 0x03, 0x07, 0x0F, 0x1F, 0x3F, 0x7F]


def random_masks(count=20, seed=0x24):
    """The 20 non-compact neighbourhoods of the L = 24 workload (the same recipe
    as the benchmark: uniform without replacement from the 120 non-compact masks)."""
    pool = [m for m in range(1, 128) if m not in COMPACT]
    rng = np.random.default_rng(seed)
    return sorted(int(m) for m in rng.choice(pool, size=count, replace=False))


def _run(jobs, ws_cap_gb=None, tune=None):
    import torch

    from paper_2607_18991_amd import nz

    total = sum(j["nsamples"] for j in jobs)
    need = nz.nz_batch_workspace_bytes(jobs, tune)
    if ws_cap_gb is not None:
        need = min(need, int(ws_cap_gb * 2**30))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    dn = torch.empty(total, dtype=torch.int32, device="cuda")
    dm = torch.empty(total, dtype=torch.int32, device="cuda")
    nz.nz_sweep_batch(jobs, ws, dn, dm, tune=tune)
    torch.cuda.synchronize()
    out = dn.cpu().numpy(), dm.cpu().numpy()
    del ws
    torch.cuda.empty_cache()
    return out


def _check_oracle(jobs, gn, gm, take):
    """take(job) -> list of (first sample offset, count) ranges to check."""
    import oracle

    off = 0
    for j in jobs:
        for a, c in take(j):
            wn, wm = oracle.sweep_many(j["L"], j["zone_mask"], j["seed"], j.get("sample0", 0) + a, c,
                                       nthreads=THREADS)
            got_n, got_m = gn[off + a:off + a + c], gm[off + a:off + a + c]
            assert (got_n == wn).all() and (got_m == wm).all(), (
                f"L={j['L']} mask={j['zone_mask']:#x} samples {a}..{a + c - 1}: {got_n[:4]} vs {wn[:4]}")
        off += j["nsamples"]


def _learned_and_plain(jobs, ws_cap_gb=None):
    from paper_2607_18991_amd import learned

    model = learned.PrefillModel.load()
    ln, lm = _run(model.plan(jobs), ws_cap_gb)
    pn, pm = _run(learned.plan_band_only(model, jobs), ws_cap_gb)
    assert (ln == pn).all() and (lm == pm).all(), "learned prefill changed an output"
    return ln, lm


def test_bench_batch_L16_compact_as_timed():
    """The benchmark's own batch (L = 16, the 7 compact masks x 1000, its
    seed) in the launch configuration it times: learned and plain plans, each
    with its tuned batch entry, narrow and wide neighbourhoods as two groups
    side by side.  Learned equals plain sample by sample; the oracle checks
    the first and the last sample of every mask."""
    from paper_2607_18991_amd import autotune, learned

    jobs = [dict(L=16, zone_mask=m, seed=0x5EED1016, nsamples=1000) for m in COMPACT]
    model = learned.PrefillModel.load()
    jl, jp = model.plan(jobs), learned.plan_band_only(model, jobs)
    ln, lm = _run(jl, tune=autotune.for_jobs(jl) or None)
    pn, pm = _run(jp, tune=autotune.for_jobs(jp) or None)
    assert (ln == pn).all() and (lm == pm).all(), "learned prefill changed an output"
    _check_oracle(jobs, ln, lm, lambda j: [(0, 1), (999, 1)])
    assert (ln > 0).all()


def test_W2_L8_compact_1e4():
    jobs = [dict(L=8, zone_mask=m, seed=0x5EED0008, nsamples=10_000) for m in COMPACT]
    gn, gm = _learned_and_plain(jobs)
    _check_oracle(jobs, gn, gm, lambda j: [(0, 96), (9_904, 96)])
    assert (gn > 0).all()


def test_W3_L16_all_masks_1e3():
    jobs = [dict(L=16, zone_mask=m, seed=0x5EED0016, nsamples=1_000) for m in range(1, 128)]
    # a workspace smaller than the batch: the batch runs in several chunks
    gn, gm = _learned_and_plain(jobs, ws_cap_gb=96)
    picked = set(COMPACT) | {0x02, 0x40, 0x55, 0x2A}
    _check_oracle(jobs, gn, gm, lambda j: [(999, 1)] if j["zone_mask"] in picked else [])
    assert (gn > 0).all()


def test_W4_uneven_batch():
    jobs = [dict(L=L, zone_mask=m, seed=0x5EED0400 + L, nsamples=500) for L in (8, 10, 12, 16, 20) for m in COMPACT]
    gn, gm = _learned_and_plain(jobs)
    _check_oracle(jobs, gn, gm, lambda j: [(0, 8), (492, 8)] if j["L"] <= 12 else
                  ([(0, 2)] if j["L"] == 16 else ([(499, 1)] if j["zone_mask"] in (0x01, 0x7F) else [])))
    # mass at n* grows with L for every neighbourhood (the fractal-dimension table)
    off = 0
    mean_mass = {}
    for j in jobs:
        mean_mass[(j["L"], j["zone_mask"])] = gm[off:off + 500].mean()
        off += 500
    for m in COMPACT:
        seq = [mean_mass[(L, m)] for L in (8, 10, 12, 16, 20)]
        assert all(b > a for a, b in zip(seq, seq[1:])), (m, seq)


def test_W5_L24_learned_vs_plain():
    masks = COMPACT + random_masks()
    assert len(set(masks)) == 27
    jobs = [dict(L=24, zone_mask=m, seed=0x5EED1024, nsamples=200) for m in masks]
    gn, gm = _learned_and_plain(jobs)
    _check_oracle(jobs, gn, gm, lambda j: [(0, 1)] if j["zone_mask"] in (0x01, 0x7F) else [])
    assert (gn > 0).all()
