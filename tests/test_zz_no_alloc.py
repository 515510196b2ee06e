"""nz_sweep_batch_static, the batch sweep inside the library's own device
buffer (no allocation by the call), against nz_sweep_batch on the same jobs:
n*, mass and backoff counts equal, on two calls in a row, the second with a
smaller batch (GPU)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

COMPACT = [0x01, 0x03, 0x07, 0x0F, 0x1F, 0x3F, 0x7F]


def _reference(jobs):
    import torch

    from paper_2607_18991_amd import nz

    total = sum(j["nsamples"] for j in jobs)
    ws = torch.empty(nz.nz_batch_workspace_bytes(jobs), dtype=torch.uint8, device="cuda")
    dn = torch.full((total,), -7, dtype=torch.int32, device="cuda")
    dm = torch.full((total,), -7, dtype=torch.int32, device="cuda")
    back = nz.nz_sweep_batch(jobs, ws, dn, dm)
    torch.cuda.synchronize()
    return dn.cpu().numpy(), dm.cpu().numpy(), back


def _static(jobs, total_alloc):
    import torch

    from paper_2607_18991_amd import nz

    total = sum(j["nsamples"] for j in jobs)
    dn = torch.full((total_alloc,), -7, dtype=torch.int32, device="cuda")
    dm = torch.full((total_alloc,), -7, dtype=torch.int32, device="cuda")
    back = nz.nz_sweep_batch_static(jobs, dn, dm)
    torch.cuda.synchronize()
    n, m = dn.cpu().numpy(), dm.cpu().numpy()
    # nothing beyond the batch's own outputs is written
    assert (n[total:] == -7).all() and (m[total:] == -7).all()
    return n[:total], m[:total], back, nz.nz_last_batch_stats()


def test_static_buffer_matches_batch_two_calls():
    from paper_2607_18991_amd import learned, nz

    assert nz.nz_static_scratch_bytes() == 256 << 20
    model = learned.PrefillModel.load()
    # first call: learned plans at L = 16 and 24 (the buffer holds a few
    # samples per chunk, so the batch runs in many chunks) and plain L = 8
    first = model.plan([dict(L=16, zone_mask=m, seed=0x57A7, nsamples=24) for m in (0x01, 0x07, 0x7F)] +
                       [dict(L=24, zone_mask=0x7F, seed=0x57A7, nsamples=3)])
    first += [dict(L=8, zone_mask=0x03, seed=0x57A7, nsamples=50)]
    rn, rm, rb = _reference(first)
    gn, gm, gb, stats = _static(first, 200)
    assert (gn == rn).all() and (gm == rm).all() and (gb == rb).all()
    assert stats["chunks"] > 1
    # second call, smaller: plain sweeps at L = 6 over the compact masks
    second = [dict(L=6, zone_mask=m, seed=0x57A8, nsamples=5) for m in COMPACT]
    rn, rm, rb = _reference(second)
    gn, gm, gb, _ = _static(second, 200)
    assert (gn == rn).all() and (gm == rm).all() and (gb == rb).all()
    assert (gn > 0).all()
