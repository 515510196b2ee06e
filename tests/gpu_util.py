"""Helpers for the GPU parity tests: run jobs through the C ABI on cuda:0 and
the same samples through the oracle."""
import os

import numpy as np

import oracle
from paper_2607_18991_amd import nz

THREADS = max(1, min(16, os.cpu_count() or 1))


def run_batch(jobs, tune=None, ws_bytes=None, fill=None):
    """fill: a byte value the workspace is set to before the batch (None:
    left as allocated)."""
    import torch

    total = sum(int(j["nsamples"]) for j in jobs)
    need = nz.nz_batch_workspace_bytes(jobs, tune)
    if fill is None:
        ws = torch.empty(ws_bytes or need, dtype=torch.uint8, device="cuda")
    else:
        ws = torch.full((ws_bytes or need,), fill, dtype=torch.uint8, device="cuda")
    dn = torch.full((max(total, 1),), -7, dtype=torch.int32, device="cuda")
    dm = torch.full((max(total, 1),), -7, dtype=torch.int32, device="cuda")
    back = nz.nz_sweep_batch(jobs, ws, dn, dm, tune=tune)
    torch.cuda.synchronize()
    return dn.cpu().numpy()[:total], dm.cpu().numpy()[:total], back, nz.nz_last_batch_stats()


def oracle_batch(jobs):
    ns, ms = [], []
    for j in jobs:
        a, b = oracle.sweep_many(j["L"], j["zone_mask"], j["seed"], j.get("sample0", 0), j["nsamples"],
                                 nthreads=THREADS, periodic=j.get("boundary", nz.NZ_FREE) == nz.NZ_PERIODIC)
        ns.append(a)
        ms.append(b)
    return np.concatenate(ns), np.concatenate(ms)


def assert_same(jobs, got_n, got_m, want_n, want_m):
    off = 0
    for j in jobs:
        n = j["nsamples"]
        gn, wn = got_n[off:off + n], want_n[off:off + n]
        gm, wm = got_m[off:off + n], want_m[off:off + n]
        bad = np.nonzero((gn != wn) | (gm != wm))[0]
        assert len(bad) == 0, (f"L={j['L']} mask={j['zone_mask']:#x} first bad sample {bad[:5]}: "
                               f"gpu n*={gn[bad[:5]]} mass={gm[bad[:5]]} oracle n*={wn[bad[:5]]} mass={wm[bad[:5]]}")
        off += n
