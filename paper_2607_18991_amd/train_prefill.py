"""Train the prefill MLP from the method's own plain sweeps and save it.

Training lattices (synthetic Philox orders, free boundaries, spanning along
axis 0): L = 4 zone 1 (1000 samples); L = 8 and the seven compact
neighbourhoods (10^4 samples each); L = 16 and all 127 neighbourhoods (1000
samples each); and L = 8, 10, 12, 16, 20 with the seven compact
neighbourhoods (500 samples each), so that the sizes the prefill is used at
(up to L = 24) are a short extrapolation in ln L rather than a long one.
Each lattice contributes ln mean and ln std of n*/N.

    python -m paper_2607_18991_amd.train_prefill [--out PATH] [--scale S]

--scale < 1 shrinks every sample count (for quick checks).
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import learned, nz

SEEDS = {4: 0x5EED0004, 8: 0x5EED0008, 16: 0x5EED0016, "uneven": 0x5EED0E4E}
COMPACT = [0x01, 0x03, 0x07, 0x0F, 0x1F, 0x3F, 0x7F]


def training_jobs(scale: float = 1.0):
    jobs = [dict(L=4, zone_mask=1, seed=SEEDS[4], nsamples=max(8, int(1000 * scale)))]
    jobs += [dict(L=8, zone_mask=m, seed=SEEDS[8], nsamples=max(8, int(10000 * scale))) for m in COMPACT]
    jobs += [dict(L=16, zone_mask=m, seed=SEEDS[16], nsamples=max(8, int(1000 * scale))) for m in range(1, 128)]
    jobs += [dict(L=L, zone_mask=m, seed=SEEDS["uneven"], nsamples=max(8, int(500 * scale)))
             for L in (8, 10, 12, 16, 20) for m in COMPACT]
    return jobs


def run_plain(jobs):
    import torch

    total = sum(j["nsamples"] for j in jobs)
    ws = torch.empty(nz.nz_batch_workspace_bytes(jobs), dtype=torch.uint8, device="cuda")
    dn = torch.zeros(total, dtype=torch.int32, device="cuda")
    dm = torch.zeros(total, dtype=torch.int32, device="cuda")
    nz.nz_sweep_batch(jobs, ws, dn, dm)
    torch.cuda.synchronize()
    return dn.cpu().numpy(), dm.cpu().numpy()


def collect(jobs):
    ns, _ = run_plain(jobs)
    pts, off = [], 0
    for j in jobs:
        pts.append(learned.aggregate(j["L"], j["zone_mask"], ns[off:off + j["nsamples"]]))
        off += j["nsamples"]
    return pts


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=learned.DEFAULT_PATH)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--steps", type=int, default=4000)
    args = ap.parse_args()
    import torch

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    pts = collect(training_jobs(args.scale))
    t1 = time.perf_counter()
    model = learned.train(pts, steps=args.steps, log_every=500)
    t2 = time.perf_counter()
    model.meta["training_points"] = pts
    model.meta["data_seconds"] = t1 - t0
    model.meta["train_seconds"] = t2 - t1
    mean, std = model.predict([p["mask"] for p in pts], [p["L"] for p in pts])
    err_u = np.log(mean) - np.log([p["mean"] for p in pts])
    err_v = np.log(std) - np.log([p["std"] for p in pts])
    model.meta["fit_rms_ln_mean"] = float(np.sqrt(np.mean(err_u**2)))
    model.meta["fit_rms_ln_std"] = float(np.sqrt(np.mean(err_v**2)))
    model.save(args.out)
    print(json.dumps({"out": args.out, "points": len(pts), "data_s": round(t1 - t0, 2), "train_s": round(t2 - t1, 2),
                      "loss": model.meta["loss_history"][-1], "rms_ln_mean": model.meta["fit_rms_ln_mean"],
                      "rms_ln_std": model.meta["fit_rms_ln_std"]}), flush=True)


if __name__ == "__main__":
    main()
