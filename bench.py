"""Benchmark of the Newman-Ziff first-spanning sweep on one MI355X.

Workload (the headline metric): L = 16 (1,048,576 sites), the seven compact
neighbourhoods sc(5)-1 .. sc(5)-1,...,7 (zone masks 0x01 .. 0x7F), 1000 samples
each, free boundaries, spanning along axis 0.  One step = the whole path over
all 7000 samples: MLP inference (learned mode), Philox keys, key-band
bucketing and sorting, bulk connected-components prefill (learned mode) and the
persistent sequential sweep, with n* and mass of every sample in HBM at the end.

Both modes are timed on the same samples; their outputs must be identical.
value = site additions per second of the learned-prefill path (sum of n* over
samples / wall time; prefilled sites count as additions, so both modes do the
same additions and the speedup is a time ratio).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

COMPACT = [0x01, 0x03, 0x07, 0x0F, 0x1F, 0x3F, 0x7F]
SEEDS = {16: 0x5EED1016, 24: 0x5EED1024}
HBM_PEAK_GBS = 8000.0


def random_masks(count=20, seed=0x24):
    """The non-compact neighbourhoods of the L = 24 table: `count` distinct
    masks drawn uniformly from the 120 non-compact ones (NumPy, fixed seed)."""
    pool = [m for m in range(1, 128) if m not in COMPACT]
    rng = np.random.default_rng(seed)
    return sorted(int(m) for m in rng.choice(pool, size=count, replace=False))


def bytes_per_addition(z: int) -> float:
    """Algorithmic HBM bytes of one sequential site addition: the site (4 B), z
    occupancy bits and its own word (z/8 + 4), its parent entry (4), about two
    parent reads per occupied-neighbour find (8 per neighbour, ~0.8 neighbours on
    average below the threshold) and a root read-modify-write per union (8)."""
    return 22.0 + z / 8.0


def base_jobs(L, samples, masks=COMPACT):
    return [dict(L=L, zone_mask=m, seed=SEEDS.get(L, 0x5EED0000 + L), nsamples=samples) for m in masks]


def run_mode(nz, torch, make_jobs, steps, warmup, tune):
    """make_jobs() is called inside every step (it runs the MLP in learned mode)."""
    jobs = make_jobs()
    total = sum(j["nsamples"] for j in jobs)
    ws_bytes = nz.nz_batch_workspace_bytes(jobs, tune)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    dn = torch.zeros(total, dtype=torch.int32, device="cuda")
    dm = torch.zeros(total, dtype=torch.int32, device="cuda")
    for _ in range(warmup):
        nz.nz_sweep_batch(make_jobs(), ws, dn, dm, tune=tune)
    torch.cuda.synchronize()
    nz.nz_set_timing(True)
    phase = {"keys_ms": 0.0, "cc_ms": 0.0, "sort_ms": 0.0, "sweep_ms": 0.0, "total_ms": 0.0, "sweep_launches": 0}
    stats = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        nz.nz_sweep_batch(make_jobs(), ws, dn, dm, tune=tune)
        t = nz.nz_last_batch_timing()
        for k in phase:
            phase[k] += t[k]
        for k, v in nz.nz_last_batch_stats().items():
            stats[k] = stats.get(k, 0) + v
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    nz.nz_set_timing(False)
    del ws
    return {"wall": wall, "ns": dn.cpu().numpy(), "ms": dm.cpu().numpy(), "phase": phase, "stats": stats,
            "jobs": jobs, "tune": tune}


def summarise(res, steps, S, z):
    ms_step = res["wall"] / steps * 1e3
    adds = int(res["ns"].astype(np.int64).sum())
    serial = res["stats"]["serial_steps"] / steps
    alg_bytes = 0.0
    # serial steps per mask are not reported separately; weight by each mask's share of n*
    masks = [j["zone_mask"] for j in res["jobs"]]
    share = np.array([res["ns"][k * S:(k + 1) * S].astype(np.float64).sum() for k in range(len(masks))])
    share = share / share.sum()
    for k, m in enumerate(masks):
        alg_bytes += serial * share[k] * bytes_per_addition(z[m])
    launches = max(res["phase"]["sweep_launches"], 1)
    sweep_ms = res["phase"]["sweep_ms"] / launches
    # neighbour checks: z per sequential addition (the sweep), z/2 per prefilled
    # site (the hook's half of the offset table); the library counts additions
    # and prefilled sites per batch, which are split over the masks by each
    # mask's n* - n0 and n0
    prefilled = res["stats"]["prefilled_sites"] / steps
    ser_w = np.zeros(len(masks))
    pre_w = np.zeros(len(masks))
    for k, j in enumerate(res["jobs"]):
        n0 = max(0, int(j.get("n0", 0) or 0))
        ns = res["ns"][k * S:(k + 1) * S].astype(np.float64)
        ser_w[k] = np.clip(ns - n0, 0, None).sum()
        pre_w[k] = n0 * S
    zs = np.array([z[m] for m in masks], dtype=np.float64)
    checks_sweep = serial * float((ser_w / max(ser_w.sum(), 1.0) * zs).sum())
    checks_pre = prefilled * float((pre_w / max(pre_w.sum(), 1.0) * np.floor(zs / 2)).sum()) if pre_w.sum() else 0.0
    ph = res["phase"]
    return {
        "ms_per_step": ms_step,
        "site_additions_per_s": adds / (ms_step / 1e3),
        "samples_per_s": len(res["ns"]) / (ms_step / 1e3),
        "sequential_steps_per_step": serial,
        "prefilled_sites_per_step": res["stats"]["prefilled_sites"] / steps,
        "backoffs_per_step": res["stats"]["backoffs"] / steps,
        "phase_ms_per_step": {k: v / steps for k, v in res["phase"].items() if k != "sweep_launches"},
        "sweep_kernel_ms": sweep_ms,
        "sweep_alg_bytes": alg_bytes,
        "neighbour_checks_per_step": {"sweep": checks_sweep, "prefill": checks_pre},
        "neighbour_checks_per_s": (checks_sweep + checks_pre) / (ms_step / 1e3),
        # per phase, over that phase's kernel time summed over the groups
        "neighbour_checks_per_s_in_phase": {
            "sweep": checks_sweep / (ph["sweep_ms"] / steps / 1e3) if ph["sweep_ms"] > 0 else None,
            "prefill": checks_pre / (ph["cc_ms"] / steps / 1e3) if ph["cc_ms"] > 0 and checks_pre else None},
        "tuning": res["tune"],
    }


def cpu_threads():
    # the oracle runs on at most 16 host threads
    return max(1, min(os.cpu_count() or 1, 16))


def cpu_baseline(jobs, per_mask):
    import oracle

    threads = cpu_threads()
    adds = 0
    res = {}
    t0 = time.perf_counter()
    for j in jobs:
        ns, ms = oracle.sweep_many(j["L"], j["zone_mask"], j["seed"], 0, per_mask, nthreads=threads)
        res[j["zone_mask"]] = (ns, ms)
        adds += int(ns.sum())
    wall = time.perf_counter() - t0
    return adds / wall, threads, res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--L", type=int, default=16)
    ap.add_argument("--samples", type=int, default=1000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-per-mask", action="store_true", help="skip the table of each compact mask on its own")
    ap.add_argument("--l24-samples", type=int, default=200, help="samples per mask of the L=24 table (0: skip)")
    ap.add_argument("--mode", choices=["both", "learned", "plain"], default="both",
                    help="profiling aid: run only one path (the JSON line then reports that path)")
    ap.add_argument("--autotune-out", default=None,
                    help="tune the benchmark's batches as a whole, add them to the tuning table and write it "
                         "to this path (no benchmark is run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; samples are independent and would shard by "
                                   "sample range across GPUs, which is not run here"}), flush=True)
        sys.exit(2)

    import torch

    from paper_2607_18991_amd import learned, nz

    from paper_2607_18991_amd import autotune

    torch.cuda.set_device(0)
    L, S = args.L, args.samples
    N = L**5
    model = learned.PrefillModel.load()
    jobs0 = base_jobs(L, S)
    masks24 = COMPACT + random_masks()
    z = {m: nz.nz_coordination(m) for m in range(1, 128)}

    if args.autotune_out:
        table = autotune.load_table()
        batches = [(f"L={L} x 7 compact x {S}, plain", learned.plan_band_only(model, jobs0)),
                   (f"L={L} x 7 compact x {S}, learned", model.plan(jobs0))]
        if args.l24_samples > 0:
            j24 = base_jobs(24, args.l24_samples, masks24)
            batches += [(f"L=24 x 27 masks x {args.l24_samples}, plain", learned.plan_band_only(model, j24)),
                        (f"L=24 x 27 masks x {args.l24_samples}, learned", model.plan(j24))]
        for name, jobs in batches:
            e = autotune.tune_batch(jobs, log=lambda m: print(f"{name}: {m}", flush=True))
            autotune.add_batch(table, jobs, e, name)
            print(f"{name}: best {e['tune']} {e['ms']} ms (default {e['default_ms']} ms)", flush=True)
        autotune.save_table(table, args.autotune_out)
        return

    if args.mode in ("both", "plain"):
        jp = learned.plan_band_only(model, jobs0)
        plain = run_mode(nz, torch, lambda: learned.plan_band_only(model, jobs0), args.steps, args.warmup,
                         autotune.for_jobs(jp) or None)
    if args.mode in ("both", "learned"):
        jl = model.plan(jobs0)
        learn = run_mode(nz, torch, lambda: model.plan(jobs0), args.steps, args.warmup,
                         autotune.for_jobs(jl) or None)
    if args.mode == "plain":
        learn = plain
    elif args.mode == "learned":
        plain = learn
    identical = bool((plain["ns"] == learn["ns"]).all() and (plain["ms"] == learn["ms"]).all())
    sp = summarise(plain, args.steps, S, z)
    sl = summarise(learn, args.steps, S, z)

    # the sweep kernel: algorithmic bytes of a step's launches over their time
    # (HIP events on the launch stream), i.e. per launch over the average
    # launch duration
    sweep_ms_step = sl["phase_ms_per_step"]["sweep_ms"]
    launches = max(1.0, learn["phase"]["sweep_launches"] / args.steps)
    kernel_ms = sweep_ms_step / launches
    achieved = sl["sweep_alg_bytes"] / (sweep_ms_step / 1e3) / 1e9
    traffic = None
    keys_traffic = None
    keys_dispatches = None   # per step, from the kernel trace of these sources (redo rounds included)
    rec_path = os.path.join(ROOT, "profiles", "nz_sweep_L16_compact_x1000_learned.json")
    if L == 16 and S == 1000 and os.path.exists(rec_path):
        from paper_2607_18991_amd import profile_summary

        rec = json.load(open(rec_path))
        if rec.get("source_sha1") == profile_summary.source_sha1():
            traffic = rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
            if "keys" in rec:
                keys_traffic = rec["keys"]["fetch_bytes_per_step"] + rec["keys"]["write_bytes_per_step"]
                keys_dispatches = rec["keys"].get("dispatches") or None
    # the keys kernel: integer VALU work of Philox4x32-10 (one block of 10
    # rounds, each two 32x32->64 products and four XORs, serves two sites) plus
    # four operations of classification per site, against 256 CUs x 64 lanes x
    # 2.4 GHz of 32-bit integer operations
    keys_ops_per_site = 10 * 6 / 2 + 4
    keyed_sites = float(N) * len(learn["ns"])
    keys_achieved = keyed_sites * keys_ops_per_site / (sl["phase_ms_per_step"]["keys_ms"] / 1e3) / 1e12
    alu_peak = 256 * 64 * 2.4e9 / 1e12
    out = {
        "metric": "site additions/s and samples/s at L=16, zones 1-7; learned-prefill vs plain speedup",
        "value": sl["site_additions_per_s"],
        "unit": "site additions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sl["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (Philox4x32-10 occupation orders)",
        "config": {"workload": f"L={L} (N={N}) x 7 compact zone masks (0x01..0x7F) x {S} samples, free boundaries, "
                               f"spanning along axis 0, learned prefill + persistent sweep",
                   "L": L, "samples_per_mask": S},
        "samples_per_s": sl["samples_per_s"],
        "neighbour_checks_per_s": sl["neighbour_checks_per_s"],
        "speedup_learned_vs_plain": sp["ms_per_step"] / sl["ms_per_step"],
        "outputs_identical_plain_vs_learned": identical,
        "learned": sl,
        "plain": sp,
        "roofline_sweep": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": "nz_sweep_kernel",
                           "kernel_ms": kernel_ms, "launches_per_step": launches,
                           "alg_bytes_per_launch": sl["sweep_alg_bytes"] / launches},
        "roofline_keys": {"bound": "alu", "achieved": keys_achieved, "peak": alu_peak, "unit": "Tops/s",
                          "frac": keys_achieved / alu_peak,
                          "traffic": keys_traffic / (keys_dispatches or launches) if keys_traffic else None,
                          "kernel": "nz_keys_kernel",
                          "kernel_ms": sl["phase_ms_per_step"]["keys_ms"] / (keys_dispatches or launches),
                          "launches_per_step": keys_dispatches or launches,
                          "ops_per_site": keys_ops_per_site},
    }
    # "roofline" is the kernel that takes the larger share of the step (a batch
    # whose narrow and wide neighbourhoods run side by side has one launch of
    # each kernel per group; rates are per launch over its own duration)
    out["roofline"] = dict(out["roofline_keys"] if sl["phase_ms_per_step"]["keys_ms"] > sweep_ms_step
                           else out["roofline_sweep"])
    def per_mask(Lm, Sm):
        # each compact neighbourhood as a batch of its own (the headline mask is
        # zones 1-7, 0x7F): learned and plain, one untimed and two timed steps
        per = {}
        for m in COMPACT:
            jm = base_jobs(Lm, Sm, [m])
            jlm, jpm = model.plan(jm), learned.plan_band_only(model, jm)
            pm_ = run_mode(nz, torch, lambda: learned.plan_band_only(model, jm), 2, 1, autotune.for_jobs(jpm) or None)
            lm_ = run_mode(nz, torch, lambda: model.plan(jm), 2, 1, autotune.for_jobs(jlm) or None)
            a, b = summarise(pm_, 2, Sm, z), summarise(lm_, 2, Sm, z)
            per[f"{m:#04x}"] = {"z": z[m], "learned_ms": b["ms_per_step"], "plain_ms": a["ms_per_step"],
                                "site_additions_per_s": b["site_additions_per_s"], "samples_per_s": b["samples_per_s"],
                                "speedup_learned_vs_plain": a["ms_per_step"] / b["ms_per_step"],
                                "outputs_identical_plain_vs_learned": bool((pm_["ns"] == lm_["ns"]).all() and
                                                                           (pm_["ms"] == lm_["ms"]).all())}
        return per

    if not args.no_per_mask and args.mode == "both":
        out["per_mask"] = per_mask(L, S)
        out["headline_mask"] = "0x7f"
    if args.l24_samples > 0:
        # the same comparison at L = 24 (7,962,624 sites): the 7 compact and 20
        # random neighbourhoods, one untimed and one timed step per mode
        j24 = base_jobs(24, args.l24_samples, masks24)
        jp24, jl24 = learned.plan_band_only(model, j24), model.plan(j24)
        p24 = run_mode(nz, torch, lambda: learned.plan_band_only(model, j24), 1, 1, autotune.for_jobs(jp24) or None)
        l24 = run_mode(nz, torch, lambda: model.plan(j24), 1, 1, autotune.for_jobs(jl24) or None)
        s24p, s24l = summarise(p24, 1, args.l24_samples, z), summarise(l24, 1, args.l24_samples, z)
        out["L24"] = {"samples_per_mask": args.l24_samples, "masks": masks24,
                      "per_mask": per_mask(24, args.l24_samples) if not args.no_per_mask else None,
                      "outputs_identical_plain_vs_learned": bool((p24["ns"] == l24["ns"]).all() and
                                                                 (p24["ms"] == l24["ms"]).all()),
                      "speedup_learned_vs_plain": s24p["ms_per_step"] / s24l["ms_per_step"],
                      "learned": s24l, "plain": s24p}
        # the learned sweep against HBM at L = 24, as at L = 16 (rate per launch
        # over the launches' own durations)
        l24_launches = max(1.0, float(l24["phase"]["sweep_launches"]))
        l24_sweep_ms = s24l["phase_ms_per_step"]["sweep_ms"]
        ach24 = s24l["sweep_alg_bytes"] / (l24_sweep_ms / 1e3) / 1e9 if l24_sweep_ms > 0 else 0.0
        out["L24"]["roofline_sweep"] = {"bound": "hbm", "achieved": ach24, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                        "frac": ach24 / HBM_PEAK_GBS, "kernel": "nz_sweep_kernel",
                                        "kernel_ms": l24_sweep_ms / l24_launches,
                                        "launches_per_step": l24_launches}
    if not args.no_cpu:
        # every thread takes the same number of samples of each mask (about
        # 10 s on 16 host cores at L = 16)
        per = min(S, cpu_threads() * (8 if L >= 16 else 32))
        cpu_rate, threads, res = cpu_baseline(jobs0, per)
        parity = all((res[m][0] == learn["ns"][k * S:k * S + per]).all() and
                     (res[m][1] == learn["ms"][k * S:k * S + per]).all() for k, m in enumerate(COMPACT))
        out["cpu_baseline"] = {"value": cpu_rate, "unit": "site additions/s", "cores": threads, "kind": "oracle",
                               "sample": f"samples 0..{per - 1} of each of the 7 masks at L={L}, spread over "
                                         f"{threads} threads (keys, full sort, serial union-find)"}
        out["parity_on_cpu_sample"] = bool(parity)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
