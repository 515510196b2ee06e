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
    cc = {"hook_ms": 0.0, "compress_ms": 0.0, "accum_ms": 0.0, "expand_ms": 0.0, "dispatches": 0}
    stats = {}
    serial = np.zeros(len(jobs), dtype=np.int64)
    prefilled = np.zeros(len(jobs), dtype=np.int64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        nz.nz_sweep_batch(make_jobs(), ws, dn, dm, tune=tune)
        t = nz.nz_last_batch_timing()
        for k in phase:
            phase[k] += t[k]
        for k, v in nz.nz_last_batch_cc_timing().items():
            cc[k] += v
        for k, v in nz.nz_last_batch_stats().items():
            stats[k] = stats.get(k, 0) + v
        a, b = nz.nz_last_batch_job_stats(len(jobs))
        serial += a
        prefilled += b
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    nz.nz_set_timing(False)
    del ws
    return {"wall": wall, "ns": dn.cpu().numpy(), "ms": dm.cpu().numpy(), "phase": phase, "cc": cc, "stats": stats,
            "serial": serial, "prefilled": prefilled, "jobs": jobs, "tune": tune}


def prefill_bytes(n0_sites: float, z: int, N: int, samples: int) -> float:
    """Algorithmic HBM bytes of the bulk labelling: per labelled site z/8
    occupancy bits and 16 bytes of hook-and-compress forest traffic, plus 8
    bytes for the size pass (the root word's update and the site's lattice
    entry), and one pass over each prefilled sample's N/8-byte bitset."""
    return n0_sites * (z / 8.0 + 24.0) + samples * N / 8.0


def summarise(res, steps, S, z):
    ms_step = res["wall"] / steps * 1e3
    adds = int(res["ns"].astype(np.int64).sum())
    jobs = res["jobs"]
    masks = [j["zone_mask"] for j in jobs]
    zs = np.array([z[m] for m in masks], dtype=np.float64)
    # per job and step: sequential additions and prefilled sites (the
    # library's own counts over the final runs of every sample)
    ser = np.asarray(res["serial"], dtype=np.float64) / steps
    pre = np.asarray(res["prefilled"], dtype=np.float64) / steps
    serial = float(ser.sum())
    sweep_bytes = float(sum(ser[k] * bytes_per_addition(z[m]) for k, m in enumerate(masks)))
    pre_bytes = float(sum(prefill_bytes(pre[k], z[m], int(j["L"]) ** 5, int(j["nsamples"]))
                          for k, (j, m) in enumerate(zip(jobs, masks)) if int(j.get("n0", -1) or -1) > 0))
    launches = max(res["phase"]["sweep_launches"], 1)
    sweep_ms = res["phase"]["sweep_ms"] / launches
    # neighbour checks: z per sequential addition (the sweep), z/2 per prefilled
    # site (the hook's half of the offset table)
    checks_sweep = float((ser * zs).sum())
    checks_pre = float((pre * np.floor(zs / 2)).sum())
    ph = res["phase"]
    cc = res.get("cc") or {}
    return {
        "ms_per_step": ms_step,
        "site_additions_per_s": adds / (ms_step / 1e3),
        "samples_per_s": len(res["ns"]) / (ms_step / 1e3),
        "sequential_steps_per_step": serial,
        "prefilled_sites_per_step": float(pre.sum()),
        "backoffs_per_step": res["stats"]["backoffs"] / steps,
        "phase_ms_per_step": {k: v / steps for k, v in ph.items() if k != "sweep_launches"},
        "labelling_ms_per_step": {k: v / steps for k, v in cc.items() if k != "dispatches"},
        "labelling_dispatches_per_step": cc.get("dispatches", 0) / steps,
        "sweep_kernel_ms": sweep_ms,
        "sweep_alg_bytes": sweep_bytes,
        "prefill_alg_bytes": pre_bytes,
        "neighbour_checks_per_step": {"sweep": checks_sweep, "prefill": checks_pre},
        "neighbour_checks_per_s": (checks_sweep + checks_pre) / (ms_step / 1e3),
        # per phase, over that phase's kernel time summed over the groups
        "neighbour_checks_per_s_in_phase": {
            "sweep": checks_sweep / (ph["sweep_ms"] / steps / 1e3) if ph["sweep_ms"] > 0 else None,
            "prefill": checks_pre / (ph["cc_ms"] / steps / 1e3) if ph["cc_ms"] > 0 and checks_pre else None},
        "tuning": res["tune"],
    }


def hbm_roofline(kernel, alg_bytes_step, ms_step, launches, traffic=None):
    """Algorithmic bytes of a step's launches over their summed duration (HIP
    events on the launch streams), i.e. bytes per launch over the average
    launch duration."""
    achieved = alg_bytes_step / (ms_step / 1e3) / 1e9 if ms_step > 0 else 0.0
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel,
            "kernel_ms": ms_step / max(launches, 1e-9), "launches_per_step": launches,
            "alg_bytes_per_launch": alg_bytes_step / max(launches, 1e-9)}


def profile_record(name):
    """Per-kernel HBM traffic of one step from the committed counter runs
    (profiles/<name>.json), if they were taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(path):
        return None
    from paper_2607_18991_amd import profile_summary

    rec = json.load(open(path))
    if rec.get("source_sha1") != profile_summary.source_sha1() or "kernels" not in rec:
        return None
    return rec


def traffic_of(prof, prefixes):
    """(HBM bytes per step, dispatches per step) of the kernels whose names
    start with any of prefixes, from a profile record."""
    if not prof:
        return None, None
    b = n = 0.0
    steps = prof.get("steps", 1)
    for k, v in prof["kernels"].items():
        if any(k.startswith(p) for p in prefixes):
            b += v["fetch_bytes"] + v["write_bytes"]
            n += v["dispatches"]
    return (b / steps if n else None), (n / steps or None)


def rooflines(summ, res, steps, N, prof):
    """HBM rooflines of the bulk labelling and the sweep, the integer-ALU
    roofline of the keys kernel, and "roofline" = the phase with the largest
    kernel time per step."""
    ph = summ["phase_ms_per_step"]
    sweep_launches = res["phase"]["sweep_launches"] / steps
    out = {}
    t, _ = traffic_of(prof, ["nz::nz_sweep_kernel"])
    out["roofline_sweep"] = hbm_roofline("nz_sweep_kernel", summ["sweep_alg_bytes"], ph["sweep_ms"],
                                         max(sweep_launches, 1.0), t / max(sweep_launches, 1.0) if t else None)
    lab = summ["labelling_ms_per_step"]
    nlab = summ["labelling_dispatches_per_step"]
    if summ["prefill_alg_bytes"] > 0 and nlab > 0:
        lab_ms = sum(lab.values())
        t, _ = traffic_of(prof, ["nz::nz_hook_kernel", "nz::nz_compress_kernel", "nz::nz_accum_kernel"])
        r = hbm_roofline("bulk labelling (nz_hook_kernel, nz_compress_kernel, nz_accum_kernel)",
                         summ["prefill_alg_bytes"], lab_ms, nlab, t / nlab if t else None)
        r["kernel_ms_split"] = {k: v / nlab for k, v in lab.items()}
        out["roofline_prefill"] = r
    keys = keys_roofline(N * len(res["ns"]), ph["keys_ms"], prof)
    out["roofline_keys"] = keys
    share = {"roofline_sweep": ph["sweep_ms"], "roofline_keys": ph["keys_ms"],
             "roofline_prefill": sum(lab.values()) if "roofline_prefill" in out else 0.0}
    out["roofline"] = dict(out[max(share, key=share.get)])
    out["roofline_share_ms_per_step"] = share
    return out


def keys_roofline(sites_step, keys_ms_step, prof):
    """Keys kernel: sites keyed per second against the chip's measured rate of
    the Philox4x32-10 arithmetic alone (profiles/alu_peak.json: ten rounds of
    two v_mad_u64_u32 and two v_bitop3_b32 per block of two sites, timed on
    every CU), or, without that file, 256 CUs x 64 lanes x 2.4 GHz over 34
    integer operations per site."""
    achieved = sites_step / (keys_ms_step / 1e3) / 1e9 if keys_ms_step > 0 else 0.0
    peak_path = os.path.join(ROOT, "profiles", "alu_peak.json")
    if os.path.exists(peak_path):
        pk = json.load(open(peak_path))
        peak, basis = pk["philox_sites_per_s"] / 1e9, "measured Philox4x32-10 block rate (profiles/alu_peak.json)"
    else:
        peak, basis = 256 * 64 * 2.4e9 / 34 / 1e9, "256 CUs x 64 lanes x 2.4 GHz / 34 operations per site"
    t, n = traffic_of(prof, ["nz::nz_keys_kernel"])
    # the whole step's keys at the peak rate: the floor the keys set under
    # ms_per_step
    return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Gsites/s", "frac": achieved / peak,
            "traffic": t / n if t else None, "kernel": "nz_keys_kernel", "launches_per_step": n,
            "kernel_ms": keys_ms_step / n if n else None, "peak_basis": basis,
            "floor_ms_per_step": sites_step / (peak * 1e9) * 1e3}


def host_cpu():
    """The host's CPU: logical CPUs, the ones this process may run on, model
    name and socket count (from /proc/cpuinfo)."""
    model, sockets = None, set()
    try:
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k = k.strip()
            if k == "model name" and model is None:
                model = v.strip()
            elif k == "physical id":
                sockets.add(v.strip())
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model,
            "sockets": len(sockets) or None}


def cpu_threads():
    """Host threads for the oracle: every CPU this process may run on, capped by
    OMP_NUM_THREADS where the host sets it (a GPU host allots a share of its
    cores to each GPU)."""
    n = len(os.sched_getaffinity(0))
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def cpu_baseline(jobs, per_mask, threads):
    """The oracle's own Newman-Ziff (keys, full sort, serial union-find) on
    samples 0..per_mask-1 of every job, one sample per thread at a time (the
    paper's ordinary work division); returns additions/s, the results and the
    keys / sort / sweep thread-seconds."""
    import oracle

    adds = 0
    res = {}
    split = np.zeros(3)
    t0 = time.perf_counter()
    for j in jobs:
        ns, ms, tm = oracle.sweep_many(j["L"], j["zone_mask"], j["seed"], 0, per_mask, nthreads=threads, times=True)
        res[j["zone_mask"]] = (ns, ms)
        adds += int(ns.sum())
        split += tm
    wall = time.perf_counter() - t0
    return adds / wall, res, {"keys_s": split[0], "sort_s": split[1], "sweep_s": split[2], "wall_s": wall}


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
    ap.add_argument("--l24-only", action="store_true",
                    help="profiling aid: time only the L=24 table (27 masks) in --mode, --steps and --warmup, and "
                         "print its figures")
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
        batches = [(f"L={L} x 7 compact x {S}, plain", learned.plan_band_only(model, jobs0), None),
                   (f"L={L} x 7 compact x {S}, learned", model.plan(jobs0),
                    lambda k, kw, sz: model.plan(jobs0, k_sigma=k, k_sigma_wide=kw, split_z=sz))]
        if args.l24_samples > 0:
            j24 = base_jobs(24, args.l24_samples, masks24)
            batches += [(f"L=24 x 27 masks x {args.l24_samples}, plain", learned.plan_band_only(model, j24), None),
                        (f"L=24 x 27 masks x {args.l24_samples}, learned", model.plan(j24),
                         lambda k, kw, sz: model.plan(j24, k_sigma=k, k_sigma_wide=kw, split_z=sz))]
        for name, jobs, replan in batches:
            e = autotune.tune_batch(jobs, log=lambda m: print(f"{name}: {m}", flush=True), replan=replan)
            autotune.add_batch(table, jobs, e, name)
            print(f"{name}: best {e['tune']} {e['ms']} ms (default {e['default_ms']} ms)", flush=True)
        autotune.save_table(table, args.autotune_out)
        return

    if args.l24_only:
        j24 = base_jobs(24, args.l24_samples, masks24)
        S24 = args.l24_samples
        res = {}
        for mode in (("plain", "learned") if args.mode == "both" else (args.mode,)):
            p24 = autotune.plan_for(model.plan(j24))
            mk = (lambda: learned.plan_band_only(model, j24)) if mode == "plain" else (lambda: model.plan(j24, **p24))
            r = run_mode(nz, torch, mk, args.steps, args.warmup, autotune.for_jobs(mk()) or None)
            res[mode] = (r, summarise(r, args.steps, S24, z))
        out = {"workload": f"L=24 (N={24**5}) x 27 masks x {S24}", "masks": masks24}
        for mode, (r, sm) in res.items():
            out[mode] = sm
            out[mode].update(rooflines(sm, r, args.steps, 24**5,
                                       profile_record(f"nz_sweep_L24_27masks_x{S24}_{mode}")))
        print(json.dumps(out), flush=True)
        return

    if args.mode in ("both", "plain"):
        jp = learned.plan_band_only(model, jobs0)
        plain = run_mode(nz, torch, lambda: learned.plan_band_only(model, jobs0), args.steps, args.warmup,
                         autotune.for_jobs(jp) or None)
    if args.mode in ("both", "learned"):
        # the prefill depth the batch was tuned with (mean - 3 std by default)
        p16 = autotune.plan_for(model.plan(jobs0))
        jl = model.plan(jobs0, **p16)
        learn = run_mode(nz, torch, lambda: model.plan(jobs0, **p16), args.steps, args.warmup,
                         autotune.for_jobs(jl) or None)
    if args.mode == "plain":
        learn = plain
    elif args.mode == "learned":
        plain = learn
    identical = bool((plain["ns"] == learn["ns"]).all() and (plain["ms"] == learn["ms"]).all())
    sp = summarise(plain, args.steps, S, z)
    sl = summarise(learn, args.steps, S, z)

    prof = profile_record(f"nz_sweep_L{L}_compact_x{S}_learned")
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
    }
    out.update(rooflines(sl, learn, args.steps, N, prof))
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
        pl24 = autotune.plan_for(model.plan(j24))
        jp24, jl24 = learned.plan_band_only(model, j24), model.plan(j24, **pl24)
        p24 = run_mode(nz, torch, lambda: learned.plan_band_only(model, j24), 1, 1, autotune.for_jobs(jp24) or None)
        l24 = run_mode(nz, torch, lambda: model.plan(j24, **pl24), 1, 1, autotune.for_jobs(jl24) or None)
        s24p, s24l = summarise(p24, 1, args.l24_samples, z), summarise(l24, 1, args.l24_samples, z)
        out["L24"] = {"samples_per_mask": args.l24_samples, "masks": masks24,
                      "per_mask": per_mask(24, args.l24_samples) if not args.no_per_mask else None,
                      "outputs_identical_plain_vs_learned": bool((p24["ns"] == l24["ns"]).all() and
                                                                 (p24["ms"] == l24["ms"]).all()),
                      "speedup_learned_vs_plain": s24p["ms_per_step"] / s24l["ms_per_step"],
                      "learned": s24l, "plain": s24p}
        # the learned path's rooflines at L = 24, as at L = 16
        out["L24"].update(rooflines(s24l, l24, 1, 24**5,
                                    profile_record(f"nz_sweep_L24_27masks_x{args.l24_samples}_learned")))
    if not args.no_cpu:
        # the oracle on the host: all the threads this process may use (every
        # thread takes the same number of samples of each mask, about 10 s on
        # 16 host cores at L = 16), then one thread on a subset of them; the
        # GPU's n* and mass must equal the oracle's on every sample timed
        threads = cpu_threads()
        per = min(S, threads * (8 if L >= 16 else 32))
        cpu_rate, res, split = cpu_baseline(jobs0, per, threads)
        per1 = min(per, 2 if L >= 16 else 16)
        one_rate, res1, split1 = cpu_baseline(jobs0, per1, 1)
        parity = all((res[m][0] == learn["ns"][k * S:k * S + per]).all() and
                     (res[m][1] == learn["ms"][k * S:k * S + per]).all() for k, m in enumerate(COMPACT))
        parity = parity and all((res1[m][0] == learn["ns"][k * S:k * S + per1]).all() for k, m in enumerate(COMPACT))
        out["cpu_baseline"] = {"value": cpu_rate, "unit": "site additions/s", "cores": threads, "kind": "oracle",
                               "sample": f"samples 0..{per - 1} of each of the 7 masks at L={L}, one sample per "
                                         f"thread at a time on {threads} threads (keys, full sort, serial "
                                         f"union-find)",
                               "host": host_cpu(),
                               "thread_seconds": split,
                               "single_core": {"value": one_rate, "unit": "site additions/s", "threads": 1,
                                               "sample": f"samples 0..{per1 - 1} of each of the 7 masks",
                                               "thread_seconds": split1},
                               "samples_per_s": len(COMPACT) * per / split["wall_s"]}
        out["parity_on_cpu_sample"] = bool(parity)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
