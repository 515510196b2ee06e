"""Autotuner of the persistent sweep: for every (L, z-class) it times the
candidate launch shapes on the GPU -- where the per-sample state lives (HBM,
occupancy bitset in LDS, bitset and parents in LDS), waves per workgroup,
resident waves per SIMD, one site or 64 sites per wave step, and whether the
HBM-resident sweep checks the bitset summary -- and keeps the fastest in a
JSON table shipped with the package.  Tuning never changes an
output (the library guarantees it and the tests check it); it only moves time.

z-classes follow the offset chunks the kernels are compiled for: z <= 64, 128,
256, 512, 892.

    python -m paper_2607_18991_amd.autotune --out tuning_table.json

rebuilds the table (one MI355X, a few minutes).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import time

from . import nz

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_table.json")
FORMAT = "nz-tuning-1"
ZCLASSES = (64, 128, 256, 512, 892)
# a representative neighbourhood per z-class (z = 10, 80, 130, 332, 892)
REPRESENTATIVE = {64: 0x01, 128: 0x04, 256: 0x07, 512: 0x1F, 892: 0x7F}
DEFAULT_LS = (4, 8, 10, 12, 16, 20, 24)


def zclass(z: int) -> int:
    for c in ZCLASSES:
        if z <= c:
            return c
    raise ValueError(f"z = {z} above 892")


def key(L: int, zc: int) -> str:
    return f"{int(L)}:{int(zc)}"


def candidates(L: int):
    """Launch shapes worth timing at side L (LDS residencies only where the
    state can fit one wave's slice)."""
    N = L**5
    bitset_bytes = ((N + 63) // 64) * 8
    out = []
    for mode in (1, 2):
        for wps in (4, 8):
            for wg in (1, 4):
                for summary in (1, 2):
                    out.append(dict(residency=2, wg_waves=wg, waves_per_simd=wps, sweep_mode=mode, summary=summary))
        if bitset_bytes <= 150 * 1024:
            out.append(dict(residency=1, wg_waves=1, waves_per_simd=8, sweep_mode=mode))
        if bitset_bytes + 4 * N <= 150 * 1024:
            out.append(dict(residency=3, wg_waves=1, waves_per_simd=8, sweep_mode=mode))
    return out


def _time_batch(jobs, tune, reps=2):
    import torch

    total = sum(j["nsamples"] for j in jobs)
    ws = torch.empty(nz.nz_batch_workspace_bytes(jobs, tune), dtype=torch.uint8, device="cuda")
    dn = torch.empty(total, dtype=torch.int32, device="cuda")
    nz.nz_sweep_batch(jobs, ws, dn, None, tune=tune)   # warm-up
    best = float("inf")
    for _ in range(reps):
        nz.nz_set_timing(True)
        nz.nz_sweep_batch(jobs, ws, dn, None, tune=tune)
        t = nz.nz_last_batch_timing()
        nz.nz_set_timing(False)
        best = min(best, t["total_ms"])
    return best, dn.cpu().numpy()


def tune_class(L: int, zc: int, samples: int, model=None, log=None):
    """Times every candidate on `samples` samples of the class's representative
    neighbourhood (learned prefill when a model is given) and returns the
    table entry.  Every candidate must reproduce the default's outputs."""
    mask = REPRESENTATIVE[zc]
    jobs = [dict(L=L, zone_mask=mask, seed=0xA070_0000 + 131 * L + zc, nsamples=samples)]
    if model is not None:
        jobs = model.plan(jobs)
    base_ms, ref = _time_batch(jobs, None)
    best = (base_ms, None)
    tried = []
    for cand in candidates(L):
        try:
            ms, out = _time_batch(jobs, cand)
        except nz.NzError as e:
            tried.append(dict(tune=cand, error=str(e)))
            continue
        if not (out == ref).all():
            raise RuntimeError(f"tuning {cand} changed outputs at L={L}, mask {mask:#x}")
        tried.append(dict(tune=cand, ms=round(ms, 3)))
        if ms < best[0]:
            best = (ms, cand)
        if log:
            log(f"L={L} z<={zc} {cand} {ms:.3f} ms")
    return {"tune": best[1] or {}, "ms": round(best[0], 3), "default_ms": round(base_ms, 3), "mask": mask,
            "samples": samples, "tried": tried}


def samples_for(L: int) -> int:
    return 512 if L <= 12 else (256 if L <= 16 else 64)


def build_table(Ls=DEFAULT_LS, model=None, log=print):
    import torch

    entries = {}
    for L in Ls:
        for zc in ZCLASSES:
            entries[key(L, zc)] = tune_class(L, zc, samples_for(L), model, log)
    return {"format": FORMAT, "device": torch.cuda.get_device_name(0), "created": time.strftime("%Y-%m-%d"),
            "entries": entries}


# ------------------------------------------------------------------ batches
# A mixed batch runs as one sweep launch per chunk, so a batch that is run
# repeatedly (a benchmark, a production table) is tuned as a whole and its
# entry is keyed by the batch's signature.

def signature(jobs) -> str:
    parts = sorted(f"{int(j['L'])}:{int(j['zone_mask'])}:{int(j['nsamples'])}:{int(int(j.get('n0', -1)) >= 0)}"
                   for j in jobs)
    return hashlib.sha1("|".join(parts).encode()).hexdigest()[:16]


def batch_candidates():
    return [dict(residency=2, wg_waves=wg, waves_per_simd=wps, sweep_mode=mode, summary=summary)
            for mode in (0, 1, 2) for wps in (4, 8) for wg in (1, 4) for summary in (1, 2)]


# widest neighbourhood of the first group when a batch runs as two groups
SPLIT_Z = (10, 64, 130, 170, 242, 340)
# prefill depth: n0 = (mean - k std) N
K_SIGMA = (3.0, 2.5, 2.0, 1.5, 1.0)


def tune_batch(jobs, reps: int = 2, log=None, replan=None):
    """Times the batch under every batch candidate, then the best one under
    every split of the batch into two groups, then (replan(k, k_wide, split_z)
    given: the jobs planned with prefill depth mean - k std, and mean - k_wide
    std for the jobs wider than split_z) every prefill depth for all jobs, and
    then every depth for the wide jobs alone; every candidate must reproduce
    the default's outputs."""
    base_ms, ref = _time_batch(jobs, None, reps)
    best = (base_ms, None)
    tried = []

    def consider(cand, js, extra=None):
        nonlocal best
        ms, out = _time_batch(js, cand, reps)
        if not (out == ref).all():
            raise RuntimeError(f"tuning {cand} {extra} changed the outputs of the batch")
        tried.append(dict(tune=cand, ms=round(ms, 3), **({"plan": extra} if extra else {})))
        if log:
            log(f"batch {cand} {extra or ''} {ms:.3f} ms")
        return ms

    for cand in batch_candidates():
        ms = consider(cand, jobs)
        if ms < best[0]:
            best = (ms, cand)
    for sz in SPLIT_Z:
        cand = dict(best[1] or {}, split_z=sz)
        ms = consider(cand, jobs)
        if ms < best[0]:
            best = (ms, cand)
    plan = None
    if replan is not None:
        for k in K_SIGMA:
            ms = consider(best[1], replan(k, None, None), {"k_sigma": k})
            if ms < best[0]:
                best = (ms, best[1])
                plan = {"k_sigma": k}
        k0 = (plan or {}).get("k_sigma", 3.0)
        sz = (best[1] or {}).get("split_z")
        for kw in K_SIGMA:
            if kw == k0:
                continue
            extra = {"k_sigma": k0, "k_sigma_wide": kw, "split_z": sz}
            ms = consider(best[1], replan(k0, kw, sz), extra)
            if ms < best[0]:
                best = (ms, best[1])
                plan = extra
    entry = {"tune": best[1] or {}, "ms": round(best[0], 3), "default_ms": round(base_ms, 3), "tried": tried,
             "samples": int(sum(int(j["nsamples"]) for j in jobs))}
    if plan:
        entry["plan"] = plan
    return entry


def add_batch(table, jobs, entry, name: str):
    table.setdefault("batches", {})[signature(jobs)] = dict(entry, name=name)


# ------------------------------------------------------------------ lookup
_table = None


def load_table(path: str = TABLE_PATH):
    global _table
    if _table is None or path != TABLE_PATH:
        if not os.path.exists(path):
            return {"format": FORMAT, "entries": {}}
        with open(path) as f:
            t = json.load(f)
        if t.get("format") != FORMAT:
            raise ValueError(f"{path}: unknown tuning table format {t.get('format')!r}")
        if path != TABLE_PATH:
            return t
        _table = t
    return _table


def lookup(L: int, zone_mask: int, table=None, nsamples: int | None = None):
    """Tuning dict for one (L, neighbourhood); {} (library defaults) if the
    table has no entry for it.  The summary choice depends on how many samples
    share the chip, so it is kept only for batches of at most as many samples
    as the entry was timed on (larger ones get the library's choice)."""
    t = table or load_table()
    e = t["entries"].get(key(L, zclass(nz.nz_coordination(zone_mask))))
    if not e:
        return {}
    tune = dict(e["tune"])
    if nsamples is not None and nsamples > int(e.get("samples", 0)):
        tune.pop("summary", None)
    return tune


# an LDS-resident sample takes a whole CU's LDS, so such residencies pay only
# while the batch has no more samples than there are CUs
LDS_RESIDENT_MAX_SAMPLES = 256


def for_jobs(jobs, table=None):
    """One tuning for a batch (the sweep is one launch per chunk): the batch's
    own entry if it was tuned as a whole, else the class entry of the job whose
    samples take longest -- the largest lattice, and among those the smallest
    neighbourhood, whose threshold lies highest -- kept in HBM residency when
    the batch has more samples than CUs."""
    if not jobs:
        return {}
    t = table or load_table()
    e = t.get("batches", {}).get(signature(jobs))
    if e:
        return dict(e["tune"])
    j = max(jobs, key=lambda j: (int(j["L"]), -nz.nz_coordination(int(j["zone_mask"]))))
    total = sum(int(j["nsamples"]) for j in jobs)
    tune = lookup(int(j["L"]), int(j["zone_mask"]), t, total)
    if tune.get("residency") in (1, 3) and total > LDS_RESIDENT_MAX_SAMPLES:
        tune.update(residency=2, wg_waves=1)
    return tune


def plan_for(jobs, table=None) -> dict:
    """Planner settings ({'k_sigma': ..., and possibly 'k_sigma_wide' and
    'split_z'}) of the batch's own entry, if it was tuned as a whole with
    them; {} otherwise.  They are the keyword arguments of
    learned.PrefillModel.plan."""
    t = table or load_table()
    e = t.get("batches", {}).get(signature(jobs)) if jobs else None
    return {k: v for k, v in e.get("plan", {}).items() if v is not None} if e else {}


def save_table(table, path: str = TABLE_PATH):
    global _table
    with open(path, "w") as f:
        json.dump(table, f, indent=1)
    if path == TABLE_PATH:
        _table = None


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", default=TABLE_PATH)
    ap.add_argument("--L", type=int, nargs="*", default=list(DEFAULT_LS))
    ap.add_argument("--plain", action="store_true", help="time plain sweeps instead of learned-prefill ones")
    args = ap.parse_args()
    import torch

    from . import learned

    torch.cuda.set_device(0)
    model = None if args.plain else learned.PrefillModel.load()
    table = build_table(args.L, model, log=lambda s: print(s, flush=True))
    if os.path.exists(args.out):
        with open(args.out) as f:
            old = json.load(f)
        table["batches"] = old.get("batches", {})   # tuned batches are kept
    save_table(table, args.out)
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
