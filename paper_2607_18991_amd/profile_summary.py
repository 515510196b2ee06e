"""Summaries of rocprofv3 runs of the benchmark for the profiles/ folder.

From a kernel-trace run (--kernel-trace --stats) and two counter runs
(--pmc FETCH_SIZE, --pmc WRITE_SIZE) of the same command, it writes
profiles/<name>.md (per-kernel time and HBM traffic, with the commands) and
profiles/<name>.json, the traffic of every kernel over the counter runs'
steps together with the SHA-1 of the kernel and launch-planner sources it was
measured on; bench.py reports that traffic only while those sources are
unchanged.

Counter scaling: FETCH_SIZE and WRITE_SIZE are KiB per dispatch; a plain
device copy of 1 GiB reads FETCH_SIZE = 0.5 GiB and WRITE_SIZE = 1 GiB on
this chip (copy_calibration.py measures it), so fetched bytes are
FETCH_SIZE * 1024 * FETCH_SCALE and written bytes WRITE_SIZE * 1024 *
WRITE_SCALE.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
# the kernels and the host planner that decides their launches
KERNEL_SOURCES = (os.path.join(HERE, "csrc", "nz_kernels.hip"), os.path.join(HERE, "csrc", "nz_api.cpp"))
FETCH_SCALE = 2.0
WRITE_SCALE = 1.0


def source_sha1(paths=KERNEL_SOURCES) -> str:
    h = hashlib.sha1()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short(name: str) -> str:
    n = name[5:] if name.startswith("void ") else name
    return n.split("(")[0]


def _find(dirname: str, suffix: str) -> str:
    for root, _, files in os.walk(dirname):
        for f in files:
            if f.endswith(suffix):
                return os.path.join(root, f)
    raise FileNotFoundError(f"no *{suffix} under {dirname}")


def kernel_stats(dirname: str):
    rows = []
    for r in csv.DictReader(open(_find(dirname, "kernel_stats.csv"))):
        rows.append(dict(kernel=short(r["Name"]), calls=int(r["Calls"]), total_ms=float(r["TotalDurationNs"]) / 1e6,
                         avg_ms=float(r["AverageNs"]) / 1e6, pct=float(r["Percentage"])))
    return rows


def counters(dirname: str, counter: str):
    """Per kernel: (dispatches, summed counter value in KiB)."""
    agg = defaultdict(lambda: [0, 0.0])
    for r in csv.DictReader(open(_find(dirname, "counter_collection.csv"))):
        if r["Counter_Name"] != counter:
            continue
        k = short(r["Kernel_Name"])
        agg[k][0] += 1
        agg[k][1] += float(r["Counter_Value"])
    return agg


def timeline(dirname: str, marker: str = "nzmlp::mlp_forward_kernel"):
    """The last bench step of a kernel-trace run as one row per dispatch:
    (queue, kernel, start ms, end ms) relative to the step's first dispatch.
    Steps start with the prefill MLP's forward kernel (every step plans its
    jobs), so the last step is everything from the last such dispatch on."""
    rows = []
    for r in csv.DictReader(open(_find(dirname, "kernel_trace.csv"))):
        q = r.get("Stream_Id") or r.get("Queue_Id") or "0"
        rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), q, short(r["Kernel_Name"])))
    rows.sort()
    starts = [i for i, row in enumerate(rows) if row[3].startswith(marker)]
    first = starts[-1] if starts else 0
    t0 = rows[first][0]
    return [(q, k, (a - t0) / 1e6, (b - t0) / 1e6) for a, b, q, k in rows[first:]]


def timeline_md(rows, title: str):
    """Markdown of timeline(): per queue, its kernels in start order, plus the
    busy span of each queue."""
    lines = [f"### {title}", "", "| queue | kernel | start ms | end ms | ms |", "|---|---|---|---|---|"]
    for q in sorted(set(r[0] for r in rows), key=str):
        mine = [r for r in rows if r[0] == q]
        for _, k, a, b in mine:
            if b - a >= 0.05:
                lines.append(f"| {q} | `{k}` | {a:.2f} | {b:.2f} | {b - a:.2f} |")
        lines.append(f"| {q} | **span** | {min(r[2] for r in mine):.2f} | {max(r[3] for r in mine):.2f} | "
                     f"{max(r[3] for r in mine) - min(r[2] for r in mine):.2f} |")
    return lines


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--stats", required=True, help="output folder of the --kernel-trace --stats run")
    ap.add_argument("--fetch", required=True, help="output folder of the --pmc FETCH_SIZE run")
    ap.add_argument("--write", required=True, help="output folder of the --pmc WRITE_SIZE run")
    ap.add_argument("--name", required=True)
    ap.add_argument("--title", required=True)
    ap.add_argument("--commands", required=True, help="text file with the commands")
    ap.add_argument("--l2", default=None, help="output folder of a --pmc TCC_HIT_sum TCC_MISS_sum run (optional)")
    ap.add_argument("--steps", type=int, default=2, help="bench steps in the stats run (warm-up included)")
    ap.add_argument("--sweep", default="nz::nz_sweep_kernel")
    ap.add_argument("--counter-steps", type=int, default=1, help="bench steps in each counter run")
    ap.add_argument("--outdir", default=os.path.join(HERE, "..", "profiles"))
    ap.add_argument("--timeline", action="store_true",
                    help="add the last step's dispatches per queue from the --stats run's kernel trace")
    args = ap.parse_args()

    stats = kernel_stats(args.stats)
    fetch = counters(args.fetch, "FETCH_SIZE")
    write = counters(args.write, "WRITE_SIZE")
    lines = [f"# {args.title}", "", "Commands (on an MI355X, from the repository root):", "", "```"]
    lines += open(args.commands).read().strip().splitlines()
    lines += ["```", "", f"Kernel time ({args.steps} bench steps in the trace run):", "",
              "| kernel | calls | total ms | average ms | % |", "|---|---|---|---|---|"]
    for r in stats:
        lines.append(f"| `{r['kernel']}` | {r['calls']} | {r['total_ms']:.3f} | {r['avg_ms']:.3f} | {r['pct']:.1f} |")
    lines += ["", f"HBM traffic (one step; FETCH_SIZE x {FETCH_SCALE:g}, WRITE_SIZE x {WRITE_SCALE:g}, "
                  "calibrated on a 1 GiB device copy):", "",
              "| kernel | dispatches | fetched GB | written GB |", "|---|---|---|---|"]
    for k in sorted(set(fetch) | set(write), key=lambda k: -(fetch.get(k, [0, 0])[1] + write.get(k, [0, 0])[1])):
        f_gb = fetch.get(k, [0, 0.0])[1] * 1024 * FETCH_SCALE / 1e9
        w_gb = write.get(k, [0, 0.0])[1] * 1024 * WRITE_SCALE / 1e9
        n = max(fetch.get(k, [0, 0])[0], write.get(k, [0, 0])[0])
        if f_gb + w_gb < 1e-3:
            continue
        lines.append(f"| `{k}` | {n} | {f_gb:.2f} | {w_gb:.2f} |")
    if args.l2:
        hit = counters(args.l2, "TCC_HIT_sum")
        miss = counters(args.l2, "TCC_MISS_sum")
        lines += ["", "L2 (one step; TCC_HIT_sum and TCC_MISS_sum, requests summed over the dispatches):", "",
                  "| kernel | dispatches | L2 requests (M) | hit rate |", "|---|---|---|---|"]
        for k in sorted(set(hit) | set(miss), key=lambda k: -(hit.get(k, [0, 0])[1] + miss.get(k, [0, 0])[1])):
            h, mi = hit.get(k, [0, 0.0])[1], miss.get(k, [0, 0.0])[1]
            if h + mi < 1e5:
                continue
            n = max(hit.get(k, [0, 0])[0], miss.get(k, [0, 0])[0])
            lines.append(f"| `{k}` | {n} | {(h + mi) / 1e6:.1f} | {h / (h + mi):.3f} |")
    if args.timeline:
        lines += [""] + timeline_md(timeline(args.stats), "Timeline of the last step (dispatches of 0.05 ms or more)")
    # per kernel (template instances summed): dispatches and bytes over the
    # counter runs, which time args.counter_steps bench steps
    kern = defaultdict(lambda: {"dispatches": 0, "fetch_bytes": 0.0, "write_bytes": 0.0})
    for k, (n, v) in fetch.items():
        base = k.split("<")[0]
        kern[base]["dispatches"] += n
        kern[base]["fetch_bytes"] += v * 1024 * FETCH_SCALE
    for k, (n, v) in write.items():
        base = k.split("<")[0]
        kern[base]["write_bytes"] += v * 1024 * WRITE_SCALE
    rec = {"steps": args.counter_steps, "kernels": dict(kern), "source_sha1": source_sha1()}
    sw = kern.get(args.sweep, {"dispatches": 0, "fetch_bytes": 0.0, "write_bytes": 0.0})
    launches = max(1, sw["dispatches"])
    lines += ["", f"Sweep kernel per launch: {sw['fetch_bytes'] / launches / 1e9:.3f} GB fetched, "
                  f"{sw['write_bytes'] / launches / 1e9:.3f} GB written over {launches} launches; kernel source "
                  f"SHA-1 {rec['source_sha1'][:12]}.", ""]
    os.makedirs(args.outdir, exist_ok=True)
    with open(os.path.join(args.outdir, args.name + ".md"), "w") as f:
        f.write("\n".join(lines))
    with open(os.path.join(args.outdir, args.name + ".json"), "w") as f:
        json.dump(rec, f, indent=1)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
