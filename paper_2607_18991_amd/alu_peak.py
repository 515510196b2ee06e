"""Measured integer peak of the keys kernel's arithmetic on this GPU.

Runs the issue-rate microbenchmarks of libnzpeak.so (csrc/alu_peak.hip) on
every compute unit: chains of v_mad_u64_u32, chains of v_bitop3_b32, and whole
Philox4x32-10 blocks (ten rounds of two of each, four blocks interleaved per
lane).  The Philox block rate times two (a block keys two sites) is the
ceiling the keys kernel is reported against: it is the chip's rate for the
Philox arithmetic alone, before any classification or store.

    python3 -m paper_2607_18991_amd.alu_peak --out profiles/alu_peak

writes profiles/alu_peak.json (the figures bench.py reads) and
profiles/alu_peak.md.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnzpeak.so")
CLOCK_HZ = 2.4e9
LANES = 64

KINDS = {0: "v_mad_u64_u32", 1: "v_bitop3_b32", 2: "Philox4x32-10 block"}


def run(which: int, grid: int, iters: int, reps: int = 5):
    import torch  # noqa: F401  (one HIP runtime per process: torch's)

    lib = ctypes.CDLL(LIB_PATH)
    lib.nzpeak_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.nzpeak_run.restype = ctypes.c_int
    ms, units = ctypes.c_double(), ctypes.c_double()
    rc = lib.nzpeak_run(which, grid, iters, reps, ctypes.byref(ms), ctypes.byref(units))
    if rc != 0:
        raise RuntimeError(f"nzpeak_run({which}) failed with code {rc}")
    return ms.value, units.value


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", default=os.path.join(HERE, "..", "profiles", "alu_peak"))
    ap.add_argument("--wgs-per-cu", type=int, default=8)
    args = ap.parse_args()
    import torch

    torch.cuda.set_device(0)
    props = torch.cuda.get_device_properties(0)
    cus = props.multi_processor_count
    grid = cus * args.wgs_per_cu
    lane_ops = cus * LANES * CLOCK_HZ
    rows = {}
    for which, iters in ((0, 4096), (1, 8192), (2, 256)):
        ms, units = run(which, grid, iters)
        rate = units / (ms / 1e3)
        rows[KINDS[which]] = {"ms": ms, "units_per_launch": units, "per_s": rate}
        print(f"{KINDS[which]}: {ms:.3f} ms, {rate:.4g} per s", flush=True)
    mad = rows["v_mad_u64_u32"]["per_s"]
    b3 = rows["v_bitop3_b32"]["per_s"]
    blocks = rows["Philox4x32-10 block"]["per_s"]
    rec = {"device": props.name, "cus": cus, "grid": grid, "clock_hz_assumed": CLOCK_HZ,
           "v_mad_u64_u32_per_s": mad, "v_bitop3_b32_per_s": b3,
           "v_mad_u64_u32_lanes_per_clock_per_cu": mad / cus / CLOCK_HZ,
           "v_bitop3_b32_lanes_per_clock_per_cu": b3 / cus / CLOCK_HZ,
           "philox_blocks_per_s": blocks, "philox_sites_per_s": 2.0 * blocks,
           "philox_block_from_rates_per_s": 1.0 / (20.0 / mad + 20.0 / b3), "runs": rows}
    lines = ["# Integer issue rates of the keys kernel's instructions (one MI355X)", "",
             "Command (from the repository root):", "", "```",
             "python3 -m paper_2607_18991_amd.alu_peak --out profiles/alu_peak", "```", "",
             f"{cus} CUs, {grid} workgroups of 256 lanes, fastest of 5 timed launches (HIP events); "
             f"rates in lane-instructions per second.", "",
             "| instruction | per second | lanes / clock / CU at 2.4 GHz | fraction of 64 lanes / clock |",
             "|---|---|---|---|"]
    for k, r in (("v_mad_u64_u32", mad), ("v_bitop3_b32", b3)):
        lines.append(f"| `{k}` | {r:.4g} | {r / cus / CLOCK_HZ:.2f} | {r / lane_ops:.3f} |")
    lines += ["", f"Philox4x32-10 (20 `v_mad_u64_u32` + 20 `v_bitop3_b32` per block, 4 blocks per lane): "
                  f"{blocks:.4g} blocks/s = **{2 * blocks:.4g} sites/s** (two sites per block); the two rates "
                  f"above would allow {1.0 / (20.0 / mad + 20.0 / b3):.4g} blocks/s if the instructions did "
                  f"not overlap.", ""]
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    with open(args.out + ".md", "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


if __name__ == "__main__":
    main()
