"""A plain device copy of known size, to calibrate the HBM traffic counters.

The profiles scale rocprofv3's FETCH_SIZE and WRITE_SIZE (KiB per dispatch)
into bytes with one factor each; this copy measures those factors.  It copies
a 1 GiB int32 tensor into another three times (1 GiB read and 1 GiB written
per dispatch):

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT_F -o c -- python3 -m paper_2607_18991_amd.copy_calibration
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT_W -o c -- python3 -m paper_2607_18991_amd.copy_calibration
    python -m paper_2607_18991_amd.copy_calibration --summarize OUT_F OUT_W --commands FILE

The last command writes profiles/copy_calibration_1GiB.md: per kernel, the
counters' bytes per dispatch beside the bytes the copy moves, and the factor
that maps one onto the other.
"""
from __future__ import annotations

import argparse
import os

BYTES = 1 << 30
REPEATS = 3


def run_copy():
    import torch

    torch.cuda.set_device(0)
    a = torch.ones(BYTES // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(REPEATS):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {BYTES} bytes x {REPEATS}", flush=True)


def summarize(fetch_dir: str, write_dir: str, commands: str, out: str):
    from .profile_summary import counters

    fetch = counters(fetch_dir, "FETCH_SIZE")
    write = counters(write_dir, "WRITE_SIZE")
    lines = ["# Traffic counter calibration: a 1 GiB device copy", "",
             "Commands (on an MI355X, from the repository root):", "", "```"]
    lines += open(commands).read().strip().splitlines()
    lines += ["```", "", f"Each dispatch of the copy reads {BYTES} bytes and writes {BYTES} bytes.", "",
              "| kernel | dispatches | FETCH_SIZE bytes / dispatch | read / FETCH | WRITE_SIZE bytes / dispatch | "
              "written / WRITE |", "|---|---|---|---|---|---|"]
    for k in sorted(set(fetch) | set(write)):
        nf, kf = fetch.get(k, [0, 0.0])
        nw, kw = write.get(k, [0, 0.0])
        fb = kf * 1024 / nf if nf else 0.0
        wb = kw * 1024 / nw if nw else 0.0
        if fb < BYTES / 16 or wb < BYTES / 16:
            continue   # not the copy (the tensor fill writes only)
        lines.append(f"| `{k}` | {max(nf, nw)} | {fb:.4g} | {BYTES / fb if fb else float('nan'):.3f} | "
                     f"{wb:.4g} | {BYTES / wb if wb else float('nan'):.3f} |")
    lines += ["", "The profiles' traffic figures use these two factors (FETCH_SIZE x 2, WRITE_SIZE x 1).", ""]
    with open(out, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--summarize", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--commands")
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", "profiles",
                                                  "copy_calibration_1GiB.md"))
    args = ap.parse_args()
    if args.summarize:
        if not args.commands:
            ap.error("--summarize needs --commands")
        summarize(args.summarize[0], args.summarize[1], args.commands, args.out)
    else:
        run_copy()


if __name__ == "__main__":
    main()
