"""Host-side measurement code on synthetic inputs (CPU): the benchmark's
neighbour-check accounting, the profile summaries (time, traffic, L2 tables
and the per-launch record the benchmark reads) and the counter calibration."""
import csv
import json
import os

import numpy as np

import bench
from paper_2607_18991_amd import copy_calibration, profile_summary


def test_neighbour_checks_split_by_mask():
    # two masks (z = 10 and 50), two samples each; the library counts 40
    # sequential additions and 150 prefilled sites for the batch
    res = {"wall": 0.5, "ns": np.array([100, 110, 50, 60]),
           "stats": {"serial_steps": 40, "prefilled_sites": 150, "backoffs": 0},
           "jobs": [dict(zone_mask=1, n0=80), dict(zone_mask=3, n0=40)],
           "phase": {"keys_ms": 1.0, "cc_ms": 2.0, "sort_ms": 1.0, "sweep_ms": 4.0, "total_ms": 8.0,
                     "sweep_launches": 1},
           "tune": None}
    out = bench.summarise(res, 1, 2, {1: 10, 3: 50})
    # sweep: additions split 50:30 (n* - n0), z = 10 and 50
    assert np.isclose(out["neighbour_checks_per_step"]["sweep"], 40 * (50 / 80 * 10 + 30 / 80 * 50))
    # prefill: sites split 160:80 (n0 per sample), half the offsets each
    assert np.isclose(out["neighbour_checks_per_step"]["prefill"], 150 * (2 / 3 * 5 + 1 / 3 * 25))
    total = out["neighbour_checks_per_step"]["sweep"] + out["neighbour_checks_per_step"]["prefill"]
    assert np.isclose(out["neighbour_checks_per_s"], total / 0.5)
    assert np.isclose(out["neighbour_checks_per_s_in_phase"]["sweep"],
                      out["neighbour_checks_per_step"]["sweep"] / 4e-3)
    # plain runs have no prefill checks
    plain = dict(res, jobs=[dict(zone_mask=1, n0=-1), dict(zone_mask=3)],
                 stats=dict(res["stats"], prefilled_sites=0))
    out = bench.summarise(plain, 1, 2, {1: 10, 3: 50})
    assert out["neighbour_checks_per_step"]["prefill"] == 0.0
    assert out["neighbour_checks_per_s_in_phase"]["prefill"] is None


_COLS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _counter_dir(root, name, rows):
    d = root / name
    d.mkdir()
    with open(d / "c_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=_COLS)
        w.writeheader()
        for i, (kernel, counter, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": kernel, "Counter_Name": counter, "Counter_Value": value})
    return str(d)


def test_profile_summary_tables_and_record(tmp_path, monkeypatch):
    sweep, keys = "void nz::nz_sweep_kernel<1, 0, true, 1, false>(NzSweepArgs, nz::SweepOut)", "nz::nz_keys_kernel"
    stats = tmp_path / "stats"
    stats.mkdir()
    with open(stats / "m16_kernel_stats.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"])
        w.writerow([sweep, 2, 20e6, 10e6, 60.0])
        w.writerow([keys, 4, 12e6, 3e6, 40.0])
    fetch = _counter_dir(tmp_path, "f", [(sweep, "FETCH_SIZE", 1000.0), (keys, "FETCH_SIZE", 10.0),
                                         (keys, "FETCH_SIZE", 10.0)])
    write = _counter_dir(tmp_path, "w", [(sweep, "WRITE_SIZE", 500.0), (keys, "WRITE_SIZE", 300.0),
                                         (keys, "WRITE_SIZE", 100.0)])
    l2 = _counter_dir(tmp_path, "l2", [(sweep, "TCC_HIT_sum", 2e6), (sweep, "TCC_MISS_sum", 6e6),
                                       (keys, "TCC_HIT_sum", 3e6), (keys, "TCC_MISS_sum", 1e6)])
    cmds = tmp_path / "cmds.txt"
    cmds.write_text("rocprofv3 ...\n")
    out = tmp_path / "out"
    monkeypatch.setattr("sys.argv", ["x", "--stats", str(stats), "--fetch", fetch, "--write", write, "--l2", l2,
                                     "--name", "t", "--title", "T", "--commands", str(cmds), "--outdir", str(out)])
    profile_summary.main()
    md = (out / "t.md").read_text()
    assert "rocprofv3 ..." in md
    assert "| `nz::nz_sweep_kernel<1, 0, true, 1, false>` | 1 | 8.0 | 0.250 |" in md
    assert "| `nz::nz_keys_kernel` | 1 | 4.0 | 0.750 |" in md
    rec = json.loads((out / "t.json").read_text())
    # one sweep dispatch: FETCH_SIZE KiB x 1024 x 2, WRITE_SIZE KiB x 1024
    assert rec["launches"] == 1
    assert rec["fetch_bytes_per_launch"] == 1000 * 1024 * profile_summary.FETCH_SCALE
    assert rec["write_bytes_per_launch"] == 500 * 1024 * profile_summary.WRITE_SCALE
    assert rec["keys"]["dispatches"] == 2
    assert rec["keys"]["write_bytes_per_step"] == 400 * 1024 * profile_summary.WRITE_SCALE
    assert rec["source_sha1"] == profile_summary.source_sha1()


def test_copy_calibration_factors(tmp_path):
    kib = copy_calibration.BYTES / 1024
    fetch = _counter_dir(tmp_path, "f", [("__amd_rocclr_copyBuffer", "FETCH_SIZE", kib / 2)] * 3 +
                         [("fill", "FETCH_SIZE", 1.0)])
    write = _counter_dir(tmp_path, "w", [("__amd_rocclr_copyBuffer", "WRITE_SIZE", kib)] * 3 +
                         [("fill", "WRITE_SIZE", kib)])
    cmds = tmp_path / "cmds.txt"
    cmds.write_text("rocprofv3 ...\n")
    out = tmp_path / "cal.md"
    copy_calibration.summarize(fetch, write, str(cmds), str(out))
    md = out.read_text()
    assert "| `__amd_rocclr_copyBuffer` | 3 |" in md and "| 2.000 |" in md and "| 1.000 |" in md
    assert "fill" not in md   # writes only: not a copy
    assert os.path.getsize(out) > 0
