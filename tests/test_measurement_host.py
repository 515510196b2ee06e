"""Host-side measurement code on synthetic inputs (CPU): the benchmark's
neighbour-check accounting, the profile summaries (time, traffic, L2 tables
and the per-launch record the benchmark reads) and the counter calibration."""
import csv
import json
import os

import numpy as np

import bench
from paper_2607_18991_amd import copy_calibration, profile_summary


def test_per_job_accounting_bytes_and_checks():
    # two masks (z = 10 and 50), two samples each; the library counts, per
    # job, 25 and 15 sequential additions and 100 and 50 prefilled sites
    res = {"wall": 0.5, "ns": np.array([100, 110, 50, 60]),
           "stats": {"serial_steps": 40, "prefilled_sites": 150, "backoffs": 0},
           "serial": np.array([25, 15]), "prefilled": np.array([100, 50]),
           "jobs": [dict(L=4, zone_mask=1, nsamples=2, n0=80), dict(L=4, zone_mask=3, nsamples=2, n0=40)],
           "phase": {"keys_ms": 1.0, "cc_ms": 2.0, "sort_ms": 1.0, "sweep_ms": 4.0, "total_ms": 8.0,
                     "sweep_launches": 1},
           "cc": {"hook_ms": 1.0, "compress_ms": 0.25, "accum_ms": 0.25, "expand_ms": 0.5, "dispatches": 2},
           "tune": None}
    out = bench.summarise(res, 1, 2, {1: 10, 3: 50})
    # sweep: z per sequential addition of each job
    assert np.isclose(out["neighbour_checks_per_step"]["sweep"], 25 * 10 + 15 * 50)
    # prefill: half the offsets per prefilled site
    assert np.isclose(out["neighbour_checks_per_step"]["prefill"], 100 * 5 + 50 * 25)
    total = out["neighbour_checks_per_step"]["sweep"] + out["neighbour_checks_per_step"]["prefill"]
    assert np.isclose(out["neighbour_checks_per_s"], total / 0.5)
    assert np.isclose(out["neighbour_checks_per_s_in_phase"]["sweep"],
                      out["neighbour_checks_per_step"]["sweep"] / 4e-3)
    # bytes: 22 + z/8 per sequential addition; n0 (z/8 + 24) + N/8 per
    # prefilled sample for the labelling
    assert np.isclose(out["sweep_alg_bytes"], 25 * (22 + 10 / 8) + 15 * (22 + 50 / 8))
    assert np.isclose(out["prefill_alg_bytes"], 100 * (10 / 8 + 24) + 50 * (50 / 8 + 24) + 2 * 2 * 1024 / 8)
    r = bench.rooflines(out, res, 1, 1024, None)
    assert np.isclose(r["roofline_sweep"]["achieved"], out["sweep_alg_bytes"] / 4e-3 / 1e9)
    assert np.isclose(r["roofline_prefill"]["achieved"], out["prefill_alg_bytes"] / 2e-3 / 1e9)
    assert np.isclose(r["roofline_prefill"]["kernel_ms"], 1.0)
    assert r["roofline"]["kernel"] == "nz_sweep_kernel"    # 4 ms of sweep against 2 of labelling
    # plain runs have no prefill checks and no labelling roofline
    plain = dict(res, jobs=[dict(L=4, zone_mask=1, nsamples=2, n0=-1), dict(L=4, zone_mask=3, nsamples=2)],
                 prefilled=np.array([0, 0]), cc={"dispatches": 0})
    out = bench.summarise(plain, 1, 2, {1: 10, 3: 50})
    assert out["neighbour_checks_per_step"]["prefill"] == 0.0
    assert out["neighbour_checks_per_s_in_phase"]["prefill"] is None
    assert "roofline_prefill" not in bench.rooflines(out, plain, 1, 1024, None)


def test_cpu_threads_respect_the_host_share(monkeypatch):
    monkeypatch.setenv("OMP_NUM_THREADS", "3")
    assert bench.cpu_threads() == min(3, len(os.sched_getaffinity(0)))
    monkeypatch.delenv("OMP_NUM_THREADS")
    assert bench.cpu_threads() == len(os.sched_getaffinity(0))
    h = bench.host_cpu()
    assert h["nproc"] >= 1 and h["affinity"] >= 1


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
    # per kernel over the counter run's one step: FETCH_SIZE KiB x 1024 x 2,
    # WRITE_SIZE KiB x 1024
    sw = rec["kernels"]["nz::nz_sweep_kernel"]
    assert sw["dispatches"] == 1
    assert sw["fetch_bytes"] == 1000 * 1024 * profile_summary.FETCH_SCALE
    assert sw["write_bytes"] == 500 * 1024 * profile_summary.WRITE_SCALE
    assert rec["kernels"]["nz::nz_keys_kernel"]["dispatches"] == 2
    assert rec["kernels"]["nz::nz_keys_kernel"]["write_bytes"] == 400 * 1024 * profile_summary.WRITE_SCALE
    assert rec["source_sha1"] == profile_summary.source_sha1() and rec["steps"] == 1
    # the benchmark's reading of the record
    b, n = bench.traffic_of(rec, ["nz::nz_keys_kernel"])
    assert n == 2 and b == 2 * 10 * 1024 * profile_summary.FETCH_SCALE + 400 * 1024 * profile_summary.WRITE_SCALE


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


def test_profile_timeline_last_step(tmp_path):
    """The step timeline: dispatches of the last step (from the last MLP
    forward on), per queue, relative to the step's start."""
    d = tmp_path / "trace"
    d.mkdir()
    rows = [("nzmlp::mlp_forward_kernel", 1, 0, 10_000), ("nz::nz_keys_kernel", 1, 20_000, 3_020_000),
            ("nzmlp::mlp_forward_kernel", 1, 5_000_000, 5_010_000), ("nz::nz_keys_kernel", 1, 5_020_000, 8_020_000),
            ("nz::nz_keys_kernel", 2, 5_030_000, 9_030_000), ("nz::nz_sweep_kernel<1, 0, true, 1, false>", 2,
                                                              9_100_000, 20_000_000)]
    with open(d / "m_kernel_trace.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Queue_Id", "Start_Timestamp", "End_Timestamp"])
        for k, q, a, b in rows:
            w.writerow([k, q, a, b])
    tl = profile_summary.timeline(str(d))
    assert [r[1] for r in tl] == ["nzmlp::mlp_forward_kernel", "nz::nz_keys_kernel", "nz::nz_keys_kernel",
                                  "nz::nz_sweep_kernel<1, 0, true, 1, false>"]
    assert tl[0][2] == 0.0 and np.isclose(tl[-1][3], 15.0)
    md = "\n".join(profile_summary.timeline_md(tl, "T"))
    assert "| 2 | **span** | 0.03 | 15.00 | 14.97 |" in md
