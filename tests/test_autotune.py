"""Host side of the autotuner: z-classes, candidate shapes the library accepts,
table lookup and the choice for a mixed batch (not GPU)."""
import json

import numpy as np
import pytest

from paper_2607_18991_amd import autotune, nz


def test_zclass_follows_offset_chunks():
    assert [autotune.zclass(z) for z in (10, 64, 65, 128, 130, 256, 332, 512, 572, 892)] == \
        [64, 64, 128, 128, 256, 256, 512, 512, 892, 892]
    for zc, mask in autotune.REPRESENTATIVE.items():
        assert autotune.zclass(nz.nz_coordination(mask)) == zc


@pytest.mark.parametrize("L", [4, 8, 16, 24])
def test_candidates_are_accepted_by_the_library(L):
    jobs = [dict(L=L, zone_mask=1, seed=1, nsamples=2)]
    for cand in autotune.candidates(L):
        assert nz.nz_batch_workspace_bytes(jobs, cand) > 0
    # LDS residencies only where the state fits
    res = {c["residency"] for c in autotune.candidates(L)}
    assert (1 in res) == (L <= 16) and (3 in res) == (L <= 8)


def test_lookup_and_batch_choice(tmp_path):
    table = {"format": autotune.FORMAT, "entries": {
        "16:64": {"tune": {"residency": 2, "wg_waves": 4, "waves_per_simd": 8, "sweep_mode": 2}},
        "16:892": {"tune": {"residency": 1, "wg_waves": 1, "waves_per_simd": 8, "sweep_mode": 1}},
        "8:64": {"tune": {"residency": 3, "wg_waves": 1, "waves_per_simd": 8, "sweep_mode": 2}}}}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(table))
    t = autotune.load_table(str(p))
    assert autotune.lookup(16, 0x7F, t)["residency"] == 1
    assert autotune.lookup(16, 0x01, t)["sweep_mode"] == 2
    assert autotune.lookup(12, 0x01, t) == {}
    jobs = [dict(L=8, zone_mask=1, nsamples=10), dict(L=16, zone_mask=0x7F, nsamples=10), dict(L=16, zone_mask=0x01, nsamples=10)]
    assert autotune.for_jobs(jobs, t) == table["entries"]["16:64"]["tune"]
    assert autotune.for_jobs([], t) == {}


def test_shipped_table_is_valid():
    t = autotune.load_table()
    assert t["format"] == autotune.FORMAT
    for k, e in t["entries"].items():
        L, zc = (int(x) for x in k.split(":"))
        assert zc in autotune.ZCLASSES
        nz.nz_batch_workspace_bytes([dict(L=L, zone_mask=autotune.REPRESENTATIVE[zc], seed=1, nsamples=1)],
                                    e["tune"] or None)
        assert e["ms"] <= e["default_ms"] * 1.0001


def test_batch_entries_and_lds_guard():
    table = {"format": autotune.FORMAT, "entries": {
        "16:64": {"tune": {"residency": 1, "wg_waves": 1, "waves_per_simd": 8, "sweep_mode": 2}}}}
    few = [dict(L=16, zone_mask=1, seed=1, nsamples=100)]
    many = [dict(L=16, zone_mask=1, seed=1, nsamples=1000)]
    assert autotune.for_jobs(few, table)["residency"] == 1
    assert autotune.for_jobs(many, table)["residency"] == 2
    autotune.add_batch(table, many, {"tune": {"residency": 2, "wg_waves": 4, "waves_per_simd": 4, "sweep_mode": 1}},
                       "L16 x 1000")
    assert autotune.for_jobs(many, table)["wg_waves"] == 4
    # the signature ignores the planned n0 values but not whether a prefill is used
    assert autotune.signature([dict(L=16, zone_mask=1, nsamples=10, n0=5)]) == \
        autotune.signature([dict(L=16, zone_mask=1, nsamples=10, n0=7)])
    assert autotune.signature([dict(L=16, zone_mask=1, nsamples=10, n0=5)]) != \
        autotune.signature([dict(L=16, zone_mask=1, nsamples=10)])
    for c in autotune.batch_candidates():
        assert nz.nz_batch_workspace_bytes(many, c) > 0


def test_summary_choice_kept_only_for_batches_like_the_timed_one():
    """The summary's worth depends on how many samples share the chip: a class
    entry's choice applies to batches no larger than the one it was timed on."""
    table = {"format": autotune.FORMAT, "entries": {
        "16:892": {"tune": {"residency": 2, "wg_waves": 1, "waves_per_simd": 8, "sweep_mode": 2, "summary": 2},
                   "samples": 256}}}
    small = [dict(L=16, zone_mask=0x7F, seed=1, nsamples=200)]
    large = [dict(L=16, zone_mask=0x7F, seed=1, nsamples=4000)]
    assert autotune.for_jobs(small, table)["summary"] == 2
    assert "summary" not in autotune.for_jobs(large, table)
    assert autotune.for_jobs(large, table)["sweep_mode"] == 2
    hbm = [c for c in autotune.candidates(16) if c["residency"] == 2]
    assert {c["summary"] for c in hbm} == {1, 2}
    assert {c.get("summary") for c in autotune.batch_candidates()} == {1, 2}


def test_batch_plan_and_split_candidates():
    """A batch entry may carry the planner's prefill depth; the split
    candidates are accepted by the library and change only the grouping."""
    table = {"format": autotune.FORMAT, "entries": {}}
    jobs = [dict(L=16, zone_mask=m, seed=1, nsamples=500, n0=1000) for m in (0x01, 0x7F)]
    assert autotune.plan_for(jobs, table) == {}
    autotune.add_batch(table, jobs, {"tune": {"residency": 2, "split_z": 130}, "plan": {"k_sigma": 2.0}}, "b")
    assert autotune.plan_for(jobs, table) == {"k_sigma": 2.0}
    assert autotune.for_jobs(jobs, table)["split_z"] == 130
    assert autotune.plan_for([], table) == {}
    for sz in autotune.SPLIT_Z:
        assert nz.nz_batch_workspace_bytes(jobs, dict(split_z=sz)) > 0
    with pytest.raises(nz.NzError):
        nz.nz_batch_workspace_bytes(jobs, dict(split_z=5))
    assert all(k > 0 for k in autotune.K_SIGMA)
    # a plan with its own depth for the wide jobs: None values are dropped
    autotune.add_batch(table, jobs, {"tune": {}, "plan": {"k_sigma": 2.5, "k_sigma_wide": 1.5, "split_z": None}}, "b")
    assert autotune.plan_for(jobs, table) == {"k_sigma": 2.5, "k_sigma_wide": 1.5}


def test_plan_outputs_wide_depth():
    """learned.plan_outputs plans the jobs wider than split_z with their own
    prefill depth and the rest as nz_prefill_plan does, in the callers' order."""
    from paper_2607_18991_amd import learned

    jobs = [dict(L=16, zone_mask=m, seed=1, nsamples=10) for m in (0x01, 0x7F, 0x03, 0x3F)]
    y = np.array([[np.log(0.14), np.log(0.004)], [np.log(0.0019), np.log(0.0002)],
                  [np.log(0.033), np.log(0.001)], [np.log(0.003), np.log(0.0003)]], dtype=np.float32)
    same = learned.plan_outputs(y, jobs, 2.5)
    assert same == nz.nz_prefill_plan(y, jobs, 2.5, 5.0)
    mixed = learned.plan_outputs(y, jobs, 2.5, k_sigma_wide=1.0, split_z=64)
    wide = nz.nz_prefill_plan(y, jobs, 1.0, 5.0)
    for i, j in enumerate(jobs):
        expect = wide[i] if nz.nz_coordination(j["zone_mask"]) > 64 else same[i]
        assert mixed[i] == expect
    assert mixed[1]["n0"] > same[1]["n0"] and mixed[0]["n0"] == same[0]["n0"]
    # the split defaults to the library's own (zones 1 and 1-2 narrow)
    assert learned.plan_outputs(y, jobs, 2.5, k_sigma_wide=1.0) == mixed
