"""Host-side checks of the counter post-processing (bench_profiles.py) on a
small hand-made counter file: the calibration copy is found among other
copies, the factors and per-launch figures follow their definitions, and
launches are keyed by (lanes, atoms per lane, block, grid blocks)."""
import csv
import os

import pytest

import bench_profiles as BP

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
          "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
          "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _write(path, dispatches):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for did, name, grid, ms, counters in dispatches:
            for cname, val in counters.items():
                w.writerow({k: 0 for k in FIELDS} | dict(
                    Dispatch_Id=did, Kernel_Name=name, Grid_Size=grid, Counter_Name=cname, Counter_Value=val,
                    Start_Timestamp=1_000_000, End_Timestamp=1_000_000 + int(ms * 1e6)))


def _sampler(lanes, apl):
    return "void dock::sample_kernel<%d, %d, 256, 0>(dock::SampleArgs)" % (lanes, apl)


def test_calibration_and_launch_records(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    launches = [(10 + k, _sampler(*la), grid, ms) for k, (la, grid, ms) in enumerate(
        [((32, 2), 196608, 100.0), ((64, 2), 131072, 40.0), ((32, 1), 196608, 30.0), ((64, 2), 196608, 20.0),
         ((16, 1), 196608, 10.0), ((32, 2), 131072, 5.0)])]
    a = [(3, copy, 131072, 0.1, {"FETCH_SIZE": 131072.0, "SQ_INSTS_VALU": 0.0}),      # calibration copy
         (9, copy, 131072, 0.1, {"FETCH_SIZE": 172000.0, "SQ_INSTS_VALU": 0.0})]      # another copy
    b = [(3, copy, 131072, 0.1, {"WRITE_SIZE": 262144.0}),
         (9, copy, 131072, 0.1, {"WRITE_SIZE": 344064.0})]
    for did, name, grid, ms in launches:
        a.append((did, name, grid, ms, {"FETCH_SIZE": 1000.0 * ms, "SQ_INSTS_VALU": 6e9 * ms}))
        b.append((did, name, grid, ms, {"WRITE_SIZE": 10.0 * ms, "TCC_REQ_sum": 4e6 * ms, "TCC_HIT_sum": 3e6 * ms,
                                        "SQ_LDS_IDX_ACTIVE": 3e8 * ms, "SQ_LDS_BANK_CONFLICT": 1e8 * ms}))
    # the initial-pose launch of the first bucket: shorter, same kernel and grid
    a.append((40, _sampler(32, 2), 196608, 1.0, {"FETCH_SIZE": 5.0, "SQ_INSTS_VALU": 1.0}))
    b.append((40, _sampler(32, 2), 196608, 1.0, {"WRITE_SIZE": 1.0, "TCC_REQ_sum": 1.0, "TCC_HIT_sum": 1.0,
                                                 "SQ_LDS_IDX_ACTIVE": 1.0, "SQ_LDS_BANK_CONFLICT": 0.0}))
    _write(str(tmp_path / "pmc_a" / "pmc_counter_collection.csv"), a)
    _write(str(tmp_path / "pmc_b" / "pmc_counter_collection.csv"), b)
    out = tmp_path / "out"
    out.mkdir()
    t = BP.counter_summaries(str(tmp_path), str(out))
    assert t["fetch_calibration"] == pytest.approx(2.0) and t["write_calibration"] == pytest.approx(1.0)
    assert t["source_sha256"] == BP.source_sha256()
    recs = t["workloads"]["C5"]
    assert set(recs) == {"32,2,256,768", "64,2,256,512", "32,1,256,768", "64,2,256,768", "16,1,256,768",
                         "32,2,256,512"}
    r = recs["32,2,256,768"]
    assert r["ms"] == pytest.approx(100.0)                      # the MC-step launch, not the initial one
    assert r["hbm_bytes"] == pytest.approx(1e5 * 1024 * 2.0 + 1e3 * 1024 * 1.0)
    assert r["l2_hit"] == pytest.approx(0.75)
    assert r["valu_busy"] == pytest.approx(round(6e11 * 4 / (0.1 * 2.4e9 * 1024), 3))
    assert r["lds_busy"] == pytest.approx(round(3e10 / (0.1 * 2.4e9 * 256), 3))
    assert r["bank_conflict"] == pytest.approx(round(1 / 3, 3))
    assert (out / "sample_kernel_mixed16_counters.md").exists() and (out / "traffic.json").exists()


def test_missing_calibration_copy_is_an_error(tmp_path):
    a = [(3, _sampler(32, 2), 196608, 1.0, {"FETCH_SIZE": 5.0, "SQ_INSTS_VALU": 1.0})]
    b = [(3, _sampler(32, 2), 196608, 1.0, {"WRITE_SIZE": 1.0})]
    _write(str(tmp_path / "pmc_a" / "pmc_counter_collection.csv"), a)
    _write(str(tmp_path / "pmc_b" / "pmc_counter_collection.csv"), b)
    with pytest.raises(SystemExit):
        BP.counter_summaries(str(tmp_path), str(tmp_path))
