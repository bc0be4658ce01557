"""Host logic of the benchmark's measurement records (no GPU): the counter
records built from rocprofv3 counter CSVs, their scaling by the copy probe,
the per-launch and per-apply division, the matrix-core figures, and the
rule that a record counts only for the kernel source it was taken on."""
import csv
import json
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

COLS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size", "Kernel_Id",
        "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count",
        "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _csv(path, rows):
    """rows: (dispatch, kernel, counter, value, start_ns, end_ns)"""
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(COLS)
        for d, k, c, v, t0, t1 in rows:
            w.writerow([d, d, "Agent 1", 2, 1, 1, 256, 1, k, 256, 0, 0, 8, 0, 16, c, float(v), t0, t1])
    return str(path)


def test_traffic_record_scales_and_divides(tmp_path):
    gib = 1 << 30
    # the copy probe: FETCH_SIZE sees half of a 1 GiB copy, WRITE_SIZE all of it (KiB)
    cf = _csv(tmp_path / "cf.csv", [(1, "copy", "FETCH_SIZE", gib / 2 / 1024, 0, 1)])
    cw = _csv(tmp_path / "cw.csv", [(1, "copy", "WRITE_SIZE", gib / 1024, 0, 1)])
    # two dispatches of kernel A (one of them counted on two rows: summed per
    # dispatch), one of kernel B
    f = _csv(tmp_path / "f.csv", [(7, "void acr::mv_seg_kernel<float>(x)", "FETCH_SIZE", 100, 0, 1),
                                  (7, "void acr::mv_seg_kernel<float>(x)", "FETCH_SIZE", 50, 0, 1),
                                  (8, "void acr::mv_seg_kernel<float>(x)", "FETCH_SIZE", 250, 0, 1),
                                  (9, "void acr::mv_coef_kernel<float>(x)", "FETCH_SIZE", 40, 0, 1)])
    w = _csv(tmp_path / "w.csv", [(7, "void acr::mv_seg_kernel<float>(x)", "WRITE_SIZE", 10, 0, 1),
                                  (8, "void acr::mv_seg_kernel<float>(x)", "WRITE_SIZE", 30, 0, 1),
                                  (9, "void acr::mv_coef_kernel<float>(x)", "WRITE_SIZE", 4, 0, 1)])
    rec = bench.traffic_record("apply", f, w, cf, cw, float(gib),
                               [("seg", "mv_seg_kernel<float>"), ("all", "mv_/4")], ["cmd"])
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    seg = rec["kernels"]["seg"]
    assert seg["dispatches"] == 2 and seg["units"] == 2.0
    assert seg["fetch_kib_per_launch"] == pytest.approx(200.0)  # (150 + 250) / 2
    assert seg["traffic_bytes_per_launch"] == pytest.approx(200 * 1024 * 2.0 + 20 * 1024 * 1.0)
    allk = rec["kernels"]["all"]
    assert allk["units"] == 4.0  # the "/4" divisor (e.g. per application), not the dispatch count
    assert allk["traffic_bytes_per_launch"] == pytest.approx((440 * 2.0 + 44 * 1.0) * 1024 / 4)
    assert rec["source_sha256"] == bench.kernel_source_hash(bench.TRAFFIC_RECORDS["apply"][1])


def test_mfma_record(tmp_path):
    k = "void acr::kc38::accum_dense_kernel<float, false>(acr::AccumArgs<float>)"
    rows = []
    # dispatch 1: 1 us, 1000 MOPS (512,000 flops), 2% busy; dispatch 2: 3 us, 3000 MOPS, 6% busy
    for d, ns, mops, util in ((1, 1000, 1000, 2.0), (2, 3000, 3000, 6.0)):
        rows += [(d, k, "SQ_INSTS_VALU_MFMA_MOPS_F32", mops, 10_000, 10_000 + ns),
                 (d, k, "SQ_INSTS_VALU_MFMA_MOPS_F64", 0, 10_000, 10_000 + ns),
                 (d, k, "SQ_INSTS_VALU_MFMA_MOPS_BF16", 0, 10_000, 10_000 + ns),
                 (d, k, "MfmaUtil", util, 10_000, 10_000 + ns)]
    rows.append((3, "void acr::kc38::accum_kernel<float, false>(x)", "MfmaUtil", 50.0, 0, 5))
    rec = bench.mfma_record(_csv(tmp_path / "m.csv", rows), [("dense", "accum_dense_kernel<float")], ["cmd"])
    r = rec["kernels"]["dense"]
    assert r["dispatches"] == 2
    assert r["mfma_flops_per_launch"] == pytest.approx(4000 * 512 / 2)
    assert r["mfma_tflops"] == pytest.approx(round(4000 * 512 / 4e-6 / 1e12, 4))
    assert r["mfma_util_pct"] == pytest.approx((2.0 * 1000 + 6.0 * 3000) / 4000)  # weighted by duration
    assert rec["source_sha256"] == bench.kernel_source_hash(bench.MFMA_RECORD[1])


def test_records_count_only_for_their_source(tmp_path, monkeypatch):
    path = tmp_path / "rec.json"
    good = {"source_sha256": bench.kernel_source_hash(("k_harith.hip", "hprog.h")),
            "kernels": {"accum_kernel": {"traffic_bytes_per_launch": 123.0, "mfma_util_pct": 1.5,
                                         "mfma_tflops": 0.5, "mfma_flops_per_launch": 7.0}}}
    path.write_text(json.dumps(good))
    monkeypatch.setitem(bench.TRAFFIC_RECORDS, "accum", (str(path), ("k_harith.hip", "hprog.h")))
    monkeypatch.setattr(bench, "MFMA_RECORD", (str(path), ("k_harith.hip", "hprog.h")))
    assert bench.measured_traffic("accum", "accum_kernel") == 123.0
    roof = bench.kernel_roofline("accum_kernel", 10, 2.0, 1e12, 78.6, abytes=41.0)
    assert roof["traffic"] == 123 and roof["algorithmic_bytes_per_launch"] == 4
    assert roof["traffic_over_algorithmic"] == pytest.approx(123 / 4.1, rel=1e-3)
    assert roof["mfma"] == {"mfma_util_pct": 1.5, "mfma_tflops": 0.5, "mfma_flops_per_launch": 7.0}
    assert roof["achieved"] == pytest.approx(1e11 / 0.2 / 1e12, rel=1e-3)
    good["source_sha256"] = "0" * 64  # taken on another source: ignored
    path.write_text(json.dumps(good))
    assert bench.measured_traffic("accum", "accum_kernel") is None
    roof = bench.kernel_roofline("accum_kernel", 10, 2.0, 1e12, 78.6)
    assert roof["traffic"] is None and "mfma" not in roof and roof["algorithmic_bytes_per_launch"] is None
