"""CPU tests of the rocprofv3 summaries in paper_1805_01559_amd.profiling, on
small CSV files written here in rocprofv3's column layout: the copy-calibrated
traffic figure, the per-cell VALU count over working dispatches only, and the
host/kernel timeline window."""

import csv
import json

import pytest

from paper_1805_01559_amd import profiling as P

COUNTER_COLS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
                "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
                "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp",
                "End_Timestamp"]


def write_counters(path, rows):
    path.mkdir(parents=True, exist_ok=True)
    with open(path / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=COUNTER_COLS)
        w.writeheader()
        for k, (disp, name, counter, value) in enumerate(rows):
            r = {c: 0 for c in COUNTER_COLS}
            r.update(Correlation_Id=k + 1, Dispatch_Id=disp, Kernel_Name=name, Counter_Name=counter,
                     Counter_Value=value)
            w.writerow(r)


def test_traffic_is_scaled_by_the_copy(tmp_path):
    # the copy of 2 x 1 MiB reads 1024 KiB by FETCH_SIZE and writes 2048 KiB
    # by WRITE_SIZE: factors 1 and 0.5; the kernel's medians are 3000 and 500
    write_counters(tmp_path / "f", [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 1024.0),
                                    (2, "k_x<1>", "FETCH_SIZE", 2000.0), (3, "k_x<1>", "FETCH_SIZE", 3000.0),
                                    (4, "k_x<1>", "FETCH_SIZE", 4000.0)])
    write_counters(tmp_path / "w", [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 2048.0),
                                    (2, "k_x<1>", "WRITE_SIZE", 500.0), (3, "k_x<1>", "WRITE_SIZE", 500.0),
                                    (4, "k_x<1>", "WRITE_SIZE", 900.0)])
    t = P.traffic(str(tmp_path / "f"), str(tmp_path / "w"), "k_x<1>", alg_bytes=1e6, copy_bytes=2 * (1 << 20))
    assert t["fetch"]["factor"] == pytest.approx(1.0) and t["write"]["factor"] == pytest.approx(0.5)
    assert t["hbm_bytes"] == pytest.approx(3000 * 1024 + 0.5 * 500 * 1024)
    assert t["ratio"] == pytest.approx(t["hbm_bytes"] / 1e6)
    # --first keeps the first dispatches only
    t2 = P.traffic(str(tmp_path / "f"), str(tmp_path / "w"), "k_x<1>", 1e6, 2 * (1 << 20), first=1)
    assert t2["fetch"]["median_kib"] == 2000.0
    json.dumps(t)


def test_valu_counts_working_dispatches_only(tmp_path):
    # dispatches 3 and 4 exit at once (a chunk's launches after the stop)
    rows = []
    for disp, v in [(1, 1000.0), (2, 1100.0), (3, 4.0), (4, 6.0), (5, 900.0)]:
        rows += [(disp, "k_y", "SQ_INSTS_VALU", v), (disp, "k_y", "SQ_INSTS_VALU_TRANS_F32", v / 10)]
    rows.append((6, "k_other", "SQ_INSTS_VALU", 5e6))
    write_counters(tmp_path, rows)
    v = P.valu(str(tmp_path), "k_y", cells=64.0)
    c = v["counters"]["SQ_INSTS_VALU"]
    assert c["dispatches"] == 3 and c["median_wave_insts"] == 1000.0
    assert c["lane_insts_per_cell"] == pytest.approx(1000.0)
    assert v["counters"]["SQ_INSTS_VALU_TRANS_F32"]["median_wave_insts"] == pytest.approx(100.0)
    assert v["kernels_matched"] == ["k_y"]


def test_timeline_window(tmp_path):
    with open(tmp_path / "run_kernel_trace.csv", "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for name, s, e in [("k_a(int)", 0, 1000), ("k_big(int)", 3000, 9000), ("k_b(int)", 9500, 10000),
                           ("k_a(int)", 20000, 21000), ("k_big(int)", 23000, 29000)]:
            w.writerow([name, s, e])
    with open(tmp_path / "run_hip_api_trace.csv", "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Domain", "Function", "Start_Timestamp", "End_Timestamp"])
        for name, s, e in [("hipLaunchKernel", 1500, 2500), ("hipEventSynchronize", 9000, 10500),
                           ("hipLaunchKernel", 40000, 41000)]:
            w.writerow(["HIP_RUNTIME_API_EXT", name, s, e])
    out = P.timeline(str(tmp_path), "k_big", index=0, after=1)
    lines = out.splitlines()[2:]
    # from the end of the dispatch before (1000 ns) to the end of the next one
    assert [ln.split("|")[3].strip() for ln in lines] == ["API", "GPU", "API", "GPU"]
    assert lines[0].split("|")[1].strip() == "0.0" and lines[1].split("|")[1].strip() == "1.5"
    assert "k_big" in lines[1] and "k_b" in lines[3]
