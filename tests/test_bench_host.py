"""Host-side logic of bench.py: the one-GPU contract and the counter summary
(scaling of FETCH_SIZE / WRITE_SIZE by the calibration copy).  No GPU."""
import csv
import json
import os
import re
import subprocess
import sys

import bench
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _counter_csv(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "p_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_traffic_summary_scales_counters_by_the_copy(tmp_path):
    xk = "void enomr::k_euler_sweep<4, 9, 0, 64, 4, 0>(enomr::SweepIn, enomr::StageOut)"
    yk = "void enomr::k_euler_sweep<4, 9, 1, 64, 4, 0>(enomr::SweepIn, enomr::StageOut)"
    cp = "__amd_rocclr_copyBuffer"
    # two dispatches per sweep, each counter split over two instances; the
    # copy of 1024 MiB reads as 512 MiB fetched and 1024 MiB written
    def rows(counter, xv, yv, copy):
        out = []
        for d, k, v in ((1, xk, xv), (2, xk, xv), (3, yk, yv), (4, yk, yv), (5, cp, copy), (6, cp, 1.0)):
            out += [{"Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": counter, "Counter_Value": v / 2}] * 2
        return out
    _counter_csv(str(tmp_path / "fetch"), rows("FETCH_SIZE", 1000.0, 3000.0, 512 * 1024.0))
    _counter_csv(str(tmp_path / "write"), rows("WRITE_SIZE", 2000.0, 500.0, 1024 * 1024.0))
    _counter_csv(str(tmp_path / "valu"), rows("SQ_INSTS_VALU", 7.0, 9.0, 1.0))
    text = bench.traffic_summary(str(tmp_path / "fetch"), str(tmp_path / "write"), str(tmp_path / "valu"),
                                 1024, "cmd")
    rec = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
    assert rec["calibration"]["fetch_scale"] == 2.0 and rec["calibration"]["write_scale"] == 1.0
    assert rec["bytes_per_launch"]["k_euler_sweep (x faces)"] == (1000.0 * 2 + 2000.0) * 1024
    assert rec["bytes_per_launch"]["k_euler_sweep (y faces)"] == (3000.0 * 2 + 500.0) * 1024
    assert rec["valu_wave_instr_per_launch"] == {"k_euler_sweep (x faces)": 7.0, "k_euler_sweep (y faces)": 9.0}
    assert rec["source_sha256"] == bench.sweep_source_hash()


def test_face_count_grows_with_order_and_pairs_cost_more_past_the_full_stencil():
    prev = 0
    for order in (5, 9, 13, 17):
        f = bench.face_ops(order)
        assert f > prev
        prev = f
        nc = oracle.ncand(order)
        t = bench.pair_ops_table(order)
        assert t[0] == bench.IS0_OPS + 2 * order + 1
        assert (t[1:nc] > t[0]).all() and not t[nc:].any()
        # minmod after every stencil with m, n >= 1 failed: all their chains were scanned
        assert t[nc - 1] == t[nc - 2] == t[nc - 3]


def _pmc_csv(path, rows):
    os.makedirs(path, exist_ok=True)
    names = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Scratch_Size", "LDS_Block_Size"]
    with open(os.path.join(path, "p_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=names)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_stall_summary_shares_and_mix(tmp_path):
    xk = "void enomr::k_euler_sweep<4, 9, 0, 64, 4, 0>(enomr::SweepIn, enomr::StageOut)"
    yk = "void enomr::k_euler_sweep<4, 9, 1, 64, 4, 0>(enomr::SweepIn, enomr::StageOut)"
    groups = [
        {"SQ_WAVES": 100, "SQ_WAVE_CYCLES": 1000, "SQ_BUSY_CYCLES": 1, "SQ_WAIT_ANY": 450, "SQ_WAIT_INST_ANY": 250,
         "SQ_ACTIVE_INST_ANY": 300, "SQ_ACTIVE_INST_VALU": 200, "SQ_ACTIVE_INST_LDS": 50},
        {"LdsLatency": 66, "LdsUtil": 50.0, "LDSBankConflict": 13.0, "VALUUtilization": 88.0},
        {"VmemLatency": 1000, "MeanOccupancyPerCU": 13.0},
        {"SQ_INSTS_VALU_FMA_F64": 40, "SQ_INSTS_VALU_ADD_F64": 20, "SQ_INSTS_VALU_MUL_F64": 10,
         "SQ_INSTS_VALU_TRANS_F64": 1, "SQ_INSTS_VALU_INT32": 6, "SQ_INSTS_VALU_INT64": 4, "SQ_INSTS_VALU": 100,
         "SQ_INSTS_LDS": 16}]
    dirs = []
    for i, g in enumerate(groups):
        rows = []
        for d, k, f in ((1, xk, 1.0), (2, xk, 1.0), (3, yk, 2.0)):
            for c, v in g.items():
                rows.append({"Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v * f,
                             "Scratch_Size": 0, "LDS_Block_Size": 39424})
        dirs.append(str(tmp_path / ("p%d" % i)))
        _pmc_csv(dirs[-1], rows)
    text = bench.stall_summary(dirs, "cmd")
    row = {l.split("|")[1].strip(): [c.strip() for c in l.split("|")[2:4]] for l in text.splitlines()
           if l.startswith("| ") and not l.startswith("| counter")}
    # shares are ratios of counters, so the y sweep's doubled counters give the same shares
    assert row["share of a wave's cycles issuing VALU (SQ_ACTIVE_INST_VALU)"] == ["20.0%", "20.0%"]
    assert row["waiting on memory, LDS or a barrier (SQ_WAIT_ANY)"] == ["45.0%", "45.0%"]
    assert row["waves per launch"] == ["100", "200"]
    assert row["of which FP64 FMA / add / mul"] == ["40.0% / 20.0% / 10.0%"] * 2
    assert row["of which other (compares, selects, min/max, moves, divide and square-root steps)"] == ["20.0%"] * 2
    assert row["scratch bytes per lane, LDS bytes per workgroup"] == ["0, 39424"] * 2
