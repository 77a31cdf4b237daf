"""Host-side parts of bench.py: the one-GPU guard and the all-cores oracle
figure (point ranges of the random streams compose exactly)."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_all_cores_oracle_figure_covers_every_splat():
    import bench
    import oracle
    import workloads as W
    w = W.cfs_square(n_points=(1 << 13) + 7, side=256)
    r, img = bench.cpu_baseline_all_cores(w, max_threads=3)
    assert r["kind"] == "oracle" and 1 <= r["cores"] <= 3 and r["value"] > 0
    assert r["host"]["nproc"] >= 1 and r["host"]["affinity"] >= 1
    ref = oracle.chaos_count(w["system"], w["run"], w["image"])
    total = int(ref["image"].astype(np.int64).sum())
    assert r["splats"] == total == ((1 << 13) + 7) * 24 - ref["dropped"]
    assert np.array_equal(img["image"], ref["image"])
    err = bench.parity_error({"image": ref["image"], "dropped": ref["dropped"]}, img)
    assert err["rel_l1"] == 0.0 and err["dropped_equal"]


def test_all_cores_depth_figure_is_the_oracle_image():
    import bench
    import oracle
    import workloads as W
    w = W.menger(n_points=(1 << 12) + 3, side=256)
    r, img = bench.cpu_baseline_all_cores(w, max_threads=3)
    ref = oracle.chaos_depth(w["system"], w["run"], w["image"], w["image"]["near"])
    assert np.array_equal(img["depth"], ref["depth"])
    assert np.array_equal(img["density"], ref["density"])
    err = bench.parity_error(dict(ref), img)
    assert err["keys_differing"] == 0 and err["density_rel_l1"] == 0.0


# ---------------------------------------------------------------------------
# The profile summarisers, on synthetic rocprofv3 outputs with known figures
# ---------------------------------------------------------------------------
def _write_csv(path, header, rows):
    import csv
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(header)
        w.writerows(rows)


def _counter_rows(counter, items):
    return [[i + 1, i + 1, "Agent 1", 1, 1, 1, 64, 1, name, 256, 0, 0, 8, 0, 16, counter,
             float(v), 0, 1] for i, (name, v) in enumerate(items)]


_COUNTER_HEADER = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id",
                   "Thread_Id", "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size",
                   "LDS_Block_Size", "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count",
                   "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp",
                   "End_Timestamp"]


def test_summarise_pmc_scales_by_the_copy(tmp_path):
    """Bytes per step = sum over the three profiled steps' dispatches / 3,
    in KiB, times the factor that makes the 256 MiB copy read 256 MiB."""
    import bench
    chaos = "void cfs::k_chaos_depth_binned<double, true, 2>(args)"
    acc = "cfs::k_depth_accumulate(args)"
    copy = "__amd_rocclr_copyBuffer"
    # the counter reads half the copy: the factor is 2
    fetch = [(copy, 131072.0)] + [(chaos, 10.0)] * 12 + [(acc, 3000.0)] * 12
    write = [(copy, 262144.0)] + [(chaos, 2000.0)] * 12 + [(acc, 50.0)] * 12
    _write_csv(str(tmp_path / "f" / "vm" / "1_counter_collection.csv"), _COUNTER_HEADER,
               _counter_rows("FETCH_SIZE", fetch))
    _write_csv(str(tmp_path / "w" / "vm" / "1_counter_collection.csv"), _COUNTER_HEADER,
               _counter_rows("WRITE_SIZE", write))
    bench.summarise_pmc(str(tmp_path / "f"), str(tmp_path / "w"), "menger", "f64",
                        out_dir=str(tmp_path))
    out = json.load(open(tmp_path / "traffic_menger_f64.json"))
    assert out["calibration"]["FETCH_SIZE"]["scale"] == 2.0
    assert out["calibration"]["WRITE_SIZE"]["scale"] == 1.0
    k = out["kernels"]
    assert k["chaos_kernel"]["FETCH_SIZE"] == 12 * 10.0 / 3 * 1024 * 2
    assert k["tile_accumulate"]["FETCH_SIZE"] == 12 * 3000.0 / 3 * 1024 * 2
    assert k["chaos_kernel"]["WRITE_SIZE"] == 12 * 2000.0 / 3 * 1024
    assert out["source_digest"] == bench.source_digest()


def test_summarise_valu_per_point_iteration(tmp_path):
    """VALU wave-instructions per point-iteration from the per-dispatch
    counters, with the launches per step read off SQ_WAVES."""
    import bench
    import workloads as W
    w = W.menger()
    N, T = w["run"]["n_points"], w["run"]["n_iters"]
    chaos = "void cfs::k_chaos_depth_binned<double, true, 2>(args)"
    waves = N / 64 / 4            # four launches per step
    insts = 90.0 * N * T / 64 / 4  # 90 per point-iteration
    rows = []
    for c, v in (("SQ_INSTS_VALU", insts), ("SQ_ACTIVE_INST_VALU", insts), ("SQ_WAVES", waves)):
        rows += _counter_rows(c, [(chaos, v)] * 12)
    _write_csv(str(tmp_path / "v" / "vm" / "1_counter_collection.csv"), _COUNTER_HEADER, rows)
    bench.summarise_valu(str(tmp_path / "v"), "menger", "f64", out_dir=str(tmp_path))
    out = json.load(open(tmp_path / "valu_menger_f64.json"))
    assert out["launches_per_step"] == 4
    assert abs(out["valu_insts_per_point_iteration"] - 90.0) < 1e-9


def test_summarise_trace_fraction(tmp_path):
    """The roofline kernel's mean over the timed steps' launches, and the
    fraction of the VALU model that mean gives."""
    import bench
    chaos = "void cfs::k_chaos_depth_binned<double, true, 2>(args)"
    steps, warmup, per = 5, 2, 4
    trace_header = ["Kind", "Agent_Id", "Queue_Id", "Stream_Id", "Thread_Id", "Dispatch_Id",
                    "Kernel_Id", "Kernel_Name", "Correlation_Id", "Start_Timestamp",
                    "End_Timestamp", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
                    "Accum_VGPR_Count", "SGPR_Count", "Workgroup_Size_X", "Workgroup_Size_Y",
                    "Workgroup_Size_Z", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"]
    rows, t = [], 0
    for i in range((steps + warmup) * per):
        dur = 3_000_000 if i < warmup * per else 1_500_000  # ns: warm-up launches slower
        rows.append(["KERNEL_DISPATCH", "Agent 1", 1, 0, 1, i + 1, 7, chaos, i + 1, t, t + dur,
                     145408, 0, 128, 0, 112, 1024, 1, 1, 1 << 24, 1, 1])
        t += dur + 1000
    _write_csv(str(tmp_path / "t" / "m_kernel_trace.csv"), trace_header, rows)
    _write_csv(str(tmp_path / "t" / "m_kernel_stats.csv"),
               ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs",
                "StdDev"],
               [[chaos, len(rows), 1.0, 1.0, 100.0, 1.0, 1.0, 0.0]])
    line = {"metric": "m", "ms_per_step": 7.0, "config": {"workload": "menger: test"},
            "phase_ms": {"chaos_kernel": 6.0, "table_transpose": 0.3, "tile_accumulate": 0.7},
            "roofline": {"lane_ops_per_step": 1.2e11, "peak": 40.0, "frac": 0.5}}
    log = tmp_path / "run.log"
    log.write_text("profiler noise\n" + json.dumps(line) + "\nmore noise\n")
    bench.summarise_trace(str(tmp_path / "t"), str(log), "menger", "f64", out_dir=str(tmp_path))
    text = (tmp_path / "trace_menger_f64.md").read_text()
    # 4 timed launches of 1.5 ms per step: 6.0 ms; 1.2e11 / 6 ms / 40 T = 0.5
    assert "6.000 ms per step in the trace" in text
    assert "**0.500**" in text


def test_summarise_trace_refuses_a_trace_without_the_kernel(tmp_path):
    """A trace whose kernels do not include the workload's roofline kernel
    (here the Sierpinski configuration's binned chaos kernel) is refused,
    not summarised as a zero-length step."""
    import pytest
    import bench
    assert bench.STEP_KERNELS["sierpinski"][0][0] == "k_chaos_binned"
    other = "void cfs::k_chaos<float, 2, 0, true, false, false>(args)"
    header = ["Kind", "Agent_Id", "Queue_Id", "Stream_Id", "Thread_Id", "Dispatch_Id",
              "Kernel_Id", "Kernel_Name", "Correlation_Id", "Start_Timestamp", "End_Timestamp",
              "LDS_Block_Size", "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count",
              "Workgroup_Size_X", "Workgroup_Size_Y", "Workgroup_Size_Z", "Grid_Size_X",
              "Grid_Size_Y", "Grid_Size_Z"]
    rows = [["KERNEL_DISPATCH", "Agent 1", 1, 0, 1, i + 1, 7, other, i + 1, 1000 * i,
             1000 * i + 500, 0, 0, 32, 0, 32, 512, 1, 1, 1 << 16, 1, 1] for i in range(7)]
    _write_csv(str(tmp_path / "t" / "s_kernel_trace.csv"), header, rows)
    _write_csv(str(tmp_path / "t" / "s_kernel_stats.csv"),
               ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs",
                "StdDev"], [[other, 7, 3500.0, 500.0, 100.0, 500.0, 500.0, 0.0]])
    line = {"metric": "m", "ms_per_step": 0.07, "config": {"workload": "sierpinski: test"},
            "phase_ms": {"chaos_kernel": 0.03}, "roofline": {"lane_ops_per_step": 1.8e8,
                                                             "peak": 39.3, "frac": 0.13}}
    log = tmp_path / "run.log"
    log.write_text(json.dumps(line) + "\n")
    with pytest.raises(SystemExit, match="no k_chaos_binned launches"):
        bench.summarise_trace(str(tmp_path / "t"), str(log), "sierpinski", "f32",
                              out_dir=str(tmp_path))


def test_summarise_pmc_reads_the_newest_run_only(tmp_path):
    """An output folder reused by two profiled runs holds two counter files;
    only the newer run's dispatches count (an older run would double the
    bytes per step)."""
    import time
    import bench
    chaos = "void cfs::k_chaos_depth_binned<double, true, 2>(args)"
    copy = "__amd_rocclr_copyBuffer"
    for sub, v in (("f", 10.0), ("w", 2000.0)):
        counter = "FETCH_SIZE" if sub == "f" else "WRITE_SIZE"
        old = [(copy, 262144.0)] + [(chaos, 999.0 * v)] * 3
        new = [(copy, 262144.0)] + [(chaos, v)] * 3
        _write_csv(str(tmp_path / sub / "vm" / "1_counter_collection.csv"), _COUNTER_HEADER,
                   _counter_rows(counter, old))
        time.sleep(0.05)
        _write_csv(str(tmp_path / sub / "vm" / "2_counter_collection.csv"), _COUNTER_HEADER,
                   _counter_rows(counter, new))
        os.utime(str(tmp_path / sub / "vm" / "1_counter_collection.csv"), (1.0e9, 1.0e9))
    bench.summarise_pmc(str(tmp_path / "f"), str(tmp_path / "w"), "menger", "f64",
                        out_dir=str(tmp_path))
    k = json.load(open(tmp_path / "traffic_menger_f64.json"))["kernels"]
    assert k["chaos_kernel"]["FETCH_SIZE"] == 3 * 10.0 / 3 * 1024
    assert k["chaos_kernel"]["WRITE_SIZE"] == 3 * 2000.0 / 3 * 1024
