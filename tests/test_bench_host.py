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
