"""Benchmark of the CFS chaos-game hot path on one MI355X.

A step is one pass of the whole hot path over the CFS-square workload:
clear the 4 x 2048 x 2048 u32 image, then run the fused chaos game of 2^24
points x 32 iterations (8 burn-in) -- random streams, selection, the 4-map
square, the swirl + translation of a copy, and the 4-channel count splat.
The timed region holds exactly K steps between two device synchronisations.

Prints one JSON line with point-iterations/s (value), splats/s, the roofline
of the dominant kernel (timed with HIP events on the stream it runs on) and
the FP64 oracle's rate on a bounded sample of the same workload on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peak figures of MI355X (public specification): 256 CUs at 2.4 GHz, each
# issuing one 64-lane vector instruction per clock across its 4 SIMDs.
VALU_LANE_OPS_PEAK = 256 * 64 * 2.4e9  # 3.93e13 lane-ops/s (full-rate ops)
HBM_PEAK_GBS = 8000.0


# Algorithmic VALU work per unit (full-rate-equivalent lane operations): a
# point-iteration is a quarter of a Philox4x32-10 block (10 rounds of two
# quarter-rate 32x32->64 multiplies and two xors: 25), the selection (4), the
# 2D map (4 FMA) and loop control (3) = 36; a splat adds binning and address
# (10) and, for the swirl, its square root and sine/cosine (20).  FP64
# transcendentals cost more than this counts, so the fraction is conservative.
PER_POINT_ITERATION = 36
PER_SPLAT = {"identity": 10, "swirl": 30, "stretch": 25}


def valu_model(final_kind, n_points, n_iters, burn_in):
    splats = n_points * (n_iters - burn_in)
    return n_points * n_iters * PER_POINT_ITERATION + splats * PER_SPLAT[final_kind]


def source_digest():
    """Digest of the HIP sources; traffic counters are valid only for it."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2606_02226_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(precision):
    """HBM bytes per launch of the binned chaos kernels from the committed
    FETCH_SIZE / WRITE_SIZE counter runs, or None when the sources changed
    since they were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_cfs_square_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_digest") != source_digest():
        return None
    return t.get("bytes_per_launch")


def measured_valu(precision):
    """VALU instruction counts of the chaos kernel from a rocprofv3 --pmc run
    (profiles/valu_cfs_square_<precision>.json), or None when the sources
    changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"valu_cfs_square_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        v = json.load(fh)
    if v.get("source_digest") != source_digest():
        return None
    return v


def _pmc_rows(directory, counter):
    """(kernel name, value) of every dispatch in a rocprofv3 --pmc CSV run."""
    import csv
    import glob
    rows = []
    for path in glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True):
        with open(path, newline="") as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") == counter:
                    rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    if not rows:
        raise SystemExit(f"no {counter} rows under {directory}")
    return rows


def summarise_valu(directory, precision):
    """Write profiles/valu_cfs_square_<precision>.json from a rocprofv3 --pmc
    run of this benchmark with SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU and SQ_WAVES:
    mean per chaos-kernel dispatch, and the VALU wave-instructions issued per
    point-iteration (the guard against a kernel that is busy but bloated)."""
    import workloads
    w = workloads.cfs_square()
    N, T = w["run"]["n_points"], w["run"]["n_iters"]
    out = {"source_digest": source_digest(), "precision": precision, "kernel": "k_chaos_binned",
           "counters": {}}
    for counter in ("SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_WAVES"):
        vals = [v for k, v in _pmc_rows(directory, counter) if "k_chaos_binned" in k]
        if not vals:
            raise SystemExit(f"no k_chaos_binned {counter} rows under {directory}")
        out["counters"][counter] = float(np.mean(vals))
    wave_pt_its = N * T / 64.0
    out["valu_insts_per_point_iteration"] = out["counters"]["SQ_INSTS_VALU"] / wave_pt_its
    out["command"] = ("rocprofv3 --pmc SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_WAVES --output-format csv "
                      "-d DIR -- python3 bench.py --steps 2 --warmup 1 --no-cpu-baseline "
                      f"--no-forms --precision {precision}")
    path = os.path.join(ROOT, "profiles", f"valu_cfs_square_{precision}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def summarise_pmc(fetch_dir, write_dir, precision):
    """Write profiles/traffic_cfs_square_<precision>.json from two rocprofv3
    --pmc runs of this benchmark with --calibration-copy (FETCH_SIZE, then
    WRITE_SIZE; both in KiB per dispatch).  Each counter is scaled by the
    factor that makes the 256 MiB calibration copy read and write 256 MiB."""
    copy_bytes = 256 << 20
    out = {"source_digest": source_digest(), "precision": precision,
           "unit": "bytes per launch", "calibration": {}, "kernels": {}}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _pmc_rows(d, counter)
        copies = [v for k, v in rows if "copyBuffer" in k or "copy" in k.lower()]
        scale = copy_bytes / (max(copies) * 1024.0)
        out["calibration"][counter] = {"copy_kib": max(copies), "scale": scale}
        for name, key in (("k_chaos_binned", "chaos_kernel"), ("k_transpose", "table_transpose"),
                          ("k_tile_accumulate", "tile_accumulate")):
            vals = [v for k, v in rows if name in k]
            if vals:
                out["kernels"].setdefault(key, {})[counter] = \
                    float(np.mean(vals)) * 1024.0 * scale
    ck = out["kernels"].get("chaos_kernel", {})
    out["bytes_per_launch"] = ck.get("FETCH_SIZE", 0.0) + ck.get("WRITE_SIZE", 0.0)
    out["command"] = ("rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) --output-format csv -d DIR "
                      "-- python3 bench.py --steps 2 --warmup 1 --no-cpu-baseline --no-forms "
                      f"--calibration-copy --precision {precision}")
    path = os.path.join(ROOT, "profiles", f"traffic_cfs_square_{precision}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def cpu_baseline(w, n_sample):
    import oracle
    oracle.build(force=False)
    run = dict(w["run"], n_points=n_sample)
    t0 = time.perf_counter()
    oracle.chaos_count(w["system"], run, w["image"])
    dt = time.perf_counter() - t0
    return {"value": n_sample * run["n_iters"] / dt, "unit": "point-iterations/s",
            "cores": 1, "kind": "oracle",
            "sample": f"{n_sample} of {w['run']['n_points']} points (all iterations, "
                      f"full image), single-threaded FP64, {dt:.1f} s"}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_all_cores(w, max_threads=16):
    """The oracle on every host core: threads take equal point ranges of the
    whole workload (the random streams are keyed by point id, so the range
    images sum to the full image exactly); ctypes releases the GIL around the
    oracle call."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    oracle.build(force=False)
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    threads = max(1, min(cores, max_threads))
    n = w["run"]["n_points"]
    bounds = [n * i // threads for i in range(threads + 1)]

    def part(i):
        run = dict(w["run"], n_points=bounds[i + 1] - bounds[i], point_offset=bounds[i])
        return oracle.chaos_count(w["system"], run, w["image"])["image"]

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        images = list(ex.map(part, range(threads)))
    dt = time.perf_counter() - t0
    total = images[0].astype(np.uint64)
    for im in images[1:]:
        total += im
    return {"value": n * w["run"]["n_iters"] / dt, "unit": "point-iterations/s",
            "cores": threads, "kind": "oracle",
            "sample": f"the whole workload ({n} points), {threads} threads over equal point "
                      f"ranges, FP64, {dt:.1f} s, CPU: {_cpu_model()}",
            "splats": int(total.sum())}


def _timed(fn, reps, stream):
    import torch
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def forms(dev, precision):
    """The batched and differentiable forms next to the plain chaos game."""
    import torch
    import workloads
    from paper_2606_02226_amd import api
    stream = torch.cuda.current_stream()
    out = {}
    # batched: 256 heterogeneous systems in one graph launch vs 256 plain calls
    entries = workloads.batched()
    images = [api.Image(w["image"], device=dev) for w in entries]
    batch = api.Batch(entries, images, precision=precision)
    graph_ms = _timed(batch.run, 5, stream)
    ws = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    systems = [api.System(w["system"]) for w in entries]

    def sequential():
        for w, s_, img in zip(entries, systems, images):
            img.clear()
            api.chaos_game(s_, w["run"], img, precision=precision, workspace=ws)

    seq_ms = _timed(sequential, 3, stream)
    pt_its = sum(w["run"]["n_points"] * w["run"]["n_iters"] for w in entries)
    splats = sum(w["run"]["n_points"] * (w["run"]["n_iters"] - w["run"]["burn_in"]) for w in entries)
    out["batched"] = {
        "workload": "256 random affine systems, 2..16 maps, 2^12..2^20 points x 32 "
                    "iterations (8 burn-in), 256^2..1024^2 u32 images",
        "precision": precision, "point_iterations": pt_its, "graph_ms": graph_ms,
        "point_iterations_per_s": pt_its / (graph_ms * 1e-3),
        "splats_per_s": splats / (graph_ms * 1e-3),
        "sequential_plain_ms": seq_ms, "speedup_vs_sequential_plain": seq_ms / graph_ms,
        "plan": batch.plan(), "error": "each instance bit-identical to its plain run"}
    batch.close()
    del images, ws
    # differentiable: forward + adjoint vs the plain count chaos game, same N, T
    w = workloads.differentiable()
    N, T = w["run"]["n_points"], w["run"]["n_iters"]
    img = api.Image(w["image"], device=dev)
    every = w["ckpt_every"]
    ckpt = torch.empty((api.n_checkpoints(T, every), N, 2), dtype=torch.float32, device=dev)
    G = torch.randn((512, 512), dtype=torch.float32, device=dev)
    sys_d = api.System(w["system"])

    def fwd():
        img.clear()
        api.splat(sys_d, w["run"], img, w["sigma_px"], ckpt=ckpt, ckpt_every=every)

    def bwd():
        api.splat_backward(sys_d, w["run"], img, w["sigma_px"], G, ckpt, every)

    fwd_ms = _timed(fwd, 10, stream)
    bwd_ms = _timed(bwd, 10, stream)
    cimg = api.Image({"kind": "u32_count", "width": 512, "height": 512, "channels": 1,
                      "lo": [0, 0], "hi": [1, 1]}, device=dev)

    def plain():
        cimg.clear()
        api.chaos_game(sys_d, w["run"], cimg, precision="f32")

    plain_ms = _timed(plain, 10, stream)
    out["grad"] = {
        "workload": "4-map affine system, 2^20 points x 32 iterations (8 burn-in), "
                    "Gaussian splat sigma 1 px into 512x512 FP32, checkpoints every 8",
        "forward_ms": fwd_ms, "backward_ms": bwd_ms, "forward_backward_ms": fwd_ms + bwd_ms,
        "plain_count_ms": plain_ms, "ratio_vs_plain": (fwd_ms + bwd_ms) / plain_ms,
        "checkpoint_bytes": int(ckpt.numel() * 4),
        "full_trajectory_bytes": int(N * (T + 1) * 2 * 4),
        "error": "gradient within 1e-4 rel. L2 of the FP64 adjoint and 1e-3 of FD (tests)"}
    del ckpt, img, cimg
    # several objects from one primitive: the 1920x1080 four-object scene
    w = workloads.space_scene()
    simg = api.Image(w["image"], device=dev)
    sws = torch.empty(api.scene_workspace_bytes(w["system"], w["objects"], w["run"], simg,
                                                precision), dtype=torch.uint8, device=dev)
    sys_s = api.System(w["system"])

    def scene():
        simg.clear()
        api.chaos_scene(sys_s, w["objects"], w["run"], simg, precision=precision, workspace=sws)

    scene_ms = _timed(scene, 10, stream)
    N, T, B = w["run"]["n_points"], w["run"]["n_iters"], w["run"]["burn_in"]
    n_obj = len(w["objects"])
    out["scene"] = {
        "workload": "circle IFS primitive, 4 objects (planet, rings, 512 stars, comet), "
                    "2^22 points x 32 iterations (8 burn-in), 4 x 1920x1080 u32",
        "precision": precision, "frame_ms": scene_ms,
        "point_iterations_per_s": N * T / (scene_ms * 1e-3),
        "splats_per_s": N * (T - B) * n_obj / (scene_ms * 1e-3),
        "error": "FP64: within 1e-4 rel. L1 of the oracle; direct and binned bit-identical (tests)"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["f32", "f64"], default="f64")
    ap.add_argument("--points-log2", type=int, default=24)
    ap.add_argument("--splat-path", choices=["auto", "direct", "binned"], default="auto")
    ap.add_argument("--cpu-sample-log2", type=int, default=23)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="copy 256 MiB once before timing (for counter calibration)")
    ap.add_argument("--summarise-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/traffic_cfs_square_<precision>.json from two "
                         "rocprofv3 --pmc output folders and exit (no GPU needed)")
    ap.add_argument("--summarise-valu", metavar="VALU_DIR",
                    help="write profiles/valu_cfs_square_<precision>.json from a rocprofv3 "
                         "--pmc SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_WAVES output folder and "
                         "exit (no GPU needed)")
    args = ap.parse_args()
    if args.summarise_pmc or args.summarise_valu:
        if args.summarise_pmc:
            summarise_pmc(*args.summarise_pmc, args.precision)
        if args.summarise_valu:
            summarise_valu(args.summarise_valu, args.precision)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; "
                                   "multi-GPU runs are not part of this build"}))
        sys.exit(2)

    import torch
    import workloads
    from paper_2606_02226_amd import _lib, api

    if not os.path.exists(_lib.LIB_PATH):
        from paper_2606_02226_amd import build as _b
        _b.build()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = workloads.cfs_square(n_points=1 << args.points_log2)
    run = w["run"]
    N, T, B = run["n_points"], run["n_iters"], run["burn_in"]
    sysc = api.System(w["system"])
    img = api.Image(w["image"], device=dev)
    stream = torch.cuda.current_stream()
    ws_bytes = api.chaos_workspace_bytes(sysc, run, img, args.precision, args.splat_path)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)

    def step(ev=None):
        img.clear()
        if ev is not None:
            ev[0].record(stream)
        api.chaos_game(sysc, run, img, precision=args.precision, splat_path=args.splat_path,
                       workspace=ws)
        if ev is not None:
            ev[1].record(stream)

    if args.calibration_copy:
        src = torch.empty(64 << 20, dtype=torch.int32, device=dev).fill_(1)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    api.timing_read()                       # drop anything recorded before
    api.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    api.timing_enable(False)
    phases = api.timing_read()              # [steps][chaos kernel, transpose, accumulate] ms
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    chaos_ms, transpose_ms, accumulate_ms = (float(v) for v in phases.mean(axis=0))

    # parity guard on the last step: exact total, no drops
    out = img.to_numpy()
    total = int(out["image"].astype(np.int64).sum())
    assert total == N * (T - B) and out["dropped"] == 0, (total, out["dropped"])

    pt_its = N * T
    splats = N * (T - B)
    value = pt_its * args.steps / elapsed
    lane_ops = valu_model("swirl", N, T, B)
    achieved = lane_ops / (chaos_ms * 1e-3) / 1e12
    peak = VALU_LANE_OPS_PEAK / 1e12
    result = {
        "metric": "point-iterations/s + splats/s on 1 MI355X; batched/grad vs plain at fixed err",
        "value": value,
        "unit": "point-iterations/s",
        "splats_per_s": splats * args.steps / elapsed,
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "kernel_ms": kernel_ms,
        "phase_ms": {"chaos_kernel": chaos_ms, "table_transpose": transpose_ms,
                     "tile_accumulate": accumulate_ms},
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic",
        "config": {"workload": "cfs_square: 4-map square + swirl/translate copy, "
                               "4-channel u32 2048x2048, 2^%d points x %d iterations "
                               "(%d burn-in)" % (args.points_log2, T, B),
                   "points": N, "iterations": T, "burn_in": B,
                   "image": [4, 2048, 2048], "precision": args.precision},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak,
                     "unit": "Tlane-op/s", "frac": achieved / peak,
                     "traffic": measured_traffic(args.precision),
                     "kernel": "k_chaos_binned (FP64 swirl, 4-channel count): the chaos "
                               "game with the LDS tile sort of its splats",
                     "lane_ops_per_launch": lane_ops,
                     "timing": "HIP events recorded by the library around the chaos kernel "
                               "on its stream (cfs_timing_enable), mean over the timed steps"},
    }
    valu = measured_valu(args.precision)
    if valu is not None and chaos_ms > 0:
        # a wave64 VALU instruction occupies its SIMD for 4 cycles: the share of
        # the kernel's SIMD cycles (1024 SIMDs at 2.4 GHz) that issue takes
        issue = valu["counters"]["SQ_INSTS_VALU"] * 4.0 / (1024 * 2.4e9 * chaos_ms * 1e-3)
        result["roofline"]["valu_counters"] = {
            "insts_per_point_iteration": valu["valu_insts_per_point_iteration"],
            "issue_share": issue,
            "source": f"profiles/valu_cfs_square_{args.precision}.json"}
    if not args.no_forms:
        result["forms"] = forms(dev, args.precision)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, 1 << args.cpu_sample_log2)
        result["cpu_baseline_all_cores"] = cpu_baseline_all_cores(w)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
