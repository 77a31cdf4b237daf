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


def valu_model(dim, final_kind, precision, n_points, n_iters, burn_in):
    """Algorithmic full-rate-equivalent lane-ops of the chaos game.

    Per point-iteration: a quarter of a Philox4x32-10 block (10 rounds x
    (2 quarter-rate 32x32->64 multiplies + 2 xors) = 100 per block), one
    quarter-rate mul_hi for the selection, d*d FMAs for the map, one for the
    loop.  Per point: one more Philox block for the initial point and d
    conversions.  Per splat: the composed transform, the binning and the
    atomic's address (constants per kind below)."""
    per_it = 25 + 4 + dim * dim + 1
    per_point = 100 + 2 * dim
    splat_cost = {("identity", "f32"): 12, ("identity", "f64"): 12,
                  ("swirl", "f32"): 12 + 30, ("swirl", "f64"): 12 + 45,
                  ("stretch", "f32"): 12 + 20, ("stretch", "f64"): 12 + 30}
    per_splat = splat_cost.get((final_kind, precision), 40)
    splats = n_points * (n_iters - burn_in)
    return n_points * n_iters * per_it + n_points * per_point + splats * per_splat


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["f32", "f64"], default="f64")
    ap.add_argument("--points-log2", type=int, default=24)
    ap.add_argument("--splat-path", choices=["auto", "direct", "binned"], default="auto")
    ap.add_argument("--cpu-sample-log2", type=int, default=21)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
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

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))

    # parity guard on the last step: exact total, no drops
    out = img.to_numpy()
    total = int(out["image"].astype(np.int64).sum())
    assert total == N * (T - B) and out["dropped"] == 0, (total, out["dropped"])

    pt_its = N * T
    splats = N * (T - B)
    value = pt_its * args.steps / elapsed
    lane_ops = valu_model(2, "swirl", args.precision, N, T, B)
    achieved = lane_ops / (kernel_ms * 1e-3) / 1e12
    peak = VALU_LANE_OPS_PEAK / 1e12
    result = {
        "metric": "point-iterations/s + splats/s on 1 MI355X; batched/grad vs plain at fixed err",
        "value": value,
        "unit": "point-iterations/s",
        "splats_per_s": splats * args.steps / elapsed,
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "kernel_ms": kernel_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic",
        "config": {"workload": "cfs_square: 4-map square + swirl/translate copy, "
                               "4-channel u32 2048x2048, 2^%d points x %d iterations "
                               "(%d burn-in)" % (args.points_log2, T, B),
                   "points": N, "iterations": T, "burn_in": B,
                   "image": [4, 2048, 2048], "precision": args.precision},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak,
                     "unit": "Tlane-op/s", "frac": achieved / peak, "traffic": None,
                     "kernel": "k_chaos (swirl, 4-channel count)",
                     "lane_ops_per_launch": lane_ops},
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, 1 << args.cpu_sample_log2)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
