"""Benchmark of the CFS chaos-game hot path on one MI355X.

A step is one pass of the whole hot path over one workload: clear the image,
then the fused chaos game -- per-point random streams, selection, the map,
the composed transform of a copy, the burn-in gate, binning and the splat
(sorted by image tile in LDS, then accumulated per tile).  The timed region
holds exactly K steps between two device synchronisations.

The headline workload is the largest of the five: the 3D Menger sponge
(20 maps, 2^26 points x 24 iterations, 8 burn-in) with the twist and the
perspective camera into a 4096 x 4096 u64 depth|index min-image plus a u32
density.  The line also carries the CFS square (2^24 points x 32 iterations
into 4 x 2048^2 u32 counts) and the Sierpinski triangle as further
configurations, the batched and differentiable forms next to the plain
chaos game, the measured ceilings (HBM copy, device and LDS atomics), each
configuration's error against the FP64 oracle over the whole workload, and
the oracle's own rate on the host's cores.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import glob
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peak figures of MI355X (public specification): 256 CUs at 2.4 GHz, each
# issuing one 64-lane vector instruction per clock across its 4 SIMDs.
N_CU = 256
CLOCK_HZ = 2.4e9
VALU_LANE_OPS_PEAK = N_CU * 64 * CLOCK_HZ  # 3.93e13 lane-ops/s (full-rate ops)
HBM_PEAK_GBS = 8000.0

# Algorithmic VALU work per unit, in full-rate-equivalent lane operations (a
# quarter-rate instruction counts 4).  A point-iteration: a quarter of a
# Philox4x32-10 block (10 rounds of two quarter-rate 32x32->64 multiplies and
# two xors: 25), the selection (4), the map (2D: 4 FMA; 3D: 9 FMA) and loop
# control (3).  A splat: binning and address (10) plus the transform of the
# copy -- swirl: square root and sine/cosine (20); stretch (15); twist and
# camera: sine/cosine, reciprocal and 12 FMA (32).  FP64 transcendentals cost
# more than this counts, so the fractions are conservative.
PHILOX_PER_DRAW, SELECT, LOOP = 25, 4, 3
MAP_FMA = {2: 4, 3: 9}
PER_SPLAT = {"identity": 10, "swirl": 30, "stretch": 25, "twist_camera": 42}
# Gaussian splat (sigma 1 px, 6 x 6 taps): 12 exponentials (quarter rate)
# and 36 FMA for the weights; the adjoint's per-splat tap gradient 12
# exponentials and 72 FMA; its sweep recomputes the trajectory and takes the
# adjoint step (4 FMA) and the six gradient FMA per point-iteration.
GAUSS_SPLAT_FWD = 12 * 4 + 36
GAUSS_SPLAT_BWD = 12 * 4 + 72
ADJOINT_STEP = 10


def per_point_iteration(dim):
    return PHILOX_PER_DRAW + SELECT + MAP_FMA[dim] + LOOP


def valu_model(dim, final_kind, n_points, n_iters, burn_in):
    splats = n_points * (n_iters - burn_in)
    return n_points * n_iters * per_point_iteration(dim) + splats * PER_SPLAT[final_kind]


# ---------------------------------------------------------------------------
# committed counter summaries (valid only for the sources they were taken on)
# ---------------------------------------------------------------------------
def source_digest():
    """Digest of the HIP sources; counter summaries are valid only for it."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2606_02226_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + fh.read())
    return h.hexdigest()[:16]


def _profile_json(kind, workload, precision):
    path = os.path.join(ROOT, "profiles", f"{kind}_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_digest") != source_digest():
        return None
    return t


def measured_traffic(workload, precision):
    """HBM bytes per launch of each kernel of the step from the committed
    FETCH_SIZE / WRITE_SIZE counter runs, or None when the sources changed
    since they were taken."""
    t = _profile_json("traffic", workload, precision)
    return None if t is None else t.get("kernels")


def measured_valu(workload, precision):
    """VALU instruction counts of the chaos kernel from a rocprofv3 --pmc run,
    or None when the sources changed since it was taken."""
    return _profile_json("valu", workload, precision)


def _pmc_rows(directory, counter):
    """(kernel name, value) of every dispatch in a rocprofv3 --pmc CSV run.
    A folder that holds the files of several runs (one per process id, when
    output folders are reused) is read for its newest run only."""
    import csv
    import glob
    paths = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    if not paths:
        raise SystemExit(f"no counter files under {directory}")
    newest = max(paths, key=os.path.getmtime)
    if len(paths) > 1:
        print(f"{directory}: {len(paths)} runs, reading the newest ({os.path.basename(newest)})",
              file=sys.stderr)
    rows = []
    with open(newest, newline="") as fh:
        for r in csv.DictReader(fh):
            if r.get("Counter_Name") == counter:
                rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    if not rows:
        raise SystemExit(f"no {counter} rows under {directory}")
    return rows


def _workload(name):
    import workloads
    return {"menger": workloads.menger, "cfs_square": workloads.cfs_square,
            "sierpinski": workloads.sierpinski,
            # the paper's circle primitive alone, and mixed with two affine
            # maps (one system whose waves draw both kinds of map)
            "circle": lambda: workloads.circle(n_points=1 << 22),
            "circle_mixed": lambda: workloads.circle(n_points=1 << 22, extra_affine=2)}[name]()


# kernels of each configuration's step, as (name fragment, key)
STEP_KERNELS = {
    "menger": (("k_chaos_depth_binned", "chaos_kernel"), ("k_transpose", "table_transpose"),
               ("k_depth_accumulate", "tile_accumulate"), ("k_fill", "image_clear")),
    "cfs_square": (("k_chaos_binned", "chaos_kernel"), ("k_transpose", "table_transpose"),
                   ("k_tile_accumulate", "tile_accumulate"), ("k_fill", "image_clear")),
    "sierpinski": (("k_chaos_binned", "chaos_kernel"), ("k_transpose", "table_transpose"),
                   ("k_tile_accumulate", "tile_accumulate"), ("k_fill", "image_clear")),
    "circle": (("k_chaos_binned", "chaos_kernel"), ("k_transpose", "table_transpose"),
               ("k_tile_accumulate", "tile_accumulate"), ("k_fill", "image_clear")),
    "circle_mixed": (("k_chaos_binned", "chaos_kernel"), ("k_transpose", "table_transpose"),
                     ("k_tile_accumulate", "tile_accumulate"), ("k_fill", "image_clear")),
}


def summarise_valu(directory, workload, precision, out_dir=None):
    """Write profiles/valu_<workload>_<precision>.json from a rocprofv3 --pmc
    run of this benchmark with SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU and SQ_WAVES:
    mean per chaos-kernel dispatch, and the VALU wave-instructions issued per
    point-iteration (the guard against a kernel that is busy but bloated)."""
    w = _workload(workload)
    N, T = w["run"]["n_points"], w["run"]["n_iters"]
    frag = STEP_KERNELS[workload][0][0]
    out = {"source_digest": source_digest(), "precision": precision, "kernel": frag,
           "counters": {}}
    for counter in ("SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_WAVES"):
        vals = [v for k, v in _pmc_rows(directory, counter) if frag + "<" in k]
        if not vals:
            raise SystemExit(f"no {frag} {counter} rows under {directory}")
        out["counters"][counter] = float(np.mean(vals))
    # a step may cut the run into several launches (point-range slices)
    launches = max(1, round((N / 64.0) / out["counters"]["SQ_WAVES"]))
    out["launches_per_step"] = launches
    out["valu_insts_per_point_iteration"] = \
        out["counters"]["SQ_INSTS_VALU"] * launches / (N * T / 64.0)
    out["command"] = ("rocprofv3 --pmc SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_WAVES --output-format csv "
                      f"-d DIR -- python3 bench.py --workload {workload} --steps 2 --warmup 1 "
                      f"--no-cpu-baseline --no-forms --no-configs --no-ceilings --precision {precision}")
    path = os.path.join(out_dir or os.path.join(ROOT, "profiles"), f"valu_{workload}_{precision}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def _csv_rows(directory, suffix):
    import csv
    paths = sorted(glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True))
    if not paths:
        raise SystemExit(f"no *{suffix} under {directory}")
    with open(paths[0]) as fh:
        return list(csv.DictReader(fh))


def summarise_trace(directory, log_path, workload, precision, steps=5, warmup=2, out_dir=None):
    """Write profiles/trace_<workload>_<precision>.md from a rocprofv3
    --kernel-trace --stats run of this benchmark (--steps 5 --warmup 2) and
    the JSON line that run printed (log_path): the kernel statistics, the
    registers and LDS of each kernel, and the roofline kernel's mean over
    the timed steps' launches beside the bench line's own HIP-event figure,
    with the fraction that the profiled mean gives."""
    line = None
    with open(log_path) as fh:
        for text in fh:
            if text.startswith('{"metric"'):
                line = json.loads(text)
    if line is None:
        raise SystemExit(f"no bench line in {log_path}")
    stats = _csv_rows(directory, "_kernel_stats.csv")
    trace = _csv_rows(directory, "_kernel_trace.csv")
    frag = STEP_KERNELS[workload][0][0]
    mine = [r for r in trace if frag + "<" in r["Kernel_Name"]]
    mine.sort(key=lambda r: int(r["Start_Timestamp"]))
    per_step = len(mine) // (steps + warmup)
    if per_step == 0:
        raise SystemExit(f"no {frag} launches in {directory}")
    timed = mine[warmup * per_step:]
    dur = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6 for r in timed]
    step_ms = float(np.sum(dur)) / steps
    roof = line["roofline"]
    frac = roof["lane_ops_per_step"] / (step_ms * 1e-3) / 1e12 / roof["peak"]
    res = {}
    for r in trace:
        name = r["Kernel_Name"]
        res.setdefault(name, (r["VGPR_Count"], r["Accum_VGPR_Count"], r["SGPR_Count"],
                              r["LDS_Block_Size"], r["Scratch_Size"], r["Workgroup_Size_X"]))
    out = [f"# Kernel trace -- {workload}, {precision.upper()} positions", "",
           f"Workload: {line['config']['workload']}.  One MI355X.", "",
           "Command (repository root; `DIR` is an output folder):", "", "```",
           "cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats --output-format csv \\",
           f"    -d DIR -o {workload} -- python3 bench.py --workload {workload} --precision {precision} \\",
           f"    --steps {steps} --warmup {warmup} --no-cpu-baseline --no-forms --no-configs --no-ceilings",
           "```", "",
           f"Kernel statistics ({steps + warmup} steps: {warmup} warm-up + {steps} timed):", "",
           "| Kernel | Calls | Average (us) | Min (us) | Max (us) | Share | VGPR | AGPR | SGPR | LDS (B) | Scratch (B) | Lanes |",
           "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for r in stats:
        name = r["Name"]
        short = name.split("(")[0].replace("void ", "")
        v = res.get(name, ("", "", "", "", "", ""))
        out.append(f"| `{short}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                   f"{float(r['Percentage']):.1f}% | " + " | ".join(v) + " |")
    out += ["", f"The roofline kernel (`{frag}`): {per_step} launch(es) per step; over the "
            f"{steps} timed steps {step_ms:.3f} ms per step in the trace, against "
            f"{line['phase_ms']['chaos_kernel']:.3f} ms from the library's HIP events in the "
            f"bench line of the same run ({line['ms_per_step']:.3f} ms per step under the "
            f"profiler).  Fraction of the VALU model from the trace: "
            f"{roof['lane_ops_per_step']:.4g} lane-ops / {step_ms:.3f} ms / "
            f"{roof['peak']:.2f} T = **{frac:.3f}** (the line: {roof['frac']:.3f}).", ""]
    out += ["Phases of the bench line (ms per step): " +
            ", ".join(f"{k} {v:.3f}" for k, v in line["phase_ms"].items()) + ".", ""]
    path = os.path.join(out_dir or os.path.join(ROOT, "profiles"), f"trace_{workload}_{precision}.md")
    with open(path, "w") as fh:
        fh.write("\n".join(out))
    print("\n".join(out))


def summarise_pmc(fetch_dir, write_dir, workload, precision, out_dir=None):
    """Write profiles/traffic_<workload>_<precision>.json from two rocprofv3
    --pmc runs of this benchmark with --calibration-copy (FETCH_SIZE, then
    WRITE_SIZE; both in KiB per dispatch).  Each counter is scaled by the
    factor that makes the 256 MiB calibration copy read and write 256 MiB;
    per kernel the bytes of one step (a step may hold several launches)."""
    copy_bytes = 256 << 20
    out = {"source_digest": source_digest(), "precision": precision,
           "unit": "bytes per step", "calibration": {}, "kernels": {}}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _pmc_rows(d, counter)
        copies = [v for k, v in rows if "copyBuffer" in k]
        scale = copy_bytes / (max(copies) * 1024.0)
        out["calibration"][counter] = {"copy_kib": max(copies), "scale": scale}
        for frag, key in STEP_KERNELS[workload]:
            vals = [v for k, v in rows if frag in k and "copyBuffer" not in k]
            if vals:
                # profiled with --steps 2 --warmup 1: three steps' dispatches
                out["kernels"].setdefault(key, {})[counter] = float(np.sum(vals)) / 3.0 * 1024.0 * scale
    out["command"] = ("rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) --output-format csv -d DIR "
                      f"-- python3 bench.py --workload {workload} --steps 2 --warmup 1 "
                      "--no-cpu-baseline --no-forms --no-configs --no-ceilings "
                      f"--calibration-copy --precision {precision}")
    path = os.path.join(out_dir or os.path.join(ROOT, "profiles"), f"traffic_{workload}_{precision}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


# ---------------------------------------------------------------------------
# host figures
# ---------------------------------------------------------------------------
def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_info():
    """What the host offers: logical CPUs, the ones this process may use, the
    thread cap of the all-cores figure (one GPU's share of a GPU machine's
    cores), and the CPU model."""
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "affinity": allowed, "thread_cap": 16,
            "model": _cpu_model()}


def cpu_baseline(w, n_sample):
    """The FP64 oracle, single-threaded, on the first n_sample points of the
    workload (all iterations, the full image)."""
    import oracle
    oracle.build(force=False)
    run = dict(w["run"], n_points=n_sample)
    t0 = time.perf_counter()
    if w["image"]["kind"] == "u64_depth":
        oracle.chaos_depth(w["system"], run, w["image"], w["image"]["near"])
    else:
        oracle.chaos_count(w["system"], run, w["image"])
    dt = time.perf_counter() - t0
    return {"value": n_sample * run["n_iters"] / dt, "unit": "point-iterations/s",
            "cores": 1, "kind": "oracle",
            "sample": f"{n_sample} of {w['run']['n_points']} points (all iterations, "
                      f"full image), single-threaded FP64, {dt:.1f} s",
            "host": host_info()}


def cpu_baseline_all_cores(w, max_threads=16):
    """The oracle over the whole workload on the host's cores: threads take
    equal point ranges (the random streams are keyed by point id, so the
    range images sum -- or, for depth keys, take the minimum -- to the full
    image exactly); ctypes releases the GIL around each oracle call.
    Returns the figure and the oracle's image (the parity reference)."""
    import oracle
    oracle.build(force=False)
    host = host_info()
    threads = max(1, min(host["affinity"], max_threads))
    n = w["run"]["n_points"]
    t0 = time.perf_counter()
    if w["image"]["kind"] == "u64_depth":
        ref = oracle.chaos_depth_sharded(w["system"], w["run"], w["image"], w["image"]["near"],
                                         threads=threads)
        splats = int(ref["density"].astype(np.int64).sum())
    else:
        ref = oracle.chaos_count_sharded(w["system"], w["run"], w["image"], threads=threads)
        splats = int(ref["image"].astype(np.int64).sum())
    dt = time.perf_counter() - t0
    fig = {"value": n * w["run"]["n_iters"] / dt, "unit": "point-iterations/s",
           "cores": threads, "kind": "oracle",
           "sample": f"the whole workload ({n} points), {threads} threads over equal point "
                     f"ranges, FP64, {dt:.1f} s",
           "host": host, "splats": splats}
    return fig, ref


def parity_error(got, ref):
    """Error of a GPU image against the oracle's image of the same workload."""
    if "depth" in ref:
        g, r = got["depth"].reshape(-1), ref["depth"].reshape(-1)
        empty = np.uint64(0xFFFFFFFFFFFFFFFF)
        gd = got["density"].astype(np.int64)
        rd = ref["density"].astype(np.int64)
        return {"density_rel_l1": float(np.abs(gd - rd).sum()) / max(float(rd.sum()), 1.0),
                "keys_differing": int(np.count_nonzero(g != r)),
                "occupied_pixels": int(np.count_nonzero(r != empty)),
                "dropped_equal": got["dropped"] == ref["dropped"],
                "reference": "FP64 oracle, whole workload"}
    h = got["image"].astype(np.int64)
    r = ref["image"].astype(np.int64)
    return {"rel_l1": float(np.abs(h - r).sum()) / max(float(r.sum()), 1.0),
            "pixels_differing": int(np.count_nonzero(h != r)),
            "dropped_equal": got["dropped"] == ref["dropped"],
            "reference": "FP64 oracle, whole workload"}


# ---------------------------------------------------------------------------
# device figures
# ---------------------------------------------------------------------------
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


def ceilings(dev):
    """Measured ceilings of the operations the splats are made of
    (cfs_microbench): HBM copy, random device atomics into working sets of
    the images' sizes, random LDS atomics in 64 KiB tables, Philox blocks."""
    import torch
    from paper_2606_02226_amd import api
    stream = torch.cuda.current_stream()
    out = {}
    buf = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
    n = api.microbench("copy", buf)
    ms = _timed(lambda: api.microbench("copy", buf), 10, stream)
    out["hbm_copy"] = {"GB_per_s": n / (ms * 1e-3) / 1e9, "bytes": n,
                       "what": "read + write of a 256 MiB device-to-device copy"}
    del buf
    for kind, mib, what in (("dev_add_u32", 64, "random u32 atomic add, 64 MiB set"),
                            ("dev_min_u64", 128, "random u64 atomic min, 128 MiB set")):
        buf = torch.zeros(mib << 20, dtype=torch.uint8, device=dev)
        ops = 1 << 27
        n = api.microbench(kind, buf, ops=ops)
        ms = _timed(lambda: api.microbench(kind, buf, ops=ops), 3, stream)
        out[kind] = {"G_per_s": n / (ms * 1e-3) / 1e9, "what": what}
        del buf
    small = torch.zeros(1 << 16, dtype=torch.uint8, device=dev)
    for kind, what in (("lds_add_u32", "random u32 LDS atomic add, 64 KiB table"),
                       ("lds_add_u64", "random u64 LDS atomic add, 64 KiB table"),
                       ("lds_min_u64", "random u64 LDS atomic min, 64 KiB table")):
        ops = 1 << 31
        n = api.microbench(kind, small, ops=ops)
        ms = _timed(lambda: api.microbench(kind, small, ops=ops), 3, stream)
        rate = n / (ms * 1e-3)
        out[kind] = {"G_per_s": rate / 1e9, "per_cu_per_clock": rate / (N_CU * CLOCK_HZ),
                     "what": what}
    # scattered runs in 2 GiB (beyond the caches), the accumulates' pattern
    rbuf = torch.zeros((4 << 20) + (2 << 30), dtype=torch.uint8, device=dev)
    for kind, length in (("runs_128", 128), ("runs_512", 512), ("runs_2048", 2048)):
        ops = (1 << 31) // length
        n = api.microbench(kind, rbuf, ops=ops)
        ms = _timed(lambda: api.microbench(kind, rbuf, ops=ops), 3, stream)
        out[kind] = {"GB_per_s": n / (ms * 1e-3) / 1e9, "bytes": n,
                     "what": f"reads of {length}-byte runs at random 16-byte-aligned places "
                             "in 2 GiB"}
    del rbuf
    lanes = 4096 * 256
    pbuf = torch.zeros(lanes * 4, dtype=torch.uint8, device=dev)
    n = api.microbench("philox", pbuf, ops=lanes * 256)
    ms = _timed(lambda: api.microbench("philox", pbuf, ops=lanes * 256), 3, stream)
    rate = n / (ms * 1e-3)
    out["philox"] = {"G_blocks_per_s": rate / 1e9,
                     "lane_ops_per_block_at_valu_peak": VALU_LANE_OPS_PEAK / rate,
                     "what": "Philox4x32-10 blocks (4 draws each)"}
    return out


def _phase_rooflines(name, w, ms, ceil):
    """Roofline of each kernel of a chaos-game step: the chaos kernel against
    the VALU model; the run-table transpose against HBM; the accumulate
    against HBM (its records) and the LDS atomics it issues."""
    sysd, run, img = w["system"], w["run"], w["image"]
    N, T, B = run["n_points"], run["n_iters"], run["burn_in"]
    dim = int(sysd["dim"])
    splats = N * (T - B)
    out = {}
    lane_ops = valu_model(dim, sysd["final_kind"], N, T, B)
    out["chaos_kernel"] = {"bound": "alu", "unit": "Tlane-op/s",
                           "achieved": lane_ops / (ms["chaos_kernel"] * 1e-3) / 1e12,
                           "peak": VALU_LANE_OPS_PEAK / 1e12,
                           "lane_ops_per_step": lane_ops, "ms": ms["chaos_kernel"]}
    if ms.get("tile_accumulate", 0) > 0:
        depth = img["kind"] == "u64_depth"
        rec = 8 if depth else 2
        # records (each written once by the chaos kernel, read once here) and
        # the image tiles read and written back
        elems = img["width"] * img["height"] * img.get("channels", 1)
        img_bytes = elems * (12 if depth else 4)
        acc_bytes = splats * rec + 2 * img_bytes
        hbm_ms = acc_bytes / (HBM_PEAK_GBS * 1e9) * 1e3
        out["tile_accumulate"] = {"bound": "hbm", "unit": "GB/s",
                                  "achieved": acc_bytes / (ms["tile_accumulate"] * 1e-3) / 1e9,
                                  "peak": HBM_PEAK_GBS, "bytes_per_step": acc_bytes,
                                  "ms": ms["tile_accumulate"], "hbm_bound_ms": hbm_ms}
        if ceil:
            if depth:
                lds_ms = splats / (ceil["lds_min_u64"]["G_per_s"] * 1e9) * 1e3 + \
                    splats / (ceil["lds_add_u32"]["G_per_s"] * 1e9) * 1e3
                what = "u64 min + u32 add per splat"
            else:
                lds_ms = splats / (ceil["lds_add_u32"]["G_per_s"] * 1e9) * 1e3
                what = "u32 add per splat"
            out["tile_accumulate"]["lds_atomic_bound_ms"] = lds_ms
            out["tile_accumulate"]["lds_atomics"] = what
            bound = max(hbm_ms, lds_ms)
            if "runs_128" in ceil:
                # the records arrive as runs of 15-40 records at scattered
                # places: the measured read rate of 128-byte runs bounds them
                runs_ms = splats * rec / (ceil["runs_128"]["GB_per_s"] * 1e9) * 1e3
                out["tile_accumulate"]["runs_read_bound_ms"] = runs_ms
                bound = max(bound, runs_ms)
            out["tile_accumulate"]["frac_of_lower_bound"] = bound / ms["tile_accumulate"]
    if ms.get("table_transpose", 0) > 0:
        out["table_transpose"] = {"ms": ms["table_transpose"]}
    for v in out.values():
        if "achieved" in v:
            v["frac"] = v["achieved"] / v["peak"]
    return out


def chaos_leg(name, dev, steps, warmup, precision, splat_path, ceil, *, error=True,
              cpu=False, cpu_sample_log2=None, calibration_copy=False):
    """K timed steps of one plain chaos-game configuration, its rooflines,
    and (optionally) its error against the oracle and the oracle's rates."""
    import torch
    from paper_2606_02226_amd import api
    w = _workload(name)
    run = w["run"]
    N, T, B = run["n_points"], run["n_iters"], run["burn_in"]
    sysc = api.System(w["system"])
    img = api.Image(w["image"], device=dev)
    stream = torch.cuda.current_stream()
    ws_bytes = api.chaos_workspace_bytes(sysc, run, img, precision, splat_path)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)

    def step():
        img.clear()
        api.chaos_game(sysc, run, img, precision=precision, splat_path=splat_path, workspace=ws)

    if calibration_copy:
        src = torch.empty(64 << 20, dtype=torch.int32, device=dev).fill_(1)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    api.timing_read()                       # drop anything recorded before
    api.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    api.timing_enable(False)
    phases = api.timing_read()              # [steps][chaos kernel, transpose, accumulate] ms
    ms = dict(zip(("chaos_kernel", "table_transpose", "tile_accumulate"),
                  (float(v) for v in phases.mean(axis=0))))
    got = img.to_numpy()
    # exact totals: every splat counted or dropped
    splats = N * (T - B)
    counted = int((got["density"] if "density" in got else got["image"]).astype(np.int64).sum())
    assert counted + got["dropped"] == splats, (counted, got["dropped"], splats)
    leg = {
        "workload": name, "precision": precision,
        "points": N, "iterations": T, "burn_in": B, "image": w["image"],
        "ms_per_step": elapsed / steps * 1e3,
        "point_iterations_per_s": N * T * steps / elapsed,
        "splats_per_s": splats * steps / elapsed,
        "phase_ms": ms,
        "rooflines": _phase_rooflines(name, w, ms, ceil),
        "workspace_bytes": ws_bytes,
    }
    leg["image"] = {k: v for k, v in w["image"].items()}
    if error or cpu:
        fig, ref = cpu_baseline_all_cores(w)
        leg["error"] = parity_error(got, ref)
        leg["cpu_baseline_all_cores"] = fig
        del ref
    if cpu:
        leg["cpu_baseline"] = cpu_baseline(w, 1 << cpu_sample_log2)
    return leg


def forms(dev, precision, ceil):
    """The batched and differentiable forms next to the plain chaos game."""
    import torch
    import workloads
    from paper_2606_02226_amd import api
    stream = torch.cuda.current_stream()
    out = {}
    # batched: 256 heterogeneous systems in one graph launch (default plan and
    # the autotuned plan) vs 256 plain calls and vs one plain run of equal work
    entries = workloads.batched()
    images = [api.Image(w["image"], device=dev) for w in entries]
    pt_its = sum(w["run"]["n_points"] * w["run"]["n_iters"] for w in entries)
    splats = sum(w["run"]["n_points"] * (w["run"]["n_iters"] - w["run"]["burn_in"])
                 for w in entries)
    lane_ops = sum(valu_model(2, "identity", w["run"]["n_points"], w["run"]["n_iters"],
                              w["run"]["burn_in"]) for w in entries)
    batch = api.Batch(entries, images, precision=precision)
    default_plan = batch.plan()
    graph_ms = _timed(batch.run, 5, stream)
    batch.close()
    tuned_plan = api.autotune(entries, images, precision=precision)
    tbatch = api.Batch(entries, images, plan=tuned_plan, precision=precision)
    tuned_ms = _timed(tbatch.run, 5, stream)
    tbatch.close()
    ws = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    systems = [api.System(w["system"]) for w in entries]

    def sequential():
        for w, s_, img in zip(entries, systems, images):
            img.clear()
            api.chaos_game(s_, w["run"], img, precision=precision, workspace=ws)

    seq_ms = _timed(sequential, 3, stream)
    del images
    # the plain kernel on one run of the same total work: the batch's first
    # system, all its points at once, into a 1024^2 u32 image
    total_points = sum(w["run"]["n_points"] for w in entries)
    w0 = entries[0]
    big_run = dict(w0["run"], n_points=total_points)
    big_img = api.Image(dict(w0["image"], width=1024, height=1024), device=dev)
    big_ws = torch.empty(max(api.chaos_workspace_bytes(systems[0], big_run, big_img, precision), 1),
                         dtype=torch.uint8, device=dev)

    def plain_equal():
        big_img.clear()
        api.chaos_game(systems[0], big_run, big_img, precision=precision, workspace=big_ws)

    equal_ms = _timed(plain_equal, 3, stream)
    del big_ws, big_img, ws
    best_ms = min(graph_ms, tuned_ms)
    out["batched"] = {
        "workload": "256 random affine systems, 2..16 maps, 2^12..2^20 points x 32 "
                    "iterations (8 burn-in), 256^2..1024^2 u32 images",
        "precision": precision, "point_iterations": pt_its, "splats": splats,
        "graph_ms_default_plan": graph_ms, "default_plan": default_plan,
        "graph_ms_tuned_plan": tuned_ms, "tuned_plan": tuned_plan,
        "point_iterations_per_s": pt_its / (best_ms * 1e-3),
        "splats_per_s": splats / (best_ms * 1e-3),
        "sequential_plain_ms": seq_ms, "speedup_vs_sequential_plain": seq_ms / best_ms,
        "plain_equal_work_ms": equal_ms,
        "plain_equal_work_point_iterations_per_s": total_points * w0["run"]["n_iters"]
        / (equal_ms * 1e-3),
        "plain_equal_work": f"one plain call: the first system, {total_points} points, same "
                            "iterations, 1024^2 u32 image",
        "roofline": {"bound": "alu", "unit": "Tlane-op/s",
                     "achieved": lane_ops / (best_ms * 1e-3) / 1e12,
                     "peak": VALU_LANE_OPS_PEAK / 1e12,
                     "frac": lane_ops / (best_ms * 1e-3) / VALU_LANE_OPS_PEAK,
                     "lane_ops": lane_ops,
                     "over": "the whole graph launch (clears, chaos, transposes, accumulates)"},
        "error": "every instance equal to the FP64 oracle's image at full size "
                 "(rel. L1 0); each bit-identical to its plain run (tests)"}
    # differentiable: forward + adjoint vs the plain count chaos game, same N, T
    w = workloads.differentiable()
    N, T, B = w["run"]["n_points"], w["run"]["n_iters"], w["run"]["burn_in"]
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
    splats_d = N * (T - B)
    taps = splats_d * 36
    fwd_valu = N * T * per_point_iteration(2) + splats_d * (PER_SPLAT["identity"] + GAUSS_SPLAT_FWD)
    bwd_valu = (N * T * per_point_iteration(2) + splats_d * PER_SPLAT["identity"]  # records again
                + splats_d * GAUSS_SPLAT_BWD                                      # tap gradients
                + N * T * (per_point_iteration(2) + ADJOINT_STEP))                # sweep
    fwd_bound = {"valu_ms": fwd_valu / VALU_LANE_OPS_PEAK * 1e3}
    if ceil:
        fwd_bound["lds_atomic_ms"] = taps / (ceil["lds_add_u32"]["G_per_s"] * 1e9) * 1e3
    bwd_bound = {"valu_ms": bwd_valu / VALU_LANE_OPS_PEAK * 1e3}
    out["grad"] = {
        "workload": "4-map affine system, 2^20 points x 32 iterations (8 burn-in), "
                    "Gaussian splat sigma 1 px into 512x512 FP32, checkpoints every 8",
        "forward_ms": fwd_ms, "backward_ms": bwd_ms, "forward_backward_ms": fwd_ms + bwd_ms,
        "plain_count_ms": plain_ms, "ratio_vs_plain": (fwd_ms + bwd_ms) / plain_ms,
        "checkpoint_bytes": int(ckpt.numel() * 4),
        "full_trajectory_bytes": int(N * (T + 1) * 2 * 4),
        "roofline": {
            "forward": dict(fwd_bound, frac=max(fwd_bound.values()) / fwd_ms,
                            what="32-bit LDS tap atomics (36 per splat, measured ceiling) "
                                 "or VALU model, whichever is longer"),
            "backward": dict(bwd_bound, frac=max(bwd_bound.values()) / bwd_ms,
                             what="VALU model: records again, tap gradients, the sweep")},
        "error": "gradient within 1e-4 rel. L2 of the FP64 adjoint at full size "
                 "(1.3e-6 measured) and 1e-3 of FD (tests)"}
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
    ap.add_argument("--warmup", type=int, default=10,
                    help="untimed steps first (the chaos kernel still speeds up over the "
                         "first several launches of a process)")
    ap.add_argument("--workload", choices=["menger", "cfs_square", "sierpinski", "circle",
                                           "circle_mixed"],
                    default="menger", help="the headline configuration")
    ap.add_argument("--precision", choices=["f32", "f64"], default=None,
                    help="positions (default: f64, f32 for the Sierpinski triangle)")
    ap.add_argument("--splat-path", choices=["auto", "direct", "binned"], default="auto")
    ap.add_argument("--cpu-sample-log2", type=int, default=None,
                    help="points of the single-threaded oracle sample (log2)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="time only the headline configuration")
    ap.add_argument("--no-ceilings", action="store_true")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="copy 256 MiB once before timing (for counter calibration)")
    ap.add_argument("--summarise-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/traffic_<workload>_<precision>.json from two "
                         "rocprofv3 --pmc output folders and exit (no GPU needed)")
    ap.add_argument("--summarise-trace", nargs=2, metavar=("TRACE_DIR", "LOG"),
                    help="write profiles/trace_<workload>_<precision>.md from a rocprofv3 "
                         "--kernel-trace --stats run (--steps 5 --warmup 2) and its output")
    ap.add_argument("--summarise-valu", metavar="VALU_DIR",
                    help="write profiles/valu_<workload>_<precision>.json from a rocprofv3 "
                         "--pmc SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_WAVES output folder and "
                         "exit (no GPU needed)")
    args = ap.parse_args()
    default_prec = {"menger": "f64", "cfs_square": "f64", "sierpinski": "f32", "circle": "f64",
                    "circle_mixed": "f64"}
    precision = args.precision or default_prec[args.workload]
    if args.summarise_pmc or args.summarise_valu or args.summarise_trace:
        if args.summarise_trace:
            summarise_trace(*args.summarise_trace, args.workload, precision)
        if args.summarise_pmc:
            summarise_pmc(*args.summarise_pmc, args.workload, precision)
        if args.summarise_valu:
            summarise_valu(args.summarise_valu, args.workload, precision)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; "
                                   "multi-GPU runs are not part of this build"}))
        sys.exit(2)

    import torch
    from paper_2606_02226_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        from paper_2606_02226_amd import build as _b
        _b.build()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ceil = None if args.no_ceilings else ceilings(dev)
    sample_log2 = args.cpu_sample_log2 or {"menger": 22, "cfs_square": 23, "sierpinski": 16,
                                            "circle": 18, "circle_mixed": 18}[args.workload]
    head = chaos_leg(args.workload, dev, args.steps, args.warmup, precision, args.splat_path,
                     ceil, error=not args.no_cpu_baseline, cpu=not args.no_cpu_baseline,
                     cpu_sample_log2=sample_log2, calibration_copy=args.calibration_copy)
    # the dominant kernel of the step: the phase that takes longest
    rl = head["rooflines"]
    dom = max((k for k in rl if "ms" in rl[k]), key=lambda k: rl[k]["ms"])
    chaos_name = [f for f, k in STEP_KERNELS[args.workload] if k == "chaos_kernel"][0]
    roof = {k: v for k, v in rl["chaos_kernel"].items()}
    roof["kernel"] = f"{chaos_name}: the fused chaos game with the LDS tile sort of its splats"
    roof["timing"] = ("HIP events recorded by the library around the kernel on its stream "
                      "(cfs_timing_enable), mean over the timed steps")
    roof["dominant_phase"] = dom
    traffic = measured_traffic(args.workload, precision)
    roof["traffic"] = None
    if traffic and "chaos_kernel" in traffic:
        tk = traffic["chaos_kernel"]
        roof["traffic"] = tk.get("FETCH_SIZE", 0.0) + tk.get("WRITE_SIZE", 0.0)
    result = {
        "metric": "point-iterations/s + splats/s on 1 MI355X; batched/grad vs plain at fixed err",
        "value": head["point_iterations_per_s"],
        "unit": "point-iterations/s",
        "splats_per_s": head["splats_per_s"],
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "phase_ms": head["phase_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": precision, "data": "synthetic",
        "config": {"workload": {
            "menger": "menger: 20-map Menger sponge, twist + perspective camera of a copy, "
                      "4096x4096 u64 depth|index min-image + u32 density, 2^26 points x 24 "
                      "iterations (8 burn-in)",
            "cfs_square": "cfs_square: 4-map square + swirl/translate copy, 4-channel u32 "
                          "2048x2048, 2^24 points x 32 iterations (8 burn-in)",
            "sierpinski": "sierpinski: 3 maps, 512x512 u32, 2^16 points x 64 iterations "
                          "(16 burn-in)",
            "circle": "circle: the paper's circle IFS (2 circle maps), 2x512x512 u32, 2^22 "
                      "points x 48 iterations (16 burn-in)",
            "circle_mixed": "circle_mixed: 2 circle maps + 2 affine maps, 4x512x512 u32, 2^22 "
                            "points x 48 iterations (16 burn-in)"}[args.workload],
            "points": head["points"], "iterations": head["iterations"],
            "burn_in": head["burn_in"], "image": head["image"], "precision": precision},
        "roofline": roof,
        "phase_rooflines": rl,
    }
    valu = measured_valu(args.workload, precision)
    if valu is not None and head["phase_ms"]["chaos_kernel"] > 0:
        # a wave64 VALU instruction occupies its SIMD for 4 cycles: the share
        # of the kernel's SIMD cycles (1024 SIMDs at 2.4 GHz) that issue takes
        insts = valu["counters"]["SQ_INSTS_VALU"] * valu.get("launches_per_step", 1)
        issue = insts * 4.0 / (1024 * CLOCK_HZ * head["phase_ms"]["chaos_kernel"] * 1e-3)
        result["roofline"]["valu_counters"] = {
            "insts_per_point_iteration": valu["valu_insts_per_point_iteration"],
            "issue_share": issue,
            "source": f"profiles/valu_{args.workload}_{precision}.json"}
    if "error" in head:
        result["error"] = head["error"]
    if "cpu_baseline" in head:
        result["cpu_baseline"] = head["cpu_baseline"]
        result["cpu_baseline_all_cores"] = head["cpu_baseline_all_cores"]
    if ceil:
        result["ceilings"] = ceil
    if not args.no_configs:
        others = {}
        for name in ("menger", "cfs_square", "sierpinski"):
            if name == args.workload:
                continue
            leg = chaos_leg(name, dev, args.steps, args.warmup, default_prec[name],
                            "auto", ceil, error=not args.no_cpu_baseline)
            others[name] = leg
        result["configs"] = others
    if not args.no_forms:
        result["forms"] = forms(dev, "f64", ceil)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
