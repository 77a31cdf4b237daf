"""FP64 CPU oracle of the CFS chaos game -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's ``cpu_baseline`` leg may
import this package.  The GPU library never imports, links or calls it, and it
imports nothing from the GPU library.

The arithmetic lives in ``cfs_oracle.c`` (plain C, FP64, single thread, no FMA
contraction); this module only builds it with gcc and marshals numpy arrays.
Every function cites the part of the paper it follows in the C source.

Parity status:
  philox4x32_10      pinned: published known-answer vectors
  thresholds/select  pinned: exhaustive over all 2^32 draws, closed form
  chaos_count        pinned: invariant-measure moments, uniform square,
                     Sierpinski box dimension, address containment,
                     composition order; circle maps: invariant uniform disk
                     (moments of r^2, half-disk per index)
  chaos_depth        pinned: Menger occupancy of the 3^k grid and box
                     dimension for the 3D points; the splat coordinates by
                     inverting the camera and the twist back to the points;
                     the depth image and density by brute-force assembly
                     from those splats and the steps' map indices
  splat_gauss        pinned: total mass closed form, separable kernel sums
  splat_gauss_backward pinned: central finite differences of splat_gauss,
                     zero gradient at the target
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cfs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_cfs_oracle.so")

FINAL_KINDS = {"identity": 0, "swirl": 1, "twist_camera": 2, "stretch": 3, "ring": 4}
MAP_KINDS = {"affine": 0, "circle": 1}
COMPOSE = {"copy": 0, "reuse": 1}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain IEEE FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _System(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_maps", C.c_int32),
                ("A", C.POINTER(C.c_float)), ("b", C.POINTER(C.c_float)),
                ("prob", C.POINTER(C.c_double)), ("final_kind", C.c_int32),
                ("final_params", C.POINTER(C.c_float)), ("kind", C.POINTER(C.c_int32)),
                ("compose", C.c_int32)]


class _Run(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("instance", C.c_uint32),
                ("n_points", C.c_uint32), ("point_offset", C.c_uint32),
                ("n_iters", C.c_uint32), ("burn_in", C.c_uint32),
                ("iter_offset", C.c_uint32)]


class _Window(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32),
                ("channels", C.c_int32), ("lo", C.c_float * 2),
                ("hi", C.c_float * 2)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        lib.orc_philox4x32_10.argtypes = [P, P, P]
        lib.orc_philox_many.argtypes = [C.c_uint64, P, P, C.c_int64]
        lib.orc_thresholds.argtypes = [P, C.c_int, P]
        lib.orc_select.argtypes = [C.c_uint32, P, C.c_int]
        lib.orc_select_histogram.argtypes = [P, C.c_int, P]
        lib.orc_chaos_count.argtypes = [P, P, P, P, P, P, P, P, P]
        lib.orc_chaos_depth.argtypes = [P, P, P, C.c_float, P, P, P, P, P, P]
        lib.orc_chaos_scene.argtypes = [P, P, C.c_int, P, P, P, P, P]
        lib.orc_splat_gauss.argtypes = [P, P, P, C.c_double, P, P]
        lib.orc_splat_gauss_backward.argtypes = [P, P, P, C.c_double, P, P]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class _Keep:
    """Holds the numpy buffers a ctypes struct points into."""

    def __init__(self, system):
        d = int(system["dim"])
        self.A = np.ascontiguousarray(system["A"], dtype=np.float32).reshape(-1)
        self.b = np.ascontiguousarray(system["b"], dtype=np.float32).reshape(-1)
        n = self.b.size // d
        prob = system.get("prob")
        self.prob = None if prob is None else np.ascontiguousarray(prob, dtype=np.float64)
        fp = np.zeros(24, np.float32)
        src = np.asarray(system.get("final_params", []), np.float32).reshape(-1)
        fp[: src.size] = src
        self.fp = fp
        kinds = system.get("kind")
        self.kind = None if kinds is None else np.ascontiguousarray(
            [MAP_KINDS[k] if isinstance(k, str) else int(k) for k in kinds], dtype=np.int32)
        self.s = _System(d, n, self.A.ctypes.data_as(C.POINTER(C.c_float)),
                         self.b.ctypes.data_as(C.POINTER(C.c_float)),
                         None if self.prob is None else
                         self.prob.ctypes.data_as(C.POINTER(C.c_double)),
                         FINAL_KINDS[system.get("final_kind", "identity")],
                         self.fp.ctypes.data_as(C.POINTER(C.c_float)),
                         None if self.kind is None else
                         self.kind.ctypes.data_as(C.POINTER(C.c_int32)),
                         COMPOSE[system.get("compose", "copy")])


def _run(run):
    return _Run(int(run.get("seed", 0)), int(run.get("instance", 0)),
                int(run["n_points"]), int(run.get("point_offset", 0)),
                int(run["n_iters"]), int(run["burn_in"]), int(run.get("iter_offset", 0)))


def _start(run, start, n, d):
    """Positions of a continued run (iter_offset > 0): a copy of ``start``
    [N][d] that the oracle reads and overwrites; None for a fresh run."""
    if not int(run.get("iter_offset", 0)):
        return None
    if start is None:
        raise ValueError("a run with iter_offset > 0 needs start positions")
    fin = np.array(start, dtype=np.float64, order="C").reshape(n, d)
    return fin


def _splats_per_point(r):
    b = r.burn_in - r.iter_offset if r.burn_in > r.iter_offset else 0
    return r.n_iters - min(b, r.n_iters)


def _window(img):
    lo = (C.c_float * 2)(*[float(v) for v in img["lo"]])
    hi = (C.c_float * 2)(*[float(v) for v in img["hi"]])
    return _Window(int(img["width"]), int(img["height"]),
                   int(img.get("channels", 1)), lo, hi)


def _check(rc, name):
    if rc != 0:
        raise ValueError(f"oracle {name} rejected its arguments (rc={rc})")


# --------------------------------------------------------------------------
# Public oracle functions (numpy in, numpy out)
# --------------------------------------------------------------------------

def philox4x32_10(ctr, key):
    """One Philox4x32-10 block for a 4-word counter and a 2-word key."""
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib.orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def philox_many(seed, ctrs):
    """Philox blocks for an [n, 4] array of counters under one 64-bit seed."""
    lib = _load()
    c = np.ascontiguousarray(ctrs, dtype=np.uint32).reshape(-1, 4)
    out = np.zeros_like(c)
    lib.orc_philox_many(C.c_uint64(seed), _ptr(c), _ptr(out), c.shape[0])
    return out


def thresholds(prob, n):
    lib = _load()
    out = np.zeros(n, np.uint64)
    p = None if prob is None else np.ascontiguousarray(prob, dtype=np.float64)
    _check(lib.orc_thresholds(_ptr(p), n, _ptr(out)), "thresholds")
    return out


def select(u, thresh):
    lib = _load()
    t = np.ascontiguousarray(thresh, dtype=np.uint64)
    return int(lib.orc_select(C.c_uint32(int(u)), _ptr(t), t.size))


def select_histogram(thresh):
    """Counts of every index over all 2^32 draws (exhaustive, a few seconds)."""
    lib = _load()
    t = np.ascontiguousarray(thresh, dtype=np.uint64)
    out = np.zeros(t.size, np.uint64)
    lib.orc_select_histogram(_ptr(t), t.size, _ptr(out))
    return out


def chaos_count(system, run, image, *, want_final=False, want_last=False,
                want_indices=False, want_splats=False, out=None, start=None):
    """Plain chaos game with a u32 count image [channels][H][W].

    Returns a dict with 'image' (accumulated into ``out`` when given) and the
    optional 'final' [N][dim] (FP64), 'last' [N], 'indices' [N][T],
    'splats' [N][S][2] fractional pixel coordinates (S splatted steps of this
    call), and 'dropped'.  A run with ``iter_offset`` K > 0 continues the
    points for T more steps from ``start`` [N][dim] (their positions after K
    steps); 'final' is then always returned.
    """
    lib = _load()
    keep = _Keep(system)
    r = _run(run)
    w = _window(image)
    N, T, d = r.n_points, r.n_iters, keep.s.dim
    img = out if out is not None else np.zeros(
        (w.channels, w.height, w.width), np.uint32)
    assert img.dtype == np.uint32 and img.flags.c_contiguous
    fin = _start(run, start, N, d)
    if fin is None and want_final:
        fin = np.zeros((N, d), np.float64)
    last = np.zeros(N, np.uint8) if want_last else None
    idx = np.zeros((N, T), np.uint8) if want_indices else None
    spl = np.zeros((N, _splats_per_point(r), 2), np.float64) if want_splats else None
    dropped = np.zeros(1, np.uint64)
    rc = lib.orc_chaos_count(C.byref(keep.s), C.byref(r), C.byref(w), _ptr(img),
                             _ptr(fin), _ptr(last), _ptr(idx), _ptr(spl),
                             _ptr(dropped))
    _check(rc, "chaos_count")
    return {"image": img, "final": fin, "last": last, "indices": idx,
            "splats": spl, "dropped": int(dropped[0])}


class _Object(C.Structure):
    _fields_ = [("final_kind", C.c_int32), ("final_params", C.POINTER(C.c_float)),
                ("place", C.c_float * 6), ("channel", C.c_int32), ("n_copies", C.c_uint32),
                ("copy_lo", C.c_float * 2), ("copy_span", C.c_float * 2),
                ("scale_lo", C.c_float), ("scale_span", C.c_float)]


def _objects(objects):
    """ctypes array of the scene's objects (dicts with final_kind,
    final_params, place, channel, n_copies, copy_lo, copy_hi, scale)."""
    arr = (_Object * len(objects))()
    keep = []
    for o, ob in zip(arr, objects):
        fp = np.zeros(24, np.float32)
        src = np.asarray(ob.get("final_params", ()), np.float32).reshape(-1)
        fp[: src.size] = src
        keep.append(fp)
        o.final_kind = FINAL_KINDS[ob.get("final_kind", "identity")]
        o.final_params = fp.ctypes.data_as(C.POINTER(C.c_float))
        pl = np.asarray(ob.get("place", (1, 0, 0, 1, 0, 0)), np.float32)
        o.place = (C.c_float * 6)(*[float(v) for v in pl])
        o.channel = int(ob.get("channel", 0))
        o.n_copies = int(ob.get("n_copies", 1))
        lo = np.asarray(ob.get("copy_lo", (0, 0)), np.float32)
        hi = np.asarray(ob.get("copy_hi", (0, 0)), np.float32)
        o.copy_lo = (C.c_float * 2)(*[float(v) for v in lo])
        o.copy_span = (C.c_float * 2)(*[float(np.float32(h - l)) for l, h in zip(lo, hi)])
        sc = np.asarray(ob.get("scale", (1, 1)), np.float32)
        o.scale_lo = float(sc[0])
        o.scale_span = float(np.float32(sc[1] - sc[0]))
    return arr, keep


def chaos_scene(system, objects, run, image, *, want_splats=False, out=None):
    """Several objects from one 2D primitive (u32 count image, one channel per
    object's ``channel``).  'splats' is [N][T-B][n_objects][2] in window
    coordinates."""
    lib = _load()
    keep = _Keep(system)
    objs, okeep = _objects(objects)
    r = _run(run)
    w = _window(image)
    N, T, B = r.n_points, r.n_iters, r.burn_in
    img = out if out is not None else np.zeros((w.channels, w.height, w.width), np.uint32)
    assert img.dtype == np.uint32 and img.flags.c_contiguous
    spl = np.zeros((N, T - B, len(objects), 2), np.float64) if want_splats else None
    dropped = np.zeros(1, np.uint64)
    rc = lib.orc_chaos_scene(C.byref(keep.s), objs, len(objects), C.byref(r), C.byref(w),
                             _ptr(img), _ptr(spl), _ptr(dropped))
    _check(rc, "chaos_scene")
    return {"image": img, "splats": spl, "dropped": int(dropped[0])}


def chaos_depth(system, run, image, near, *, want_final=False, want_last=False,
                want_splats=False, depth=None, density=None, start=None):
    """3D chaos game into a u64 depth|index min-buffer and a u32 density
    (continued runs as for chaos_count)."""
    lib = _load()
    keep = _Keep(system)
    r = _run(run)
    w = _window(image)
    N = r.n_points
    if depth is None:
        depth = np.full((w.height, w.width), np.iinfo(np.uint64).max, np.uint64)
    if density is None:
        density = np.zeros((w.height, w.width), np.uint32)
    fin = _start(run, start, N, 3)
    if fin is None and want_final:
        fin = np.zeros((N, 3), np.float64)
    last = np.zeros(N, np.uint8) if want_last else None
    spl = np.zeros((N, _splats_per_point(r), 3), np.float64) if want_splats else None
    dropped = np.zeros(1, np.uint64)
    rc = lib.orc_chaos_depth(C.byref(keep.s), C.byref(r), C.byref(w),
                             C.c_float(near), _ptr(depth), _ptr(density),
                             _ptr(fin), _ptr(last), _ptr(spl), _ptr(dropped))
    _check(rc, "chaos_depth")
    return {"depth": depth, "density": density, "final": fin, "last": last,
            "splats": spl, "dropped": int(dropped[0])}


def splat_gauss(system, run, image, sigma_px, *, want_final=False):
    """FP64 Gaussian soft-splat density [H][W] (sum of weights / (N (T-B)))."""
    lib = _load()
    keep = _Keep(system)
    r = _run(run)
    w = _window(image)
    dens = np.zeros((w.height, w.width), np.float64)
    fin = np.zeros((r.n_points, 2), np.float64) if want_final else None
    rc = lib.orc_splat_gauss(C.byref(keep.s), C.byref(r), C.byref(w),
                             C.c_double(sigma_px), _ptr(dens), _ptr(fin))
    _check(rc, "splat_gauss")
    return dens if not want_final else (dens, fin)


def splat_gauss_backward(system, run, image, sigma_px, dL_dD):
    """Gradient of L w.r.t. the maps, [n_maps][6] = (a00,a01,a10,a11,b0,b1)."""
    lib = _load()
    keep = _Keep(system)
    r = _run(run)
    w = _window(image)
    g = np.ascontiguousarray(dL_dD, dtype=np.float64)
    assert g.shape == (w.height, w.width)
    grad = np.zeros((keep.s.n_maps, 6), np.float64)
    rc = lib.orc_splat_gauss_backward(C.byref(keep.s), C.byref(r), C.byref(w),
                                      C.c_double(sigma_px), _ptr(g), _ptr(grad))
    _check(rc, "splat_gauss_backward")
    return grad


def l2_loss(density, target):
    """The fitting loop's image loss (Section 4): sum (D - D*)^2 in FP64 and
    its gradient 2 (D - D*), both from the float inputs widened exactly."""
    d = np.asarray(density, np.float64).reshape(-1) - np.asarray(target, np.float64).reshape(-1)
    return float(np.dot(d, d)), 2.0 * d


def gauss_loss(system, run, image, sigma_px, target):
    """L = sum (D - D*)^2 with D from splat_gauss."""
    D = splat_gauss(system, run, image, sigma_px)
    return float(np.sum((D - target) ** 2)), D


# --------------------------------------------------------------------------
# Point-range shards of the whole workload (test infrastructure).
#
# Points are independent and every point's random stream is keyed by its
# global id, so the image of a run is the sum (counts, densities) or the
# minimum (depth keys) of the images of any partition of its points into
# ranges (Section 1: each point colours its own pixels).  The helpers below
# run the single-threaded oracle on equal point ranges in threads (ctypes
# releases the interpreter lock during each call) and combine the parts by
# that definition; no arithmetic of the method is done here.
# --------------------------------------------------------------------------

def host_threads(cap=16):
    """Threads for the sharded oracle: the cores this process may run on,
    at most ``cap`` (a GPU machine grants one GPU's share of its cores)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, cap))


def _ranges(run, parts):
    n = int(run["n_points"])
    off = int(run.get("point_offset", 0))
    parts = max(1, min(parts, n)) if n else 1
    b = [n * i // parts for i in range(parts + 1)]
    return [dict(run, n_points=b[i + 1] - b[i], point_offset=off + b[i])
            for i in range(parts) if b[i + 1] > b[i]]


def _pool_map(fn, items, threads):
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max(1, threads)) as ex:
        return list(ex.map(fn, items))


def chaos_count_sharded(system, run, image, threads=None):
    """chaos_count of the whole run as the sum of its point-range parts:
    {'image', 'dropped'} (image uint32, as chaos_count returns it)."""
    threads = threads or host_threads()
    runs = _ranges(run, threads)
    if not runs:
        return chaos_count(system, run, image)
    parts = _pool_map(lambda r: chaos_count(system, r, image), runs, threads)
    total = parts[0]["image"].astype(np.uint64)
    for p in parts[1:]:
        total += p["image"]
    assert int(total.max(initial=0)) < 2**32
    return {"image": total.astype(np.uint32), "dropped": sum(p["dropped"] for p in parts)}


def chaos_depth_sharded(system, run, image, near, threads=None):
    """chaos_depth of the whole run: key image the minimum and density the
    sum of the point-range parts: {'depth', 'density', 'dropped'}."""
    threads = threads or host_threads()
    runs = _ranges(run, threads)
    if not runs:
        return chaos_depth(system, run, image, near)
    parts = _pool_map(lambda r: chaos_depth(system, r, image, near), runs, threads)
    depth = parts[0]["depth"]
    dens = parts[0]["density"].astype(np.uint64)
    for p in parts[1:]:
        np.minimum(depth, p["depth"], out=depth)
        dens += p["density"]
    return {"depth": depth, "density": dens.astype(np.uint32),
            "dropped": sum(p["dropped"] for p in parts)}


def splat_gauss_sharded(system, run, image, sigma_px, threads=None):
    """splat_gauss of the whole run: each part is normalised by its own
    point count, so the whole density is the parts weighted by their share
    of the points."""
    threads = threads or host_threads()
    N = int(run["n_points"])
    runs = _ranges(run, threads)
    parts = _pool_map(lambda r: (r["n_points"], splat_gauss(system, r, image, sigma_px)),
                      runs, threads)
    return sum(d * (n / N) for n, d in parts)


def splat_gauss_backward_sharded(system, run, image, sigma_px, dL_dD, threads=None):
    """splat_gauss_backward of the whole run for a fixed upstream gradient:
    the gradient is a sum over points, each part normalised by its own point
    count, so the parts are weighted by their share of the points."""
    threads = threads or host_threads()
    N = int(run["n_points"])
    runs = _ranges(run, threads)
    parts = _pool_map(lambda r: (r["n_points"],
                                 splat_gauss_backward(system, r, image, sigma_px, dL_dD)),
                      runs, threads)
    return sum(g * (n / N) for n, g in parts)
