"""Python binding of the CFS chaos-game library (argument marshalling only).

Every step of the path runs in the HIP kernels of libcfs.so; this module turns
workload dicts and torch tensors into the C structs of include/cfs.h and
passes device pointers plus the current HIP stream.  PyTorch provides device
memory and streams, nothing else.

Workload dicts (see ``workloads``) carry:
  system: dim, A [n][d][d], b [n][d], prob or None, final_kind, final_params
  run:    seed, instance, n_points, point_offset, n_iters, burn_in
  image:  kind, width, height, channels, lo, hi (and near for depth images)
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import CfsImage, CfsRun, CfsSystem, check


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _scratch(nbytes, device, stream=None, dtype=torch.uint8):
    """A workspace tensor allocated here for one call.  Torch's caching
    allocator ties a block to the stream it was allocated on and may hand it
    out again as soon as this function's reference is dropped; when the
    kernels run on another stream, record that stream on the tensor so the
    block is not reused before the work queued there has finished."""
    elem = torch.empty((), dtype=dtype).element_size()
    t = torch.empty(max((int(nbytes) + elem - 1) // elem, 1), dtype=dtype, device=device)
    if stream is not None:
        t.record_stream(stream)
    return t


class System:
    """C view of a system dict; keeps the host arrays alive."""

    def __init__(self, system):
        d = int(system["dim"])
        self.A = np.ascontiguousarray(system["A"], dtype=np.float32).reshape(-1)
        self.b = np.ascontiguousarray(system["b"], dtype=np.float32).reshape(-1)
        n = self.b.size // d
        prob = system.get("prob")
        self.prob = None if prob is None else np.ascontiguousarray(prob, np.float64)
        fp = (C.c_float * 24)()
        src = np.asarray(system.get("final_params", []), np.float32).reshape(-1)
        for i, v in enumerate(src[:24]):
            fp[i] = float(v)
        kinds = system.get("kind")
        self.kind = None if kinds is None else np.ascontiguousarray(
            [_lib.MAP_KINDS[k] if isinstance(k, str) else int(k) for k in kinds], np.int32)
        self.struct = CfsSystem(
            d, n, self.A.ctypes.data_as(C.POINTER(C.c_float)),
            self.b.ctypes.data_as(C.POINTER(C.c_float)),
            None if self.prob is None else self.prob.ctypes.data_as(C.POINTER(C.c_double)),
            _lib.FINAL_KINDS[system.get("final_kind", "identity")], fp,
            None if self.kind is None else self.kind.ctypes.data_as(C.POINTER(C.c_int32)),
            _lib.COMPOSE[system.get("compose", "copy")])
        self.dim, self.n_maps = d, n


def run_struct(run, precision="f32", splat_path="auto"):
    return CfsRun(int(run.get("seed", 0)), int(run.get("instance", 0)),
                  int(run["n_points"]), int(run.get("point_offset", 0)),
                  int(run["n_iters"]), int(run["burn_in"]),
                  _lib.PRECISIONS[precision], _lib.SPLAT_PATHS[splat_path],
                  int(run.get("iter_offset", 0)))


class Image:
    """Device image of a workload's image description.

    u32_count: int32 storage [channels][H][W] (read back as uint32);
    f32_density: float32 [H][W]; u64_depth: int64 keys [H][W] (read back as
    uint64) plus int32 density [H][W].  ``dropped`` counts dropped splats.
    """

    def __init__(self, desc, device="cuda", data=None):
        self.desc = dict(desc)
        kind = desc["kind"]
        W, H, Ch = int(desc["width"]), int(desc["height"]), int(desc.get("channels", 1))
        self.kind = kind
        self.density = None
        if data is not None:
            self.data = data
        elif kind == "u32_count":
            self.data = torch.empty((Ch, H, W), dtype=torch.int32, device=device)
        elif kind == "f32_density":
            self.data = torch.empty((H, W), dtype=torch.float32, device=device)
        elif kind == "u64_depth":
            self.data = torch.empty((H, W), dtype=torch.int64, device=device)
        else:
            raise ValueError(f"unknown image kind {kind}")
        if kind == "u64_depth":
            self.density = torch.empty((H, W), dtype=torch.int32, device=device)
        self.dropped = torch.zeros(1, dtype=torch.int64, device=device)
        lo = (C.c_float * 2)(*[float(v) for v in desc["lo"]])
        hi = (C.c_float * 2)(*[float(v) for v in desc["hi"]])
        self.struct = CfsImage(_lib.IMAGE_KINDS[kind], W, H, Ch, lo, hi,
                               float(desc.get("near", 0.0)), self.data.data_ptr(),
                               None if self.density is None else self.density.data_ptr(),
                               self.dropped.data_ptr())

    def clear(self, stream=None):
        check(_lib.load().cfs_image_clear(C.byref(self.struct), _stream_handle(stream)),
              "cfs_image_clear")
        return self

    def to_numpy(self):
        """Host copies with the element types of include/cfs.h."""
        torch.cuda.synchronize()
        out = {"dropped": int(self.dropped.cpu().item())}
        a = self.data.cpu().numpy()
        if self.kind == "u32_count":
            out["image"] = a.view(np.uint32)
        elif self.kind == "u64_depth":
            out["depth"] = a.view(np.uint64)
            out["density"] = self.density.cpu().numpy().view(np.uint32)
        else:
            out["image"] = a
        return out


def image_clear(image, stream=None):
    return image.clear(stream)


def chaos_game(system, run, image, *, precision="f32", final=None, last=None,
               indices=None, splat_path="auto", workspace=None, stream=None):
    """Enqueue the plain chaos game (cfs_chaos_game) into ``image``.

    ``splat_path`` is 'auto', 'direct' or 'binned'; ``workspace`` is an
    optional uint8 device tensor reused across calls (allocated here, of the
    size for the fewest launches, when missing; a smaller one is used as it
    is, and the library cuts the run into launches that fit it).

    ``system`` is a workload system dict or a :class:`System`; ``final``
    (float32/float64 [N][dim]), ``last`` (uint8 [N]) and ``indices``
    (uint8 [N][T]) are optional device tensors.  The image accumulates.
    A run with ``iter_offset`` K > 0 (a multiple of 4) continues the points
    from the positions in ``final`` (after K steps) and leaves them there
    after its own steps.
    """
    lib = _lib.load()
    sysc = system if isinstance(system, System) else System(system)
    runc = run_struct(run, precision, splat_path)
    ws_bytes = lib.cfs_chaos_game_workspace(C.byref(sysc.struct), C.byref(runc),
                                            C.byref(image.struct))
    ws, nbytes = None, 0
    if ws_bytes:
        if workspace is not None:
            ws, nbytes = workspace, workspace.numel() * workspace.element_size()
        else:
            ws, nbytes = _scratch(ws_bytes, image.data.device, stream), ws_bytes
    rc = lib.cfs_chaos_game(C.byref(sysc.struct), C.byref(runc), C.byref(image.struct),
                            _ptr(final), _ptr(last), _ptr(indices), _ptr(ws),
                            C.c_size_t(nbytes), _stream_handle(stream))
    check(rc, "cfs_chaos_game")
    return image


def chaos_game_noalloc(system, run, image, *, precision="f32", final=None, last=None,
                       indices=None, splat_path="auto", stream=None):
    """Enqueue cfs_chaos_game_noalloc: the chaos game of :func:`chaos_game`
    with the binned splat's records in the library's fixed per-GPU array
    (no workspace, nothing allocated here or in the library).  Calls that
    overlap on one GPU race on that array."""
    lib = _lib.load()
    sysc = system if isinstance(system, System) else System(system)
    runc = run_struct(run, precision, splat_path)
    check(lib.cfs_chaos_game_noalloc(C.byref(sysc.struct), C.byref(runc), C.byref(image.struct),
                                     _ptr(final), _ptr(last), _ptr(indices),
                                     _stream_handle(stream)), "cfs_chaos_game_noalloc")
    return image


def microbench(kind, buf, ops=0, stream=None):
    """Enqueue one ceiling probe (cfs_microbench) over the uint8 device
    tensor ``buf``; returns the operations (bytes for 'copy' and the runs)
    it issues.  ``kind``: copy, dev_add_u32, dev_min_u64, lds_add_u32,
    lds_add_u64, lds_min_u64, philox, runs_128, runs_512, runs_2048."""
    done = C.c_uint64(0)
    check(_lib.load().cfs_microbench(_lib.MICROBENCH[kind], _ptr(buf),
                                     C.c_size_t(buf.numel() * buf.element_size()),
                                     C.c_uint64(int(ops)), C.byref(done),
                                     _stream_handle(stream)), "cfs_microbench")
    return int(done.value)


def timing_enable(on=True):
    """Record HIP events around the phases of every cfs_chaos_game call."""
    check(_lib.load().cfs_timing_enable(1 if on else 0), "cfs_timing_enable")


def timing_read(max_calls=256):
    """[calls][3] milliseconds (chaos kernel, transpose, accumulate) of the
    calls recorded since the last read."""
    buf = (C.c_float * (3 * max_calls))()
    n = C.c_int32(0)
    check(_lib.load().cfs_timing_read(buf, max_calls, C.byref(n)), "cfs_timing_read")
    return np.frombuffer(buf, np.float32, 3 * n.value).reshape(n.value, 3).copy()


def chaos_workspace_bytes(system, run, image, precision="f32", splat_path="auto"):
    lib = _lib.load()
    sysc = system if isinstance(system, System) else System(system)
    runc = run_struct(run, precision, splat_path)
    return int(lib.cfs_chaos_game_workspace(C.byref(sysc.struct), C.byref(runc),
                                            C.byref(image.struct)))


def objects_struct(objects):
    """ctypes array of cfs_object from object dicts (final_kind,
    final_params, place, channel, n_copies, copy_lo, copy_hi, scale)."""
    arr = (_lib.CfsObject * len(objects))()
    for o, ob in zip(arr, objects):
        o.final_kind = _lib.FINAL_KINDS[ob.get("final_kind", "identity")]
        fp = np.zeros(24, np.float32)
        src = np.asarray(ob.get("final_params", ()), np.float32).reshape(-1)
        fp[: src.size] = src
        o.final_params = (C.c_float * 24)(*[float(v) for v in fp])
        pl = np.asarray(ob.get("place", (1, 0, 0, 1, 0, 0)), np.float32)
        o.place = (C.c_float * 6)(*[float(v) for v in pl])
        o.channel = int(ob.get("channel", 0))
        o.n_copies = int(ob.get("n_copies", 1))
        lo = np.asarray(ob.get("copy_lo", (0, 0)), np.float32)
        hi = np.asarray(ob.get("copy_hi", (0, 0)), np.float32)
        o.copy_lo = (C.c_float * 2)(*[float(v) for v in lo])
        o.copy_span = (C.c_float * 2)(*[float(v) for v in (hi - lo)])
        sc = np.asarray(ob.get("scale", (1, 1)), np.float32)
        o.scale_lo = float(sc[0])
        o.scale_span = float(np.float32(sc[1] - sc[0]))
    return arr


def chaos_scene(system, objects, run, image, *, precision="f32", splat_path="auto",
                workspace=None, stream=None):
    """Several objects from one 2D primitive (cfs_chaos_scene) into the
    u32_count ``image`` (accumulates)."""
    lib = _lib.load()
    sysc = system if isinstance(system, System) else System(system)
    objs = objects_struct(objects)
    runc = run_struct(run, precision, splat_path)
    ws_bytes = lib.cfs_chaos_scene_workspace(C.byref(sysc.struct), objs, len(objects),
                                             C.byref(runc), C.byref(image.struct))
    ws = None
    if ws_bytes:
        if workspace is not None and workspace.numel() >= ws_bytes:
            ws = workspace
        else:
            ws = _scratch(ws_bytes, image.data.device, stream)
    rc = lib.cfs_chaos_scene(C.byref(sysc.struct), objs, len(objects), C.byref(runc),
                             C.byref(image.struct), _ptr(ws), C.c_size_t(ws_bytes),
                             _stream_handle(stream))
    check(rc, "cfs_chaos_scene")
    return image


def scene_workspace_bytes(system, objects, run, image, precision="f32", splat_path="auto"):
    lib = _lib.load()
    sysc = system if isinstance(system, System) else System(system)
    runc = run_struct(run, precision, splat_path)
    return int(lib.cfs_chaos_scene_workspace(C.byref(sysc.struct), objects_struct(objects),
                                             len(objects), C.byref(runc),
                                             C.byref(image.struct)))


def philox_dump(seed, ctrs, stream=None):
    """Philox4x32-10 blocks of an int32/uint32 device tensor [n][4] of counters."""
    lib = _lib.load()
    ctrs = ctrs.contiguous()
    out = torch.empty_like(ctrs)
    check(lib.cfs_philox_dump(C.c_uint64(int(seed)), _ptr(ctrs), _ptr(out),
                              C.c_uint64(ctrs.shape[0]), _stream_handle(stream)),
          "cfs_philox_dump")
    return out


# ---------------------------------------------------------------------------
# Differentiable form
# ---------------------------------------------------------------------------
def n_checkpoints(n_iters, every):
    return (int(n_iters) + int(every) - 1) // int(every)


def splat(system, run, image, sigma_px, *, ckpt=None, ckpt_every=8, workspace=None,
          stream=None):
    """Gaussian soft splat (cfs_splat) into an f32_density ``image``.

    ``ckpt`` is an optional float32 device tensor
    [ceil(T / ckpt_every)][N][2] that receives the checkpoints."""
    lib = _lib.load()
    sysc = system if isinstance(system, System) else System(system)
    runc = run_struct(run, "f32")
    need = int(lib.cfs_splat_workspace(C.byref(sysc.struct), C.byref(runc),
                                       C.byref(image.struct), C.c_float(sigma_px)))
    ws = workspace
    if need and (ws is None or ws.numel() < need):
        ws = _scratch(need, image.data.device, stream)
    rc = lib.cfs_splat(C.byref(sysc.struct), C.byref(runc), C.byref(image.struct),
                       C.c_float(sigma_px), _ptr(ckpt), C.c_int32(int(ckpt_every)),
                       _ptr(ws if need else None), C.c_size_t(need), _stream_handle(stream))
    check(rc, "cfs_splat")
    return image


def splat_backward(system, run, image, sigma_px, dL_dD, ckpt, ckpt_every=8, grad=None,
                   workspace=None, stream=None):
    """Adjoint of the Gaussian splat (cfs_splat_backward): returns the float32
    device gradient [n_maps][6] = (a00, a01, a10, a11, b0, b1)."""
    lib = _lib.load()
    sysc = system if isinstance(system, System) else System(system)
    runc = run_struct(run, "f32")
    need = int(lib.cfs_splat_backward_workspace(C.byref(sysc.struct), C.byref(runc),
                                                C.byref(image.struct), C.c_float(sigma_px)))
    dev = dL_dD.device
    if workspace is not None and workspace.numel() >= need:
        ws = workspace
    else:
        ws = _scratch(need, dev, stream)
    if grad is None:
        grad = torch.empty((sysc.n_maps, 6), dtype=torch.float32, device=dev)
        if stream is not None:
            grad.record_stream(stream)
    g = dL_dD.contiguous()
    if stream is not None and g.data_ptr() != dL_dD.data_ptr():
        g.record_stream(stream)
    rc = lib.cfs_splat_backward(C.byref(sysc.struct), C.byref(runc), C.byref(image.struct),
                                C.c_float(sigma_px), _ptr(g), _ptr(ckpt),
                                C.c_int32(int(ckpt_every)), _ptr(grad), _ptr(ws),
                                C.c_size_t(need), _stream_handle(stream))
    check(rc, "cfs_splat_backward")
    return grad


def l2_loss(density, target, *, grad=None, want_grad=True, workspace=None, stream=None):
    """cfs_l2_loss: returns (loss as a float64 device tensor [1], dL/dD or
    None).  ``density`` and ``target`` are float32 device tensors of equal
    size; ``grad`` (float32, same size) is written when given or when
    ``want_grad``."""
    lib = _lib.load()
    d = density.contiguous()
    t = target.contiguous()
    if d.dtype != torch.float32 or t.dtype != torch.float32 or d.numel() != t.numel():
        raise ValueError("density and target must be float32 tensors of equal size")
    n = d.numel()
    if stream is not None:
        # copies made by .contiguous() above are read on ``stream``
        for src, cp in ((density, d), (target, t)):
            if cp.data_ptr() != src.data_ptr():
                cp.record_stream(stream)
    if grad is None and want_grad:
        grad = torch.empty_like(d)
        if stream is not None:
            grad.record_stream(stream)
    loss = torch.empty(1, dtype=torch.float64, device=d.device)
    if stream is not None:
        loss.record_stream(stream)
    ws_bytes = int(lib.cfs_l2_loss_workspace(C.c_uint64(n)))
    if workspace is None or workspace.numel() * workspace.element_size() < ws_bytes:
        workspace = _scratch(ws_bytes, d.device, stream, dtype=torch.float64)
    check(lib.cfs_l2_loss(_ptr(d), _ptr(t), C.c_uint64(n), _ptr(grad), _ptr(loss),
                          _ptr(workspace), C.c_size_t(ws_bytes), _stream_handle(stream)),
          "cfs_l2_loss")
    return loss, grad


def theta_to_system(theta, like=None, prob=None):
    """System dict of a 2D affine IFS from parameters [n][6] =
    (a00, a01, a10, a11, b0, b1) (a host copy is taken: the map table travels
    in kernel arguments)."""
    th = theta.detach().to("cpu", torch.float32).numpy() if torch.is_tensor(theta) \
        else np.asarray(theta, np.float32)
    return {"dim": 2, "A": th[:, :4].reshape(-1, 2, 2).copy(), "b": th[:, 4:].copy(),
            "prob": prob if like is None else like.get("prob"),
            "final_kind": "identity", "final_params": np.zeros(24, np.float32)}


# ---------------------------------------------------------------------------
# Batched form
# ---------------------------------------------------------------------------
def _plan_struct(plan):
    if plan is None:
        return None
    p = _lib.CfsPlan()
    p.blocks_per_item = int(plan.get("blocks_per_item", 1))
    p.emit_grid = int(plan.get("emit_grid", 0))
    p.acc_grid = int(plan.get("acc_grid", 0))
    p.splat_path = _lib.SPLAT_PATHS[plan.get("splat_path", "binned")]
    p.direct_below = int(plan.get("direct_below", 0))
    return p


def _plan_dict(p):
    names = {v: k for k, v in _lib.SPLAT_PATHS.items()}
    return {"blocks_per_item": p.blocks_per_item, "emit_grid": p.emit_grid,
            "acc_grid": p.acc_grid, "splat_path": names[p.splat_path],
            "direct_below": int(p.direct_below)}


def _batch_items(entries, images, precision):
    n = len(entries)
    items = (_lib.CfsBatchItem * n)()
    keep = []
    for i, (w, img) in enumerate(zip(entries, images)):
        s = System(w["system"])
        keep.append(s)
        items[i].sys = s.struct
        items[i].run = run_struct(w["run"], precision)
        items[i].img = img.struct
    return items, keep


class Batch:
    """A batch of instances (workload dicts with system/run/image) rendered by
    one HIP-graph launch per ``run()`` into ``images`` (api.Image objects that
    must outlive the batch)."""

    def __init__(self, entries, images, plan=None, precision="f32"):
        lib = _lib.load()
        self.images = list(images)
        items, keep = _batch_items(entries, self.images, precision)
        handle = C.c_void_p()
        ps = _plan_struct(plan)
        check(lib.cfs_batch_create(items, len(entries), None if ps is None else C.byref(ps),
                                   C.byref(handle)), "cfs_batch_create")
        self._h = handle
        self._keep = keep

    def run(self, stream=None):
        check(_lib.load().cfs_batch_run(self._h, _stream_handle(stream)), "cfs_batch_run")

    def update(self, index, system, stream=None):
        s = System(system)
        check(_lib.load().cfs_batch_update(self._h, int(index), C.byref(s.struct),
                                           _stream_handle(stream)), "cfs_batch_update")

    def plan(self):
        p = _lib.CfsPlan()
        check(_lib.load().cfs_batch_plan(self._h, C.byref(p)), "cfs_batch_plan")
        return _plan_dict(p)

    def close(self):
        if self._h:
            _lib.load().cfs_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(entries, images, precision="f32", cache=None, stream=None):
    """Time the candidate plans on this batch (cfs_autotune); returns the
    fastest plan as a dict.  Overwrites the images.  ``cache``: path of a
    JSON Lines plan cache (a matching entry is returned without timing)."""
    lib = _lib.load()
    items, keep = _batch_items(entries, images, precision)
    p = _lib.CfsPlan()
    check(lib.cfs_autotune(items, len(entries), C.byref(p),
                           None if cache is None else str(cache).encode(),
                           _stream_handle(stream)), "cfs_autotune")
    return _plan_dict(p)
