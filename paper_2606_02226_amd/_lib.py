"""ctypes declarations of include/cfs.h and the loader of libcfs.so.

The library must have been built in-tree (``paper_2606_02226_amd/libcfs.so``);
there is no fallback of any kind: a missing library is an error.
"""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcfs.so")

CFS_OK = 0
CFS_E_INVALID = -1
CFS_E_UNSUPPORTED = -2
CFS_E_NOMEM = -3
CFS_E_DEVICE = -4
CFS_E_WORKSPACE = -5
CFS_MAX_MAPS = 64

FINAL_KINDS = {"identity": 0, "swirl": 1, "twist_camera": 2, "stretch": 3, "ring": 4}
IMAGE_KINDS = {"u32_count": 0, "f32_density": 1, "u64_depth": 2}
PRECISIONS = {"f32": 0, "f64": 1}
MAP_KINDS = {"affine": 0, "circle": 1}
COMPOSE = {"copy": 0, "reuse": 1}
SPLAT_PATHS = {"auto": 0, "direct": 1, "binned": 2}

# Every symbol include/cfs.h declares.
EXPORTS = (
    "cfs_version", "cfs_last_error", "cfs_image_clear", "cfs_chaos_game_workspace",
    "cfs_chaos_game", "cfs_splat_workspace", "cfs_splat", "cfs_splat_backward_workspace",
    "cfs_splat_backward", "cfs_batch_create", "cfs_batch_run", "cfs_batch_update",
    "cfs_batch_plan", "cfs_batch_destroy", "cfs_autotune", "cfs_philox_dump",
    "cfs_chaos_scene_workspace", "cfs_chaos_scene", "cfs_l2_loss_workspace", "cfs_l2_loss",
    "cfs_timing_enable", "cfs_timing_read", "cfs_microbench", "cfs_chaos_game_noalloc",
)
MICROBENCH = {"copy": 0, "dev_add_u32": 1, "dev_min_u64": 2, "lds_add_u32": 3,
              "lds_min_u64": 4, "philox": 5, "lds_add_u64": 6, "runs_128": 7, "runs_512": 8,
              "runs_2048": 9}


class CfsSystem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_maps", C.c_int32),
                ("A", C.POINTER(C.c_float)), ("b", C.POINTER(C.c_float)),
                ("prob", C.POINTER(C.c_double)), ("final_kind", C.c_int32),
                ("final_params", C.c_float * 24), ("kind", C.POINTER(C.c_int32)),
                ("compose", C.c_int32)]


class CfsRun(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("instance", C.c_uint32),
                ("n_points", C.c_uint32), ("point_offset", C.c_uint32),
                ("n_iters", C.c_uint32), ("burn_in", C.c_uint32),
                ("precision", C.c_int32), ("splat_path", C.c_int32),
                ("iter_offset", C.c_uint32)]


class CfsImage(C.Structure):
    _fields_ = [("kind", C.c_int32), ("width", C.c_int32), ("height", C.c_int32),
                ("channels", C.c_int32), ("lo", C.c_float * 2), ("hi", C.c_float * 2),
                ("near_plane", C.c_float), ("data", C.c_void_p),
                ("density", C.c_void_p), ("dropped", C.c_void_p)]


class CfsObject(C.Structure):
    _fields_ = [("final_kind", C.c_int32), ("final_params", C.c_float * 24),
                ("place", C.c_float * 6), ("channel", C.c_int32), ("n_copies", C.c_uint32),
                ("copy_lo", C.c_float * 2), ("copy_span", C.c_float * 2),
                ("scale_lo", C.c_float), ("scale_span", C.c_float)]


class CfsBatchItem(C.Structure):
    _fields_ = [("sys", CfsSystem), ("run", CfsRun), ("img", CfsImage)]


class CfsPlan(C.Structure):
    _fields_ = [("blocks_per_item", C.c_int32), ("emit_grid", C.c_int32),
                ("acc_grid", C.c_int32), ("splat_path", C.c_int32),
                ("direct_below", C.c_uint64)]


_lib = None


class CfsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cfs error {code}: {msg}")
        self.code = code


def load():
    """Load libcfs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -m paper_2606_02226_amd.build)")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    lib.cfs_version.restype = C.c_int
    lib.cfs_last_error.restype = C.c_char_p
    lib.cfs_image_clear.argtypes = [C.POINTER(CfsImage), P]
    lib.cfs_chaos_game_workspace.argtypes = [C.POINTER(CfsSystem), C.POINTER(CfsRun),
                                             C.POINTER(CfsImage)]
    lib.cfs_chaos_game_workspace.restype = C.c_size_t
    lib.cfs_chaos_game.argtypes = [C.POINTER(CfsSystem), C.POINTER(CfsRun),
                                   C.POINTER(CfsImage), P, P, P, P, C.c_size_t, P]
    lib.cfs_chaos_game_noalloc.argtypes = [C.POINTER(CfsSystem), C.POINTER(CfsRun),
                                           C.POINTER(CfsImage), P, P, P, P]
    lib.cfs_splat_workspace.argtypes = [C.POINTER(CfsSystem), C.POINTER(CfsRun),
                                        C.POINTER(CfsImage), C.c_float]
    lib.cfs_splat_workspace.restype = C.c_size_t
    lib.cfs_splat.argtypes = [C.POINTER(CfsSystem), C.POINTER(CfsRun), C.POINTER(CfsImage),
                              C.c_float, P, C.c_int32, P, C.c_size_t, P]
    lib.cfs_splat_backward_workspace.argtypes = [C.POINTER(CfsSystem), C.POINTER(CfsRun),
                                                 C.POINTER(CfsImage), C.c_float]
    lib.cfs_splat_backward_workspace.restype = C.c_size_t
    lib.cfs_splat_backward.argtypes = [C.POINTER(CfsSystem), C.POINTER(CfsRun),
                                       C.POINTER(CfsImage), C.c_float, P, P, C.c_int32, P,
                                       P, C.c_size_t, P]
    lib.cfs_batch_create.argtypes = [C.POINTER(CfsBatchItem), C.c_int32, C.POINTER(CfsPlan),
                                     C.POINTER(C.c_void_p)]
    lib.cfs_batch_run.argtypes = [P, P]
    lib.cfs_batch_update.argtypes = [P, C.c_int32, C.POINTER(CfsSystem), P]
    lib.cfs_batch_plan.argtypes = [P, C.POINTER(CfsPlan)]
    lib.cfs_batch_destroy.argtypes = [P]
    lib.cfs_batch_destroy.restype = None
    lib.cfs_autotune.argtypes = [C.POINTER(CfsBatchItem), C.c_int32, C.POINTER(CfsPlan),
                                 C.c_char_p, P]
    lib.cfs_philox_dump.argtypes = [C.c_uint64, P, P, C.c_uint64, P]
    lib.cfs_timing_enable.argtypes = [C.c_int32]
    lib.cfs_timing_read.argtypes = [P, C.c_int32, P]
    lib.cfs_microbench.argtypes = [C.c_int32, P, C.c_size_t, C.c_uint64,
                                   C.POINTER(C.c_uint64), P]
    lib.cfs_l2_loss_workspace.argtypes = [C.c_uint64]
    lib.cfs_l2_loss_workspace.restype = C.c_size_t
    lib.cfs_l2_loss.argtypes = [P, P, C.c_uint64, P, P, P, C.c_size_t, P]
    lib.cfs_chaos_scene_workspace.argtypes = [C.POINTER(CfsSystem), C.POINTER(CfsObject),
                                              C.c_int32, C.POINTER(CfsRun), C.POINTER(CfsImage)]
    lib.cfs_chaos_scene_workspace.restype = C.c_size_t
    lib.cfs_chaos_scene.argtypes = [C.POINTER(CfsSystem), C.POINTER(CfsObject), C.c_int32,
                                    C.POINTER(CfsRun), C.POINTER(CfsImage), P, C.c_size_t, P]
    _lib = lib
    return lib


def check(rc, what="cfs call"):
    if rc != CFS_OK:
        msg = load().cfs_last_error().decode(errors="replace")
        raise CfsError(rc, f"{what}: {msg}")
