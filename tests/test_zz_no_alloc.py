"""cfs_chaos_game_noalloc: the chaos game with the library's fixed per-GPU
scratch array in place of a caller workspace gives exactly what
cfs_chaos_game gives (integer images bit for bit, final positions and last
indices equal), over two calls in a row -- the second smaller -- so the
second call runs on the scratch that the first left behind.  The host-side
refusal of runs that cannot fit the array needs no GPU."""
import ctypes as C
import os

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")


def _lib():
    from paper_2606_02226_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_2606_02226_amd import build
        build.build()
    L.load()
    return L


def test_refuses_runs_beyond_the_scratch():
    """A depth run with 70000 splatted steps per point: one workgroup's 8-byte
    records alone (4375 chunks of 16384) take 573 MB, more than the 256 MiB
    array, while they fit cfs_chaos_game's launch budget (2^30 records).  BINNED is
    refused before anything is enqueued; nothing is dereferenced."""
    L = _lib()
    lib = L.load()
    A = np.ascontiguousarray(np.tile(np.eye(3) / 3.0, (2, 1, 1)), np.float32)
    b = np.zeros((2, 3), np.float32)
    fp = (C.c_float * 24)()
    s = L.CfsSystem(3, 2, A.ctypes.data_as(C.POINTER(C.c_float)),
                    b.ctypes.data_as(C.POINTER(C.c_float)), None, L.FINAL_KINDS["twist_camera"],
                    fp)
    img = L.CfsImage(L.IMAGE_KINDS["u64_depth"], 64, 64, 1, (C.c_float * 2)(-1, -1),
                     (C.c_float * 2)(1, 1), 0.1, C.c_void_p(256), C.c_void_p(512), None)
    steps = 70000
    binned = L.CfsRun(0, 0, 1 << 10, 0, steps + 4, 4, 1, L.SPLAT_PATHS["binned"], 0)
    # cfs_chaos_game takes it (the launch budget holds 2^30 records)
    assert lib.cfs_chaos_game_workspace(C.byref(s), C.byref(binned), C.byref(img)) > 0
    rc = lib.cfs_chaos_game_noalloc(C.byref(s), C.byref(binned), C.byref(img), None, None, None,
                                    None)
    assert rc == L.CFS_E_UNSUPPORTED
    msg = lib.cfs_last_error().decode()
    assert "workspace limit" in msg and str(256 << 20) in msg
    # invalid arguments are refused as by cfs_chaos_game
    bad = L.CfsRun(0, 0, 1 << 10, 0, 8, 4, 7, 0, 0)   # precision 7
    assert lib.cfs_chaos_game_noalloc(C.byref(s), C.byref(bad), C.byref(img), None, None, None,
                                      None) == L.CFS_E_INVALID
    assert "precision" in lib.cfs_last_error().decode()


def _api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_02226_amd import api
    return api


def _dev():
    return torch.device("cuda:0")


def _both(api, w, precision, splat_path="auto"):
    """(cfs_chaos_game result, cfs_chaos_game_noalloc result) of one workload."""
    N, d = w["run"]["n_points"], int(w["system"]["dim"])
    dt = torch.float64 if precision == "f64" else torch.float32
    out = []
    for fn in (api.chaos_game, api.chaos_game_noalloc):
        img = api.Image(w["image"], device=_dev()).clear()
        fin = torch.empty((N, d), dtype=dt, device=_dev())
        last = torch.empty((N,), dtype=torch.uint8, device=_dev())
        print(f"  {fn.__name__}: {w['name']} N={N} {precision} {splat_path}", flush=True)
        fn(w["system"], w["run"], img, precision=precision, final=fin, last=last,
           splat_path=splat_path)
        torch.cuda.synchronize()
        out.append((img.to_numpy(), fin.cpu().numpy(), last.cpu().numpy()))
    return out


def _assert_same(a, b):
    (ia, fa, la), (ib, fb, lb) = a, b
    assert ia.keys() == ib.keys()
    for k in ia:
        if k == "dropped":
            assert ia[k] == ib[k]
        else:
            assert np.array_equal(ia[k], ib[k]), k
    assert np.array_equal(fa, fb)
    assert np.array_equal(la, lb)


@pytest.mark.gpu
def test_count_image_two_calls():
    """The CFS square at full size (2^24 points, 4 x 2048^2; several launches
    of the 256 MiB array), then a smaller run (2^18 points, 4 x 512^2)."""
    api = _api()
    for w in (W.cfs_square(), W.cfs_square(n_points=(1 << 18) + 77, side=512)):
        ref, got = _both(api, w, "f64", "binned")
        _assert_same(ref, got)
        total = int(got[0]["image"].astype(np.int64).sum()) + got[0]["dropped"]
        assert total == w["run"]["n_points"] * (w["run"]["n_iters"] - w["run"]["burn_in"])


@pytest.mark.gpu
def test_depth_image_two_calls():
    """The Menger sponge at 2^22 points into 4096^2 (8-byte records: several
    launches), then 2^16 + 5 points into 1024^2."""
    api = _api()
    for w in (W.menger(n_points=1 << 22), W.menger(n_points=(1 << 16) + 5, side=1024)):
        ref, got = _both(api, w, "f64")
        _assert_same(ref, got)


@pytest.mark.gpu
def test_direct_and_small_runs():
    """Runs that take the direct splat (no scratch) and a run of fewer points
    than one workgroup, in FP32."""
    api = _api()
    for w in (W.sierpinski(n_points=4096), W.cfs_square(n_points=300, side=256)):
        ref, got = _both(api, w, "f32")
        _assert_same(ref, got)
    ref, got = _both(api, W.cfs_square(n_points=300, side=256), "f32", "binned")
    _assert_same(ref, got)
