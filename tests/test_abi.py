"""C-ABI checks that need no GPU: the library loads, exports every function
include/cfs.h declares, and rejects invalid arguments on the host before
anything is enqueued.  Every call below fails host validation by construction
(device pointers are NULL, or a placeholder address together with another
argument that is invalid), so no kernel is ever launched.""" 
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cfs.h")


@pytest.fixture(scope="module")
def L():
    from paper_2606_02226_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2606_02226_amd import build
        build.build()
    _lib.load()
    return _lib


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cfs_[a-z_0-9]+)\s*\(", text)))


def test_header_matches_binding_list(L):
    assert header_functions() == sorted(L.EXPORTS)


def test_library_exports_every_header_symbol(L):
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    defined = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [f for f in header_functions() if f not in defined]
    assert not missing, missing


def test_version(L):
    assert L.load().cfs_version() == 1


def _system(L, dim=2, n=3, A=None, b=None, prob=None, final_kind=0):
    A = np.ascontiguousarray(A if A is not None else np.tile(np.eye(dim) * 0.5, (n, 1, 1)),
                             np.float32)
    b = np.ascontiguousarray(b if b is not None else np.zeros((n, dim)), np.float32)
    keep = [A, b]
    pp = None
    if prob is not None:
        prob = np.ascontiguousarray(prob, np.float64)
        keep.append(prob)
        pp = prob.ctypes.data_as(C.POINTER(C.c_double))
    s = L.CfsSystem(dim, n, A.ctypes.data_as(C.POINTER(C.c_float)),
                    b.ctypes.data_as(C.POINTER(C.c_float)), pp, final_kind,
                    (C.c_float * 24)())
    return s, keep


def _run(L, n_points=10, n_iters=8, burn_in=2, precision=0, offset=0, iter_offset=0):
    return L.CfsRun(0, 0, n_points, offset, n_iters, burn_in, precision, 0, iter_offset)


def _image(L, kind=0, W=16, H=16, ch=1, lo=(0, 0), hi=(1, 1)):
    return L.CfsImage(kind, W, H, ch, (C.c_float * 2)(*lo), (C.c_float * 2)(*hi), 0.0,
                      None, None, None)


def _call(L, s, r, img):
    lib = L.load()
    return lib.cfs_chaos_game(C.byref(s), C.byref(r), C.byref(img), None, None, None, None,
                              0, None)


CASES = [
    ("dim", dict(sys=dict(dim=4)), "dim must be 2 or 3"),
    ("n_maps0", dict(sys=dict(n=0)), "n_maps must be"),
    ("n_maps65", dict(sys=dict(n=65)), "n_maps must be"),
    ("nanA", dict(sys=dict(A=np.full((3, 2, 2), np.nan))), "A[0] is not finite"),
    ("infb", dict(sys=dict(b=np.full((3, 2), np.inf))), "b[0] is not finite"),
    ("final", dict(sys=dict(final_kind=9)), "unknown final kind"),
    ("swirl3d", dict(sys=dict(dim=3, final_kind=1)), "needs dim 2"),
    ("camera2d", dict(sys=dict(final_kind=2)), "needs dim 3"),
    ("iters0", dict(run=dict(n_iters=0)), "n_iters must be"),
    ("iteroff", dict(run=dict(iter_offset=6)), "iter_offset must be a multiple of 4"),
    ("iterbig", dict(run=dict(iter_offset=(1 << 30) + 4)), "iter_offset must be a multiple of 4"),
    ("offset", dict(run=dict(offset=2**32 - 5)), "exceeds 2^32"),
    ("prec", dict(run=dict(precision=7)), "precision"),
    ("width", dict(img=dict(W=0)), "image size"),
    ("height", dict(img=dict(H=70000)), "image size"),
    ("window", dict(img=dict(lo=(1, 0), hi=(1, 1))), "lo < hi"),
    ("data", dict(), "image data is NULL"),
]


@pytest.mark.parametrize("name,kw,msg", CASES, ids=[c[0] for c in CASES])
def test_invalid_arguments(L, name, kw, msg):
    sk = dict(kw.get("sys", {}))
    dim = sk.get("dim", 2)
    n = sk.get("n", 3)
    if dim == 4 or n in (0, 65):
        sk.setdefault("A", np.zeros((max(n, 1), 2, 2)))
        sk.setdefault("b", np.zeros((max(n, 1), 2)))
        s, keep = _system(L, dim=2, n=max(n, 1), A=sk["A"], b=sk["b"])
        s.dim, s.n_maps = dim, n
    else:
        s, keep = _system(L, **sk)
    r = _run(L, **kw.get("run", {}))
    img = _image(L, **kw.get("img", {}))
    rc = _call(L, s, r, img)
    assert rc == L.CFS_E_INVALID
    assert msg in L.load().cfs_last_error().decode()


def test_bad_probabilities(L):
    s, keep = _system(L, prob=[0.5, 0.6, 0.1])
    rc = _call(L, s, _run(L), _image(L))
    assert rc == L.CFS_E_INVALID
    assert "sum to" in L.load().cfs_last_error().decode()
    s, keep = _system(L, prob=[0.5, -0.1, 0.6])
    assert _call(L, s, _run(L), _image(L)) == L.CFS_E_INVALID


def test_null_structs(L):
    lib = L.load()
    assert lib.cfs_chaos_game(None, None, None, None, None, None, None, 0, None) == L.CFS_E_INVALID
    assert "NULL" in lib.cfs_last_error().decode()
    assert lib.cfs_image_clear(None, None) == L.CFS_E_INVALID


def test_philox_dump_rejects_null(L):
    lib = L.load()
    assert lib.cfs_philox_dump(0, None, None, 4, None) == L.CFS_E_INVALID


PLACEHOLDER = 0x1000  # never dereferenced: each call using it fails validation


def _dens_image(L, W=16, H=16):
    return L.CfsImage(1, W, H, 1, (C.c_float * 2)(0, 0), (C.c_float * 2)(1, 1), 0.0,
                      PLACEHOLDER, None, None)


def test_splat_validation(L):
    lib = L.load()
    s, keep = _system(L, n=4)
    r = _run(L, n_points=16, n_iters=8, burn_in=2)
    img = _dens_image(L)
    # sigma outside (0, 2.5]
    assert lib.cfs_splat(C.byref(s), C.byref(r), C.byref(img), 0.0, None, 8, None, 0,
                         None) == L.CFS_E_INVALID
    assert "sigma" in lib.cfs_last_error().decode()
    assert lib.cfs_splat(C.byref(s), C.byref(r), C.byref(img), 3.0, None, 8, None, 0,
                         None) == L.CFS_E_INVALID
    # FP64 positions are not offered by the differentiable form
    r64 = _run(L, n_points=16, n_iters=8, burn_in=2, precision=1)
    assert lib.cfs_splat(C.byref(s), C.byref(r64), C.byref(img), 1.0, None, 8, None, 0,
                         None) == L.CFS_E_UNSUPPORTED
    # a count image is not a density
    cimg = _image(L)
    cimg.data = PLACEHOLDER
    assert lib.cfs_splat(C.byref(s), C.byref(r), C.byref(cimg), 1.0, None, 8, None, 0,
                         None) == L.CFS_E_INVALID


def test_splat_backward_validation(L):
    lib = L.load()
    s9, keep = _system(L, n=9)
    r = _run(L, n_points=16, n_iters=8, burn_in=2)
    img = _dens_image(L)
    img.data = None
    # image data NULL fails validation first
    assert lib.cfs_splat_backward(C.byref(s9), C.byref(r), C.byref(img), 1.0, None, None, 8,
                                  None, None, 0, None) == L.CFS_E_INVALID
    # missing upstream gradient / checkpoints (data pointer only checked for NULL)
    img.data = PLACEHOLDER
    s4, keep4 = _system(L, n=4)
    assert lib.cfs_splat_backward(C.byref(s4), C.byref(r), C.byref(img), 1.0, None, None, 8,
                                  None, None, 0, None) == L.CFS_E_INVALID
    assert "required" in lib.cfs_last_error().decode()
    # more than 8 maps
    assert lib.cfs_splat_backward(C.byref(s9), C.byref(r), C.byref(img), 1.0, None, None, 8,
                                  None, None, 0, None) == L.CFS_E_UNSUPPORTED


def test_batch_validation(L):
    lib = L.load()
    out = C.c_void_p()
    assert lib.cfs_batch_create(None, 0, None, C.byref(out)) == L.CFS_E_INVALID
    items = (L.CfsBatchItem * 1)()
    s, keep = _system(L, n=3)
    items[0].sys = s
    items[0].run = _run(L)
    items[0].img = _image(L)  # data NULL
    assert lib.cfs_batch_create(items, 1, None, C.byref(out)) == L.CFS_E_INVALID
    assert "batch item 0" in lib.cfs_last_error().decode()
    s3, keep3 = _system(L, dim=3, n=3)
    items[0].sys = s3
    assert lib.cfs_batch_create(items, 1, None, C.byref(out)) != L.CFS_OK
    assert lib.cfs_batch_run(None, None) == L.CFS_E_INVALID
    assert lib.cfs_batch_plan(None, None) == L.CFS_E_INVALID
    assert lib.cfs_batch_update(None, 0, None, None) == L.CFS_E_INVALID
    lib.cfs_batch_destroy(None)


def test_workspace_queries_on_invalid_input(L):
    lib = L.load()
    assert lib.cfs_chaos_game_workspace(None, None, None) == 0
    assert lib.cfs_splat_workspace(None, None, None, 1.0) == 0
    assert lib.cfs_splat_backward_workspace(None, None, None, 1.0) == 0


def test_bad_map_kind(L):
    lib = L.load()
    s, keep = _system(L, n=3)
    kinds = (C.c_int32 * 3)(0, 7, 0)
    s.kind = kinds
    assert _call(L, s, _run(L), _image(L)) == L.CFS_E_INVALID
    assert "not a map kind" in lib.cfs_last_error().decode()
    s3, keep3 = _system(L, dim=3, n=3)
    k3 = (C.c_int32 * 3)(1, 0, 0)
    s3.kind = k3
    assert _call(L, s3, _run(L), _image(L)) == L.CFS_E_INVALID
    assert "dim 2" in lib.cfs_last_error().decode()


def test_bad_compose(L):
    lib = L.load()
    s, keep = _system(L, n=3)
    s.compose = 2
    assert _call(L, s, _run(L), _image(L)) == L.CFS_E_INVALID
    assert "composition mode" in lib.cfs_last_error().decode()
    s3, keep3 = _system(L, dim=3, n=3)
    s3.compose = 1
    assert _call(L, s3, _run(L), _image(L)) == L.CFS_E_INVALID
    assert "dim 2" in lib.cfs_last_error().decode()


def _objects(L, n=1, **kw):
    arr = (L.CfsObject * max(n, 1))()
    for o in arr:
        o.place = (C.c_float * 6)(1, 0, 0, 1, 0, 0)
        o.n_copies = 1
        for k, v in kw.items():
            setattr(o, k, v)
    return arr


def _scene_call(L, s, objs, n, r=None, img=None):
    lib = L.load()
    r = r or _run(L)
    img = img or _image(L)
    img.data = PLACEHOLDER
    return lib.cfs_chaos_scene(C.byref(s), objs, n, C.byref(r), C.byref(img), None, 0, None)


@pytest.mark.parametrize("case,msg", [
    ("n0", "n_objects"), ("n9", "n_objects"), ("channel", "channel"), ("kind", "2D transform"),
    ("copies", "n_copies"), ("place", "place"), ("primitive", "no transform"),
    ("dim3", "2D"), ("null", "objects is NULL"), ("depth_image", "density buffer"),
])
def test_scene_validation(L, case, msg):
    lib = L.load()
    s, keep = _system(L, n=3)
    objs, n = _objects(L, 1), 1
    img = None
    if case == "n0":
        n = 0
    elif case == "n9":
        objs, n = _objects(L, 9), 9
    elif case == "channel":
        objs = _objects(L, 1, channel=1)
    elif case == "kind":
        objs = _objects(L, 1, final_kind=2)
    elif case == "copies":
        objs = _objects(L, 1, n_copies=0)
    elif case == "place":
        objs = _objects(L, 1)
        objs[0].place[4] = float("nan")
    elif case == "primitive":
        s.final_kind = 1
    elif case == "dim3":
        s, keep = _system(L, dim=3, n=3)
    elif case == "null":
        objs = None
    elif case == "depth_image":
        img = _image(L, kind=2)
    assert _scene_call(L, s, objs, n, img=img) == L.CFS_E_INVALID
    assert msg in lib.cfs_last_error().decode()


def test_scene_workspace_zero_on_invalid(L):
    lib = L.load()
    s, keep = _system(L, n=3)
    objs = _objects(L, 1, channel=5)
    assert lib.cfs_chaos_scene_workspace(C.byref(s), objs, 1, C.byref(_run(L)),
                                         C.byref(_image(L))) == 0


def test_l2_loss_validation(L):
    lib = L.load()
    assert lib.cfs_l2_loss_workspace(0) == 8
    assert lib.cfs_l2_loss_workspace(10**9) == 1024 * 8
    assert lib.cfs_l2_loss(None, None, 0, None, None, None, 0, None) == L.CFS_E_INVALID
    assert "loss is NULL" in lib.cfs_last_error().decode()
    assert lib.cfs_l2_loss(None, None, 5, None, PLACEHOLDER, None, 0, None) == L.CFS_E_INVALID
    assert lib.cfs_l2_loss(PLACEHOLDER, PLACEHOLDER, 5, None, PLACEHOLDER, None, 0,
                           None) == L.CFS_E_WORKSPACE


def test_batch_rejects_circle_maps(L):
    lib = L.load()
    out = C.c_void_p()
    items = (L.CfsBatchItem * 1)()
    s, keep = _system(L, n=3)
    kinds = (C.c_int32 * 3)(0, 1, 0)
    s.kind = kinds
    items[0].sys = s
    items[0].run = _run(L)
    img = _image(L)
    img.data = PLACEHOLDER
    items[0].img = img
    assert lib.cfs_batch_create(items, 1, None, C.byref(out)) == L.CFS_E_UNSUPPORTED
    assert "affine maps only" in lib.cfs_last_error().decode()


def test_timing_hook_without_calls(L):
    lib = L.load()
    n = C.c_int32(-1)
    buf = (C.c_float * 6)()
    assert lib.cfs_timing_enable(1) == L.CFS_OK
    assert lib.cfs_timing_read(buf, 2, C.byref(n)) == L.CFS_OK and n.value == 0
    assert lib.cfs_timing_enable(0) == L.CFS_OK
    assert lib.cfs_timing_read(None, 0, None) == L.CFS_E_INVALID


def test_binned_image_size_limit(L):
    # count images up to 2^25 elements take the binned splat; one more row
    # is refused for BINNED (and AUTO falls back to the direct splat)
    lib = L.load()
    s, keep = _system(L)
    r = L.CfsRun(0, 0, 1 << 20, 0, 8, 2, 0, 2)
    ok = _image(L, W=8192, H=4096)
    ok.data = C.c_void_p(256)  # never dereferenced: nothing is launched
    assert lib.cfs_chaos_game_workspace(C.byref(s), C.byref(r), C.byref(ok)) > 0
    big = _image(L, W=8192, H=4097)
    big.data = C.c_void_p(256)  # never dereferenced: the call fails first
    assert lib.cfs_chaos_game_workspace(C.byref(s), C.byref(r), C.byref(big)) == 0
    rc = lib.cfs_chaos_game(C.byref(s), C.byref(r), C.byref(big), None, None, None, None, 0,
                            None)
    assert rc == L.CFS_E_UNSUPPORTED
    assert "at most 33554432 elements" in lib.cfs_last_error().decode()


def test_workspace_below_one_workgroup_refused(L):
    # a workspace smaller than the fewest launches need is cut into more
    # launches; one below a single workgroup's records is refused for BINNED
    # before anything is enqueued (the pointers are never dereferenced)
    lib = L.load()
    s, keep = _system(L)
    r = L.CfsRun(0, 0, 1 << 20, 0, 8, 2, 0, 2)
    img = _image(L, W=256, H=256)
    img.data = C.c_void_p(256)
    need = lib.cfs_chaos_game_workspace(C.byref(s), C.byref(r), C.byref(img))
    assert need > 4096
    rc = lib.cfs_chaos_game(C.byref(s), C.byref(r), C.byref(img), None, None, None,
                            C.c_void_p(4096), 4096, None)
    assert rc == L.CFS_E_WORKSPACE
    assert "one workgroup" in lib.cfs_last_error().decode()
    rc = lib.cfs_chaos_game(C.byref(s), C.byref(r), C.byref(img), None, None, None, None, 0,
                            None)
    assert rc == L.CFS_E_WORKSPACE


def test_continued_run_rules(L):
    # a continued run needs final_points (its start) and is for cfs_chaos_game
    # only; burn_in beyond n_iters is refused where runs cannot be continued
    lib = L.load()
    s, keep = _system(L)
    img = _image(L)
    img.data = C.c_void_p(256)  # never dereferenced: the calls fail first
    r = _run(L, iter_offset=8)
    rc = lib.cfs_chaos_game(C.byref(s), C.byref(r), C.byref(img), None, None, None, None, 0,
                            None)
    assert rc == L.CFS_E_INVALID
    assert "reads its start from final_points" in lib.cfs_last_error().decode()
    dens = _image(L, kind=1)
    dens.data = C.c_void_p(256)
    rc = lib.cfs_splat(C.byref(s), C.byref(r), C.byref(dens), C.c_float(1.0), None, 0, None,
                       0, None)
    assert rc == L.CFS_E_UNSUPPORTED
    assert "cfs_chaos_game only" in lib.cfs_last_error().decode()
    r = _run(L, burn_in=9)
    rc = lib.cfs_splat(C.byref(s), C.byref(r), C.byref(dens), C.c_float(1.0), None, 0, None,
                       0, None)
    assert rc == L.CFS_E_INVALID
    assert "exceeds n_iters" in lib.cfs_last_error().decode()


def test_negative_near_plane_refused(L):
    # depth keys order splats by the FP32 bits of their depth, which is the
    # order of the depths only for non-negative values
    lib = L.load()
    s, keep = _system(L, dim=3, n=3, final_kind=2)
    r = _run(L)
    img = L.CfsImage(2, 16, 16, 1, (C.c_float * 2)(-1, -1), (C.c_float * 2)(1, 1), -0.5,
                     C.c_void_p(256), C.c_void_p(512), None)  # never dereferenced
    assert _call(L, s, r, img) == L.CFS_E_INVALID
    assert "near_plane" in lib.cfs_last_error().decode()
    img.near_plane = float("nan")
    assert _call(L, s, r, img) == L.CFS_E_INVALID


def test_binned_record_budget(L):
    # one workgroup's records must fit one launch's budget (2^29 16-bit
    # records): 43690 chunks of 12288, i.e. 1048560 splatted steps per point.
    # One step more is refused for BINNED and takes the direct splat for AUTO.
    lib = L.load()
    s, keep = _system(L)
    img = _image(L, W=64, H=64)
    img.data = C.c_void_p(256)  # never dereferenced: nothing is launched
    fits = L.CfsRun(0, 0, 1 << 12, 0, 1 << 20, 16, 0, 2)
    assert lib.cfs_chaos_game_workspace(C.byref(s), C.byref(fits), C.byref(img)) > 0
    over = L.CfsRun(0, 0, 1 << 12, 0, 1 << 20, 15, 0, 2)
    assert lib.cfs_chaos_game_workspace(C.byref(s), C.byref(over), C.byref(img)) == 0
    rc = lib.cfs_chaos_game(C.byref(s), C.byref(over), C.byref(img), None, None, None, None, 0,
                            None)
    assert rc == L.CFS_E_UNSUPPORTED
    assert "record budget" in lib.cfs_last_error().decode()
    auto = L.CfsRun(0, 0, 1 << 12, 0, 1 << 20, 15, 0, 0)
    assert lib.cfs_chaos_game_workspace(C.byref(s), C.byref(auto), C.byref(img)) == 0
    # a scene multiplies the records by its objects: 8 objects x 2^17 steps
    objs = _objects(L, 8)
    scene = L.CfsRun(0, 0, 1 << 12, 0, (1 << 17) + 8, 0, 0, 2)
    assert lib.cfs_chaos_scene_workspace(C.byref(s), objs, 8, C.byref(scene),
                                         C.byref(img)) == 0
    rc = lib.cfs_chaos_scene(C.byref(s), objs, 8, C.byref(scene), C.byref(img), None, 0, None)
    assert rc == L.CFS_E_UNSUPPORTED
    assert "record budget" in lib.cfs_last_error().decode()
    # depth images: 2^30 records of 8 bytes, 65536 chunks of 16384 per
    # workgroup, i.e. 1048576 splatted steps per point: the longest run
    # (n_iters = 2^20, no burn-in) fits one workgroup, with one workgroup per
    # launch (8 GiB of records)
    s3, keep3 = _system(L, dim=3, n=3, final_kind=2)
    dimg = L.CfsImage(2, 64, 64, 1, (C.c_float * 2)(-1, -1), (C.c_float * 2)(1, 1), 0.1,
                      C.c_void_p(256), C.c_void_p(512), None)  # never dereferenced
    dmax = L.CfsRun(0, 0, 1 << 12, 0, 1 << 20, 0, 0, 2)
    ws = lib.cfs_chaos_game_workspace(C.byref(s3), C.byref(dmax), C.byref(dimg))
    assert ws >= (1 << 30) * 8
    rc = lib.cfs_chaos_game(C.byref(s3), C.byref(dmax), C.byref(dimg), None, None, None, None,
                            0, None)
    assert rc == L.CFS_E_WORKSPACE  # nothing was passed; nothing is launched


def test_microbench_validation(L):
    lib = L.load()
    done = C.c_uint64(7)
    assert lib.cfs_microbench(0, None, 64, 0, C.byref(done), None) == L.CFS_E_INVALID
    assert lib.cfs_microbench(0, C.c_void_p(256), 64, 0, None, None) == L.CFS_E_INVALID
    # placeholder addresses are never dereferenced: each call fails first
    assert lib.cfs_microbench(0, C.c_void_p(255), 64, 0, C.byref(done), None) == L.CFS_E_INVALID
    assert "aligned" in lib.cfs_last_error().decode()
    assert lib.cfs_microbench(10, C.c_void_p(256), 64, 0, C.byref(done), None) == L.CFS_E_INVALID
    assert "unknown microbenchmark" in lib.cfs_last_error().decode()
    assert lib.cfs_microbench(0, C.c_void_p(256), 16, 0, C.byref(done), None) == L.CFS_E_INVALID
    assert lib.cfs_microbench(1, C.c_void_p(256), 2, 1, C.byref(done), None) == L.CFS_E_INVALID
    assert lib.cfs_microbench(3, C.c_void_p(256), 1024, 1, C.byref(done), None) == L.CFS_E_INVALID
    assert lib.cfs_microbench(5, C.c_void_p(256), 1024, 1, C.byref(done), None) == L.CFS_E_INVALID
    # run reads: 4 MiB of lane words plus at least two runs
    for kind in (7, 8, 9):
        assert lib.cfs_microbench(kind, C.c_void_p(256), 4 << 20, 1, C.byref(done),
                                  None) == L.CFS_E_INVALID
        assert "two runs" in lib.cfs_last_error().decode()
    assert done.value == 7
