"""GPU parity of the plain chaos game (cfs_chaos_game, cfs_philox_dump,
cfs_image_clear) against the FP64 oracle, through the C ABI.

Bars: Philox blocks and index sequences bit-exact; final positions within
1e-5 absolute; integer histograms within 1e-4 relative L1 of the total and
inside the guard-band interval [sure, sure + maybe] built from the oracle's
FP64 splat coordinates; totals exact.
"""
import math

import numpy as np
import pytest

import workloads as W
from parity import depth_key_diff, guard_band_images, guard_band_violations, rel_l1

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_02226_amd import api as _api
    return _api


def _dev():
    return torch.device("cuda:0")


def run_gpu(api, w, precision="f32", want_indices=False, want_final=True, system=None,
            run=None, image=None):
    system = system or w["system"]
    run = run or w["run"]
    image_desc = image or w["image"]
    N, T, d = run["n_points"], run["n_iters"], system["dim"]
    img = api.Image(image_desc, device=_dev()).clear()
    ftype = torch.float32 if precision == "f32" else torch.float64
    fin = torch.empty((N, d), dtype=ftype, device=_dev()) if want_final else None
    last = torch.empty((N,), dtype=torch.uint8, device=_dev())
    idx = torch.empty((N, T), dtype=torch.uint8, device=_dev()) if want_indices else None
    api.chaos_game(system, run, img, precision=precision, final=fin, last=last, indices=idx)
    out = img.to_numpy()
    out["final"] = None if fin is None else fin.cpu().numpy().astype(np.float64)
    out["last"] = last.cpu().numpy()
    out["indices"] = None if idx is None else idx.cpu().numpy()
    return out


def test_philox_dump_bitexact(api, orc):
    rng = np.random.default_rng(1)
    ctrs = rng.integers(0, 2**32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    ctrs[0] = 0
    ctrs[1] = 0xFFFFFFFF
    for seed in (0, 0xFFFFFFFFFFFFFFFF, 0x0123456789ABCDEF):
        dev = torch.from_numpy(ctrs.view(np.int32)).to(_dev())
        got = api.philox_dump(seed, dev).cpu().numpy().view(np.uint32)
        ref = orc.philox_many(seed, ctrs)
        assert np.array_equal(got, ref)


def test_sierpinski_full_parity(api, orc):
    """Sierpinski: 2^16 points x 64 iterations (16 burn-in), FP32 points,
    512x512 u32 over [0,1]^2 -- the full configuration."""
    w = W.sierpinski()
    N, T, B = 1 << 16, 64, 16
    got = run_gpu(api, w, "f32", want_indices=True)
    ref = orc.chaos_count(w["system"], w["run"], w["image"], want_final=True,
                          want_last=True, want_indices=True, want_splats=True)
    assert np.array_equal(got["indices"], ref["indices"])
    assert np.array_equal(got["last"], ref["last"])
    err = np.max(np.abs(got["final"] - ref["final"]))
    assert err <= 1e-5, err
    h, r = got["image"], ref["image"]
    assert int(h.astype(np.int64).sum()) == N * (T - B) == int(r.astype(np.int64).sum())
    assert got["dropped"] == 0
    l1 = rel_l1(h, r)
    print(f"sierpinski f32: max|dp|={err:.3e} relL1={l1:.3e}")
    assert l1 <= 1e-4, l1
    sure, maybe = guard_band_images(ref["splats"], 0, 512, 512, 1, eps_px=512 * 2e-6)
    assert guard_band_violations(h, sure, maybe) == (0, 0)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_cfs_square_parity(api, orc, precision):
    """CFS square + swirl + translation, 4 channels by last index, full
    2048x2048 image, 2^16 points (the oracle's share of the full run)."""
    w = W.cfs_square(n_points=1 << 16)
    N, T, B = 1 << 16, 32, 8
    got = run_gpu(api, w, precision, want_indices=True)
    ref = orc.chaos_count(w["system"], w["run"], w["image"], want_final=True,
                          want_last=True, want_indices=True, want_splats=True)
    assert np.array_equal(got["indices"], ref["indices"])
    assert np.array_equal(got["last"], ref["last"])
    err = np.max(np.abs(got["final"] - ref["final"]))
    assert err <= 1e-5, err
    h, r = got["image"], ref["image"]
    assert got["dropped"] == 0 and int(h.astype(np.int64).sum()) == N * (T - B)
    # per-channel totals depend only on the (bit-exact) indices
    assert np.array_equal(h.astype(np.int64).sum(axis=(1, 2)), r.astype(np.int64).sum(axis=(1, 2)))
    l1 = rel_l1(h, r)
    eps = 1024 * (1e-12 if precision == "f64" else 2e-6)
    chan = ref["indices"][:, B:]
    sure, maybe = guard_band_images(ref["splats"], chan, 2048, 2048, 4, eps_px=eps)
    viol = guard_band_violations(h, sure, maybe)
    print(f"cfs_square {precision}: max|dp|={err:.3e} relL1={l1:.3e} guard={viol}")
    assert viol == (0, 0)
    if precision == "f64":
        assert l1 <= 1e-4, l1


def test_point_range_split_bitexact(api):
    w = W.cfs_square(n_points=5000, side=512)
    img = api.Image(w["image"], device=_dev()).clear()
    api.chaos_game(w["system"], w["run"], img, precision="f64")
    whole = img.to_numpy()["image"].copy()
    img.clear()
    api.chaos_game(w["system"], dict(w["run"], n_points=1234), img, precision="f64")
    api.chaos_game(w["system"], dict(w["run"], n_points=5000 - 1234, point_offset=1234), img,
                   precision="f64")
    assert np.array_equal(img.to_numpy()["image"], whole)


def test_run_to_run_bitexact(api):
    w = W.cfs_square(n_points=1 << 18)
    a = run_gpu(api, w, "f32", want_final=False)["image"]
    b = run_gpu(api, w, "f32", want_final=False)["image"]
    assert np.array_equal(a, b)


@pytest.mark.parametrize("n_points,n_iters,burn_in", [
    (1, 1, 0), (1, 7, 7), (255, 5, 2), (257, 13, 3), (1000, 64, 63), (4099, 9, 0)])
def test_ragged_shapes(api, orc, n_points, n_iters, burn_in):
    w = W.sierpinski(n_points=n_points, n_iters=n_iters, burn_in=burn_in, side=64)
    got = run_gpu(api, w, "f64", want_indices=True)
    ref = orc.chaos_count(w["system"], w["run"], w["image"], want_final=True,
                          want_last=True, want_indices=True)
    assert np.array_equal(got["indices"], ref["indices"])
    assert np.array_equal(got["last"], ref["last"])
    assert np.max(np.abs(got["final"] - ref["final"])) <= 1e-12
    assert np.array_equal(got["image"], ref["image"])


def test_zero_points_is_noop(api):
    w = W.sierpinski(n_points=0, side=32)
    img = api.Image(w["image"], device=_dev()).clear()
    api.chaos_game(w["system"], w["run"], img)
    assert int(img.to_numpy()["image"].astype(np.int64).sum()) == 0


def test_unequal_probabilities_and_dead_maps(api, orc):
    # 16 maps: zero-probability maps are never drawn; a prefix that already
    # sums to one leaves every later map unreachable
    rng = np.random.default_rng(9)
    n = 16
    A = np.stack([np.eye(2) * 0.4] * n).astype(np.float32)
    b = rng.uniform(0, 0.6, size=(n, 2)).astype(np.float32)
    p_dead = rng.dirichlet(np.ones(n))
    p_dead[[3, 15]] = 0.0
    p_dead /= p_dead.sum()
    p_prefix = np.zeros(n)
    p_prefix[:2] = 0.5
    for prob in (p_dead, p_prefix, rng.dirichlet(np.ones(n))):
        system = W._system(A, b, prob=prob)
        run = {"seed": 7, "instance": 3, "n_points": 3000, "point_offset": 11,
               "n_iters": 20, "burn_in": 4}
        img = {"kind": "u32_count", "width": 128, "height": 128, "channels": 1,
               "lo": [0, 0], "hi": [1, 1]}
        got = run_gpu(api, None, "f64", want_indices=True, system=system, run=run, image=img)
        ref = orc.chaos_count(system, run, img, want_last=True, want_indices=True)
        assert np.array_equal(got["indices"], ref["indices"])
        counts = np.bincount(ref["indices"].reshape(-1), minlength=n)
        assert np.all(counts[prob == 0] == 0)
        assert np.array_equal(got["image"], ref["image"])


def test_3d_identity_counts(api, orc):
    w = W.menger(n_points=4096, side=64)
    system = dict(w["system"], final_kind="identity")
    img = {"kind": "u32_count", "width": 81, "height": 81, "channels": 1,
           "lo": [0, 0], "hi": [1, 1]}
    got = run_gpu(api, w, "f64", want_indices=True, system=system, image=img)
    ref = orc.chaos_count(system, w["run"], img, want_final=True, want_indices=True)
    assert np.array_equal(got["indices"], ref["indices"])
    assert np.max(np.abs(got["final"] - ref["final"])) <= 1e-12
    assert rel_l1(got["image"], ref["image"]) <= 1e-4


def test_stretch_transform(api, orc):
    w = W.cfs_square(n_points=4096, side=256)
    system = dict(w["system"], final_kind="stretch",
                  final_params=np.array([2.0, 1.0] + [0.0] * 22, np.float32))
    img = {"kind": "u32_count", "width": 256, "height": 256, "channels": 4,
           "lo": [0.0, -1.0], "hi": [2.0, 1.0]}
    got = run_gpu(api, w, "f64", system=system, image=img)
    ref = orc.chaos_count(system, w["run"], img)
    assert rel_l1(got["image"], ref["image"]) <= 1e-4
    assert got["dropped"] == ref["dropped"]


def test_menger_depth_parity(api, orc):
    w = W.menger(n_points=1 << 14, side=1024)
    got_img = api.Image(w["image"], device=_dev()).clear()
    api.chaos_game(w["system"], w["run"], got_img, precision="f64")
    got = got_img.to_numpy()
    ref = orc.chaos_depth(w["system"], w["run"], w["image"], w["image"]["near"])
    assert got["dropped"] == ref["dropped"]
    assert np.array_equal(got["density"], ref["density"])
    occupied, differ, occ_diff, ulps = depth_key_diff(got["depth"], ref["depth"])
    print(f"menger f64: keys differing {differ} of {occupied} (max {ulps} ulp)")
    # FP64 depths differ from the oracle's by a few FP64 ulps (other rounding
    # order and sine/cosine), so an FP32 key could differ only where a
    # pixel's winning depth lies within those ulps of an FP32 rounding
    # boundary: about 2e-9 per occupied pixel, so keys are equal exactly
    assert occ_diff == 0 and differ == 0, (differ, ulps)


def test_image_clear(api):
    desc = {"kind": "u64_depth", "width": 37, "height": 5, "channels": 1,
            "lo": [-1, -1], "hi": [1, 1], "near": 0.1}
    img = api.Image(desc, device=_dev())
    img.data.fill_(5)
    img.density.fill_(7)
    img.dropped.fill_(3)
    img.clear()
    out = img.to_numpy()
    assert np.all(out["depth"] == np.iinfo(np.uint64).max)
    assert np.all(out["density"] == 0) and out["dropped"] == 0
    # odd offsets exercise the unaligned head of the 16-byte clear
    base = torch.full((1001,), 9, dtype=torch.int32, device=_dev())
    for off in (0, 1, 2, 3):
        view = base[off:off + 997]
        d = {"kind": "u32_count", "width": 997, "height": 1, "channels": 1,
             "lo": [0, 0], "hi": [1, 1]}
        im = api.Image(d, device=_dev(), data=view)
        base.fill_(9)
        im.clear()
        host = base.cpu().numpy()
        assert np.all(host[off:off + 997] == 0)
        assert np.all(host[:off] == 9) and np.all(host[off + 997:] == 9)


# ---------------------------------------------------------------------------
# Binned splat: bit-identical to the direct splat, same parity bars
# ---------------------------------------------------------------------------
def _image_of(api, w, precision, splat_path, system=None, run=None, image=None):
    img = api.Image(image or w["image"], device=_dev()).clear()
    api.chaos_game(system or w["system"], run or w["run"], img, precision=precision,
                   splat_path=splat_path)
    return img.to_numpy()


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_binned_equals_direct_square(api, precision):
    w = W.cfs_square(n_points=(1 << 18) + 77)
    a = _image_of(api, w, precision, "direct")
    b = _image_of(api, w, precision, "binned")
    assert np.array_equal(a["image"], b["image"]) and a["dropped"] == b["dropped"] == 0


def test_binned_sierpinski_parity(api, orc):
    w = W.sierpinski()
    got = _image_of(api, w, "f32", "binned")
    ref = orc.chaos_count(w["system"], w["run"], w["image"])
    assert int(got["image"].astype(np.int64).sum()) == (1 << 16) * 48
    assert rel_l1(got["image"], ref["image"]) <= 1e-4
    assert np.array_equal(got["image"], _image_of(api, w, "f32", "direct")["image"])


def test_binned_drops_and_ragged(api, orc):
    # window cut through the attractor: splats outside are dropped and counted;
    # a ragged image (not a multiple of the tile) and ragged point count
    w = W.sierpinski(n_points=5000, n_iters=37, burn_in=5)
    image = {"kind": "u32_count", "width": 333, "height": 211, "channels": 1,
             "lo": [0.2, 0.1], "hi": [0.9, 0.7]}
    got = _image_of(api, w, "f64", "binned", image=image)
    ref = orc.chaos_count(w["system"], w["run"], image)
    assert np.array_equal(got["image"], ref["image"])
    assert got["dropped"] == ref["dropped"] > 0


@pytest.mark.parametrize("shape", [(300, 170), (128, 129), (40, 700)])
def test_binned_per_index_channels_ragged(api, orc, shape):
    """Per-index counts (one channel per map) in images whose planes are not
    multiples of the binned splat's 16384-element tiles, so tiles straddle
    two channels' planes and the last one lies partly past the image; the
    image equals the oracle's."""
    W_, H_ = shape
    w = W.sierpinski(n_points=(1 << 15) + 7, n_iters=29, burn_in=5)
    image = {"kind": "u32_count", "width": W_, "height": H_, "channels": 3,
             "lo": [-0.05, -0.05], "hi": [1.05, 0.95]}
    got = _image_of(api, w, "f64", "binned", image=image)
    ref = orc.chaos_count(w["system"], w["run"], image)
    assert np.array_equal(got["image"], ref["image"])
    assert got["dropped"] == ref["dropped"]


def test_binned_concentrated_and_empty_tiles(api):
    # the attractor covers 64x64 pixels of a 4096x4096 image: 16 of 1024 tiles
    # hold every record (runs of ~770 records: several passes of the widest
    # lane group), the rest are skipped by their record totals
    w = W.sierpinski(n_points=(1 << 16) + 3)
    image = {"kind": "u32_count", "width": 4096, "height": 4096, "channels": 1,
             "lo": [0, 0], "hi": [64, 64]}
    a = _image_of(api, w, "f32", "direct", image=image)
    b = _image_of(api, w, "f32", "binned", image=image)
    assert np.array_equal(a["image"], b["image"]) and a["dropped"] == b["dropped"]
    assert int(b["image"].astype(np.int64).sum()) + b["dropped"] == ((1 << 16) + 3) * 48
    assert not b["image"][0, 64:, :].any() and not b["image"][0, :, 64:].any()


def test_binned_on_side_stream(api):
    # two calls into one image on a stream of their own (2^22 + 517 points,
    # workspace passed in and reused), read after only that stream is waited
    # for: equal to twice the direct splat
    w = W.cfs_square(n_points=(1 << 22) + 517, side=1024)
    ref = _image_of(api, w, "f64", "direct")["image"].astype(np.int64)
    side = torch.cuda.Stream()
    img = api.Image(w["image"], device=_dev())
    ws_bytes = api.chaos_workspace_bytes(w["system"], w["run"], img, "f64", "binned")
    assert ws_bytes > 0
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=_dev())
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        img.clear(side)
        for _ in range(2):
            api.chaos_game(w["system"], w["run"], img, precision="f64", splat_path="binned",
                           workspace=ws, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    got = img.data.cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal(got, 2 * ref)


def test_binned_side_stream_own_workspace(api):
    # a call on a side stream that leaves the workspace to the binding, made
    # outside that stream's context, followed at once by allocations and
    # writes on the current stream: the binding's workspace must not be
    # handed out again while the side stream still uses it
    w = W.cfs_square(n_points=(1 << 22) + 517, side=1024)
    ref = _image_of(api, w, "f64", "binned")["image"]
    side = torch.cuda.Stream()
    img = api.Image(w["image"], device=_dev())
    side.wait_stream(torch.cuda.current_stream())
    img.clear(side)
    api.chaos_game(w["system"], w["run"], img, precision="f64", splat_path="binned", stream=side)
    ws_bytes = api.chaos_workspace_bytes(w["system"], w["run"], img, "f64", "binned")
    junk = [torch.full((ws_bytes // 4 + 1,), -1, dtype=torch.int32, device=_dev())
            for _ in range(2)]
    torch.cuda.current_stream().wait_stream(side)
    got = img.data.cpu().numpy().view(np.uint32)
    del junk
    assert np.array_equal(got, ref)


def test_binned_call_in_graph(api):
    # the binned call (clear, chaos kernel, transpose, accumulate) captured
    # into a graph: every replay, with eager calls in between, equals the
    # eager result
    w = W.cfs_square(n_points=(1 << 22) + 3, side=512)
    eager = _image_of(api, w, "f32", "binned")["image"]
    img = api.Image(w["image"], device=_dev())
    ws_bytes = api.chaos_workspace_bytes(w["system"], w["run"], img, "f32", "binned")
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=_dev())
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        with torch.cuda.graph(g, stream=cap):
            img.clear(cap)
            api.chaos_game(w["system"], w["run"], img, precision="f32", splat_path="binned",
                           workspace=ws, stream=cap)
    torch.cuda.synchronize()
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(img.to_numpy()["image"], eager)
        other = _image_of(api, w, "f32", "binned")["image"]
        assert np.array_equal(other, eager)


@pytest.mark.parametrize("px", [257, 258])
def test_binned_single_pixel(api, px):
    # one map x -> b sends every splat to pixel (px, 100): a single run per
    # chunk in a single tile, one pixel counting n * 48 (several accumulate
    # workgroups over chunk ranges, merged with device atomics); the image
    # equals the direct splat's
    n = (1 << 16) + 3
    b = [[(px + 0.5) / 512.0, 100.5 / 512.0]]
    system = W._system(np.zeros((1, 2, 2)), b)
    run = W._run(n, 64, 16)
    image = W._image("u32_count", 512, 512, 1, (0, 0), (1, 1))
    w = {"system": system, "run": run, "image": image}
    a = _image_of(api, w, "f32", "direct")
    got = _image_of(api, w, "f32", "binned")
    assert np.array_equal(a["image"], got["image"])
    assert int(got["image"][0, 100, px]) == n * 48
    assert int(got["image"].astype(np.int64).sum()) == n * 48


def test_binned_two_pixels_with_large_counts(api):
    # two maps x -> b0, b1 with probabilities 0.9 / 0.1 in a 4x4 image: one
    # tile, counts above 2^16 per pixel, compared with the oracle
    import oracle as orc
    n = 40000
    system = W._system(np.zeros((2, 2, 2)), [[0.25, 0.25], [0.75, 0.75]], prob=[0.9, 0.1])
    run = W._run(n, 40, 8)
    image = W._image("u32_count", 4, 4, 1, (0, 0), (1, 1))
    w = {"system": system, "run": run, "image": image}
    got = _image_of(api, w, "f64", "binned")
    ref = orc.chaos_count(system, run, image)
    assert np.array_equal(got["image"], ref["image"])
    assert int(got["image"].max()) > 65535


def test_binned_largest_image(api):
    # the largest count image the binned splat takes (2^25 elements: 2048
    # tiles, the last one full) against the direct splat
    w = W.sierpinski(n_points=(1 << 18) + 11)
    image = {"kind": "u32_count", "width": 8192, "height": 4096, "channels": 1,
             "lo": [0, 0], "hi": [1, 1]}
    a = _image_of(api, w, "f32", "direct", image=image)
    b = _image_of(api, w, "f32", "binned", image=image)
    assert np.array_equal(a["image"], b["image"]) and a["dropped"] == b["dropped"]
    assert int(b["image"].astype(np.int64).sum()) + b["dropped"] == ((1 << 18) + 11) * 48


def test_binned_slices_long_runs(api):
    # 1000 splats per point: the run is split into several slices that share
    # the workspace; the image must equal the direct splat's
    w = W.cfs_square(n_points=(1 << 22) + 5, n_iters=1004, burn_in=4, side=1024)
    sysw = dict(w["system"], final_kind="identity")
    image = dict(w["image"], lo=[0, 0], hi=[1, 1])
    img = api.Image(image, device=_dev())
    nbytes = api.chaos_workspace_bytes(sysw, w["run"], img, "f32", "binned")
    assert 0 < nbytes < (1 << 32)
    a = _image_of(api, w, "f32", "direct", system=sysw, image=image)
    b = _image_of(api, w, "f32", "binned", system=sysw, image=image)
    assert np.array_equal(a["image"], b["image"]) and a["dropped"] == b["dropped"]
    # FP32 can round x/2 + 1/2 up to exactly 1.0 (a tie from 1 - 2^-24), which is
    # outside the half-open window: such splats are dropped and counted
    assert int(b["image"].astype(np.int64).sum()) + b["dropped"] == ((1 << 22) + 5) * 1000


def test_binned_unequal_probabilities_3d(api, orc):
    w = W.menger(n_points=20000, side=64)
    rng = np.random.default_rng(2)
    prob = rng.dirichlet(np.ones(20))
    system = dict(w["system"], final_kind="identity", prob=prob)
    image = {"kind": "u32_count", "width": 300, "height": 300, "channels": 20,
             "lo": [0, 0], "hi": [1, 1]}
    got = _image_of(api, w, "f64", "binned", system=system, image=image)
    ref = orc.chaos_count(system, w["run"], image)
    assert np.array_equal(got["image"], ref["image"])


def test_binned_workspace_too_small(api):
    """Half the workspace of the fewest launches is enough (more launches);
    one below a single workgroup's records is refused under BINNED, with
    nothing written."""
    from paper_2606_02226_amd import _lib
    import ctypes as C
    w = W.cfs_square(n_points=1 << 16)
    img = api.Image(w["image"], device=_dev()).clear()
    sysc = api.System(w["system"])
    runc = api.run_struct(w["run"], "f64", "binned")
    need = _lib.load().cfs_chaos_game_workspace(C.byref(sysc.struct), C.byref(runc),
                                                C.byref(img.struct))
    half = torch.empty(int(need) // 2, dtype=torch.uint8, device=_dev())
    rc = _lib.load().cfs_chaos_game(C.byref(sysc.struct), C.byref(runc), C.byref(img.struct),
                                    None, None, None, C.c_void_p(half.data_ptr()),
                                    C.c_size_t(half.numel()), None)
    assert rc == _lib.CFS_OK
    torch.cuda.synchronize()
    assert np.array_equal(img.to_numpy()["image"], _image_of(api, w, "f64", "binned")["image"])
    img.clear()
    tiny = torch.empty(4096, dtype=torch.uint8, device=_dev())
    rc = _lib.load().cfs_chaos_game(C.byref(sysc.struct), C.byref(runc), C.byref(img.struct),
                                    None, None, None, C.c_void_p(tiny.data_ptr()),
                                    C.c_size_t(tiny.numel()), None)
    assert rc == _lib.CFS_E_WORKSPACE
    assert int(img.to_numpy()["image"].astype(np.int64).sum()) == 0


def test_full_size_cfs_square_sampled(api, orc):
    """The benchmark configuration (2^24 points, FP64, binned) checked on
    sampled points computed one by one by the oracle, on exact totals and
    against the direct splat bit for bit."""
    w = W.cfs_square()
    N, T, B = 1 << 24, 32, 8
    img = api.Image(w["image"], device=_dev()).clear()
    fin = torch.empty((N, 2), dtype=torch.float64, device=_dev())
    last = torch.empty((N,), dtype=torch.uint8, device=_dev())
    api.chaos_game(w["system"], w["run"], img, precision="f64", final=fin, last=last,
                   splat_path="binned")
    got = img.to_numpy()
    h = got["image"].astype(np.int64)
    assert got["dropped"] == 0 and int(h.sum()) == N * (T - B)
    tot = h.sum(axis=(1, 2))
    # per-channel totals: binomial(N (T-B), 1/4) within 6 sigma
    sd = math.sqrt(N * (T - B) * 0.25 * 0.75)
    assert np.all(np.abs(tot - N * (T - B) / 4) < 6 * sd)
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(N, size=512, replace=False))
    sample[0], sample[-1] = 0, N - 1
    fs = fin[torch.from_numpy(sample).to(_dev())].cpu().numpy()
    ls = last[torch.from_numpy(sample).to(_dev())].cpu().numpy()
    for i, pid in enumerate(sample):
        r = orc.chaos_count(w["system"], dict(w["run"], n_points=1, point_offset=int(pid)),
                            w["image"], want_final=True, want_last=True)
        assert r["last"][0] == ls[i]
        assert np.max(np.abs(r["final"][0] - fs[i])) <= 1e-12
    direct = _image_of(api, w, "f64", "direct")
    assert np.array_equal(direct["image"], got["image"])


# ---------------------------------------------------------------------------
# Binned depth splat (3D camera): bit-identical to the direct depth splat
# ---------------------------------------------------------------------------
def _depth_image(api, w, precision, splat_path, run=None):
    img = api.Image(w["image"], device=_dev()).clear()
    api.chaos_game(w["system"], run or w["run"], img, precision=precision, splat_path=splat_path)
    return img.to_numpy()


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_depth_binned_equals_direct(api, precision):
    w = W.menger(n_points=(1 << 18) + 3, side=1024)
    a = _depth_image(api, w, precision, "direct")
    b = _depth_image(api, w, precision, "binned")
    assert np.array_equal(a["depth"], b["depth"])
    assert np.array_equal(a["density"], b["density"])
    assert a["dropped"] == b["dropped"]


@pytest.mark.parametrize("shape", [(1000, 700), (200, 90), (130, 1000), (64, 64)])
def test_depth_ragged_tiles_vs_oracle(api, orc, shape):
    """Depth images whose last 8192-pixel tile of the binned splat lies
    partly past the image (and one image smaller than a tile), at other
    aspect ratios than the square workloads.  Binned keys and density equal
    the direct splat's bit for bit, and the oracle's."""
    W_, H_ = shape
    w = W.menger(n_points=(1 << 14) + 5, side=1024)
    w["image"] = dict(w["image"], width=W_, height=H_)
    got = _depth_image(api, w, "f64", "binned")
    direct = _depth_image(api, w, "f64", "direct")
    assert np.array_equal(got["depth"], direct["depth"])
    assert np.array_equal(got["density"], direct["density"])
    assert got["dropped"] == direct["dropped"]
    ref = orc.chaos_depth(w["system"], w["run"], w["image"], w["image"]["near"])
    assert got["dropped"] == ref["dropped"]
    assert np.array_equal(got["density"], ref["density"])
    occupied, differ, occ_diff, ulps = depth_key_diff(got["depth"], ref["depth"])
    assert occ_diff == 0 and differ == 0, (differ, ulps)


def test_depth_fp32_guard_band(api, orc):
    """FP32 positions and transforms for the depth image, against the FP64
    oracle: FP32 rounding moves a few splats across pixel edges and changes
    depths by a few FP32 ulps, so occupancy and density agree to within a
    small fraction, and where both images hold a key its depth agrees to
    FP32 rounding of the 24 steps and the camera (a few 1e-6 relative)
    except where another splat of nearly the same depth wins."""
    w = W.menger(n_points=1 << 15, side=1024)
    got = _depth_image(api, w, "f32", "binned")
    ref = orc.chaos_depth(w["system"], w["run"], w["image"], w["image"]["near"])
    d_got = got["density"].astype(np.int64)
    d_ref = ref["density"].astype(np.int64)
    dens_l1 = np.abs(d_got - d_ref).sum() / d_ref.sum()
    occupied, differ, occ_diff, ulps = depth_key_diff(got["depth"], ref["depth"])
    empty = np.uint64(0xFFFFFFFFFFFFFFFF)
    g = got["depth"].reshape(-1)
    r = ref["depth"].reshape(-1)
    both = (g != empty) & (r != empty)
    gd = (g[both] >> np.uint64(32)).astype(np.uint32).view(np.float32).astype(np.float64)
    rd = (r[both] >> np.uint64(32)).astype(np.uint32).view(np.float32).astype(np.float64)
    rel = np.abs(gd - rd) / rd
    print(f"menger f32: density rel L1 {dens_l1:.2e}, occupancy differs at {occ_diff} of "
          f"{occupied}, keys differ at {differ}, depth rel diff p99 {np.quantile(rel, 0.99):.2e} "
          f"max {rel.max():.2e}")
    assert int(d_got.sum()) + got["dropped"] == int(d_ref.sum()) + ref["dropped"]
    # measured: density 9.2e-5, occupancy 5 of 197689 pixels, p99 8.1e-8
    assert dens_l1 <= 5e-4
    assert occ_diff <= 2e-4 * occupied
    assert np.quantile(rel, 0.99) <= 1e-6
    assert np.count_nonzero(rel > 1e-5) <= 2e-3 * occupied


def test_small_workspace_takes_more_launches(api):
    """A workspace below what the fewest launches need: the binned splat
    runs in more point-range launches that fit it, with the same image; a
    workspace below one workgroup's records takes the direct splat under
    AUTO (the same image again)."""
    w = W.menger(n_points=(1 << 17) + 5, side=512)
    sysc = api.System(w["system"])
    full = _depth_image(api, w, "f64", "binned")
    need = api.chaos_workspace_bytes(sysc, w["run"], api.Image(w["image"], device=_dev()), "f64",
                                     "binned")
    for frac, path in ((3, "binned"), (7, "auto")):
        ws = torch.empty(need // frac, dtype=torch.uint8, device=_dev())
        img = api.Image(w["image"], device=_dev()).clear()
        api.chaos_game(sysc, w["run"], img, precision="f64", splat_path=path, workspace=ws)
        got = img.to_numpy()
        assert np.array_equal(got["depth"], full["depth"])
        assert np.array_equal(got["density"], full["density"])
        assert got["dropped"] == full["dropped"]
    tiny = torch.empty(1 << 16, dtype=torch.uint8, device=_dev())
    img = api.Image(w["image"], device=_dev()).clear()
    api.chaos_game(sysc, w["run"], img, precision="f64", splat_path="auto", workspace=tiny)
    got = img.to_numpy()
    assert np.array_equal(got["depth"], full["depth"])
    assert np.array_equal(got["density"], full["density"])


def test_depth_binned_vs_oracle(api, orc):
    w = W.menger(n_points=1 << 14, side=1024)
    got = _depth_image(api, w, "f64", "binned")
    ref = orc.chaos_depth(w["system"], w["run"], w["image"], w["image"]["near"])
    assert got["dropped"] == ref["dropped"]
    assert np.array_equal(got["density"], ref["density"])
    occupied, differ, occ_diff, ulps = depth_key_diff(got["depth"], ref["depth"])
    assert occ_diff == 0 and ulps <= 1 and differ <= 2, (differ, ulps)


def test_full_size_menger(api, orc):
    """The 3D configuration at full size (2^26 points x 24 iterations, 4096^2):
    binned == direct bit for bit, exact splat accounting, and sampled points'
    final positions and last indices equal to the oracle's one by one."""
    w = W.menger()
    N, T, B = 1 << 26, 24, 8
    img = api.Image(w["image"], device=_dev()).clear()
    fin = torch.empty((N, 3), dtype=torch.float64, device=_dev())
    last = torch.empty((N,), dtype=torch.uint8, device=_dev())
    api.chaos_game(w["system"], w["run"], img, precision="f64", final=fin, last=last,
                   splat_path="binned")
    got = img.to_numpy()
    assert int(got["density"].astype(np.int64).sum()) + got["dropped"] == N * (T - B)
    direct = _depth_image(api, w, "f64", "direct")
    assert np.array_equal(direct["depth"], got["depth"])
    assert np.array_equal(direct["density"], got["density"])
    rng = np.random.default_rng(3)
    sample = np.sort(rng.choice(N, size=256, replace=False))
    idx = torch.from_numpy(sample).to(_dev())
    fs, ls = fin[idx].cpu().numpy(), last[idx].cpu().numpy()
    for i, pid in enumerate(sample):
        r = orc.chaos_depth(w["system"], dict(w["run"], n_points=1, point_offset=int(pid)),
                            dict(w["image"], width=8, height=8), w["image"]["near"],
                            want_final=True, want_last=True)
        assert r["last"][0] == ls[i]
        assert np.max(np.abs(r["final"][0] - fs[i])) <= 1e-12


# ---------------------------------------------------------------------------
# The paper's circle primitive (non-affine maps, mixed kinds)
# ---------------------------------------------------------------------------
def _near_circle_singularity(orc, w, pid, eps):
    """Whether the oracle's FP64 trajectory of point ``pid`` enters a circle
    map within ``eps`` of the map's singular set: the origin (polar angle
    undefined; an error d in p moves the angle by about d / |p|) or the
    positive x-axis, where the polar angle taken in [0, 2 pi) jumps from 2 pi
    to 0, so the image radius sqrt(angle / 2 pi) jumps from 1 to 0.  A
    rounding difference there sends the two trajectories apart; elsewhere the
    map is smooth and the error stays at rounding level."""
    run, system = w["run"], w["system"]
    circle_maps = {i for i, k in enumerate(system["kind"]) if k == "circle"}
    T = run["n_iters"]
    one = dict(run, n_points=1, point_offset=int(pid))
    idx = orc.chaos_count(system, dict(one, burn_in=T), w["image"], want_indices=True)["indices"][0]
    for t in range(1, T):          # p_t is the input of step t + 1
        if int(idx[t]) not in circle_maps:
            continue
        p = orc.chaos_count(system, dict(one, n_iters=t, burn_in=t), w["image"],
                            want_final=True)["final"][0]
        if np.hypot(p[0], p[1]) < eps or (p[0] > -eps and abs(p[1]) < eps):
            return True
    return False


def _check_circle_positions(orc, w, got, ref, bound, eps):
    """Every final position within ``bound`` of the oracle's, except points
    whose trajectory passes within ``eps`` of a circle map's singular set
    (at most 1 in 1000)."""
    err = np.abs(got["final"] - ref["final"]).max(axis=1)
    out = np.flatnonzero(err > bound)
    assert out.size <= max(1, err.size // 1000), out.size
    for pid in out:
        assert _near_circle_singularity(orc, w, pid, eps), (int(pid), float(err[pid]))
    inside = np.delete(err, out)
    return float(inside.max(initial=0.0)), int(out.size)


def test_circle_fp64_parity(api, orc):
    w = W.circle(n_points=1 << 14)
    got = run_gpu(api, w, "f64", want_indices=True)
    ref = orc.chaos_count(w["system"], w["run"], w["image"], want_final=True,
                          want_last=True, want_indices=True)
    assert np.array_equal(got["indices"], ref["indices"])
    worst, n_out = _check_circle_positions(orc, w, got, ref, 1e-9, 1e-6)
    print(f"circle f64: max |dp| {worst:.2e} ({n_out} points past the singular set), "
          f"relL1 {rel_l1(got['image'], ref['image']):.2e}")
    assert rel_l1(got["image"], ref["image"]) <= 1e-4
    assert got["dropped"] == ref["dropped"]


def test_circle_fp32_indices_and_measure(api, orc):
    w = W.circle(n_points=1 << 14)
    got = run_gpu(api, w, "f32", want_indices=True)
    ref = orc.chaos_count(w["system"], w["run"], w["image"], want_final=True,
                          want_indices=True)
    assert np.array_equal(got["indices"], ref["indices"])
    # FP32 rounding (6e-8 relative per operation) grows to the 1e-5 bar only
    # through the 1 / |p| of the polar angle near the origin or a change of
    # side of the positive x-axis
    worst, n_out = _check_circle_positions(orc, w, got, ref, 1e-5, 1e-2)
    l1 = rel_l1(got["image"], ref["image"])
    print(f"circle f32: max |dp| {worst:.2e} ({n_out} points past the singular set), "
          f"relL1 {l1:.2e}")
    P = got["final"]
    u = P[:, 0] ** 2 + P[:, 1] ** 2
    assert np.all(u <= 1.0 + 1e-6) and abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / u.size)


@pytest.mark.parametrize("compose", ["copy", "reuse"])
@pytest.mark.parametrize("path", ["direct", "binned"])
def test_mixed_kinds_parity(api, orc, path, compose):
    """Two circle maps and two affine maps in one system, so waves hold both
    kinds at once: every point's index sequence and last index are the
    oracle's bit for bit, its final position within rounding, the image
    within the histogram bar, and a ragged last workgroup (20000 points) and
    dropped splats are accounted for."""
    w = W.circle(n_points=20000, extra_affine=2)
    if compose == "reuse":
        w = dict(w, system=dict(w["system"], final_kind="swirl",
                                final_params=np.array([0, 0, 1.5, 0, 0] + [0] * 19, np.float32),
                                compose="reuse"))
    N, T = w["run"]["n_points"], w["run"]["n_iters"]
    img = api.Image(w["image"], device=_dev()).clear()
    fin = torch.empty((N, 2), dtype=torch.float64, device=_dev())
    last = torch.empty((N,), dtype=torch.uint8, device=_dev())
    idx = torch.empty((N, T), dtype=torch.uint8, device=_dev())
    api.chaos_game(w["system"], w["run"], img, precision="f64", splat_path=path, final=fin,
                   last=last, indices=idx)
    got = img.to_numpy()
    ref = orc.chaos_count(w["system"], w["run"], w["image"], want_final=True, want_last=True,
                          want_indices=True)
    assert np.array_equal(idx.cpu().numpy(), ref["indices"])
    assert np.array_equal(last.cpu().numpy(), ref["last"])
    assert got["dropped"] == ref["dropped"]
    assert rel_l1(got["image"], ref["image"]) <= 1e-4
    # positions: within rounding, except near the circle maps' singular set
    _check_circle_positions(orc, w, {"final": fin.cpu().numpy()}, ref, 1e-9, 1e-6)


@pytest.mark.parametrize("path", ["direct", "binned"])
@pytest.mark.parametrize("compose", ["copy", "reuse"])
def test_composed_circle_parity(api, orc, compose, path):
    # Section 3's composition figure: the swirl on a copy of the point or fed back
    w = W.composed_circle(compose, n_points=20000)
    img = api.Image(w["image"], device=_dev()).clear()
    api.chaos_game(w["system"], w["run"], img, precision="f64", splat_path=path)
    got = img.to_numpy()
    ref = orc.chaos_count(w["system"], w["run"], w["image"])
    l1 = rel_l1(got["image"], ref["image"])
    print(f"composed circle {compose} {path}: relL1 {l1:.2e}")
    assert l1 <= 1e-4
    assert got["dropped"] == ref["dropped"]


def test_reuse_square_final_points(api, orc):
    # the CFS square's swirl fed back into the iteration, FP64, per point
    w = W.cfs_square(n_points=4096, side=256)
    w["system"]["compose"] = "reuse"
    got = run_gpu(api, w, "f64", want_indices=True)
    ref = orc.chaos_count(w["system"], w["run"], w["image"], want_final=True,
                          want_indices=True)
    assert np.array_equal(got["indices"], ref["indices"])
    # the swirl and the affine maps are smooth: no point leaves rounding level
    err = np.abs(got["final"] - ref["final"]).max(axis=1)
    print(f"reuse square f64: max |dp| {err.max():.2e}")
    assert err.max() <= 1e-9, err.max()
    assert rel_l1(got["image"], ref["image"]) <= 1e-4


def test_timing_hook_phases(api):
    # the measurement hook: one record per call, phases non-negative, the
    # chaos kernel of the binned path takes time, the direct path has no
    # transpose or accumulate phase
    w = W.sierpinski(n_points=1 << 16)
    img = api.Image(w["image"], device=_dev()).clear()
    api.timing_read()
    api.timing_enable(True)
    try:
        api.chaos_game(w["system"], w["run"], img, precision="f32", splat_path="binned")
        api.chaos_game(w["system"], w["run"], img, precision="f32", splat_path="direct")
    finally:
        api.timing_enable(False)
    ph = api.timing_read()
    assert ph.shape == (2, 3)
    assert np.all(ph >= 0) and ph[0, 0] > 0 and ph[1, 0] > 0
    assert ph[1, 1] < 0.05 and ph[1, 2] < 0.05
    assert api.timing_read().shape == (0, 3)


@pytest.mark.parametrize("case", ["dirichlet64", "bucket_edges", "tiny"])
def test_selection_guide_cases(api, orc, case):
    # the guide-table selection against the oracle's plain inverse CDF:
    # 64 maps (several thresholds per guide bucket), thresholds exactly on
    # bucket boundaries (multiples of 2^24), and clusters of tiny probabilities
    rng = np.random.default_rng(21)
    if case == "dirichlet64":
        n = 64
        prob = rng.dirichlet(np.ones(n) * 0.3)
    elif case == "bucket_edges":
        n = 8
        prob = np.array([1, 3, 5, 7, 64, 32, 16, 128], np.float64) / 256.0
    else:
        n = 12
        prob = np.full(n, 1e-9)
        prob[[0, 5, 11]] = (1.0 - 9e-9) / 3
    A = np.stack([np.eye(2) * 0.3] * n).astype(np.float32)
    b = rng.uniform(0, 0.7, size=(n, 2)).astype(np.float32)
    system = W._system(A, b, prob=prob)
    run = {"seed": 12345, "instance": 1, "n_points": 20000, "point_offset": 0,
           "n_iters": 32, "burn_in": 8}
    img = {"kind": "u32_count", "width": 64, "height": 64, "channels": 1,
           "lo": [0, 0], "hi": [1, 1]}
    got = run_gpu(api, None, "f32", want_indices=True, system=system, run=run, image=img)
    ref = orc.chaos_count(system, run, img, want_indices=True)
    assert np.array_equal(got["indices"], ref["indices"])
