"""GPU parity of several objects from one primitive (cfs_chaos_scene) against
the FP64 oracle, through the C ABI.

Bars: FP64 positions -- histograms within 1e-4 relative L1 and dropped counts
exact; FP32 positions -- every pixel inside the oracle's guard-band interval
and totals exact; the direct and binned splats bit-identical; point-range
splits add up exactly at the full 1920x1080 scene size.
"""
import numpy as np
import pytest

import workloads as W
from parity import guard_band_images, guard_band_violations, rel_l1

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


def _scene_gpu(api, w, precision, path, run=None):
    img = api.Image(w["image"], device=_dev()).clear()
    api.chaos_scene(w["system"], w["objects"], run or w["run"], img, precision=precision,
                    splat_path=path)
    return img.to_numpy()


def _small_scene(n_points=1 << 14):
    # the space scene at a quarter of its size, so that the oracle runs in seconds
    return W.space_scene(n_points=n_points, width=480, height=270, n_stars=64)


@pytest.mark.parametrize("path", ["direct", "binned"])
def test_scene_fp64_parity(api, orc, path):
    w = _small_scene()
    got = _scene_gpu(api, w, "f64", path)
    ref = orc.chaos_scene(w["system"], w["objects"], w["run"], w["image"])
    l1 = rel_l1(got["image"], ref["image"])
    print(f"scene f64 {path}: relL1 {l1:.2e}, dropped {got['dropped']} / {ref['dropped']}")
    assert l1 <= 1e-4
    assert got["dropped"] == ref["dropped"]


def test_scene_fp32_guard_band(api, orc):
    w = _small_scene()
    got = _scene_gpu(api, w, "f32", "binned")
    ref = orc.chaos_scene(w["system"], w["objects"], w["run"], w["image"], want_splats=True)
    im = w["image"]
    q = ref["splats"]                                   # [N][T-B][n_obj][2]
    fx = (q[..., 0] - im["lo"][0]) * im["width"] / (im["hi"][0] - im["lo"][0])
    fy = (q[..., 1] - im["lo"][1]) * im["height"] / (im["hi"][1] - im["lo"][1])
    ch = np.array([o["channel"] for o in w["objects"]])[None, None, :]
    sure, maybe = guard_band_images(np.stack([fx, fy], -1), ch, im["width"], im["height"],
                                    im["channels"], eps_px=0.02)
    low, high = guard_band_violations(got["image"], sure, maybe)
    l1 = rel_l1(got["image"], ref["image"])
    print(f"scene f32: relL1 {l1:.2e}, guard-band violations {low}/{high}")
    assert (low, high) == (0, 0)
    N, T_rec = w["run"]["n_points"], w["run"]["n_iters"] - w["run"]["burn_in"]
    assert int(got["image"].sum()) + got["dropped"] == N * T_rec * len(w["objects"])


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_scene_direct_equals_binned(api, precision):
    w = _small_scene(n_points=50000)
    a = _scene_gpu(api, w, precision, "direct")
    b = _scene_gpu(api, w, precision, "binned")
    assert np.array_equal(a["image"], b["image"])
    assert a["dropped"] == b["dropped"]


def test_single_object_equals_plain_chaos_game(api):
    w = W.circle(n_points=30000, extra_affine=1)
    img = {"kind": "u32_count", "width": 300, "height": 200, "channels": 1,
           "lo": [-1.5, -1.0], "hi": [1.5, 1.0]}
    for kind, fp in (("swirl", (0.1, 0.0, 4.0, 0.0, 0.1)), ("ring", (0.5, 0.9))):
        scene = {"system": w["system"], "run": w["run"], "image": img,
                 "objects": [{"final_kind": kind, "final_params": fp}]}
        got = _scene_gpu(api, scene, "f64", "binned")
        s2 = W._system(w["system"]["A"], w["system"]["b"], kind=w["system"]["kind"],
                       final_kind=kind, final_params=fp)
        plain = api.Image(img, device=_dev()).clear()
        api.chaos_game(s2, w["run"], plain, precision="f64", splat_path="binned")
        assert np.array_equal(got["image"], plain.to_numpy()["image"])


def test_ragged_and_empty(api, orc):
    w = _small_scene(n_points=1000)      # not a multiple of the 512-lane block
    w["run"]["n_iters"], w["run"]["burn_in"] = 13, 5
    for path in ("direct", "binned"):
        got = _scene_gpu(api, w, "f64", path)
        ref = orc.chaos_scene(w["system"], w["objects"], w["run"], w["image"])
        assert rel_l1(got["image"], ref["image"]) <= 1e-4
    w["run"]["n_points"] = 0
    got = _scene_gpu(api, w, "f64", "binned")
    assert int(got["image"].sum()) == 0 and got["dropped"] == 0


def test_full_size_scene_splits_and_sample(api, orc):
    # the 1920x1080 space scene at 2^22 points: point-range halves add up to
    # the whole run exactly, and a sampled range matches the oracle
    w = W.space_scene()
    N = w["run"]["n_points"]
    whole = _scene_gpu(api, w, "f64", "auto")
    T_rec = w["run"]["n_iters"] - w["run"]["burn_in"]
    assert int(whole["image"].sum()) + whole["dropped"] == N * T_rec * 4
    img = api.Image(w["image"], device=_dev()).clear()
    for off, n in ((0, N // 2), (N // 2, N - N // 2)):
        r = dict(w["run"], point_offset=off, n_points=n)
        api.chaos_scene(w["system"], w["objects"], r, img, precision="f64")
    halves = img.to_numpy()
    assert np.array_equal(whole["image"], halves["image"])
    sample = dict(w["run"], point_offset=N - 3000, n_points=3000)
    got = _scene_gpu(api, w, "f64", "binned", run=sample)
    ref = orc.chaos_scene(w["system"], w["objects"], sample, w["image"])
    assert rel_l1(got["image"], ref["image"]) <= 1e-4
    assert got["dropped"] == ref["dropped"]


def test_scene_copy_tables_and_streamed_copies(api, orc):
    # three duplicated objects whose copies overflow the workgroup's table
    # of copy placements: the first (300 copies) and the third (200) get
    # table rows, the second (300) no longer fits and draws every copy's
    # placement per splat; FP64 binned and direct against the oracle
    w = _small_scene(n_points=(1 << 13) + 9)
    a = 480 / 270
    star = lambda n, ch: {"final_kind": "identity", "place": W._place(1.0), "channel": ch,
                          "n_copies": n, "copy_lo": (-a, -1.0), "copy_hi": (a, 1.0),
                          "scale": (0.004, 0.01)}
    w["objects"] = [star(300, 0), star(300, 1), star(200, 2), dict(w["objects"][0], channel=3)]
    ref = orc.chaos_scene(w["system"], w["objects"], w["run"], w["image"])
    for path in ("direct", "binned"):
        got = _scene_gpu(api, w, "f64", path)
        assert rel_l1(got["image"], ref["image"]) <= 1e-4, path
        assert got["dropped"] == ref["dropped"], path
