"""GPU parity of the batched form (cfs_batch_*, cfs_autotune): every instance
of a batch is bit-identical to the plain cfs_chaos_game of that instance
(same random streams, same device functions), FP64 instances match the
oracle, graph replays are exact, updates take effect without re-capture."""
import numpy as np
import pytest

import workloads as W
from parity import rel_l1

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


def plain_image(api, w, precision="f32", splat_path="auto"):
    img = api.Image(w["image"], device=_dev()).clear()
    api.chaos_game(w["system"], w["run"], img, precision=precision, splat_path=splat_path)
    return img.to_numpy()


def small_batch(n=32, max_points=1 << 14):
    return W.batched(n_instances=n, max_points=max_points)


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("path", ["binned", "direct", "mixed"])
def test_batch_equals_plain(api, precision, path):
    """Every instance equals its plain run, whether the batch's instances
    all take the binned splat, all the direct one, or each the one the plan's
    threshold gives it (mixed: instances below 2^18 splats direct)."""
    entries = small_batch()
    images = [api.Image(w["image"], device=_dev()) for w in entries]
    plan = {"splat_path": "binned" if path == "mixed" else path, "blocks_per_item": 2}
    if path == "mixed":
        plan["direct_below"] = 1 << 18
        splats = [w["run"]["n_points"] * (w["run"]["n_iters"] - w["run"]["burn_in"])
                  for w in entries]
        assert min(splats) < 1 << 18 <= max(splats)   # both strategies are exercised
    b = api.Batch(entries, images, plan=plan, precision=precision)
    assert b.plan()["direct_below"] == plan.get("direct_below", 0)
    b.run()
    for w, img in zip(entries, images):
        got = img.to_numpy()
        ref = plain_image(api, w, precision)
        assert np.array_equal(got["image"], ref["image"]), w["name"]
        assert got["dropped"] == ref["dropped"]
    b.close()


def test_batch_fp64_vs_oracle(api, orc):
    entries = small_batch(n=12, max_points=1 << 13)
    images = [api.Image(w["image"], device=_dev()) for w in entries]
    b = api.Batch(entries, images, precision="f64")
    b.run()
    for w, img in zip(entries, images):
        got = img.to_numpy()
        ref = orc.chaos_count(w["system"], w["run"], w["image"])
        assert rel_l1(got["image"], ref["image"]) <= 1e-4, w["name"]
        assert got["dropped"] == ref["dropped"]
    b.close()


def test_graph_replays_exact(api):
    entries = small_batch(n=16)
    images = [api.Image(w["image"], device=_dev()) for w in entries]
    b = api.Batch(entries, images)
    b.run()
    first = [img.to_numpy()["image"].copy() for img in images]
    for _ in range(3):
        # eager work and a host sync between replays
        scratch = torch.ones(1 << 20, device=_dev()).sum()
        torch.cuda.synchronize()
        b.run()
        for f, img in zip(first, images):
            assert np.array_equal(img.to_numpy()["image"], f)
    assert scratch.item() == float(1 << 20)
    b.close()


def test_update_without_recapture(api):
    entries = small_batch(n=8)
    images = [api.Image(w["image"], device=_dev()) for w in entries]
    b = api.Batch(entries, images)
    b.run()
    before = [img.to_numpy()["image"].copy() for img in images]
    rng = np.random.default_rng(77)
    n5 = entries[5]["system"]["b"].shape[0]
    A, bb = W.random_affine_maps(rng, n5)
    A, bb = W.normalise_to_unit_square(A, bb)
    new_sys = W._system(A, bb, prob=rng.dirichlet(np.ones(n5)))
    b.update(5, new_sys)
    b.run()
    for i, img in enumerate(images):
        got = img.to_numpy()["image"]
        if i == 5:
            ref = plain_image(api, dict(entries[5], system=new_sys))["image"]
            assert np.array_equal(got, ref)
            assert not np.array_equal(got, before[5])
        else:
            assert np.array_equal(got, before[i])
    b.close()


def test_batch_edge_instances(api):
    base = small_batch(n=3)
    entries = [dict(base[0], run=dict(base[0]["run"], n_points=0)),
               dict(base[1], run=dict(base[1]["run"], n_iters=9, burn_in=9)),
               dict(base[2], image=dict(base[2]["image"], width=333, height=77)),
               dict(base[0], run=dict(base[0]["run"], n_points=1025, instance=9))]
    images = [api.Image(w["image"], device=_dev()) for w in entries]
    b = api.Batch(entries, images)
    b.run()
    for w, img in zip(entries, images):
        assert np.array_equal(img.to_numpy()["image"], plain_image(api, w)["image"])
    b.close()


def test_autotune_plan_is_valid(api, tmp_path):
    """The tuned plan renders every instance exactly; it is written to the
    cache file under the device's architecture, CU count and the batch's
    signature, and a second call returns it from the cache without running
    anything (the images it would overwrite keep their contents)."""
    import json
    entries = small_batch(n=16)
    images = [api.Image(w["image"], device=_dev()) for w in entries]
    cache = tmp_path / "plans.jsonl"
    plan = api.autotune(entries, images, cache=cache)
    assert plan["splat_path"] in ("binned", "direct") and plan["blocks_per_item"] >= 1
    lines = cache.read_text().splitlines()
    assert len(lines) == 1
    entry = json.loads(lines[0])
    props = torch.cuda.get_device_properties(_dev())
    assert entry["cus"] == props.multi_processor_count
    assert entry["arch"].startswith("gfx950")
    assert entry["plan"]["blocks_per_item"] == plan["blocks_per_item"]
    assert entry["plan"]["direct_below"] == plan["direct_below"]
    assert entry["ms"] > 0
    for img in images:
        img.data.fill_(7)
    again = api.autotune(entries, images, cache=cache)
    torch.cuda.synchronize()
    assert again == plan
    assert all(int(img.data.min()) == 7 == int(img.data.max()) for img in images)
    assert len(cache.read_text().splitlines()) == 1
    # another batch shape misses the cache and appends its own line
    other = small_batch(n=5)
    oimgs = [api.Image(w["image"], device=_dev()) for w in other]
    api.autotune(other, oimgs, cache=cache)
    assert len(cache.read_text().splitlines()) == 2
    b = api.Batch(entries, images, plan=plan)
    b.run()
    for w, img in zip(entries, images):
        assert np.array_equal(img.to_numpy()["image"], plain_image(api, w)["image"])
    b.close()


def test_full_size_batch(api):
    """The batched configuration at full size: 256 systems, 2..16 maps,
    2^12..2^20 points, 256^2..1024^2 images, one graph launch.  Exact totals
    for every instance; a sample of instances bit-identical to plain runs."""
    entries = W.batched()
    images = [api.Image(w["image"], device=_dev()) for w in entries]
    b = api.Batch(entries, images)
    b.run()
    torch.cuda.synchronize()
    for w, img in zip(entries, images):
        out = img.to_numpy()
        r = w["run"]
        assert int(out["image"].astype(np.int64).sum()) + out["dropped"] == \
            r["n_points"] * (r["n_iters"] - r["burn_in"])
    for i in (0, 1, 2, 100, 255):
        assert np.array_equal(images[i].to_numpy()["image"], plain_image(api, entries[i])["image"])
    b.close()
