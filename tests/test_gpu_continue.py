"""Continued runs on the GPU (cfs_run.iter_offset): a chaos game cut into
calls -- each point continued from the positions the previous call left in
final_points -- gives the images (summed), index sequences and final
positions of the uncut game, bit for bit, on both splat paths and for depth
images; and a continued call matches the oracle's continued call."""
import numpy as np
import pytest

import workloads as W

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


def _game(api, w, run, precision, path, final=None, image=None):
    img = image or api.Image(w["image"], device=_dev()).clear()
    N, T = run["n_points"], run["n_iters"]
    dt = torch.float64 if precision == "f64" else torch.float32
    d = w["system"]["dim"]
    fin = final if final is not None else torch.zeros((N, d), dtype=dt, device=_dev())
    idx = torch.empty((N, T), dtype=torch.uint8, device=_dev())
    api.chaos_game(w["system"], run, img, precision=precision, final=fin, indices=idx,
                   splat_path=path)
    torch.cuda.synchronize()
    return img, fin, idx


@pytest.mark.parametrize("precision", ["f32", "f64"])
@pytest.mark.parametrize("path", ["direct", "binned"])
@pytest.mark.parametrize("cut", [4, 12, 28])
def test_cut_game_equals_whole(api, precision, path, cut):
    w = W.cfs_square(n_points=(1 << 15) + 33, side=512)
    run = dict(w["run"], n_iters=32, burn_in=8)
    img_w, fin_w, idx_w = _game(api, w, run, precision, path)
    whole = img_w.to_numpy()
    img, fin, idx1 = _game(api, w, dict(run, n_iters=cut), precision, path)
    img, fin, idx2 = _game(api, w, dict(run, n_iters=32 - cut, iter_offset=cut), precision, path,
                           final=fin, image=img)
    got = img.to_numpy()
    assert np.array_equal(got["image"], whole["image"])
    assert got["dropped"] == whole["dropped"]
    assert torch.equal(fin, fin_w)
    assert torch.equal(torch.cat([idx1, idx2], dim=1), idx_w)


def test_continued_call_matches_oracle(api, orc):
    # start positions from the oracle's first 16 steps, then 16 more steps
    # on the GPU (FP64, binned) against the oracle's continued call
    w = W.cfs_square(n_points=5000, side=256)
    run = dict(w["run"], n_iters=16, burn_in=8)
    first = orc.chaos_count(w["system"], run, w["image"], want_final=True)
    cont = dict(run, iter_offset=16)
    ref = orc.chaos_count(w["system"], cont, w["image"], start=first["final"], want_indices=True)
    start = torch.from_numpy(first["final"]).to(_dev())
    img, fin, idx = _game(api, w, cont, "f64", "binned", final=start)
    got = img.to_numpy()
    assert np.array_equal(got["image"], ref["image"])
    assert np.array_equal(idx.cpu().numpy(), ref["indices"])
    assert np.max(np.abs(fin.cpu().numpy() - ref["final"])) <= 1e-9


@pytest.mark.parametrize("path", ["direct", "binned"])
def test_depth_game_cut(api, path):
    w = W.menger(n_points=(1 << 14) + 5, side=256)
    run = w["run"]
    T = run["n_iters"]

    def depth_game(r, fin, img):
        api.chaos_game(w["system"], r, img, precision="f64", final=fin, splat_path=path)
        torch.cuda.synchronize()

    whole = api.Image(w["image"], device=_dev()).clear()
    fw = torch.zeros((run["n_points"], 3), dtype=torch.float64, device=_dev())
    depth_game(run, fw, whole)
    img = api.Image(w["image"], device=_dev()).clear()
    f = torch.zeros_like(fw)
    depth_game(dict(run, n_iters=8), f, img)
    depth_game(dict(run, n_iters=4, iter_offset=8), f, img)
    depth_game(dict(run, n_iters=T - 12, iter_offset=12), f, img)
    a, b = img.to_numpy(), whole.to_numpy()
    assert np.array_equal(a["depth"], b["depth"]) and np.array_equal(a["density"], b["density"])
    assert torch.equal(f, fw)
