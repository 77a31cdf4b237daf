"""Continued runs (iteration_offset): the chaos game of a point is one
sequence of steps (Section 3), so a game cut into calls -- the second
starting from the first's final positions, with the steps' global numbers --
must give the same draws, indices, positions and splats as one call; the
burn-in counts global steps.  Pinned against the uncut oracle game, and
against its defining property: the image of the whole game is the sum of
the images of the pieces."""
import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("cut", [4, 12, 13, 30])
def test_count_game_cut_anywhere(orc, cut):
    w = W.cfs_square(n_points=700, side=128)
    run = dict(w["run"], n_iters=32, burn_in=8)
    whole = orc.chaos_count(w["system"], run, w["image"], want_final=True, want_indices=True)
    first = orc.chaos_count(w["system"], dict(run, n_iters=cut), w["image"], want_final=True,
                            want_indices=True)
    second = orc.chaos_count(w["system"], dict(run, n_iters=32 - cut, iter_offset=cut),
                             w["image"], start=first["final"], want_indices=True)
    assert np.array_equal(first["image"].astype(np.int64) + second["image"], whole["image"])
    assert np.array_equal(np.concatenate([first["indices"], second["indices"]], axis=1),
                          whole["indices"])
    assert np.array_equal(second["final"], whole["final"])
    assert first["dropped"] + second["dropped"] == whole["dropped"]
    # the burn-in lies in the first piece when cut >= 8, across both otherwise
    assert int(first["image"].sum()) == 700 * max(0, cut - 8)


def test_burn_in_spanning_calls(orc):
    # a call that lies inside the burn-in splats nothing but moves the points
    w = W.sierpinski(n_points=300, n_iters=40, burn_in=20)
    run = w["run"]
    a = orc.chaos_count(w["system"], dict(run, n_iters=8), w["image"], want_final=True)
    assert int(a["image"].sum()) == 0
    b = orc.chaos_count(w["system"], dict(run, n_iters=32, iter_offset=8), w["image"],
                        start=a["final"])
    whole = orc.chaos_count(w["system"], run, w["image"])
    assert np.array_equal(b["image"], whole["image"])


def test_depth_game_cut(orc):
    w = W.menger(n_points=500, side=64)
    run = w["run"]
    T = run["n_iters"]
    near = w["image"]["near"]
    whole = orc.chaos_depth(w["system"], run, w["image"], near, want_final=True)
    a = orc.chaos_depth(w["system"], dict(run, n_iters=10), w["image"], near, want_final=True)
    b = orc.chaos_depth(w["system"], dict(run, n_iters=T - 10, iter_offset=10), w["image"],
                        near, start=a["final"], depth=a["depth"].copy(),
                        density=a["density"].copy())
    assert np.array_equal(b["depth"], whole["depth"])
    assert np.array_equal(b["density"], whole["density"])
    assert np.array_equal(b["final"], whole["final"])


def test_continued_run_needs_start(orc):
    w = W.sierpinski(n_points=10)
    with pytest.raises(ValueError):
        orc.chaos_count(w["system"], dict(w["run"], iter_offset=4), w["image"])
