"""The oracle over point-range shards equals the oracle over the whole run:
counts and depth keys exactly, FP64 densities and gradients to rounding.
(The full-size GPU parity tests and the benchmark's error figures rely on
it.)"""
import numpy as np

import workloads as W


def test_count_shards_equal_whole(orc):
    w = W.cfs_square(n_points=20000, side=256)
    a = orc.chaos_count(w["system"], w["run"], w["image"])
    for threads in (1, 3, 7):
        b = orc.chaos_count_sharded(w["system"], w["run"], w["image"], threads=threads)
        assert np.array_equal(a["image"], b["image"]) and a["dropped"] == b["dropped"]


def test_count_shards_keep_offset_and_drops(orc):
    w = W.sierpinski(n_points=5001, n_iters=20, burn_in=4)
    run = dict(w["run"], point_offset=123)
    image = dict(w["image"], lo=[0.2, 0.1], hi=[0.9, 0.7], width=97, height=61)
    a = orc.chaos_count(w["system"], run, image)
    b = orc.chaos_count_sharded(w["system"], run, image, threads=4)
    assert a["dropped"] > 0
    assert np.array_equal(a["image"], b["image"]) and a["dropped"] == b["dropped"]


def test_depth_shards_equal_whole(orc):
    w = W.menger(n_points=6000, side=200)
    near = w["image"]["near"]
    a = orc.chaos_depth(w["system"], w["run"], w["image"], near)
    b = orc.chaos_depth_sharded(w["system"], w["run"], w["image"], near, threads=5)
    assert np.array_equal(a["depth"], b["depth"])
    assert np.array_equal(a["density"], b["density"]) and a["dropped"] == b["dropped"]


def test_gauss_shards_equal_whole(orc):
    w = W.differentiable(n_points=3001, n_iters=12, burn_in=3, side=48)
    a = orc.splat_gauss(w["system"], w["run"], w["image"], 1.5)
    b = orc.splat_gauss_sharded(w["system"], w["run"], w["image"], 1.5, threads=4)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(a)
    G = np.random.default_rng(7).standard_normal((48, 48))
    ga = orc.splat_gauss_backward(w["system"], w["run"], w["image"], 1.5, G)
    gb = orc.splat_gauss_backward_sharded(w["system"], w["run"], w["image"], 1.5, G, threads=4)
    assert np.max(np.abs(ga - gb)) <= 1e-12 * np.max(np.abs(ga))
