"""Pins of the oracle's composed transforms (copy semantics).

The swirl r, th -> r, th + kappa r followed by a translation t is checked in
polar form: the copy keeps the distance to the swirl centre and turns by
exactly kappa r (sign included); with kappa = 0 it is a pure translation, so
the image is the identity image shifted by t (an exact pixel shift here).
Copy semantics: the iterated point itself is unchanged by the transform, so
final positions and indices do not depend on it.
"""
import math

import numpy as np

import workloads as W


def _last_splat_world(r, image):
    sx = image["width"] / (image["hi"][0] - image["lo"][0])
    sy = image["height"] / (image["hi"][1] - image["lo"][1])
    fx = r["splats"][:, -1, 0] / sx + image["lo"][0]
    fy = r["splats"][:, -1, 1] / sy + image["lo"][1]
    return np.stack([fx, fy], axis=1)


def test_swirl_polar_form(orc):
    w = W.cfs_square(n_points=4096)
    r = orc.chaos_count(w["system"], w["run"], w["image"], want_final=True,
                        want_splats=True)
    c = np.array([0.5, 0.5])
    t = np.array([0.5, 0.5])
    kappa = 2.0
    q = _last_splat_world(r, w["image"])  # copy of p_T after the transform
    p = r["final"]
    rp = np.linalg.norm(p - c, axis=1)
    rq = np.linalg.norm(q - (c + t), axis=1)
    assert np.max(np.abs(rp - rq)) < 1e-12
    ang_p = np.arctan2(p[:, 1] - c[1], p[:, 0] - c[0])
    ang_q = np.arctan2(q[:, 1] - c[1] - t[1], q[:, 0] - c[0] - t[0])
    turn = np.mod(ang_q - ang_p - kappa * rp + math.pi, 2 * math.pi) - math.pi
    assert np.max(np.abs(turn[rp > 1e-6])) < 1e-9
    # whole image inside the window: nothing dropped, exact total
    assert r["dropped"] == 0
    assert int(r["image"].sum()) == 4096 * 24


def test_swirl_copy_semantics(orc):
    w = W.cfs_square(n_points=2048, side=256)
    plain = dict(w["system"], final_kind="identity")
    a = orc.chaos_count(w["system"], w["run"], w["image"], want_final=True,
                        want_indices=True)
    b = orc.chaos_count(plain, w["run"], w["image"], want_final=True,
                        want_indices=True)
    assert np.array_equal(a["final"], b["final"])
    assert np.array_equal(a["indices"], b["indices"])
    # per-channel totals depend only on the indices
    assert np.array_equal(a["image"].sum(axis=(1, 2)), b["image"].sum(axis=(1, 2)))


def test_swirl_kappa_zero_is_translation(orc):
    side = 256  # 128 px per unit: t = (0.5, 0.5) is a 64 px shift
    w = W.cfs_square(n_points=4096, side=side, kappa=0.0)
    sw = orc.chaos_count(w["system"], w["run"], w["image"])["image"]
    plain = dict(w["system"], final_kind="identity")
    idn = orc.chaos_count(plain, w["run"], w["image"])["image"]
    shifted = np.zeros_like(idn)
    shifted[:, 64:, 64:] = idn[:, :side - 64, :side - 64]
    assert int(idn[:, side - 64:, :].sum() + idn[:, :, side - 64:].sum()) == 0
    diff = np.abs(sw.astype(np.int64) - shifted.astype(np.int64)).sum()
    assert diff == 0


def test_stretch_special_values(orc):
    # x2 = sx x, y2 = y - sy cos x on the unit square; with sx = 2, sy = 1
    # the copy of a point at x = 0 drops by exactly 1 and x doubles.
    w = W.cfs_square(n_points=1024, side=256)
    system = dict(w["system"], final_kind="stretch",
                  final_params=np.array([2.0, 1.0] + [0.0] * 22, np.float32))
    image = {"width": 256, "height": 256, "channels": 1, "lo": [0.0, -1.0],
             "hi": [2.0, 1.0]}
    r = orc.chaos_count(system, w["run"], image, want_final=True, want_splats=True)
    q = _last_splat_world(r, image)
    p = r["final"]
    assert np.allclose(q[:, 0], 2.0 * p[:, 0], rtol=0, atol=1e-12)
    # y2 - y = -cos(x): compare with the cosine's Taylor series bounds
    dy = q[:, 1] - p[:, 1]
    x = p[:, 0]
    lower = -(1 - x**2 / 2 + x**4 / 24)
    upper = -(1 - x**2 / 2 + x**4 / 24 - x**6 / 720)
    assert np.all(dy >= lower - 1e-12) and np.all(dy <= upper + 1e-12)
