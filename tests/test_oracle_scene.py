"""Pins of the oracle's multiple-objects form (Section 3, several objects from
one primitive).

 - one object with the identity placement and no copies is the plain chaos
   game with that object's transform (images equal bit for bit);
 - the ring transform sends the uniform disk to the uniform annulus: the
   squared radius is U[r_in^2, r_out^2) and the angle U[0, 2 pi);
 - a placement q -> s R q + t of the uniform disk has mean t and
   E|q - t|^2 = s^2 / 2;
 - duplication: every splat lies in the disk of radius scale_c around
   offset_c of one copy c, and the copies are hit uniformly (chi-square),
   also for a second duplicated object (the odd-multiplier draw);
 - totals: splats + dropped = N (T - B) per object.
"""
import math

import numpy as np
import pytest

import workloads as W

PLAIN_IMG = {"width": 96, "height": 96, "channels": 1, "lo": [-1.5, -1.5], "hi": [1.5, 1.5]}


@pytest.mark.parametrize("kind,params", [("identity", ()), ("swirl", (0.1, -0.2, 3.0, 0.1, 0.0)),
                                         ("stretch", (0.75, 0.25)), ("ring", (0.5, 1.0))])
def test_single_object_is_plain_chaos_game(orc, kind, params):
    w = W.circle(n_points=2048, n_iters=20, burn_in=4, extra_affine=1)
    s = dict(w["system"])
    scene = orc.chaos_scene(s, [{"final_kind": kind, "final_params": params}], w["run"],
                            PLAIN_IMG)
    s2 = W._system(s["A"], s["b"], kind=s["kind"], final_kind=kind, final_params=params)
    plain = orc.chaos_count(s2, w["run"], PLAIN_IMG)
    assert np.array_equal(scene["image"], plain["image"])
    assert scene["dropped"] == plain["dropped"]


def test_ring_uniform_annulus(orc):
    ri, ro = 0.4, 0.9
    w = W.circle(n_points=1 << 14, n_iters=40, burn_in=32)
    r = orc.chaos_scene(w["system"], [{"final_kind": "ring", "final_params": (ri, ro)}],
                        w["run"], PLAIN_IMG, want_splats=True)
    q = r["splats"][:, -1, 0, :]          # one splat per point: independent samples
    R2 = (q ** 2).sum(axis=1)
    N = R2.size
    assert R2.min() >= ri * ri * (1 - 1e-12) and R2.max() < ro * ro
    mean, var = (ri * ri + ro * ro) / 2, (ro * ro - ri * ri) ** 2 / 12
    assert abs(R2.mean() - mean) < 5 * math.sqrt(var / N)
    ang = np.mod(np.arctan2(q[:, 1], q[:, 0]), 2 * math.pi) / (2 * math.pi)
    assert abs(ang.mean() - 0.5) < 5 * math.sqrt(1 / 12 / N)
    cnt = np.bincount(np.floor(ang * 16).astype(int), minlength=16)
    chi2 = float(((cnt - N / 16) ** 2 / (N / 16)).sum())
    assert chi2 < 15 + 6 * math.sqrt(30)


def test_placement_moments(orc):
    s, ang, t = 0.3, 0.7, (0.25, -0.5)
    w = W.circle(n_points=1 << 14, n_iters=40, burn_in=32)
    ob = {"final_kind": "identity", "place": W._place(s, ang, *t)}
    r = orc.chaos_scene(w["system"], [ob], w["run"], PLAIN_IMG, want_splats=True)
    q = r["splats"][:, -1, 0, :]
    N = q.shape[0]
    d = q - np.asarray(t)
    # uniform disk of radius s: E[x] = 0, Var[x] = s^2 / 4 per axis, E|d|^2 = s^2 / 2
    for c in range(2):
        assert abs(d[:, c].mean()) < 5 * math.sqrt(s * s / 4 / N)
    r2 = (d ** 2).sum(axis=1)
    assert r2.max() <= s * s * (1 + 1e-9)
    assert abs(r2.mean() - s * s / 2) < 5 * math.sqrt(s ** 4 / 12 / N)


def _copy_places(orc, seed, n_copies, obj_index, lo, hi, scale, instance=0):
    ctrs = np.zeros((n_copies, 4), np.uint32)
    ctrs[:, 0] = np.arange(n_copies)
    ctrs[:, 1] = obj_index
    ctrs[:, 2] = instance
    ctrs[:, 3] = 3
    wds = orc.philox_many(seed, ctrs)
    e = (wds[:, :3] >> 8).astype(np.float64) * 2.0 ** -24
    lo = np.asarray(lo, np.float32).astype(np.float64)
    span = (np.asarray(hi, np.float32) - np.asarray(lo, np.float32)).astype(np.float64)
    off = lo + span * e[:, :2]
    sc = np.float64(np.float32(scale[0])) + np.float64(np.float32(scale[1] - scale[0])) * e[:, 2]
    return off, sc


def test_duplication_copies_and_uniform_draw(orc):
    nc = 16
    w = W.circle(n_points=1 << 13, n_iters=24, burn_in=8)
    objs = [
        {"final_kind": "identity", "channel": 0},
        {"final_kind": "identity", "n_copies": nc, "copy_lo": (-1.2, -1.2),
         "copy_hi": (1.2, 1.2), "scale": (0.004, 0.008), "channel": 0},
        {"final_kind": "swirl", "final_params": (0, 0, 2.0, 0, 0), "n_copies": nc,
         "copy_lo": (-1.2, -1.2), "copy_hi": (1.2, 1.2), "scale": (0.002, 0.005), "channel": 0},
    ]
    r = orc.chaos_scene(w["system"], objs, w["run"], PLAIN_IMG, want_splats=True)
    N, T_rec = w["run"]["n_points"], w["run"]["n_iters"] - w["run"]["burn_in"]
    assert int(r["image"].sum()) + r["dropped"] == N * T_rec * len(objs)
    for o in (1, 2):
        off, sc = _copy_places(orc, w["run"]["seed"], nc, o, objs[o]["copy_lo"],
                               objs[o]["copy_hi"], objs[o]["scale"])
        dmin = min(np.linalg.norm(off[i] - off[j]) for i in range(nc) for j in range(i))
        assert dmin > 2 * sc.max()      # the copies do not overlap for this seed
        q = r["splats"][:, :, o, :].reshape(-1, 2)
        dist = np.linalg.norm(q[:, None, :] - off[None, :, :], axis=2)
        c = dist.argmin(axis=1)
        assert np.all(dist[np.arange(c.size), c] <= sc[c] * (1 + 1e-9))
        cnt = np.bincount(c, minlength=nc)
        exp = c.size / nc
        chi2 = float(((cnt - exp) ** 2 / exp).sum())
        assert chi2 < (nc - 1) + 6 * math.sqrt(2 * (nc - 1))


def test_space_scene_totals(orc):
    w = W.space_scene(n_points=2048)
    r = orc.chaos_scene(w["system"], w["objects"], w["run"], w["image"])
    N, T_rec = w["run"]["n_points"], w["run"]["n_iters"] - w["run"]["burn_in"]
    per = r["image"].sum(axis=(1, 2))
    assert int(per.sum()) + r["dropped"] == N * T_rec * 4
    for ch in (0, 1, 3):            # planet, rings and comet are fully in frame
        assert per[ch] == N * T_rec
