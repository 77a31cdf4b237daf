"""Pins of the two composition modes of Section 3 (the composition figure:
the transform applied to a copy of the point, or the transformed point fed
back into the iteration).

 - with the identity transform both modes are the same computation;
 - reuse of a linear transform G (the stretch with no cosine term) is the
   chaos game of the affine maps G A_k, G b_k in copy mode;
 - reuse of a pure translation t (the swirl with kappa = 0) is the chaos
   game of the maps A_k, b_k + t;
 - for Sierpinski-type maps x/2 + c_k fed back through x -> x + t the
   invariant measure has the mean 2 (mean(c) + t) (fixed point of the mean
   recursion m = m/2 + mean(c) + t).
"""
import math

import numpy as np

import workloads as W

IMG = {"width": 64, "height": 64, "channels": 1, "lo": [-4, -4], "hi": [4, 4]}


def _sys(A, b, final_kind="identity", fp=(), compose="copy", kind=None):
    return W._system(A, b, final_kind=final_kind, final_params=fp, compose=compose, kind=kind)


def _maps(seed=3, n=4):
    rng = np.random.default_rng(seed)
    A, b = W.random_affine_maps(rng, n)
    return np.asarray(A, np.float32), np.asarray(b, np.float32)


def test_reuse_identity_is_copy(orc):
    A, b = _maps()
    run = W._run(2048, 24, 4, seed=5)
    a = orc.chaos_count(_sys(A, b), run, IMG, want_final=True)
    c = orc.chaos_count(_sys(A, b, compose="reuse"), run, IMG, want_final=True)
    assert np.array_equal(a["image"], c["image"])
    assert np.array_equal(a["final"], c["final"])


def test_reuse_linear_stretch_is_affine(orc):
    A, b = _maps(seed=4)
    # a power-of-two factor keeps the products G A_k, G b_k exact in float32
    sx = np.float32(0.5)
    G = np.diag([sx, np.float32(1)]).astype(np.float32)
    A2 = np.einsum("ij,kjl->kil", G, A).astype(np.float32)
    b2 = (b @ G.T).astype(np.float32)
    assert np.array_equal(A2.astype(np.float64), np.einsum("ij,kjl->kil", G.astype(np.float64),
                                                           A.astype(np.float64)))
    run = W._run(2048, 24, 4, seed=6)
    reuse = orc.chaos_count(_sys(A, b, "stretch", (sx, 0.0), "reuse"), run, IMG,
                            want_final=True)
    ref = orc.chaos_count(_sys(A2, b2), run, IMG, want_final=True)
    assert np.max(np.abs(reuse["final"] - ref["final"])) < 1e-12
    assert abs(int(reuse["image"].sum()) - int(ref["image"].sum())) <= 2
    assert np.abs(reuse["image"].astype(np.int64) - ref["image"]).sum() <= 8


def test_reuse_translation_is_shifted_maps(orc):
    A, b = _maps(seed=5)
    # offsets on a 2^-16 grid, so that b + t is exact in float32
    b = (np.round(b.astype(np.float64) * 65536) / 65536).astype(np.float32)
    t = np.array([0.25, -0.125], np.float32)
    run = W._run(2048, 24, 4, seed=7)
    reuse = orc.chaos_count(_sys(A, b, "swirl", (0.0, 0.0, 0.0, t[0], t[1]), "reuse"), run,
                            IMG, want_final=True)
    ref = orc.chaos_count(_sys(A, (b + t).astype(np.float32)), run, IMG, want_final=True)
    assert np.max(np.abs(reuse["final"] - ref["final"])) < 1e-12


def test_reuse_translation_mean_closed_form(orc):
    w = W.sierpinski(n_points=1 << 15, n_iters=40, burn_in=39)
    s = w["system"]
    t = (0.125, 0.0625)
    sys = _sys(s["A"], s["b"], "swirl", (0.0, 0.0, 0.0) + t, "reuse")
    r = orc.chaos_count(sys, w["run"], IMG, want_final=True)
    P = r["final"]
    cbar = np.asarray(s["b"], np.float64).mean(axis=0)
    want = 2.0 * (cbar + np.asarray(t))
    # the stationary law has per-coordinate variance below (extent)^2 / 4
    N = P.shape[0]
    for c in range(2):
        assert abs(P[:, c].mean() - want[c]) < 6 * 0.5 / math.sqrt(N)


def test_copy_and_reuse_differ_for_circle(orc):
    """The composition figure's point: with the swirl as the transform the
    two modes give different pictures (copy keeps the disk's area; reuse
    does not), while the identity gives the same one."""
    a = W.composed_circle("copy", n_points=1 << 14)
    c = W.composed_circle("reuse", n_points=1 << 14)
    ra = orc.chaos_count(a["system"], a["run"], a["image"], want_final=True)
    rc = orc.chaos_count(c["system"], c["run"], c["image"], want_final=True)
    # a swirl about the origin keeps |q|, so copy mode keeps the uniform disk's radii
    ua = (ra["final"] ** 2).sum(axis=1)
    assert np.all(ua < 1.0)
    assert not np.array_equal(ra["image"], rc["image"])
