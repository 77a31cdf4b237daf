"""Pins of the oracle's circle map (the paper's circle equation, under the
reading that swaps the two uniform coordinates u = r^2 and v = angle / 2 pi).

 - the uniform measure on the unit disk is invariant: r^2 and angle / 2 pi
   are independent U[0, 1) after many steps (moments, chi-square);
 - map f sends the disk onto its upper (f = 0) or lower (f = 1) half;
 - composition order: the binary digits of angle / 2 pi are the indices
   f_T, f_{T-2}, f_{T-4}, ... and those of r^2 are f_{T-1}, f_{T-3}, ...
"""
import math

import numpy as np

import workloads as W


def _run_circle(orc, n=1 << 15, T=48):
    w = W.circle(n_points=n, n_iters=T, burn_in=T - 1)
    img = {"width": 8, "height": 8, "channels": 1, "lo": [-1, -1], "hi": [1, 1]}
    r = orc.chaos_count(w["system"], w["run"], img, want_final=True, want_indices=True,
                        want_last=True)
    P = r["final"]
    u = P[:, 0] ** 2 + P[:, 1] ** 2
    v = np.mod(np.arctan2(P[:, 1], P[:, 0]), 2 * math.pi) / (2 * math.pi)
    return r, u, v


def test_circle_invariant_uniform_disk(orc):
    r, u, v = _run_circle(orc)
    N = u.size
    assert np.all(u < 1.0)
    for x in (u, v):
        assert abs(x.mean() - 0.5) < 5 * math.sqrt(1 / 12 / N)
        assert abs(x.var() - 1 / 12) < 5 * math.sqrt((1 / 80 - 1 / 144) / N)
    assert abs(np.mean(u < 0.25) - 0.25) < 5 * math.sqrt(0.25 * 0.75 / N)  # P(r < 1/2)
    cells = np.floor(u * 8).astype(int) * 8 + np.floor(v * 8).astype(int)
    cnt = np.bincount(cells, minlength=64)
    exp = N / 64
    chi2 = float(((cnt - exp) ** 2 / exp).sum())
    assert chi2 < 63 + 6 * math.sqrt(2 * 63)


def test_circle_half_disk_per_index(orc):
    r, u, v = _run_circle(orc, n=4096)
    P, last = r["final"], r["last"]
    assert np.all(P[last == 0, 1] >= -1e-15)
    assert np.all(P[last == 1, 1] <= 1e-15)


def test_circle_composition_digits(orc):
    r, u, v = _run_circle(orc, n=4096)
    idx = r["indices"].astype(np.int64)
    k = 10
    dv = np.zeros(idx.shape[0], np.int64)
    du = np.zeros(idx.shape[0], np.int64)
    for j in range(k):
        dv = dv * 2 + idx[:, -1 - 2 * j]
        du = du * 2 + idx[:, -2 - 2 * j]
    got_v = np.floor(v * 2**k).astype(np.int64)
    got_u = np.floor(u * 2**k).astype(np.int64)
    # points within rounding of a dyadic cell edge are not classified
    clear = (np.abs(v * 2**k - np.round(v * 2**k)) > 1e-6) & \
            (np.abs(u * 2**k - np.round(u * 2**k)) > 1e-6)
    assert clear.mean() > 0.99
    assert np.array_equal(got_v[clear], dv[clear])
    assert np.array_equal(got_u[clear], du[clear])


def test_mixed_kinds_accepted(orc):
    w = W.circle(n_points=256, extra_affine=2)
    img = {"width": 16, "height": 16, "channels": 4, "lo": [-1, -1], "hi": [1, 1]}
    r = orc.chaos_count(w["system"], w["run"], img, want_indices=True)
    assert set(np.unique(r["indices"])) == {0, 1, 2, 3}
