"""Pins of the oracle's plain chaos game against closed forms.

 - invariant-measure first and second moments of affine systems from their
   linear systems (Sierpinski, square, random contractive systems);
 - the 4-map square: uniform invariant measure, channel i supported on
   quadrant i, binary-digit structure of the positions (composition order);
 - Sierpinski: address containment at depth k (brute force over all 3^k
   addresses), box-counting dimension log 3 / log 2, exact totals.
"""
import math

import numpy as np
import pytest

import workloads as W


def invariant_moments(A, b, p):
    """Mean and covariance of the invariant measure of x -> A_i x + b_i chosen
    with probability p_i: mu = (I - sum p A)^-1 sum p b and
    (I - sum p A (x) A) vec M2 = vec sum p (A mu b^T + b mu^T A^T + b b^T)."""
    A = np.asarray(A, np.float64)
    b = np.asarray(b, np.float64)
    d = b.shape[1]
    Abar = np.einsum("i,ijk->jk", p, A)
    mu = np.linalg.solve(np.eye(d) - Abar, np.einsum("i,ij->j", p, b))
    K = sum(p[i] * np.kron(A[i], A[i]) for i in range(len(p)))
    rhs = sum(p[i] * (np.outer(A[i] @ mu, b[i]) + np.outer(b[i], A[i] @ mu)
                      + np.outer(b[i], b[i])) for i in range(len(p)))
    M2 = np.linalg.solve(np.eye(d * d) - K, rhs.reshape(-1)).reshape(d, d)
    return mu, M2 - np.outer(mu, mu)


def _probs(system):
    n = system["b"].shape[0]
    return np.full(n, 1.0 / n) if system["prob"] is None else system["prob"]


def _check_moments(final, mu, cov, nsig=5.0):
    N = final.shape[0]
    m = final.mean(axis=0)
    se = final.std(axis=0) / math.sqrt(N)
    assert np.all(np.abs(m - mu) < nsig * se + 1e-12), (m, mu, se)
    d = final.shape[1]
    for a in range(d):
        for c in range(d):
            f = (final[:, a] - mu[a]) * (final[:, c] - mu[c])
            se_f = f.std() / math.sqrt(N)
            assert abs(f.mean() - cov[a, c]) < nsig * se_f, (a, c, f.mean(), cov[a, c])


def test_closed_form_moments_match_hand_values():
    w = W.sierpinski()
    mu, cov = invariant_moments(w["system"]["A"], w["system"]["b"], np.full(3, 1 / 3))
    v = np.asarray(W.SIERPINSKI_VERTICES)
    v = v.astype(np.float32).astype(np.float64)  # b stored as FP32 v/2
    assert np.allclose(mu, (0.5, np.float32(0.433) * 2 / 3), atol=1e-7)
    assert np.allclose(cov, np.cov(v.T, bias=True) / 3, atol=1e-7)
    s = W.cfs_square()
    mu, cov = invariant_moments(s["system"]["A"], s["system"]["b"], np.full(4, 0.25))
    assert np.allclose(mu, (0.5, 0.5)) and np.allclose(cov, np.eye(2) / 12)
    m = W.menger(n_points=1)
    mu, cov = invariant_moments(m["system"]["A"], m["system"]["b"], np.full(20, 0.05))
    assert np.allclose(mu, (0.5, 0.5, 0.5)) and np.allclose(cov, np.eye(3) / 10)


@pytest.mark.parametrize("name", ["sierpinski", "square", "random0", "random1", "random2"])
def test_invariant_moments(orc, name):
    if name == "sierpinski":
        w = W.sierpinski(n_points=1 << 16)
        system, run = w["system"], w["run"]
    elif name == "square":
        w = W.cfs_square(n_points=1 << 16, n_iters=64)
        system = dict(w["system"], final_kind="identity")
        run = w["run"]
    else:
        inst = W.batched(n_instances=3)[int(name[-1])]
        system = inst["system"]
        run = dict(inst["run"], n_points=1 << 16, n_iters=64)
    img = {"width": 8, "height": 8, "channels": 1, "lo": [0, 0], "hi": [1, 1]}
    r = orc.chaos_count(system, run, img, want_final=True)
    mu, cov = invariant_moments(system["A"], system["b"], _probs(system))
    _check_moments(r["final"], mu, cov)


def test_square_uniform_and_channels(orc):
    w = W.cfs_square(n_points=1 << 16, n_iters=32, burn_in=8, side=64)
    system = dict(w["system"], final_kind="identity")
    image = dict(w["image"], lo=[0, 0], hi=[1, 1])
    r = orc.chaos_count(system, w["run"], image, want_final=True)
    img = r["image"]
    N, T, B = 1 << 16, 32, 8
    assert r["dropped"] == 0 and int(img.sum()) == N * (T - B)
    # channel i (last map index i) only inside quadrant i = corner_i / 2 + [0, 1/2)^2
    for i, (cx, cy) in enumerate(W.SQUARE_CORNERS):
        q = np.zeros((64, 64), bool)
        q[int(cy) * 32:int(cy) * 32 + 32, int(cx) * 32:int(cx) * 32 + 32] = True
        assert img[i][~q].sum() == 0 and img[i][q].sum() > 0
    # final positions iid uniform on [0,1)^2: chi-square over 16x16 cells
    cells = np.floor(r["final"] * 16).astype(int)
    cnt = np.bincount(cells[:, 1] * 16 + cells[:, 0], minlength=256)
    exp = N / 256
    chi2 = float(((cnt - exp) ** 2 / exp).sum())
    assert chi2 < 255 + 6 * math.sqrt(2 * 255), chi2


def test_square_binary_digits_give_composition_order(orc):
    # p_T = f_{k_T}(... f_{k_1}(p_0)) with f_i(x) = x/2 + c_i/2, so the first k
    # binary digits of p_T.x are the x-bits of c_{k_T}, c_{k_{T-1}}, ...
    w = W.cfs_square(n_points=4096, n_iters=32, burn_in=8)
    system = dict(w["system"], final_kind="identity")
    img = {"width": 8, "height": 8, "channels": 1, "lo": [0, 0], "hi": [1, 1]}
    r = orc.chaos_count(system, w["run"], img, want_final=True, want_indices=True,
                        want_last=True)
    idx = r["indices"].astype(np.int64)
    assert np.array_equal(r["last"], r["indices"][:, -1])
    corners = np.asarray(W.SQUARE_CORNERS, np.int64)
    for k in (1, 2, 5, 12):
        digits_x = np.zeros(idx.shape[0], np.int64)
        digits_y = np.zeros(idx.shape[0], np.int64)
        for j in range(1, k + 1):
            kk = idx[:, -j]
            digits_x += corners[kk, 0] << (k - j)
            digits_y += corners[kk, 1] << (k - j)
        assert np.array_equal(np.floor(r["final"][:, 0] * 2**k).astype(np.int64), digits_x)
        assert np.array_equal(np.floor(r["final"][:, 1] * 2**k).astype(np.int64), digits_y)


def _sub_triangle(word, verts):
    """Vertices of f_{w_1} o f_{w_2} o ... (triangle) for x -> (x + v_i)/2."""
    tri = verts.copy()
    for i in reversed(word):
        tri = (tri + verts[i]) / 2.0
    return tri


def test_sierpinski_addresses_brute_force(orc):
    w = W.sierpinski(n_points=1 << 14)
    r = orc.chaos_count(w["system"], w["run"], w["image"], want_final=True,
                        want_indices=True)
    verts = (2.0 * w["system"]["b"].astype(np.float64))  # v_i = 2 b_i
    k = 5
    words = [tuple(int(c) for c in np.base_repr(a, 3).zfill(k)) for a in range(3**k)]
    tris = np.stack([_sub_triangle(wd, verts) for wd in words])  # [3^k][3][2]
    # barycentric coordinates of every final point in every depth-k triangle
    P = r["final"]
    v0, v1, v2 = tris[:, 0], tris[:, 1], tris[:, 2]
    den = (v1[:, 1] - v2[:, 1]) * (v0[:, 0] - v2[:, 0]) + (v2[:, 0] - v1[:, 0]) * (v0[:, 1] - v2[:, 1])
    l0 = ((v1[None, :, 1] - v2[None, :, 1]) * (P[:, None, 0] - v2[None, :, 0])
          + (v2[None, :, 0] - v1[None, :, 0]) * (P[:, None, 1] - v2[None, :, 1])) / den
    l1 = ((v2[None, :, 1] - v0[None, :, 1]) * (P[:, None, 0] - v2[None, :, 0])
          + (v0[None, :, 0] - v2[None, :, 0]) * (P[:, None, 1] - v2[None, :, 1])) / den
    l2 = 1 - l0 - l1
    inside = (l0 > -1e-9) & (l1 > -1e-9) & (l2 > -1e-9)
    # the address of point n is its last k indices, most recent first
    idx = r["indices"].astype(np.int64)
    addr = np.zeros(P.shape[0], np.int64)
    for j in range(k):
        addr = addr * 3 + idx[:, -1 - j]
    assert np.all(inside[np.arange(P.shape[0]), addr])
    # sub-triangles of one depth meet only at vertices: no point lies in two
    assert np.all(inside.sum(axis=1) == 1)
    # multinomial frequencies over the 3^k addresses
    cnt = np.bincount(addr, minlength=3**k)
    exp = P.shape[0] / 3**k
    chi2 = float(((cnt - exp) ** 2 / exp).sum())
    dof = 3**k - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


def test_sierpinski_box_dimension_and_totals(orc):
    w = W.sierpinski()
    r = orc.chaos_count(w["system"], w["run"], w["image"])
    img = r["image"][0]
    N, T, B = 1 << 16, 64, 16
    assert r["dropped"] == 0 and int(img.sum()) == N * (T - B)
    occ = img > 0
    xs, ys = [], []
    for s in range(3, 10):
        f = 512 // 2**s
        pooled = occ.reshape(2**s, f, 2**s, f).any(axis=(1, 3))
        xs.append(s)
        ys.append(math.log2(pooled.sum()))
    slope = np.polyfit(xs, ys, 1)[0]
    assert abs(slope - math.log(3) / math.log(2)) < 0.03, slope


def test_point_range_split_is_exact(orc):
    # the streams are keyed by global point id: two half runs sum to the whole
    w = W.cfs_square(n_points=2048, side=128)
    whole = orc.chaos_count(w["system"], w["run"], w["image"])["image"]
    a = orc.chaos_count(w["system"], dict(w["run"], n_points=1000), w["image"])["image"]
    b = orc.chaos_count(w["system"], dict(w["run"], n_points=1048, point_offset=1000),
                        w["image"])["image"]
    assert np.array_equal(whole, a + b)
