"""Pins of the oracle's 3D chaos game (Menger sponge + twist + camera).

 - occupancy of the 3^k grid by the iterated points: exactly the 20^k cells of
   the sponge (k <= 3), never a centre or face cell; the last map index names
   the depth-1 cell (composition order);
 - the twist is a rotation about the vertical axis through the cube centre by
   kappa (y - 1/2): recovered from the depth buffer's splats by inverting the
   camera, it keeps the height and the distance to the axis and turns by that
   angle;
 - depth keys decode to depths inside the bounding sphere's depth range;
   pixels with density > 0 are exactly those with a key.
The projected image itself is parity unpinned beyond the oracle.
"""
import math

import numpy as np

import workloads as W


def test_menger_occupancy(orc):
    w = W.menger(n_points=1 << 18, side=64)
    r = orc.chaos_depth(w["system"], w["run"], w["image"], w["image"]["near"],
                        want_final=True, want_last=True)
    P = r["final"]
    allowed1 = set(W.menger_offsets())
    for k in (1, 2, 3):
        # the maps are FP32-rounded (1/3 is not exact), which moves sub-cube
        # edges by ~1e-8: points that close to a grid plane are not classified
        x = P * 3**k
        clear = np.all(np.abs(x - np.round(x)) > 1e-5, axis=1)
        cells = np.floor(x[clear]).astype(np.int64)
        assert clear.mean() > 0.99
        assert cells.min() >= 0 and cells.max() < 3**k
        occ = {tuple(c) for c in np.unique(cells, axis=0)}
        assert len(occ) == 20**k
        for c in occ:
            digits = [tuple((np.array(c) // 3**(k - 1 - j)) % 3) for j in range(k)]
            assert all(d in allowed1 for d in digits)
    # depth-1 cell of p_T is the offset of the last map applied
    offs = np.asarray(W.menger_offsets())
    x = P * 3
    clear = np.all(np.abs(x - np.round(x)) > 1e-5, axis=1)
    cell1 = np.floor(x).astype(np.int64)
    assert np.array_equal(cell1[clear], offs[r["last"]][clear])


def test_twist_and_camera_inverse(orc):
    w = W.menger(n_points=2048, side=512)
    fp = w["system"]["final_params"].astype(np.float64)
    kappa, c = fp[0], fp[1:4]
    M = fp[4:16].reshape(3, 4)
    fx, fy = fp[16], fp[17]
    r = orc.chaos_depth(w["system"], w["run"], w["image"], w["image"]["near"],
                        want_final=True, want_splats=True)
    img = w["image"]
    s = r["splats"][:, -1, :]  # last splat = copy of p_T
    ok = np.isfinite(s[:, 0])
    assert ok.mean() > 0.99
    scale = img["width"] / (img["hi"][0] - img["lo"][0])
    ndc_x = s[:, 0] / scale + img["lo"][0]
    ndc_y = s[:, 1] / scale + img["lo"][1]
    z = s[:, 2]
    v = np.stack([ndc_x * z / fx, ndc_y * z / fy, z], axis=1)
    R, tr = M[:, :3], M[:, 3]
    wv = (v - tr) @ np.linalg.inv(R).T  # twisted, centred world point
    p = r["final"] - c
    ok &= True
    assert np.allclose(wv[ok, 1], p[ok, 1], atol=1e-6)
    rad_w = np.hypot(wv[:, 0], wv[:, 2])
    rad_p = np.hypot(p[:, 0], p[:, 2])
    assert np.allclose(rad_w[ok], rad_p[ok], atol=1e-6)
    ang = np.arctan2(wv[:, 2], wv[:, 0]) - np.arctan2(p[:, 2], p[:, 0])
    turn = np.mod(ang - kappa * p[:, 1] + math.pi, 2 * math.pi) - math.pi
    sel = ok & (rad_p > 1e-3)
    assert np.max(np.abs(turn[sel])) < 1e-5


def test_depth_keys(orc):
    w = W.menger(n_points=1 << 14, side=256)
    r = orc.chaos_depth(w["system"], w["run"], w["image"], w["image"]["near"])
    depth, dens = r["depth"], r["density"]
    has = depth != np.iinfo(np.uint64).max
    assert np.array_equal(has, dens > 0)
    keys = depth[has]
    colour = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
    assert colour.max() < 20
    zb = (keys >> np.uint64(32)).astype(np.uint32)
    z = zb.view(np.float32).astype(np.float64)
    dist = np.linalg.norm(np.array([2.0, 1.5, 2.5]))
    rad = math.sqrt(3) / 2
    assert z.min() >= dist - rad - 1e-5 and z.max() <= dist + rad + 1e-5
    assert int(dens.sum()) + r["dropped"] == (1 << 14) * 16


def test_depth_image_from_splats_brute_force(orc):
    # the depth image assembled by brute force from the oracle's own splat
    # coordinates and the map index of each step (drawn by the same random
    # streams, so the count game of the untransformed system gives them):
    # drop depth <= near and pixels outside the window, key = FP32 bits of
    # the depth << 32 | index, minimum per pixel, density = splats per pixel
    w = W.menger(n_points=3000, side=64)
    run, image, near = w["run"], w["image"], w["image"]["near"]
    r = orc.chaos_depth(w["system"], run, image, near, want_splats=True)
    plain = dict(w["system"], final_kind="identity")
    idx = orc.chaos_count(plain, run, {"kind": "u32_count", "width": 4, "height": 4,
                                       "channels": 1, "lo": [0, 0], "hi": [1, 1]},
                          want_indices=True)["indices"]
    B = run["burn_in"]
    s = r["splats"].reshape(-1, 3)
    k = idx[:, B:].reshape(-1).astype(np.uint64)
    H, Wd = image["height"], image["width"]
    fin = np.isfinite(s).all(axis=1)
    z = np.where(fin, s[:, 2], 0.0)
    px = np.floor(np.where(fin, s[:, 0], -1.0)).astype(np.int64)
    py = np.floor(np.where(fin, s[:, 1], -1.0)).astype(np.int64)
    keep = fin & (z > near) & (px >= 0) & (px < Wd) & (py >= 0) & (py < H)
    zb = np.float32(z[keep]).view(np.uint32).astype(np.uint64)
    key = (zb << np.uint64(32)) | k[keep]
    flat = py[keep] * Wd + px[keep]
    depth = np.full(H * Wd, np.iinfo(np.uint64).max, np.uint64)
    np.minimum.at(depth, flat, key)
    dens = np.bincount(flat, minlength=H * Wd).astype(np.uint32)
    assert np.array_equal(depth.reshape(H, Wd), r["depth"])
    assert np.array_equal(dens.reshape(H, Wd), r["density"])
    assert r["dropped"] == int((~keep).sum())
    assert keep.mean() > 0.9
