"""Comparison helpers for GPU-vs-oracle parity (tests only)."""
from __future__ import annotations

import numpy as np


def rel_l1(got, ref):
    got = np.asarray(got, np.int64)
    ref = np.asarray(ref, np.int64)
    tot = float(ref.sum())
    return float(np.abs(got - ref).sum()) / max(tot, 1.0)


def guard_band_images(splats, channel, width, height, channels, eps_px):
    """Interval images from the oracle's FP64 splat pixel coordinates.

    splats: [..., 2] fractional pixel coordinates (NaN = dropped);
    channel: same leading shape, channel of every splat.
    Returns (sure, maybe): ``sure`` counts splats farther than eps_px from
    every pixel edge; ``maybe`` adds each remaining splat to every pixel it
    could land in with a position error of at most eps_px.  Any correct
    rounding-perturbed histogram H satisfies sure <= H <= sure + maybe.
    """
    xy = splats.reshape(-1, 2)
    ch = np.broadcast_to(channel, splats.shape[:-1]).reshape(-1).astype(np.int64)
    sure = np.zeros((channels, height, width), np.int64)
    maybe = np.zeros((channels, height, width), np.int64)
    fx, fy = xy[:, 0], xy[:, 1]
    ok = np.isfinite(fx) & np.isfinite(fy)
    fx, fy, ch = fx[ok], fy[ok], ch[ok]
    ix_lo = np.floor(fx - eps_px).astype(np.int64)
    ix_hi = np.floor(fx + eps_px).astype(np.int64)
    iy_lo = np.floor(fy - eps_px).astype(np.int64)
    iy_hi = np.floor(fy + eps_px).astype(np.int64)
    clear = (ix_lo == ix_hi) & (iy_lo == iy_hi)
    inside = (ix_lo >= 0) & (ix_lo < width) & (iy_lo >= 0) & (iy_lo < height)
    s = clear & inside
    np.add.at(sure, (ch[s], iy_lo[s], ix_lo[s]), 1)
    amb = ~clear
    for ix in (ix_lo, ix_hi):
        for iy in (iy_lo, iy_hi):
            m = amb & (ix >= 0) & (ix < width) & (iy >= 0) & (iy < height)
            # the same pixel may be listed twice when only one axis is ambiguous
            np.add.at(maybe, (ch[m], iy[m], ix[m]), 1)
    return sure, maybe


def guard_band_violations(hist, sure, maybe):
    h = np.asarray(hist, np.int64).reshape(sure.shape)
    low = int(np.count_nonzero(h < sure))
    high = int(np.count_nonzero(h > sure + maybe))
    return low, high


def depth_key_diff(got, ref):
    """Compare two u64 depth|index key images (key = FP32 bits of a positive
    depth << 32 | map index; all ones = empty).  Returns (occupied pixels,
    pixels whose keys differ, pixels whose occupancy differs, largest
    difference of the depth bits among differing occupied pixels).  Positive
    FP32 values order as their bit patterns, so one unit of the depth bits is
    one FP32 ulp of the depth."""
    g = np.asarray(got, np.uint64).reshape(-1)
    r = np.asarray(ref, np.uint64).reshape(-1)
    empty = np.uint64(0xFFFFFFFFFFFFFFFF)
    occ_g, occ_r = g != empty, r != empty
    occ_diff = int(np.count_nonzero(occ_g != occ_r))
    both = occ_g & occ_r
    diff = both & (g != r)
    gd = (g[diff] >> np.uint64(32)).astype(np.int64)
    rd = (r[diff] >> np.uint64(32)).astype(np.int64)
    ulps = int(np.max(np.abs(gd - rd))) if gd.size else 0
    return int(np.count_nonzero(occ_r)), int(np.count_nonzero(diff)), occ_diff, ulps
