"""Algorithmic cost of the cutting voxel projector, for roofline figures.

The operator is bound by plain VALU arithmetic, so its roofline is counted in
FP32 VALU lane-operations per voxel-view (one per lane instruction; a
reciprocal counts 4 because the transcendental unit runs at quarter rate).
The count is that of the minimal per-voxel algorithm, independent of any
particular kernel:

  per voxel-view     relaxed: r^2, reciprocal, scale      7   (exact: 1)
  per column piece   Y position 3, row range 6, coef 1,
                     first row boundary C_b               10 + C_b
  per row piece      next boundary C_b, difference,
                     weight, accumulate                   C_b + 3
                     exact form: centroid height and
                     1/r^2 per piece                       +12
  column stage       FP64 polygon moments, amortised
                     over the column's n3 voxels           400 / n3 per piece
  C_b = 6 without, 24 with the elevation correction (box average).

n_c (column pieces) and n_p (row pieces) per voxel-view come from the
geometry: estimate_counts() samples voxel-views and counts the detector
columns and rows their footprint spans (numpy, independent of the kernels).
"""
import math

import numpy as np

PEAK_LANE_OPS = 256 * 64 * 2.4e9   # CUs x lanes x clock: 3.93e13 lane-op/s (FP32, non-packed)


def ops_per_voxel_view(n_c, n_p, exact, ec, n3):
    cb = 24.0 if ec else 6.0
    per_vox = 1.0 if exact else 7.0
    per_row = cb + 3.0 + (12.0 if exact else 0.0)
    return per_vox + n_c * (10.0 + cb) + n_p * per_row + n_c * 400.0 / n3


def estimate_counts(p, nsample=20000, seed=0):
    """Mean detector-column pieces and row pieces per voxel-view (voxels whose
    footprint lies on the detector)."""
    rng = np.random.default_rng(seed)
    n1, n2, n3 = p["vol_dims"]
    a1, a2, a3 = p["voxel_mm"]
    o = p.get("vol_offset_mm", (0.0, 0.0, 0.0))
    M, N = p["det_cols"], p["det_rows"]
    b1, b2 = p["pitch_mm"]
    pp = p.get("principal_px")
    c1, c2 = ((M - 1) / 2, (N - 1) / 2) if pp is None else pp
    D, f = p["sid_mm"], p["sdd_mm"]
    ang = np.asarray(p["angles_rad"])
    i = rng.integers(0, n1, nsample)
    j = rng.integers(0, n2, nsample)
    k = rng.integers(0, n3, nsample)
    lam = ang[rng.integers(0, len(ang), nsample)]
    x1 = o[0] + (i + 0.5 - n1 / 2) * a1
    x2 = o[1] + (j + 0.5 - n2 / 2) * a2
    x3 = o[2] + (k + 0.5 - n3 / 2) * a3
    cl, sl = np.cos(lam), np.sin(lam)
    s1, s2 = D * cl, D * sl
    chi = []
    for dx in (-0.5, 0.5):
        for dy in (-0.5, 0.5):
            r1, r2 = x1 + dx * a1 - s1, x2 + dy * a2 - s2
            chi.append(c1 + (f / b1) * (-sl * r1 + cl * r2) / (-cl * r1 - sl * r2))
    chi = np.array(chi)
    ulo = np.floor(chi.min(axis=0) + 0.5)
    uhi = np.floor(chi.max(axis=0) + 0.5)
    depth = -cl * (x1 - s1) - sl * (x2 - s2)
    ytop = c2 - (x3 + 0.5 * a3) * f / (b2 * depth)
    ybot = c2 - (x3 - 0.5 * a3) * f / (b2 * depth)
    vlo = np.floor(ytop + 0.5)
    vhi = np.floor(ybot + 0.5)
    on = (ulo >= 0) & (uhi < M) & (vlo >= 0) & (vhi < N)
    n_c = (uhi - ulo + 1)[on]
    n_r = (vhi - vlo + 1)[on]
    return float(n_c.mean()), float((n_c * n_r).mean())


def roofline(p, exact, ec, seconds_per_launch):
    """ALU roofline figures of one operator launch."""
    n_c, n_p = estimate_counts(p)
    n1, n2, n3 = p["vol_dims"]
    vv = n1 * n2 * n3 * len(p["angles_rad"])
    ops = ops_per_voxel_view(n_c, n_p, exact, ec, n3)
    achieved = vv * ops / seconds_per_launch
    return dict(n_c=n_c, n_p=n_p, ops_per_vv=ops, voxel_views=vv,
                achieved=achieved, peak=PEAK_LANE_OPS, frac=achieved / PEAK_LANE_OPS)
