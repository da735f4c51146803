"""Algorithmic cost of the cutting voxel projector, for roofline figures.

The operator is bound by plain VALU arithmetic (its compulsory HBM traffic,
4 (N_vox + V M N) bytes per application, is a few hundred times below what
the arithmetic takes), so its roofline is counted in FP32 VALU lane-operations
per voxel-view.  The count is fixed here, independent of any kernel, from the
steps of the method (Sec. III-A column polygons, row extents and cut volumes;
Sec. III-B elevation correction; Sec. II-F 1/r^2; eq. cvpsu sums), with a
reciprocal or square root counted as 4 and an FMA as 1:

  ops/vv = (C_COL + n_b C_BND + n_c C_COLFIN) / K      column stage, shared
         + n_c C_VOX  [+ C_VOX_RELAXED]               per voxel and column piece
         + n_p C_PIX  [+ n_e C_PIX_EC_EDGE]            per voxel and pixel

  C_COL = 36          corners of the voxel base, chi1 range of the column
  C_BND = 50 (70 EC)  one column boundary: the half-plane polygon moments
                      (area, centroid; with EC the second moments too)
  C_COLFIN = 14       one column piece: area and centroid from two prefixes,
                      depth, row scale
  C_VOX = 8           one voxel in one column piece: row position, row range,
                      coefficient
  C_VOX_RELAXED = 7   relaxed form: r^2 at the voxel centre, its reciprocal
                      and the scale, once per voxel-view
  C_PIX = 12 / 16     one (voxel, pixel) weight: row boundary, x3 extent,
                      volume, accumulation (exact form: the piece centroid's
                      height and its 1/r^2 add 4)
  C_PIX_EC_EDGE = 15  elevation correction at a top or bottom pixel of a
                      piece: the box average of the boundary (Sec. III-B)

n_c, n_p: column pieces and (voxel, pixel) weights per voxel-view; n_b = n_c
+ 1 column boundaries; n_e: pixels at the first or last row of a piece's row
range (every row of a piece of at most two rows); K: voxels sharing one column
computation, n3 by the column identity of Sec. III-A (chi1 does not depend on
x3).  estimate_counts() samples the geometry (numpy, independent of the
kernels); a CPU test checks its counts against the oracle's weights.
"""
import numpy as np

PEAK_LANE_OPS = 256 * 64 * 2.4e9   # CUs x lanes x clock: 3.93e13 lane-op/s (FP32, non-packed)

C_COL = 36.0
C_BND, C_BND_EC = 50.0, 70.0
C_COLFIN = 14.0
C_VOX = 8.0
C_VOX_RELAXED = 7.0
C_PIX_RELAXED, C_PIX_EXACT = 12.0, 16.0
C_PIX_EC_EDGE = 15.0


def ops_per_voxel_view(n_c, n_p, n_e, exact, ec, K):
    """Algorithmic FP32 VALU lane-operations per voxel-view."""
    n_b = n_c + 1.0
    col = (C_COL + n_b * (C_BND_EC if ec else C_BND) + n_c * C_COLFIN) / K
    vox = n_c * C_VOX + (0.0 if exact else C_VOX_RELAXED)
    pix = n_p * (C_PIX_EXACT if exact else C_PIX_RELAXED) + (n_e * C_PIX_EC_EDGE if ec else 0.0)
    return col + vox + pix


def estimate_counts(p, nsample=20000, seed=0):
    """Mean column pieces n_c, pixels n_p and edge pixels n_e per voxel-view,
    over voxel-views whose footprint lies on the detector: the detector
    columns the voxel base's corners span, and per column the rows between
    the top and bottom faces at the voxel centre's depth."""
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
    return float(n_c.mean()), float((n_c * n_r).mean()), float((n_c * np.minimum(n_r, 2)).mean())


def roofline(p, exact, ec, seconds_per_launch, counts=None):
    """ALU roofline figures of one operator launch (algorithmic ops per
    voxel-view times voxel-views per launch over the launch time)."""
    n_c, n_p, n_e = counts if counts is not None else estimate_counts(p)
    n1, n2, n3 = p["vol_dims"]
    vv = n1 * n2 * n3 * len(p["angles_rad"])
    ops = ops_per_voxel_view(n_c, n_p, n_e, exact, ec, n3)
    achieved = vv * ops / seconds_per_launch
    return dict(n_c=n_c, n_p=n_p, n_e=n_e, ops_per_vv=ops, voxel_views=vv,
                achieved=achieved, peak=PEAK_LANE_OPS, frac=achieved / PEAK_LANE_OPS)
