"""FP64 oracle of the TT separable-footprint projector, the footprint
projector the paper compares the cutting voxel projector with (Sec. I, the
separable footprints of Long, Fessler & Balter, IEEE TMI 29(11) 2010;
Sec. IV, the comparison; Sec. V-C, the same method on the voxel-wise GPU
structure).

TEST INFRASTRUCTURE (see the package docstring): only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use
it; it shares no code with the HIP product path.

The projector, per view and voxel, in the order of the published method:

1. transaxial footprint: the chi1 coordinates of the four corners of the
   voxel's x1x2 base, sorted, t0 <= t1 <= t2 <= t3, are the vertices of a
   trapezoid of height 1 (chi1 does not depend on x3, eq.
   columnprojectionidentity);
2. axial footprint: the chi2 coordinates of the voxel's bottom and top
   faces (x3 = z0, z1) at its nearest and farthest depth (the smallest and
   largest d.(x - s) over the base corners), sorted, are the vertices of a
   second trapezoid of height 1 (the "TT" variant; the "TR" variant takes
   one rectangle between the two faces at the depth of the voxel centre);
3. amplitude: the chord of the ray through the voxel centre across the
   voxel, taken as if the ray left through the voxel's side faces:
   min(a1 / |r1|, a2 / |r2|) |r| with r = centre - source (the method's
   amplitude from the central ray; for a1 = a2 it is a / max(|cos phi|,
   |sin phi|) / cos(theta));
4. detector blur: each footprint is integrated over the pixel, [u - 1/2,
   u + 1/2] x [v - 1/2, v + 1/2] in pixel-index units (unit width), so
   pixel (u, v) receives mu * amplitude * F1(u) * F2(v), the estimate of the
   pixel's area-averaged line integral (eq. integ).

Pixels outside the detector are dropped, as in the cutting voxel oracle.
Conventions (orbit, frames, chi2 opposite to x3, camera matrices) are those
of the package.  Parity of the footprint shapes against the authors' own TT
implementation is unpinned (the paper does not print its formulas); the
method is pinned by its parallel-beam exactness, by the exact cut integrals
and by the paper's accuracy claim against CVP (tests/test_oracle_tt.py).
"""
import math

import numpy as np

from . import frames_from_matrices

_MUTATION = 0   # planted mistakes for the pin tests (0 = none)


def set_mutation(m):
    global _MUTATION
    _MUTATION = int(m)


def trapezoid_integral(t, x0, x1):
    """Integral over [x0, x1] of the height-1 trapezoid with sorted vertices
    t[..., 0..3] (rise on [t0, t1], 1 on [t1, t2], fall on [t2, t3]):
    each linear piece clipped to the interval, integrated as its length times
    its value at the clipped midpoint."""
    t0, t1, t2, t3 = t[..., 0], t[..., 1], t[..., 2], t[..., 3]
    out = np.zeros(np.broadcast(t0, x0, x1).shape)
    lo, hi = np.maximum(x0, t0), np.minimum(x1, t1)
    ok = (hi > lo) & (t1 > t0)
    with np.errstate(divide="ignore", invalid="ignore"):
        out += np.where(ok, (hi - lo) * (0.5 * (lo + hi) - t0) / (t1 - t0), 0.0)
    out += np.maximum(np.minimum(x1, t2) - np.maximum(x0, t1), 0.0)
    lo, hi = np.maximum(x0, t2), np.minimum(x1, t3)
    ok = (hi > lo) & (t3 > t2)
    with np.errstate(divide="ignore", invalid="ignore"):
        out += np.where(ok, (hi - lo) * (t3 - 0.5 * (lo + hi)) / (t3 - t2), 0.0)
    return out


def _views(geom):
    """Per view: source s[3], e1 (x1, x2), d (x1, x2), f/b1, f/b2, c1, c2."""
    M, N = int(geom["det_cols"]), int(geom["det_rows"])
    if "matrices" in geom:
        o = np.asarray(geom.get("vol_offset_mm", (0, 0, 0)), dtype=np.float64)
        out = []
        for fr in frames_from_matrices(geom["matrices"], o):
            s1, s2, s3, e1x, e1y, dx, dy, fb1, fb2, c1, c2 = fr
            out.append((np.array([s1, s2, s3]), np.array([e1x, e1y]), np.array([dx, dy]), fb1, fb2, c1, c2))
        return out
    pp = geom.get("principal_px")
    c1, c2 = ((M - 1) / 2.0, (N - 1) / 2.0) if pp is None else (float(pp[0]), float(pp[1]))
    b1, b2 = (float(v) for v in geom["pitch_mm"])
    D, f = float(geom["sid_mm"]), float(geom["sdd_mm"])
    out = []
    for lam in np.asarray(geom["angles_rad"], dtype=np.float64):
        s = np.array([D * math.cos(lam), D * math.sin(lam), 0.0])
        e1 = np.array([-math.sin(lam), math.cos(lam)])
        d = np.array([-math.cos(lam), -math.sin(lam)])
        out.append((s, e1, d, f / b1, f / b2, c1, c2))
    return out


def _grid(geom):
    n1, n2, n3 = (int(v) for v in geom["vol_dims"])
    a = np.array(geom["voxel_mm"], dtype=np.float64)
    o = np.array(geom.get("vol_offset_mm", (0, 0, 0)), dtype=np.float64)
    lo = o - 0.5 * np.array([n1, n2, n3]) * a
    return (n1, n2, n3), a, lo


def _weights(geom, view_geom, ii, jj, kk, axial="TT"):
    """The (voxel, pixel, weight) triples of the voxels (ii[n], jj[n], kk[n])
    in one view, as flat arrays in chunks: position in the voxel list, pixel
    index v*M + u, weight."""
    _, a, lo = _grid(geom)
    M, N = int(geom["det_cols"]), int(geom["det_rows"])
    s, e1, d, fb1, fb2, c1, c2 = view_geom
    # the voxel's column (i, j): base corners, chi1 and depth
    xc1 = lo[0] + (ii + 0.5) * a[0]
    xc2 = lo[1] + (jj + 0.5) * a[1]
    chi, dep = [], []
    for q1 in (-0.5, 0.5):
        for q2 in (-0.5, 0.5):
            p1 = xc1 + q1 * a[0] - s[0]
            p2 = xc2 + q2 * a[1] - s[1]
            D = d[0] * p1 + d[1] * p2
            dep.append(D)
            chi.append(c1 + fb1 * (e1[0] * p1 + e1[1] * p2) / D)
    chi = np.stack(chi, axis=-1)                        # [n][4], corner order
    tau = chi if _MUTATION == 4 else np.sort(chi, axis=-1)
    dep = np.stack(dep, axis=-1)
    Dn, Df = dep.min(axis=-1), dep.max(axis=-1)
    Dc = d[0] * (xc1 - s[0]) + d[1] * (xc2 - s[1])
    # amplitude: chord of the central ray
    r1, r2 = xc1 - s[0], xc2 - s[1]
    with np.errstate(divide="ignore"):
        if _MUTATION == 1:
            lphi = np.maximum(a[0] / np.abs(r1), a[1] / np.abs(r2))
        else:
            lphi = np.minimum(a[0] / np.abs(r1), a[1] / np.abs(r2))
    half = 0.0 if _MUTATION == 3 else 0.5
    # the voxel's slice: bottom face z0, top face z1, centre zc
    z0 = lo[2] + kk * a[2]
    Z0 = z0 - s[2]
    Z1 = Z0 + a[2]
    zr = Z0 + 0.5 * a[2]
    if axial == "TT" and _MUTATION != 2:
        ts = np.stack([c2 - fb2 * Z1 / Dn, c2 - fb2 * Z1 / Df, c2 - fb2 * Z0 / Dn, c2 - fb2 * Z0 / Df], axis=-1)
        ts = np.sort(ts, axis=-1)                       # [n][4]
    else:   # TR: a rectangle between the faces at the centre depth
        top = c2 - fb2 * Z1 / Dc
        bot = c2 - fb2 * Z0 / Dc
        ts = np.stack([top, top, bot, bot], axis=-1)
    amp = lphi * np.sqrt(r1 ** 2 + r2 ** 2 + zr ** 2)

    ulo = np.floor(tau[:, 0] + 0.5).astype(np.int64)
    uhi = np.floor(tau[:, 3] + 0.5).astype(np.int64)
    vlo = np.floor(ts[:, 0] + 0.5).astype(np.int64)
    vhi = np.floor(ts[:, 3] + 0.5).astype(np.int64)
    if len(ii) == 0:
        return
    nu = int((uhi - ulo).max()) + 1
    nv = int((vhi - vlo).max()) + 1
    pos = np.arange(len(ii))
    # the axial factors of every row offset, then the transaxial ones
    rows = []
    for dv in range(nv):
        v = vlo + dv
        F2 = trapezoid_integral(ts, v - half, v + 1.0 - half)
        rows.append((v, amp * F2, (v <= vhi) & (v >= 0) & (v < N) & (F2 != 0.0)))
    for du in range(nu):
        u = ulo + du
        F1 = trapezoid_integral(tau, u - half, u + 1.0 - half)
        okc = (u <= uhi) & (u >= 0) & (u < M) & (F1 != 0.0)
        if not okc.any():
            continue
        for v, aF2, okv in rows:
            ok = okc & okv
            if not ok.any():
                continue
            yield pos[ok], v[ok] * M + u[ok], (aF2 * F1)[ok]


def _view_weights(geom, view_geom, axial="TT", chunk=1 << 22):
    """All (voxel, pixel, weight) triples of one view, voxels in chunks of
    whole slices: voxel index k*n2*n1 + j*n1 + i, pixel index v*M + u."""
    (n1, n2, n3), _, _ = _grid(geom)
    per = max(1, chunk // (n1 * n2))
    jj0, ii0 = np.divmod(np.arange(n1 * n2), n1)
    for k0 in range(0, n3, per):
        k1 = min(n3, k0 + per)
        kk = np.repeat(np.arange(k0, k1), n1 * n2)
        ii = np.tile(ii0, k1 - k0)
        jj = np.tile(jj0, k1 - k0)
        base = k0 * n1 * n2
        for p, pix, w in _weights(geom, view_geom, ii, jj, kk, axial):
            yield base + p, pix, w


def project(geom, x, views=None, axial="TT"):
    """b = A_TT x in FP64, [views][N][M]."""
    (n1, n2, n3), _, _ = _grid(geom)
    M, N = int(geom["det_cols"]), int(geom["det_rows"])
    vg = _views(geom)
    lo, hi = (0, len(vg)) if views is None else views
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    out = np.zeros((hi - lo, N, M))
    for q, view in enumerate(range(lo, hi)):
        acc = np.zeros(N * M)
        for vox, pix, w in _view_weights(geom, vg[view], axial):
            acc += np.bincount(pix, weights=w * x[vox], minlength=N * M)
        out[q] = acc.reshape(N, M)
    return out


def backproject(geom, b, views=None, axial="TT"):
    """x = A_TT^T b in FP64, [n3][n2][n1]; b holds the views [lo, hi)."""
    (n1, n2, n3), _, _ = _grid(geom)
    M, N = int(geom["det_cols"]), int(geom["det_rows"])
    vg = _views(geom)
    lo, hi = (0, len(vg)) if views is None else views
    b = np.asarray(b, dtype=np.float64).reshape(hi - lo, N * M)
    acc = np.zeros(n1 * n2 * n3)
    for q, view in enumerate(range(lo, hi)):
        for vox, pix, w in _view_weights(geom, vg[view], axial):
            acc += np.bincount(vox, weights=w * b[q][pix], minlength=n1 * n2 * n3)
    return acc.reshape(n3, n2, n1)


def backproject_voxels(geom, b, idx, views=None, axial="TT"):
    """(A_TT^T b) at the listed linear voxel indices (k*n2*n1 + j*n1 + i)."""
    (n1, n2, n3), _, _ = _grid(geom)
    M, N = int(geom["det_cols"]), int(geom["det_rows"])
    vg = _views(geom)
    lo, hi = (0, len(vg)) if views is None else views
    b = np.asarray(b, dtype=np.float64).reshape(hi - lo, N * M)
    idx = np.asarray(idx, dtype=np.int64)
    kk, rem = np.divmod(idx, n1 * n2)
    jj, ii = np.divmod(rem, n1)
    out = np.zeros(len(idx))
    for q, view in enumerate(range(lo, hi)):
        for p, pix, w in _weights(geom, vg[view], ii, jj, kk, axial):
            out += np.bincount(p, weights=w * b[q][pix], minlength=len(idx))
    return out
