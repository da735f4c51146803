"""Plain definitions that the cutting voxel projector approximates.

TEST INFRASTRUCTURE (see the package docstring).  These functions pin the
step-by-step oracle; they share no code with it:

* pixel-averaged line integrals by K x K equally spaced rays per pixel
  (the SiddonK construction of Sec. II-D; K -> infinity gives eq. integ for
  area weighting and eq. integub for unit-sphere weighting);
* the exact volume of a voxel cut by a pixel's ray pyramid and the exact
  integral of 1/r^2 over it (the quantities of eq. extinction / eq. intcut),
  by vertex enumeration, convex hull and tetrahedral quadrature;
* closed forms of the solid angle of a flat rectangular pixel, including the
  paper's spherical-quadrilateral formula (Sec. II-E).

Coordinates follow the same conventions as the oracle (circular orbit about
+x3, chi2 opposite to x3), written out again here from the definitions.  A
geometry with camera matrices (``matrices`` [views][3][4], Sec. III-C) is
used through the matrices themselves: pixel boundaries are the planes
(P_row1 - t P_row3) . [x; 1] = 0, rays run along M^-1 (chi1, chi2, 1), the
source is -M^-1 p4 (no decomposition into frames).
"""
import itertools
import math

import numpy as np


def camera(geom, view):
    """The view's camera matrix, signed so that points in front of the source
    (the volume) have a positive third homogeneous coordinate."""
    P = np.array(geom["matrices"][view], dtype=np.float64)
    n = np.array(geom["vol_dims"], dtype=np.float64)
    a = np.array(geom["voxel_mm"], dtype=np.float64)
    o = np.array(geom.get("vol_offset_mm", (0, 0, 0)), dtype=np.float64)
    if P[2] @ np.append(o, 1.0) < 0:
        P = -P
    return P


def source(geom, view):
    if "matrices" in geom:
        P = camera(geom, view)
        return -np.linalg.solve(P[:, :3], P[:, 3])
    return frame(geom, view)[0]


def frame(geom, view):
    lam = float(np.asarray(geom["angles_rad"])[view])
    D = float(geom["sid_mm"])
    s = np.array([D * math.cos(lam), D * math.sin(lam), 0.0])
    e1 = np.array([-math.sin(lam), math.cos(lam), 0.0])
    e2 = np.array([0.0, 0.0, -1.0])
    d = np.array([-math.cos(lam), -math.sin(lam), 0.0])
    return s, e1, e2, d


def principal(geom):
    pp = geom.get("principal_px")
    if pp is None:
        return (geom["det_cols"] - 1) / 2.0, (geom["det_rows"] - 1) / 2.0
    return float(pp[0]), float(pp[1])


def voxel_box(geom, i, j, k):
    n = np.array(geom["vol_dims"], dtype=np.float64)
    a = np.array(geom["voxel_mm"], dtype=np.float64)
    o = np.array(geom.get("vol_offset_mm", (0, 0, 0)), dtype=np.float64)
    lo = o - 0.5 * n * a + np.array([i, j, k]) * a
    return lo, lo + a


def detector_point(geom, view, chi1, chi2):
    """World position of detector coordinate (chi1, chi2) (pixel-index units)."""
    s, e1, e2, d = frame(geom, view)
    c1, c2 = principal(geom)
    b1, b2 = geom["pitch_mm"]
    f = float(geom["sdd_mm"])
    chi1 = np.asarray(chi1, dtype=np.float64)
    chi2 = np.asarray(chi2, dtype=np.float64)
    return (s + f * d)[None, :] + ((chi1 - c1) * b1).reshape(-1, 1) * e1[None, :] + \
        ((chi2 - c2) * b2).reshape(-1, 1) * e2[None, :]


def chord_lengths(src, dirs, lo, hi):
    """Length of each half-line src + t*dir (t >= 0, |dir| = 1) inside the box
    [lo, hi] (slab method)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / dirs
        t0 = (lo[None, :] - src[None, :]) * inv
        t1 = (hi[None, :] - src[None, :]) * inv
    tmin = np.minimum(t0, t1)
    tmax = np.maximum(t0, t1)
    # rays parallel to a slab: inside if src within the slab, else empty
    par = dirs == 0
    inside = (src[None, :] >= lo[None, :]) & (src[None, :] <= hi[None, :])
    tmin = np.where(par, np.where(inside, -np.inf, np.inf), tmin)
    tmax = np.where(par, np.where(inside, np.inf, -np.inf), tmax)
    enter = np.maximum(tmin.max(axis=1), 0.0)
    leave = tmax.min(axis=1)
    return np.maximum(leave - enter, 0.0)


def pixel_solid_angle_arctan(f, x0, x1, y0, y1):
    """Solid angle of the rectangle [x0,x1]x[y0,y1] on a plane at distance f,
    F(X,Y) = atan(XY / (f sqrt(X^2 + Y^2 + f^2)))."""
    def F(X, Y):
        return math.atan(X * Y / (f * math.sqrt(X * X + Y * Y + f * f)))
    return F(x1, y1) - F(x0, y1) - F(x1, y0) + F(x0, y0)


def pixel_solid_angle_paper(f, x0, x1, y0, y1):
    """The paper's spherical-quadrilateral area: 2 pi minus the sum of the
    angles between consecutive great-circle planes through the corner
    directions t_0..t_3 (counter-clockwise)."""
    t = [np.array([x0, y0, f]), np.array([x1, y0, f]), np.array([x1, y1, f]),
         np.array([x0, y1, f])]
    t = [v / np.linalg.norm(v) for v in t]
    acc = 0.0
    for i in range(4):
        a = np.cross(t[i], t[(i + 1) % 4])
        b = np.cross(t[(i + 1) % 4], t[(i + 2) % 4])
        c = np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b))
        acc += math.acos(max(-1.0, min(1.0, c)))
    return 2 * math.pi - acc


def pixel_edges_mm(geom, u, v):
    c1, c2 = principal(geom)
    b1, b2 = geom["pitch_mm"]
    return ((u - 0.5 - c1) * b1, (u + 0.5 - c1) * b1, (v - 0.5 - c2) * b2, (v + 0.5 - c2) * b2)


def supersample_voxel(geom, view, ijk, pixels, K, weighting="solid_angle"):
    """Pixel-averaged chord length of voxel ijk for each (u, v) in pixels,
    from K x K equally spaced rays per pixel (midpoints of a K x K grid).

    weighting 'area': plain mean over the grid points (area average, eq. integ);
    weighting 'solid_angle': each ray weighted by its solid-angle element
    f / R^3 dA, normalised by the pixel's exact solid angle (eq. integub)."""
    s, e1, e2, d = frame(geom, view)
    lo, hi = voxel_box(geom, *ijk)
    f = float(geom["sdd_mm"])
    b1, b2 = geom["pitch_mm"]
    g = (np.arange(K) + 0.5) / K - 0.5
    G1, G2 = np.meshgrid(g, g, indexing="xy")
    out = []
    for (u, v) in pixels:
        P = detector_point(geom, view, u + G1.ravel(), v + G2.ravel())
        R = P - s[None, :]
        Rn = np.linalg.norm(R, axis=1)
        L = chord_lengths(s, R / Rn[:, None], lo, hi)
        if weighting == "area":
            out.append(L.mean())
        else:
            w = f / Rn ** 3 * (b1 * b2 / (K * K))
            x0, x1, y0, y1 = pixel_edges_mm(geom, u, v)
            out.append(float(np.sum(w * L)) / pixel_solid_angle_arctan(f, x0, x1, y0, y1))
    return np.array(out)


# ------------------------------------------------------------ exact cuts

def _halfspaces(geom, view, ijk, u, v):
    """Rows (n, c) of the constraints n.x <= c describing voxel ijk cut by the
    ray pyramid of pixel (u, v)."""
    lo, hi = voxel_box(geom, *ijk)
    if "matrices" in geom:
        P = camera(geom, view)
        H = []
        for ax in range(3):
            n = np.zeros(3); n[ax] = 1.0
            H.append((n, hi[ax]))
            H.append((-n, -lo[ax]))
        # chi_r <= t  <=>  (P_r - t P_3) . [x; 1] <= 0 in front of the source
        for r, lo_t, hi_t in ((0, u - 0.5, u + 0.5), (1, v - 0.5, v + 0.5)):
            ph = P[r] - hi_t * P[2]
            H.append((ph[:3], -ph[3]))
            pl = -(P[r] - lo_t * P[2])
            H.append((pl[:3], -pl[3]))
        return H
    s, e1, e2, d = frame(geom, view)
    c1, c2 = principal(geom)
    b1, b2 = geom["pitch_mm"]
    f = float(geom["sdd_mm"])
    H = []
    for ax in range(3):
        n = np.zeros(3); n[ax] = 1.0
        H.append((n, hi[ax]))
        H.append((-n, -lo[ax]))
    # chi1 <= t  <=>  ((f/b1) e1 - (t - c1) d).(x - s) <= 0, same for chi2 with e2
    for (e, b, c, lo_t, hi_t) in ((e1, b1, c1, u - 0.5, u + 0.5), (e2, b2, c2, v - 0.5, v + 0.5)):
        nh = (f / b) * e - (hi_t - c) * d
        H.append((nh, nh @ s))
        nl = -((f / b) * e - (lo_t - c) * d)
        H.append((nl, nl @ s))
    return H


def cut_polytope(geom, view, ijk, u, v):
    """Vertices of voxel ijk intersected with the ray pyramid of pixel (u, v)
    (vertex enumeration over all plane triples)."""
    H = _halfspaces(geom, view, ijk, u, v)
    lo, hi = voxel_box(geom, *ijk)
    scale = float(np.max(hi - lo))
    pts = []
    for a, b, c in itertools.combinations(range(len(H)), 3):
        A = np.array([H[a][0], H[b][0], H[c][0]])
        if abs(np.linalg.det(A)) < 1e-12 * np.prod([np.linalg.norm(r) for r in A]):
            continue
        x = np.linalg.solve(A, np.array([H[a][1], H[b][1], H[c][1]]))
        ok = all(n @ x <= cc + 1e-9 * scale * max(1.0, np.linalg.norm(n)) for n, cc in H)
        if ok:
            pts.append(x)
    if len(pts) < 4:
        return np.zeros((0, 3))
    return np.unique(np.round(np.array(pts), 12), axis=0)


# degree-2 four-point rule on the reference tetrahedron
_TA, _TB = 0.5854101966249685, 0.1381966011250105
_TET_BARY = np.array([[_TA, _TB, _TB, _TB], [_TB, _TA, _TB, _TB],
                      [_TB, _TB, _TA, _TB], [_TB, _TB, _TB, _TA]])


def cut_integrals(geom, view, ijk, u, v):
    """(|V^(ijk)_(uv)|, integral of 1/r^2, integral of R^3/(f r^2)) over the
    voxel cut by the ray pyramid of pixel (u, v); r = |x - s| and R = f r /
    (d.(x - s)) is the distance from the source to where the ray through x
    meets the detector.  The second integral equals the solid-angle integral
    of the chord length over the pixel (eq. intcut); the third equals the
    detector-area integral of the chord length (dS = R^3/f dOmega, eq. voxat)."""
    from scipy.spatial import ConvexHull, Delaunay, QhullError
    P = cut_polytope(geom, view, ijk, u, v)
    if len(P) < 4:
        return 0.0, 0.0, 0.0
    try:
        vol = ConvexHull(P).volume
        tri = Delaunay(P)
    except QhullError:
        return 0.0, 0.0, 0.0
    if "matrices" in geom:
        s = source(geom, view)
        i_sa = 0.0
        for simp in tri.simplices:
            T = P[simp]
            tv = abs(np.linalg.det(T[1:] - T[0])) / 6.0
            q = _TET_BARY @ T - s[None, :]
            i_sa += tv * np.mean(1.0 / np.sum(q * q, axis=1))
        return vol, i_sa, float("nan")
    s, e1, e2, d = frame(geom, view)
    f = float(geom["sdd_mm"])
    i_sa = 0.0
    i_area = 0.0
    for simp in tri.simplices:
        T = P[simp]
        tv = abs(np.linalg.det(T[1:] - T[0])) / 6.0
        q = _TET_BARY @ T - s[None, :]
        r2 = np.sum(q * q, axis=1)
        depth = q @ d
        i_sa += tv * np.mean(1.0 / r2)
        i_area += tv * np.mean(f * f * np.sqrt(r2) / depth ** 3)
    return vol, i_sa, i_area


def voxel_definition(geom, view, ijk, pixels, weighting="solid_angle"):
    """Exact pixel-averaged extinction of a unit-attenuation voxel: the
    solid-angle average (eq. integub) or the area average (eq. integ) of the
    chord length, through the exact cut integrals."""
    f = float(geom["sdd_mm"])
    b1, b2 = geom["pitch_mm"]
    out = []
    for (u, v) in pixels:
        vol, i_sa, i_area = cut_integrals(geom, view, ijk, u, v)
        if weighting == "area":
            out.append(i_area / (b1 * b2))
        else:
            x0, x1, y0, y1 = pixel_edges_mm(geom, u, v)
            out.append(i_sa / pixel_solid_angle_arctan(f, x0, x1, y0, y1))
    return np.array(out)


# ------------------------------------------------------------ SiddonK on volumes

def siddon_project(geom, x, K, views=None):
    """SiddonK projection of a whole volume (Sec. II-D): for every pixel the
    mean over K x K rays (towards the midpoints of a K x K grid of equal
    cells on the pixel) of the line integral of mu, each line integral the
    sum over voxels of mu times the exact chord length (slab method, every
    voxel tested; no traversal).  x: [n3][n2][n1].  Returns [views][N][M]
    in FP64.  Brute force over voxels x rays: for tiny grids only."""
    x = np.asarray(x, dtype=np.float64)
    n3, n2, n1 = x.shape
    nz = np.argwhere(x != 0.0)                       # (k, j, i) of non-zero voxels
    mu = x[nz[:, 0], nz[:, 1], nz[:, 2]]
    a = np.array(geom["voxel_mm"], dtype=np.float64)
    o = np.array(geom.get("vol_offset_mm", (0, 0, 0)), dtype=np.float64)
    base = o - 0.5 * np.array([n1, n2, n3]) * a
    lo = base[None, :] + nz[:, ::-1] * a[None, :]    # (i, j, k) order -> x1, x2, x3
    hi = lo + a[None, :]
    M, N = int(geom["det_cols"]), int(geom["det_rows"])
    V = len(geom["angles_rad"])
    views = range(V) if views is None else range(*views)
    g = (np.arange(K) + 0.5) / K - 0.5
    G1, G2 = np.meshgrid(g, g, indexing="xy")
    out = np.zeros((len(views), N, M))
    for vi, view in enumerate(views):
        s = frame(geom, view)[0]
        for v in range(N):
            for u in range(M):
                P = detector_point(geom, view, u + G1.ravel(), v + G2.ravel())
                R = P - s[None, :]
                dirs = R / np.linalg.norm(R, axis=1)[:, None]
                # chord of every ray in every voxel box: (rays, voxels)
                with np.errstate(divide="ignore", invalid="ignore"):
                    inv = 1.0 / dirs
                    t0 = (lo[None, :, :] - s[None, None, :]) * inv[:, None, :]
                    t1 = (hi[None, :, :] - s[None, None, :]) * inv[:, None, :]
                tmin = np.minimum(t0, t1)
                tmax = np.maximum(t0, t1)
                par = (dirs == 0)[:, None, :]
                inside = (s[None, None, :] >= lo[None, :, :]) & (s[None, None, :] <= hi[None, :, :])
                tmin = np.where(par, np.where(inside, -np.inf, np.inf), tmin)
                tmax = np.where(par, np.where(inside, np.inf, -np.inf), tmax)
                enter = np.maximum(tmin.max(axis=2), 0.0)
                leave = tmax.min(axis=2)
                L = np.maximum(leave - enter, 0.0)
                out[vi, v, u] = float(np.sum(L @ mu)) / (K * K)
    return out


def pixel_solid_angle_matrix(geom, view, u, v):
    """Solid angle of pixel (u, v) seen from the source of a camera-matrix
    view: the spherical quadrilateral spanned by the rays through the pixel's
    corners, M^-1 (u +- 1/2, v +- 1/2, 1) (the paper's formula: 2 pi minus
    the angles between consecutive great-circle planes)."""
    P = camera(geom, view)
    Minv = np.linalg.inv(P[:, :3])
    t = [Minv @ np.array([u + du, v + dv, 1.0]) for du, dv in ((-0.5, -0.5), (0.5, -0.5), (0.5, 0.5), (-0.5, 0.5))]
    t = [x / np.linalg.norm(x) for x in t]
    acc = 0.0
    for i in range(4):
        a = np.cross(t[i], t[(i + 1) % 4])
        b = np.cross(t[(i + 1) % 4], t[(i + 2) % 4])
        c = np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b))
        acc += math.acos(max(-1.0, min(1.0, c)))
    return 2 * math.pi - acc
