"""FP64 CPU oracle of the cutting voxel projector (CVP).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP product path and never imports it.

Two parts:

* the paper's algorithm step by step in FP64 (``cvp_oracle.c`` through
  ctypes: :func:`project`, :func:`backproject`, :func:`voxel_weights`, ...);
* plain definitions that CVP approximates, used only to pin the first part
  (``definition.py``: ray supersampling, exact polyhedral cut volumes,
  closed-form pixel solid angles);
* the solvers run on these operators (``cgls.py``, ``lsqr.py``,
  ``sart.py``) and the TT separable-footprint projector the paper compares
  CVP with (``tt.py``).

Geometry is passed as a plain dict with the keys of :data:`GEOM_KEYS`, or,
for a general trajectory (Sec. III-C: one camera matrix per view), with
``matrices`` ([views][3][4], world mm -> homogeneous pixel-index coordinates)
in place of the orbit keys; the matrices are taken apart here (RQ
decomposition) into each view's frame and intrinsics.
"""
import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libcvp_oracle.so")
_lib = None

GEOM_KEYS = ("vol_dims", "voxel_mm", "vol_offset_mm", "det_cols", "det_rows",
             "pitch_mm", "principal_px", "sid_mm", "sdd_mm", "angles_rad")


class _Geom(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("n3", ctypes.c_int32),
                ("a1", ctypes.c_double), ("a2", ctypes.c_double), ("a3", ctypes.c_double),
                ("o1", ctypes.c_double), ("o2", ctypes.c_double), ("o3", ctypes.c_double),
                ("ncols", ctypes.c_int32), ("nrows", ctypes.c_int32),
                ("b1", ctypes.c_double), ("b2", ctypes.c_double),
                ("c1", ctypes.c_double), ("c2", ctypes.c_double),
                ("sid", ctypes.c_double), ("sdd", ctypes.c_double),
                ("nviews", ctypes.c_int32),
                ("angles", ctypes.POINTER(ctypes.c_double)),
                ("frames", ctypes.POINTER(ctypes.c_double))]


class _Opts(ctypes.Structure):
    _fields_ = [("exact", ctypes.c_int32), ("ec", ctypes.c_int32),
                ("scaling", ctypes.c_int32), ("raw_volume", ctypes.c_int32)]


class _Piece(ctypes.Structure):
    _fields_ = [("u", ctypes.c_int32), ("area", ctypes.c_double),
                ("cm1", ctypes.c_double), ("cm2", ctypes.c_double),
                ("depth", ctypes.c_double), ("h", ctypes.c_double)]


SCALINGS = {"solid_angle": 0, "cos": 1, "none": 2}


@dataclass
class Options:
    """exact: r at the cut centroid (else at the voxel centre, the relaxed
    form); ec: elevation correction; scaling: 'solid_angle' (eq. cvpus),
    'cos' (eq. cvp) or 'none'; raw_volume: weight = cut volume."""
    exact: bool = True
    ec: bool = True
    scaling: str = "solid_angle"
    raw_volume: bool = False

    def _c(self):
        return _Opts(int(self.exact), int(self.ec), SCALINGS[self.scaling],
                     int(self.raw_volume))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or (
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(os.path.join(HERE, "cvp_oracle.c"))):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        G, O = ctypes.POINTER(_Geom), ctypes.POINTER(_Opts)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        lp = ctypes.POINTER(ctypes.c_int64)
        L.orc_project.argtypes = [G, O, dp, dp, ctypes.c_int, ctypes.c_int]
        L.orc_backproject.argtypes = [G, O, dp, dp, ctypes.c_int, ctypes.c_int]
        L.orc_backproject_voxels.argtypes = [G, O, dp, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int64, lp, dp]
        L.orc_voxel_weights.argtypes = [G, O, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, ip, ip, dp, ctypes.c_int]
        L.orc_column_pieces.argtypes = [G, O, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(_Piece), ctypes.c_int]
        L.orc_row_length.argtypes = [G, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_row_length.restype = ctypes.c_double
        L.orc_pixel_scale.argtypes = [G, ctypes.c_int, dp]
        L.orc_pixel_scale_view.argtypes = [G, ctypes.c_int, ctypes.c_int, dp]
        L.orc_pixel_solid_angle.argtypes = [G, ctypes.c_int, ctypes.c_int]
        L.orc_pixel_solid_angle.restype = ctypes.c_double
        L.orc_project_point.argtypes = [G, ctypes.c_int, dp, dp]
        L.orc_view_frame.argtypes = [G, ctypes.c_int, dp, dp, dp, dp]
        L.orc_set_mutation.argtypes = [ctypes.c_int]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def frames_from_matrices(P, centre, tol=1e-9):
    """Per-view frames of camera matrices P [V][3][4] (x~ = P [x; 1] in
    homogeneous pixel-index coordinates): M = K R by RQ decomposition (K
    upper triangular with a positive diagonal, R orthogonal), the source s =
    -M^-1 p4, and the sign of P fixed so that the volume centre (in front of
    the source) has positive depth.  The convention of Sec. III-A is required: rows e1
    and d of R horizontal, e2 = (0, 0, -1) (chi2 opposite to x3), no skew.
    Returns [V][11]: s1, s2, s3, e1x, e1y, dx, dy, f/b1, f/b2, c1, c2."""
    from scipy.linalg import rq
    P = np.asarray(P, dtype=np.float64)
    out = np.zeros((len(P), 11))
    for v, Pv in enumerate(P):
        if Pv[2] @ np.append(centre, 1.0) < 0:
            Pv = -Pv
        Mv, p4 = Pv[:, :3], Pv[:, 3]
        s = -np.linalg.solve(Mv, p4)
        K, R = rq(Mv)
        D = np.diag(np.sign(np.diag(K)))
        K, R = K @ D, D @ R                 # positive diagonal of K
        if K[2, 2] < 0:
            raise ValueError("view %d: degenerate camera matrix" % v)
        K = K / K[2, 2]
        e1, e2, d = R
        if (abs(e1[2]) > tol or abs(d[2]) > tol or abs(e2[2] + 1.0) > tol
                or abs(K[0, 1]) > tol * K[0, 0]):
            raise ValueError("view %d: chi1 must not depend on x3 and chi2 must run opposite to x3 "
                             "(Sec. III-A convention)" % v)
        out[v] = (s[0], s[1], s[2], e1[0], e1[1], d[0], d[1], K[0, 0], K[1, 1], K[0, 2], K[1, 2])
    return out


class Geometry:
    """Oracle-side geometry built from a plain parameter dict."""

    def __init__(self, p):
        self.p = dict(p)
        n1, n2, n3 = (int(v) for v in p["vol_dims"])
        a1, a2, a3 = (float(v) for v in p["voxel_mm"])
        o = p.get("vol_offset_mm", (0.0, 0.0, 0.0))
        M, N = int(p["det_cols"]), int(p["det_rows"])
        if "matrices" in p:
            self.frames = np.ascontiguousarray(frames_from_matrices(p["matrices"], np.asarray(o, dtype=np.float64)))
            nv = len(self.frames)
            self.angles = np.zeros(nv)
            b1 = b2 = c1 = c2 = sid = sdd = 0.0      # unused: every view has its frame
            fp = _dptr(self.frames)
        else:
            b1, b2 = (float(v) for v in p["pitch_mm"])
            pp = p.get("principal_px")
            c1, c2 = ((M - 1) / 2.0, (N - 1) / 2.0) if pp is None else (float(pp[0]), float(pp[1]))
            self.angles = np.ascontiguousarray(np.asarray(p["angles_rad"], dtype=np.float64))
            sid, sdd = float(p["sid_mm"]), float(p["sdd_mm"])
            fp = ctypes.POINTER(ctypes.c_double)()
        self.c = _Geom(n1, n2, n3, a1, a2, a3, float(o[0]), float(o[1]), float(o[2]),
                       M, N, b1, b2, c1, c2, sid, sdd,
                       len(self.angles), _dptr(self.angles), fp)
        self.vol_shape = (n3, n2, n1)
        self.nviews = len(self.angles)
        self.proj_shape = (self.nviews, N, M)

    def ref(self):
        return ctypes.byref(self.c)


def _geom(g):
    return g if isinstance(g, Geometry) else Geometry(g)


def project(geom, opts: Options, x, views=None):
    """b = A x (FP64) for views [lo, hi) (default: all)."""
    g = _geom(geom)
    lo, hi = (0, g.nviews) if views is None else views
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(g.vol_shape))
    b = np.zeros((hi - lo,) + g.proj_shape[1:], dtype=np.float64)
    rc = lib().orc_project(g.ref(), ctypes.byref(opts._c()), _dptr(x), _dptr(b), lo, hi)
    if rc != 0:
        raise RuntimeError("orc_project failed: %d" % rc)
    return b


def backproject(geom, opts: Options, b, views=None):
    """x = A^T b (FP64); b holds the views [lo, hi)."""
    g = _geom(geom)
    lo, hi = (0, g.nviews) if views is None else views
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape((hi - lo,) + g.proj_shape[1:]))
    x = np.zeros(g.vol_shape, dtype=np.float64)
    rc = lib().orc_backproject(g.ref(), ctypes.byref(opts._c()), _dptr(b), _dptr(x), lo, hi)
    if rc != 0:
        raise RuntimeError("orc_backproject failed: %d" % rc)
    return x


def backproject_voxels(geom, opts: Options, b, idx, views=None):
    """(A^T b) at the listed linear voxel indices."""
    g = _geom(geom)
    lo, hi = (0, g.nviews) if views is None else views
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape((hi - lo,) + g.proj_shape[1:]))
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    out = np.zeros(len(idx), dtype=np.float64)
    rc = lib().orc_backproject_voxels(g.ref(), ctypes.byref(opts._c()), _dptr(b), lo, hi,
                                      len(idx), idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      _dptr(out))
    if rc != 0:
        raise RuntimeError("orc_backproject_voxels failed: %d" % rc)
    return out


def voxel_weights(geom, opts: Options, view, i, j, k, max_out=4096):
    """(u, v, w) arrays: voxel (i,j,k)'s weights in S (no mu, no pixel scale)."""
    g = _geom(geom)
    us = np.zeros(max_out, np.int32)
    vs = np.zeros(max_out, np.int32)
    ws = np.zeros(max_out, np.float64)
    n = lib().orc_voxel_weights(g.ref(), ctypes.byref(opts._c()), view, i, j, k,
                                us.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                vs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                _dptr(ws), max_out)
    if n < 0:
        raise RuntimeError("orc_voxel_weights overflow")
    return us[:n].copy(), vs[:n].copy(), ws[:n].copy()


def column_pieces(geom, opts: Options, view, i, j):
    """List of dicts (u, area, cm1, cm2, depth, h) for column (i,j)."""
    g = _geom(geom)
    arr = (_Piece * 64)()
    n = lib().orc_column_pieces(g.ref(), ctypes.byref(opts._c()), view, i, j, arr, 64)
    if n < 0:
        raise RuntimeError("orc_column_pieces overflow")
    return [dict(u=arr[q].u, area=arr[q].area, cm1=arr[q].cm1, cm2=arr[q].cm2,
                 depth=arr[q].depth, h=arr[q].h) for q in range(n)]


def row_length(geom, s3, v, depth, h, z0, z1, view=0):
    g = _geom(geom)
    return lib().orc_row_length(g.ref(), view, s3, v, depth, h, z0, z1)


def pixel_scale(geom, scaling, view=0):
    g = _geom(geom)
    out = np.zeros(g.proj_shape[1:], np.float64)
    lib().orc_pixel_scale_view(g.ref(), view, SCALINGS[scaling], _dptr(out))
    return out


def pixel_solid_angle(geom, u, v):
    g = _geom(geom)
    return lib().orc_pixel_solid_angle(g.ref(), u, v)


def project_point(geom, view, x):
    g = _geom(geom)
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    chi = np.zeros(2)
    lib().orc_project_point(g.ref(), view, _dptr(x), _dptr(chi))
    return chi


def view_frame(geom, view):
    g = _geom(geom)
    s, e1, e2, d = (np.zeros(3) for _ in range(4))
    lib().orc_view_frame(g.ref(), view, _dptr(s), _dptr(e1), _dptr(e2), _dptr(d))
    return s, e1, e2, d


def set_mutation(m: int):
    """Switch on a planted mistake (mutation tests only); 0 restores."""
    lib().orc_set_mutation(int(m))


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n: int):
    """OpenMP threads of the oracle's loops (timing only)."""
    lib().orc_set_num_threads(int(n))
