"""ctypes loader of the in-tree HIP library (libcvp.so) and its C ABI.

There is no fallback: if the library is missing or fails to load, every
operator raises.  Build it with ``__graft_entry__.build()`` (or
``python paper_2110_09841_amd/build.py``).
"""
import ctypes
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcvp.so")

CVP_OK, CVP_E_INVALID, CVP_E_NOMEM, CVP_E_DEVICE, CVP_E_UNSUPPORTED, CVP_E_BREAKDOWN = range(6)
CVP_FLAG_RAW_VOLUME = 1

_lib = None


class CVPError(RuntimeError):
    def __init__(self, status, detail):
        self.status = status
        super().__init__("%s: %s" % (status_string(status) if _lib else status, detail))


class GeometryDesc(ctypes.Structure):
    _fields_ = [("vol_dims", ctypes.c_int32 * 3),
                ("voxel_mm", ctypes.c_double * 3),
                ("vol_offset_mm", ctypes.c_double * 3),
                ("det_cols", ctypes.c_int32), ("det_rows", ctypes.c_int32),
                ("pitch_mm", ctypes.c_double * 2),
                ("principal_px", ctypes.c_double * 2),
                ("source_iso_mm", ctypes.c_double),
                ("source_det_mm", ctypes.c_double),
                ("n_views", ctypes.c_int32),
                ("angles_rad", ctypes.POINTER(ctypes.c_double))]


class MatricesDesc(ctypes.Structure):
    _fields_ = [("vol_dims", ctypes.c_int32 * 3),
                ("voxel_mm", ctypes.c_double * 3),
                ("vol_offset_mm", ctypes.c_double * 3),
                ("det_cols", ctypes.c_int32), ("det_rows", ctypes.c_int32),
                ("n_views", ctypes.c_int32),
                ("matrices", ctypes.POINTER(ctypes.c_double))]


class OptionsC(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("elevation_correction", ctypes.c_int32),
                ("scaling", ctypes.c_int32), ("flags", ctypes.c_uint32)]


def lib():
    """Load libcvp.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libcvp.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    st = ctypes.c_int
    L.cvp_geometry_from_views.argtypes = [ctypes.POINTER(GeometryDesc), ctypes.POINTER(vp)]
    L.cvp_geometry_from_views.restype = st
    L.cvp_geometry_from_matrices.argtypes = [ctypes.POINTER(MatricesDesc), ctypes.POINTER(vp)]
    L.cvp_geometry_from_matrices.restype = st
    L.cvp_geometry_destroy.argtypes = [vp]
    L.cvp_geometry_destroy.restype = None
    for name in ("cvp_project", "cvp_backproject"):
        f = getattr(L, name)
        f.argtypes = [vp, ctypes.POINTER(OptionsC), vp, vp, vp]
        f.restype = st
    L.cvp_geometry_sizes.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    L.cvp_geometry_sizes.restype = st
    L.cvp_status_string.argtypes = [st]
    L.cvp_status_string.restype = ctypes.c_char_p
    L.cvp_last_error_detail.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
    L.cvp_last_error_detail.restype = st
    _register_extra(L)
    _lib = L
    return L


class LaunchC(ctypes.Structure):
    _fields_ = [("proj_band_cols", ctypes.c_int32), ("bp_stack_cols", ctypes.c_int32), ("bp_passes", ctypes.c_int32),
                ("bp_workgroups_per_cu", ctypes.c_int32), ("bp_shared_window", ctypes.c_int32)]


def _register_extra(L):
    """Signatures of the solver, batch and input-generation entry points
    (present in the same library)."""
    vp = ctypes.c_void_p
    st = ctypes.c_int
    specs = {
        "cvp_batch_create": ([ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(vp)], st),
        "cvp_batch_destroy": ([vp], None),
        "cvp_project_batched": ([vp, ctypes.POINTER(OptionsC), ctypes.POINTER(vp), ctypes.POINTER(vp), vp], st),
        "cvp_backproject_batched": ([vp, ctypes.POINTER(OptionsC), ctypes.POINTER(vp), ctypes.POINTER(vp), vp], st),
        "cvp_cgls_workspace_size": ([ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)], st),
        "cvp_cgls_start": ([vp, ctypes.POINTER(OptionsC), vp, vp, vp, vp, vp, vp, vp, vp], st),
        "cvp_cgls_iterate": ([vp, ctypes.POINTER(OptionsC), ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp], st),
        "cvp_cgls_batched_start": ([vp, ctypes.POINTER(OptionsC)] + [ctypes.POINTER(vp)] * 7 + [vp], st),
        "cvp_cgls_batched_iterate": ([vp, ctypes.POINTER(OptionsC), ctypes.c_int32] + [ctypes.POINTER(vp)] * 6
                                     + [vp], st),
        "cvp_project_workspace_size": ([vp, ctypes.POINTER(ctypes.c_int64)], st),
        "cvp_project_ws": ([vp, ctypes.POINTER(OptionsC), vp, vp, vp, ctypes.c_int64, vp], st),
        "cvp_project_noalloc": ([vp, ctypes.POINTER(OptionsC), vp, vp, vp], st),
        "cvp_project_siddon": ([vp, ctypes.c_int32, vp, vp, vp], st),
        "cvp_project_views": ([vp, ctypes.POINTER(OptionsC), vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                               vp, ctypes.c_int64, vp], st),
        "cvp_backproject_views": ([vp, ctypes.POINTER(OptionsC), vp, vp, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, vp], st),
        "cvp_sart_setup": ([vp, ctypes.POINTER(OptionsC), ctypes.c_int32, vp, vp, vp, vp], st),
        "cvp_sart_iterate": ([vp, ctypes.POINTER(OptionsC), ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                              ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp], st),
        "cvp_lsqr_workspace_size": ([ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)], st),
        "cvp_lsqr_start": ([vp, ctypes.POINTER(OptionsC)] + [vp] * 8 + [vp], st),
        "cvp_lsqr_iterate": ([vp, ctypes.POINTER(OptionsC), ctypes.c_int32] + [vp] * 7 + [vp], st),
        "cvp_dot": ([vp, vp, ctypes.c_int64, vp, vp, vp], st),
        "cvp_cgls_set_tolerance": ([vp, ctypes.c_double, ctypes.c_double, vp], st),
        "cvp_synth_ellipsoids": ([vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                                  vp, vp], st),
        "cvp_synth_add_gaussian": ([vp, ctypes.c_int64, ctypes.c_float, ctypes.c_uint64, vp], st),
        "cvp_geometry_get_launch": ([vp, ctypes.POINTER(LaunchC)], st),
        "cvp_geometry_set_launch": ([vp, ctypes.POINTER(LaunchC)], st),
        "cvp_geometry_cache_records": ([vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), vp], st),
    }
    for name, (args, res) in specs.items():
        if hasattr(L, name):
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res


def status_string(s):
    return lib().cvp_status_string(int(s)).decode()


def last_error():
    buf = ctypes.create_string_buffer(512)
    lib().cvp_last_error_detail(buf, 512)
    return buf.value.decode()


def check(status):
    if status != CVP_OK:
        raise CVPError(status, last_error())


def make_matrices_desc(p):
    """MatricesDesc from a dict with vol_dims, voxel_mm, vol_offset_mm,
    det_cols, det_rows and matrices ([views][3][4])."""
    import numpy as np
    m = np.ascontiguousarray(np.asarray(p["matrices"], dtype=np.float64).reshape(-1, 12))
    d = MatricesDesc()
    d.vol_dims[:] = [int(v) for v in p["vol_dims"]]
    d.voxel_mm[:] = [float(v) for v in p["voxel_mm"]]
    d.vol_offset_mm[:] = [float(v) for v in p.get("vol_offset_mm", (0.0, 0.0, 0.0))]
    d.det_cols, d.det_rows = int(p["det_cols"]), int(p["det_rows"])
    d.n_views = len(m)
    d.matrices = m.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return d, m


def make_desc(p):
    """GeometryDesc from a plain parameter dict (keys as in synth.geometry)."""
    angles = (ctypes.c_double * len(p["angles_rad"]))(*[float(a) for a in p["angles_rad"]])
    d = GeometryDesc()
    d.vol_dims[:] = [int(v) for v in p["vol_dims"]]
    d.voxel_mm[:] = [float(v) for v in p["voxel_mm"]]
    d.vol_offset_mm[:] = [float(v) for v in p.get("vol_offset_mm", (0.0, 0.0, 0.0))]
    d.det_cols, d.det_rows = int(p["det_cols"]), int(p["det_rows"])
    d.pitch_mm[:] = [float(v) for v in p["pitch_mm"]]
    pp = p.get("principal_px")
    d.principal_px[:] = [math.nan, math.nan] if pp is None else [float(pp[0]), float(pp[1])]
    d.source_iso_mm = float(p["sid_mm"])
    d.source_det_mm = float(p["sdd_mm"])
    d.n_views = len(p["angles_rad"])
    d.angles_rad = ctypes.cast(angles, ctypes.POINTER(ctypes.c_double))
    return d, angles
