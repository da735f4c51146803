"""Python binding of the cutting voxel projector (argument marshalling only).

Every step runs in the HIP kernels of libcvp.so; PyTorch provides device
memory and the current stream.  Layouts: volume [n3, n2, n1], projections
[views, rows, cols], float32, contiguous, on the geometry's device.
"""
import ctypes
from dataclasses import dataclass

import torch

from . import _lib

VARIANTS = {"exact": 0, "relaxed": 1, "tt": 2}
SCALINGS = {"solid_angle": 0, "cos": 1, "none": 2}


@dataclass(frozen=True)
class Options:
    """variant: 'exact' (r at the cut centroid), 'relaxed' (r at the voxel
    centre) or 'tt' (the TT separable-footprint projector, which takes ec
    False and scaling 'cos': see TT); ec: elevation correction (Sec. III-B);
    scaling: 'solid_angle' (eq. cvpus), 'cos' (eq. cvp) or 'none';
    raw_volume: weight = cut volume."""
    variant: str = "exact"
    ec: bool = True
    scaling: str = "solid_angle"
    raw_volume: bool = False

    def c(self):
        return _lib.OptionsC(VARIANTS[self.variant], int(bool(self.ec)), SCALINGS[self.scaling],
                             _lib.CVP_FLAG_RAW_VOLUME if self.raw_volume else 0)


# Options of the TT separable-footprint projector (the comparator of Sec. I
# and IV): it estimates the area-averaged line integral, the quantity of the
# flat-panel scaling.
TT = Options(variant="tt", ec=False, scaling="cos")


class Geometry:
    """Cone-beam geometry, built on the current HIP device.

    ``params`` is a plain dict: a circular orbit (see ``synth.geometry``:
    vol_dims, voxel_mm, vol_offset_mm, det_cols, det_rows, pitch_mm,
    principal_px, sid_mm, sdd_mm, angles_rad), or a general trajectory with
    ``matrices`` ([views][3][4] camera matrices, see
    ``synth.matrix_geometry``) in place of the orbit keys."""

    def __init__(self, params):
        self.params = dict(params)
        h = ctypes.c_void_p()
        if "matrices" in params:
            desc, self._angles = _lib.make_matrices_desc(params)
            _lib.check(_lib.lib().cvp_geometry_from_matrices(ctypes.byref(desc), ctypes.byref(h)))
            nv = desc.n_views
        else:
            desc, self._angles = _lib.make_desc(params)
            _lib.check(_lib.lib().cvp_geometry_from_views(ctypes.byref(desc), ctypes.byref(h)))
            nv = len(params["angles_rad"])
        self.handle = h
        self.records_cached = False
        n1, n2, n3 = (int(v) for v in params["vol_dims"])
        self.vol_shape = (n3, n2, n1)
        self.proj_shape = (nv, int(params["det_rows"]), int(params["det_cols"]))
        self.device = torch.device("cuda", torch.cuda.current_device())
        nbytes = ctypes.c_int64()
        _lib.check(_lib.lib().cvp_project_workspace_size(h, ctypes.byref(nbytes)))
        self.project_work_words = max(1, (nbytes.value + 3) // 4)

    def __del__(self):
        h = getattr(self, "handle", None)
        L = getattr(_lib, "_lib", None) if _lib is not None else None   # None at interpreter exit
        if h is not None and h.value and L is not None:
            L.cvp_geometry_destroy(h)
            self.handle = None

    @property
    def n_voxels(self):
        n3, n2, n1 = self.vol_shape
        return n1 * n2 * n3

    @property
    def n_views(self):
        return self.proj_shape[0]

    @property
    def launch(self):
        """Launch plan in use: (projection band columns, backprojection
        stack columns, backprojection passes per stack)."""
        lp = _lib.LaunchC()
        _lib.check(_lib.lib().cvp_geometry_get_launch(self.handle, ctypes.byref(lp)))
        return int(lp.proj_band_cols), int(lp.bp_stack_cols), int(lp.bp_passes)

    @property
    def bp_workgroups_per_cu(self):
        """Backprojection workgroups per compute unit the plan's LDS budget
        is sized for (3 or 4 with cached records; 3 without)."""
        lp = _lib.LaunchC()
        _lib.check(_lib.lib().cvp_geometry_get_launch(self.handle, ctypes.byref(lp)))
        return int(lp.bp_workgroups_per_cu)

    @property
    def bp_shared_window(self):
        """True when the cached-record backprojection stages one detector
        window per workgroup instead of one per wave."""
        lp = _lib.LaunchC()
        _lib.check(_lib.lib().cvp_geometry_get_launch(self.handle, ctypes.byref(lp)))
        return bool(lp.bp_shared_window)

    def set_launch(self, proj_band_cols=0, bp_stack_cols=0, bp_passes=0, bp_workgroups_per_cu=0,
                   bp_shared_window=False):
        """Replace the launch plan (0 selects the planner's default for that
        field).  Raises CVPError if the plan does not fit."""
        lp = _lib.LaunchC(int(proj_band_cols), int(bp_stack_cols), int(bp_passes), int(bp_workgroups_per_cu),
                          int(bool(bp_shared_window)))
        _lib.check(_lib.lib().cvp_geometry_set_launch(self.handle, ctypes.byref(lp)))

    def cache_records(self, enable=True):
        """Compute the cut-piece records of every (view, voxel column) once
        and keep them on the device (cvp_geometry_cache_records): the
        cutting voxel operators then read them instead of recomputing them
        in every launch, with bitwise the same results.  enable=False frees
        them.  Returns the table's size in bytes (0 when freed)."""
        nb = ctypes.c_int64()
        _lib.check(_lib.lib().cvp_geometry_cache_records(self.handle, int(bool(enable)), ctypes.byref(nb), _stream()))
        self.records_cached = nb.value > 0
        return int(nb.value)


def _check_tensor(t, shape, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("%s must be a contiguous float32 tensor on the GPU" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def project(x, geom: Geometry, opts: Options = Options(), out=None):
    """b = A x (overwrites ``out`` if given).  Runs cvp_project_ws with its
    small scratch (the per-group maxima of |x|) from torch's caching
    allocator on the current stream."""
    _check_tensor(x, geom.vol_shape, "x")
    if out is None:
        out = torch.empty(geom.proj_shape, dtype=torch.float32, device=x.device)
    _check_tensor(out, geom.proj_shape, "out")
    work = torch.empty(geom.project_work_words, dtype=torch.int32, device=x.device)
    o = opts.c()
    _lib.check(_lib.lib().cvp_project_ws(geom.handle, ctypes.byref(o), ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(work.data_ptr()),
                                         4 * work.numel(), _stream()))
    return out


def project_siddon(x, geom: Geometry, K: int, out=None):
    """Reference ray-driven projection SiddonK: the mean line integral over
    K x K rays per pixel (cvp_project_siddon)."""
    _check_tensor(x, geom.vol_shape, "x")
    if out is None:
        out = torch.empty(geom.proj_shape, dtype=torch.float32, device=x.device)
    _check_tensor(out, geom.proj_shape, "out")
    _lib.check(_lib.lib().cvp_project_siddon(geom.handle, int(K), ctypes.c_void_p(x.data_ptr()),
                                             ctypes.c_void_p(out.data_ptr()), _stream()))
    return out


def backproject(b, geom: Geometry, opts: Options = Options(), out=None):
    """x = A^T b (overwrites ``out`` if given)."""
    _check_tensor(b, geom.proj_shape, "b")
    if out is None:
        out = torch.empty(geom.vol_shape, dtype=torch.float32, device=b.device)
    _check_tensor(out, geom.vol_shape, "out")
    o = opts.c()
    _lib.check(_lib.lib().cvp_backproject(geom.handle, ctypes.byref(o), ctypes.c_void_p(b.data_ptr()),
                                          ctypes.c_void_p(out.data_ptr()), _stream()))
    return out


class Batch:
    """Several geometries served by one persistent launch per direction."""

    def __init__(self, geoms):
        self.geoms = list(geoms)
        arr = (ctypes.c_void_p * len(self.geoms))(*[g.handle.value for g in self.geoms])
        h = ctypes.c_void_p()
        _lib.check(_lib.lib().cvp_batch_create(arr, len(self.geoms), ctypes.byref(h)))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        L = getattr(_lib, "_lib", None) if _lib is not None else None   # None at interpreter exit
        if h is not None and h.value and L is not None:
            L.cvp_batch_destroy(h)
            self.handle = None

    def __len__(self):
        return len(self.geoms)


def _ptr_array(ts):
    return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])


def project_batched(xs, batch: Batch, opts: Options = Options(), outs=None):
    """[A_q x_q for each problem q] in one persistent launch."""
    if len(xs) != len(batch):
        raise ValueError("expected %d volumes" % len(batch))
    for x, g in zip(xs, batch.geoms):
        _check_tensor(x, g.vol_shape, "x")
    if outs is None:
        outs = [torch.empty(g.proj_shape, dtype=torch.float32, device=x.device) for x, g in zip(xs, batch.geoms)]
    for o, g in zip(outs, batch.geoms):
        _check_tensor(o, g.proj_shape, "out")
    oc = opts.c()
    _lib.check(_lib.lib().cvp_project_batched(batch.handle, ctypes.byref(oc), _ptr_array(xs),
                                              _ptr_array(outs), _stream()))
    return outs


def backproject_batched(bs, batch: Batch, opts: Options = Options(), outs=None):
    """[A_q^T b_q for each problem q] in one persistent launch."""
    if len(bs) != len(batch):
        raise ValueError("expected %d projection stacks" % len(batch))
    for b, g in zip(bs, batch.geoms):
        _check_tensor(b, g.proj_shape, "b")
    if outs is None:
        outs = [torch.empty(g.vol_shape, dtype=torch.float32, device=b.device) for b, g in zip(bs, batch.geoms)]
    for o, g in zip(outs, batch.geoms):
        _check_tensor(o, g.vol_shape, "out")
    oc = opts.c()
    _lib.check(_lib.lib().cvp_backproject_batched(batch.handle, ctypes.byref(oc), _ptr_array(bs),
                                                  _ptr_array(outs), _stream()))
    return outs


# The solver and the differentiable operators under the same namespace
# (imported last: both modules build on the definitions above).
from .cgls import CGLS, BatchedCGLS, cgls  # noqa: E402,F401
from .autograd import BackProject, Project  # noqa: E402,F401
