"""LSQR and OS-SART on the GPU through the C ABI (the paper's other solvers on
the same operators, Sec. V-E), with HIP-graph capture.

Every step runs in libcvp.so: operator launches, FP64 dot products, fused
vector updates, the scalar recurrences (LSQR) and the subset updates
(OS-SART).  The host only reads the residual histories.
"""
import ctypes

import torch

from . import _lib
from .cvp import Geometry, Options, _check_tensor, _stream

LSQR_SCALARS = 16
HISTORY = 4096


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


def project_views(x, geom: Geometry, view0, view_stride, n_views, out, opts: Options = Options()):
    """Writes A x for views view0, view0 + view_stride, ... (n_views of them)
    into those views of the full-size projection tensor ``out``; the other
    views of ``out`` are left untouched."""
    _check_tensor(x, geom.vol_shape, "x")
    _check_tensor(out, geom.proj_shape, "out")
    work = torch.empty(geom.project_work_words, dtype=torch.int32, device=x.device)
    o = opts.c()
    _lib.check(_lib.lib().cvp_project_views(geom.handle, ctypes.byref(o), _vp(x), _vp(out), int(view0),
                                            int(view_stride), int(n_views), _vp(work), 4 * work.numel(),
                                            _stream()))
    return out


def backproject_views(b, geom: Geometry, view0, view_stride, n_views, out=None, opts: Options = Options()):
    """A^T restricted to views view0, view0 + view_stride, ... of the
    full-size projection tensor ``b``."""
    _check_tensor(b, geom.proj_shape, "b")
    if out is None:
        out = torch.empty(geom.vol_shape, dtype=torch.float32, device=b.device)
    _check_tensor(out, geom.vol_shape, "out")
    o = opts.c()
    _lib.check(_lib.lib().cvp_backproject_views(geom.handle, ctypes.byref(o), _vp(b), _vp(out), int(view0),
                                                int(view_stride), int(n_views), _stream()))
    return out


class _Captured:
    graph = None
    graph_iters = 0

    def capture(self, n: int):
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                self.iterate(n)
        torch.cuda.current_stream().wait_stream(side)
        self.graph, self.graph_iters = g, n

    def replay(self):
        self.graph.replay()


class LSQR(_Captured):
    """Paige-Saunders LSQR: x minimises |b - A x| over growing Krylov spaces.
    Vectors x, v, w, s (volume) and u, q (projections); scalars and the
    |r|, |A^T r| estimate histories on the device."""

    def __init__(self, geom: Geometry, opts: Options, b, x0=None):
        _check_tensor(b, geom.proj_shape, "b")
        self.geom, self.opts, self.b = geom, opts, b
        dev = b.device
        self.x = torch.zeros(geom.vol_shape, dtype=torch.float32, device=dev) if x0 is None \
            else x0.detach().clone().contiguous()
        _check_tensor(self.x, geom.vol_shape, "x0")
        self.v, self.w, self.s = (torch.empty(geom.vol_shape, dtype=torch.float32, device=dev) for _ in range(3))
        self.u, self.q = (torch.empty(geom.proj_shape, dtype=torch.float32, device=dev) for _ in range(2))
        nbytes = ctypes.c_int64()
        _lib.check(_lib.lib().cvp_lsqr_workspace_size(geom.n_voxels, self.u.numel(), ctypes.byref(nbytes)))
        self.work = torch.zeros(nbytes.value // 8, dtype=torch.float64, device=dev)
        self._o = opts.c()

    def _ptrs(self):
        return [_vp(t) for t in (self.x, self.u, self.v, self.w, self.q, self.s, self.work)]

    def start(self):
        x, u, v, w, q, s, wk = self._ptrs()
        _lib.check(_lib.lib().cvp_lsqr_start(self.geom.handle, ctypes.byref(self._o), _vp(self.b), x, u, v, w, q, s,
                                             wk, _stream()))

    def iterate(self, n: int):
        x, u, v, w, q, s, wk = self._ptrs()
        _lib.check(_lib.lib().cvp_lsqr_iterate(self.geom.handle, ctypes.byref(self._o), int(n), x, u, v, w, q, s,
                                               wk, _stream()))

    def iterations(self):
        return int(self.work[6].item())

    def histories(self):
        """(|b - A x_k|, |A^T (b - A x_k)|) estimates for k = 0 .. iterations."""
        k = min(self.iterations(), HISTORY - 1)
        h = self.work[LSQR_SCALARS:LSQR_SCALARS + 2 * HISTORY].cpu().numpy()
        return h[:k + 1], h[HISTORY:HISTORY + k + 1]


class OSSART(_Captured):
    """OS-SART over n_subsets interleaved view subsets (t, t + T, ...):
    x <- x + lam A_t^T ((b_t - A_t x) / R_t) / C_t per subset, R = A 1 and
    C_t = A_t^T 1 computed once by setup(); nonneg clips x at 0."""

    def __init__(self, geom: Geometry, opts: Options, b, n_subsets, lam=1.0, nonneg=False, x0=None):
        _check_tensor(b, geom.proj_shape, "b")
        self.geom, self.opts, self.b = geom, opts, b
        self.T, self.lam, self.nonneg = int(n_subsets), float(lam), bool(nonneg)
        dev = b.device
        self.x = torch.zeros(geom.vol_shape, dtype=torch.float32, device=dev) if x0 is None \
            else x0.detach().clone().contiguous()
        _check_tensor(self.x, geom.vol_shape, "x0")
        self.rowsum = torch.empty(geom.proj_shape, dtype=torch.float32, device=dev)
        self.colsum = torch.empty((self.T,) + tuple(geom.vol_shape), dtype=torch.float32, device=dev)
        self.q = torch.empty(geom.proj_shape, dtype=torch.float32, device=dev)
        self.z = torch.empty(geom.vol_shape, dtype=torch.float32, device=dev)
        self._o = opts.c()

    def setup(self):
        _lib.check(_lib.lib().cvp_sart_setup(self.geom.handle, ctypes.byref(self._o), self.T, _vp(self.rowsum),
                                             _vp(self.colsum), _vp(self.q), _stream()))

    def iterate(self, n_sweeps: int):
        _lib.check(_lib.lib().cvp_sart_iterate(self.geom.handle, ctypes.byref(self._o), self.T, int(n_sweeps),
                                               ctypes.c_float(self.lam), int(self.nonneg), _vp(self.b), _vp(self.x),
                                               _vp(self.rowsum), _vp(self.colsum), _vp(self.q), _vp(self.z),
                                               _stream()))

