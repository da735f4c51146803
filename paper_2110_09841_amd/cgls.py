"""CGLS on the GPU through the C ABI, with HIP-graph capture.

The whole iteration (two operator launches, FP64 dot products, fused vector
updates and the scalar recurrences) runs on the device; the host only reads
the residual history between graph replays.  Relative residual:
rho_k = |A^T (b - A x_k)| / |A^T (b - A x_0)|.
"""
import ctypes
import time

import numpy as np
import torch

from . import _lib
from .cvp import Batch, Geometry, Options, _check_tensor, _ptr_array, _stream

N_SCALARS = 16
HISTORY = 4096
STOP = 8


class CGLS:
    def __init__(self, geom: Geometry, opts: Options, b, x0=None):
        _check_tensor(b, geom.proj_shape, "b")
        self.geom, self.opts = geom, opts
        self.b = b
        dev = b.device
        self.x = torch.zeros(geom.vol_shape, dtype=torch.float32, device=dev) if x0 is None \
            else x0.detach().clone().contiguous()
        _check_tensor(self.x, geom.vol_shape, "x0")
        self.r = torch.empty(geom.proj_shape, dtype=torch.float32, device=dev)
        self.q = torch.empty(geom.proj_shape, dtype=torch.float32, device=dev)
        self.s = torch.empty(geom.vol_shape, dtype=torch.float32, device=dev)
        self.p = torch.empty(geom.vol_shape, dtype=torch.float32, device=dev)
        nbytes = ctypes.c_int64()
        _lib.check(_lib.lib().cvp_cgls_workspace_size(geom.n_voxels, self.r.numel(), ctypes.byref(nbytes)))
        self.work = torch.zeros(nbytes.value // 8, dtype=torch.float64, device=dev)
        self._o = opts.c()
        self.graph = None
        self.graph_iters = 0

    def _ptrs(self):
        return [ctypes.c_void_p(t.data_ptr()) for t in (self.x, self.r, self.s, self.p, self.q, self.work)]

    def start(self):
        """r = b - A x0, s = A^T r, p = s, gamma0 = |s|^2."""
        x, r, s, p, q, w = self._ptrs()
        _lib.check(_lib.lib().cvp_cgls_start(self.geom.handle, ctypes.byref(self._o),
                                             ctypes.c_void_p(self.b.data_ptr()), x, r, s, p, q, w, _stream()))

    def iterate(self, n: int):
        x, r, s, p, q, w = self._ptrs()
        _lib.check(_lib.lib().cvp_cgls_iterate(self.geom.handle, ctypes.byref(self._o), int(n),
                                               x, r, s, p, q, w, _stream()))

    def capture(self, n: int):
        """Capture n iterations in one HIP graph (replayed by replay())."""
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

    def scalars(self):
        return self.work[:N_SCALARS].cpu().numpy()

    def gamma_history(self):
        """|s_k|^2 for k = 0 .. iterations done."""
        sc = self.scalars()
        k = int(sc[6])
        return self.work[N_SCALARS:N_SCALARS + min(k, HISTORY - 1) + 1].cpu().numpy()

    def residual_history(self):
        """|r_k|^2 = |b - A x_k|^2 for k = 1 .. iterations done."""
        k = int(self.scalars()[6])
        off = N_SCALARS + HISTORY
        return self.work[off:off + min(k, HISTORY)].cpu().numpy()

    def rho(self):
        g = self.gamma_history()
        return np.sqrt(np.maximum(g, 0.0) / g[0])

    def breakdown(self):
        return bool(self.scalars()[7] != 0.0)

    def stopped(self):
        """The device-side stop flag (tolerance met or breakdown)."""
        return bool(self.scalars()[STOP] != 0.0)

    def set_tolerance(self, tol, gamma_ref=None):
        """Stop on the device once |s_k|^2 <= tol^2 gamma_ref (gamma_ref:
        |s_0|^2 of the run by default); 0 never stops.  Takes effect at the
        next start()."""
        _lib.check(_lib.lib().cvp_cgls_set_tolerance(ctypes.c_void_p(self.work.data_ptr()), float(tol),
                                                     float(gamma_ref or 0.0), _stream()))

    def reset(self, b=None, x0=None):
        """New right-hand side and/or starting point in the same buffers (a
        captured graph stays valid)."""
        if b is not None:
            self.b.copy_(b)
        if x0 is None:
            self.x.zero_()
        else:
            self.x.copy_(x0)

    def run(self, tol=1e-3, max_iter=400, per_graph=20, use_graph=True, gamma_ref=None, start=True):
        """Iterate until rho_k <= tol or max_iter.  rho_k = |s_k| /
        sqrt(gamma_ref), by default gamma_ref = |s_0|^2 of this run.  The
        stop is taken on the device (cvp_cgls_set_tolerance): once rho_k <=
        tol the remaining iterations of a graph replay do nothing, so the run
        costs the iterations it needs; the host checks the flag once per
        replay of per_graph iterations.  Returns (iterations, seconds, rho
        history); time counts from the start call to the replay boundary
        where the flag is seen."""
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if start:
            self.set_tolerance(tol, gamma_ref)
            self.start()
        if use_graph and (self.graph is None or self.graph_iters != per_graph):
            self.capture(per_graph)
        done = 0
        while True:
            g = self.gamma_history()      # synchronises
            ref = g[0] if gamma_ref is None else gamma_ref
            rho = np.sqrt(np.maximum(g, 0.0) / ref)
            if rho[-1] <= tol or self.breakdown() or self.stopped() or done >= max_iter:
                break
            if use_graph:
                self.replay()
            else:
                self.iterate(per_graph)
            done += per_graph
        t1 = time.perf_counter()
        hit = np.nonzero(rho <= tol)[0]
        return (int(hit[0]) if len(hit) else len(rho) - 1), t1 - t0, rho


def cgls(geom: Geometry, b, opts: Options = Options(), x0=None, tol=1e-3, max_iter=400, per_graph=20,
         use_graph=True):
    """Least-squares solution of A x = b by CGLS from x0 (zero by default)
    until rho_k <= tol or max_iter iterations.  Returns (x, info) with info
    = {"iterations", "seconds", "rho", "breakdown"}; rho is the residual
    history (one entry per iteration run)."""
    solver = CGLS(geom, opts, b, x0)
    it, sec, rho = solver.run(tol=tol, max_iter=max_iter, per_graph=per_graph, use_graph=use_graph)
    return solver.x, {"iterations": it, "seconds": sec, "rho": rho, "breakdown": solver.breakdown()}


class BatchedCGLS:
    """CGLS on every problem of a Batch at once: each problem keeps its own
    vectors, scalars and history (those of CGLS on it alone, bitwise), and
    the two operator steps of an iteration are one batched launch each."""

    def __init__(self, batch: Batch, opts: Options, bs, x0s=None):
        n = len(batch)
        if len(bs) != n or (x0s is not None and len(x0s) != n):
            raise ValueError("expected %d right-hand sides / starting points" % n)
        self.batch, self.opts = batch, opts
        self.b = list(bs)
        for b, g in zip(self.b, batch.geoms):
            _check_tensor(b, g.proj_shape, "b")
        dev = self.b[0].device
        self.x, self.r, self.q, self.s, self.p, self.work = [], [], [], [], [], []
        nbytes = ctypes.c_int64()
        for k, g in enumerate(batch.geoms):
            x = torch.zeros(g.vol_shape, dtype=torch.float32, device=dev) if x0s is None \
                else x0s[k].detach().clone().contiguous()
            _check_tensor(x, g.vol_shape, "x0")
            self.x.append(x)
            self.r.append(torch.empty(g.proj_shape, dtype=torch.float32, device=dev))
            self.q.append(torch.empty(g.proj_shape, dtype=torch.float32, device=dev))
            self.s.append(torch.empty(g.vol_shape, dtype=torch.float32, device=dev))
            self.p.append(torch.empty(g.vol_shape, dtype=torch.float32, device=dev))
            _lib.check(_lib.lib().cvp_cgls_workspace_size(g.n_voxels, self.r[-1].numel(), ctypes.byref(nbytes)))
            self.work.append(torch.zeros(nbytes.value // 8, dtype=torch.float64, device=dev))
        self._o = opts.c()
        self._arrs = [_ptr_array(v) for v in (self.x, self.r, self.s, self.p, self.q, self.work)]
        self._b = _ptr_array(self.b)
        self.graph = None
        self.graph_iters = 0

    def __len__(self):
        return len(self.x)

    def start(self):
        _lib.check(_lib.lib().cvp_cgls_batched_start(self.batch.handle, ctypes.byref(self._o), self._b,
                                                     *self._arrs, _stream()))

    def iterate(self, n: int):
        _lib.check(_lib.lib().cvp_cgls_batched_iterate(self.batch.handle, ctypes.byref(self._o), int(n),
                                                       *self._arrs, _stream()))

    def capture(self, n: int):
        """Capture n batched iterations in one HIP graph."""
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

    def gamma_histories(self):
        """Per problem: |s_k|^2 for k = 0 .. iterations done."""
        out = []
        for w in self.work:
            sc = w[:N_SCALARS].cpu().numpy()
            k = int(sc[6])
            out.append(w[N_SCALARS:N_SCALARS + min(k, HISTORY - 1) + 1].cpu().numpy())
        return out

    def rho(self):
        return [np.sqrt(np.maximum(g, 0.0) / g[0]) for g in self.gamma_histories()]

    def breakdown(self):
        return [bool(float(w[7]) != 0.0) for w in self.work]

    def stopped(self):
        return [bool(float(w[STOP]) != 0.0) for w in self.work]

    def set_tolerance(self, tol, gamma_refs=None):
        """Per-problem device-side stop (see CGLS.set_tolerance); a stopped
        problem's work items are skipped by the batched launches."""
        for k, w in enumerate(self.work):
            ref = 0.0 if gamma_refs is None else float(gamma_refs[k])
            _lib.check(_lib.lib().cvp_cgls_set_tolerance(ctypes.c_void_p(w.data_ptr()), float(tol), ref, _stream()))

    def run(self, tol=1e-3, max_iter=400, per_graph=20, use_graph=True, gamma_refs=None):
        """Iterate all problems until each has rho_k <= tol (or broke down),
        or max_iter; each problem stops on the device when it meets the
        tolerance (its later work items are skipped), the host checks once
        per replay.  rho_k = |s_k| / sqrt(gamma_ref) with gamma_refs per
        problem (default: each run's own |s_0|^2).  Returns (per-problem
        iterations to reach tol, or the last iteration if not reached;
        seconds; per-problem rho histories)."""
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.set_tolerance(tol, gamma_refs)
        self.start()
        if use_graph and (self.graph is None or self.graph_iters != per_graph):
            self.capture(per_graph)
        done = 0
        while True:
            gh = self.gamma_histories()          # synchronises
            refs = [g[0] for g in gh] if gamma_refs is None else list(gamma_refs)
            rhos = [np.sqrt(np.maximum(g, 0.0) / r) for g, r in zip(gh, refs)]
            brk, stp = self.breakdown(), self.stopped()
            if all(r[-1] <= tol or b or s for r, b, s in zip(rhos, brk, stp)) or done >= max_iter:
                break
            if use_graph:
                self.replay()
            else:
                self.iterate(per_graph)
            done += per_graph
        t1 = time.perf_counter()
        its = []
        for r in rhos:
            hit = np.nonzero(r <= tol)[0]
            its.append(int(hit[0]) if len(hit) else len(r) - 1)
        return its, t1 - t0, rhos
