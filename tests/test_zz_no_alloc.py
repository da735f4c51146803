"""cvp_project_noalloc (the projection whose per-group maxima live in the
library's fixed device scratch, for callers that cannot allocate) against
cvp_project_ws with a caller buffer, through the C ABI: bitwise equal on two
calls in a row, the second with a smaller problem (the scratch keeps the
first call's contents), then again after the larger one; sizes beyond the
fixed scratch are rejected before anything is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
from paper_2110_09841_amd import _lib, cvp, synth

from gpu_util import assert_parity, needs_gpu, say

pytestmark = [pytest.mark.gpu, needs_gpu]


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _noalloc(G, opts, x):
    out = torch.full(G.proj_shape, float("nan"), dtype=torch.float32, device="cuda")
    o = opts.c()
    st = _lib.lib().cvp_project_noalloc(G.handle, ctypes.byref(o), ctypes.c_void_p(x.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), _stream())
    _lib.check(st)
    return out


def _ws(G, opts, x):
    out = torch.empty(G.proj_shape, dtype=torch.float32, device="cuda")
    need = ctypes.c_int64()
    _lib.check(_lib.lib().cvp_project_workspace_size(G.handle, ctypes.byref(need)))
    work = torch.empty(max(1, need.value // 4), dtype=torch.int32, device="cuda")
    o = opts.c()
    _lib.check(_lib.lib().cvp_project_ws(G.handle, ctypes.byref(o), ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(work.data_ptr()),
                                         need.value, _stream()))
    return out


def test_noalloc_projection_equals_workspace_projection():
    big = synth.geometry((96, 80, 40), 0.8, 120, 60, 1.2, 300.0, 480.0, 12, 360.0)
    small = synth.geometry((37, 29, 20), (0.9, 1.1, 0.7), 53, 41, 1.3, 260.0, 430.0, 5, 200.0,
                           vol_offset_mm=(1.5, -2.0, 3.0))
    cases = [(big, 31, "relaxed"), (small, 32, "exact"), (big, 33, "exact")]
    for g, seed, variant in cases:
        G = cvp.Geometry(g)
        x = torch.from_numpy(synth.uniform_volume(G.vol_shape, seed=seed)).cuda()
        x[G.vol_shape[0] // 2, 2, 3] = 1e4            # one bright voxel: a large wedge maximum
        opts = cvp.Options(variant=variant, ec=True)
        say("noalloc", g["vol_dims"], variant)
        a = _noalloc(G, opts, x)
        b = _ws(G, opts, x)
        torch.cuda.synchronize()
        assert torch.equal(a, b), (g["vol_dims"], variant)
        if g is small:
            o = O.Options(exact=variant == "exact", ec=True)
            assert_parity(a.cpu().numpy(), O.project(g, o, x.cpu().numpy()), "noalloc small %s" % variant)


def test_noalloc_rejects_oversized_volume():
    # n2 * ceil(n1 / 16) = 257 * 1024 = 263168 > 262144 words of scratch
    g = synth.geometry((16384, 257, 1), 0.01, 64, 16, 1.0, 750.0, 1200.0, 2, 360.0)
    G = cvp.Geometry(g)
    x = torch.zeros(G.vol_shape, dtype=torch.float32, device="cuda")
    out = torch.zeros(G.proj_shape, dtype=torch.float32, device="cuda")
    o = cvp.Options().c()
    st = _lib.lib().cvp_project_noalloc(G.handle, ctypes.byref(o), ctypes.c_void_p(x.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), _stream())
    assert st == _lib.CVP_E_UNSUPPORTED and "scratch" in _lib.last_error()
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0     # nothing was enqueued
