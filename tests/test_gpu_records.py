"""Cached cut-piece records (cvp_geometry_cache_records): with the table the
operators read the FP64 records of every (view, voxel column) that a
one-off pass computed, instead of computing them in each launch; the
results must be bitwise those without it -- both forms, EC on and off,
record strides 4 and 8, view subsets, either LDS budget of the
backprojection, the allocation-free projection and CGLS -- and the TT projector, which keeps its own records, is unaffected.
Geometries whose voxels span more than 8 columns are refused."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2110_09841_amd import _lib, cvp, solvers, synth

from gpu_util import needs_gpu, say

pytestmark = [pytest.mark.gpu, needs_gpu]

COMBOS = [("exact", True), ("relaxed", True), ("exact", False), ("relaxed", False)]


def geoms():
    # record stride 4 (a C-arm like geometry) and 8 (about 5 columns per voxel)
    g4 = synth.geometry((37, 29, 30), (0.9, 1.1, 0.7), 61, 47, 1.3, 260.0, 430.0, 12, 200.0,
                        vol_offset_mm=(1.5, -2.0, 3.0))
    g8 = synth.geometry((21, 19, 17), 1.0, 160, 120, 0.45, 300.0, 520.0, 9, 360.0, vol_offset_mm=(0.5, 1.0, -1.5))
    return {"pmax4": g4, "pmax8": g8}


def noalloc(x, G, opts):
    out = torch.empty(G.proj_shape, dtype=torch.float32, device="cuda")
    o = opts.c()
    _lib.check(_lib.lib().cvp_project_noalloc(G.handle, ctypes.byref(o), ctypes.c_void_p(x.data_ptr()),
                                              ctypes.c_void_p(out.data_ptr()), cvp._stream()))
    return out


@pytest.mark.parametrize("name", ["pmax4", "pmax8"])
def test_cached_records_give_the_same_bits(name):
    g = geoms()[name]
    G = cvp.Geometry(g)
    x = torch.from_numpy(synth.ellipsoid_phantom(g["vol_dims"], g["voxel_mm"], 6, seed=91,
                                                 semi_axes_mm=(2.0, 9.0))).cuda()
    b = torch.from_numpy(synth.uniform_projections(G.proj_shape, seed=92)).cuda()
    ref = {}
    for variant, ec in COMBOS:
        opts = cvp.Options(variant=variant, ec=ec)
        ref[variant, ec] = (cvp.project(x, G, opts), cvp.backproject(b, G, opts), noalloc(x, G, opts),
                            solvers.backproject_views(b, G, 1, 3, 3, opts=opts))
    tt = (cvp.project(x, G, cvp.TT), cvp.backproject(b, G, cvp.TT))
    nb = G.cache_records()
    n3, n2, n1 = G.vol_shape
    say(name, "record table %d bytes, launch %s" % (nb, G.launch))
    assert nb >= G.n_views * n2 * n1 * 4 * (4 * 12 + 1)
    assert G.cache_records() == nb            # a second enable keeps the table
    for variant, ec in COMBOS:
        opts = cvp.Options(variant=variant, ec=ec)
        got = (cvp.project(x, G, opts), cvp.backproject(b, G, opts), noalloc(x, G, opts),
               solvers.backproject_views(b, G, 1, 3, 3, opts=opts))
        for what, r, t in zip(("A x", "A^T b", "A x (no alloc)", "A^T b (views 1, 4, 7)"), ref[variant, ec], got):
            assert torch.equal(r, t), (name, variant, ec, what)
    # the backprojection's LDS budget (workgroups per CU) changes only the split
    assert G.bp_workgroups_per_cu == (4 if name == "pmax4" else 3)
    for wpc in (3, 4):
        G.set_launch(0, 0, 0, wpc)
        assert G.bp_workgroups_per_cu == wpc
        for variant, ec in COMBOS[:2]:
            opts = cvp.Options(variant=variant, ec=ec)
            assert torch.equal(cvp.backproject(b, G, opts), ref[variant, ec][1]), (name, wpc, variant)
    if name == "pmax8":
        # pixels small against the voxels: one window per workgroup for 8- and
        # 16-column stacks (4-column ones keep their own), and each wave's own
        # windows, partly read from global memory
        shared = []
        for gw, kp, shw in ((8, 1, True), (16, 1, True), (4, 1, True), (8, 1, False), (4, 2, False)):
            G.set_launch(0, gw, kp, 3, shw)
            shared.append(G.bp_shared_window)
            for variant, ec in COMBOS:
                opts = cvp.Options(variant=variant, ec=ec)
                assert torch.equal(cvp.backproject(b, G, opts), ref[variant, ec][1]), (gw, kp, variant, ec)
            opts = cvp.Options(variant="relaxed", ec=True)
            assert torch.equal(solvers.backproject_views(b, G, 1, 3, 3, opts=opts), ref["relaxed", True][3])
        say("one window per workgroup:", shared)
        assert shared == [True, True, False, False, False]
    G.set_launch()
    out = torch.full(G.proj_shape, 3.0, device="cuda")
    solvers.project_views(x, G, 2, 4, 2, out, cvp.Options(variant="relaxed", ec=True))
    full = ref["relaxed", True][0]
    for v in range(G.n_views):
        assert torch.equal(out[v], full[v] if v in (2, 6) else torch.full_like(out[v], 3.0))
    assert torch.equal(cvp.project(x, G, cvp.TT), tt[0]) and torch.equal(cvp.backproject(b, G, cvp.TT), tt[1])
    assert G.cache_records(False) == 0
    opts = cvp.Options(variant="exact", ec=True)
    assert torch.equal(cvp.project(x, G, opts), ref["exact", True][0])


def test_cgls_with_cached_records():
    g = geoms()["pmax4"]
    G = cvp.Geometry(g)
    opts = cvp.Options(variant="relaxed", ec=True)
    xt = torch.from_numpy(synth.ellipsoid_phantom(g["vol_dims"], g["voxel_mm"], 5, seed=93,
                                                  semi_axes_mm=(2.0, 9.0))).cuda()
    b = cvp.project(xt, G, opts)
    A = cvp.CGLS(G, opts, b)
    A.start()
    A.iterate(6)
    G.cache_records()
    B = cvp.CGLS(G, opts, b)
    B.start()
    B.iterate(6)
    torch.cuda.synchronize()
    assert torch.equal(A.x, B.x)


def test_wide_footprints_refused():
    g = synth.geometry((5, 4, 3), 1.0, 616, 480, 0.154, 749.0, 1198.0, 3, 360.0)
    G = cvp.Geometry(g)
    with pytest.raises(_lib.CVPError) as ei:
        G.cache_records()
    assert ei.value.status == _lib.CVP_E_UNSUPPORTED


def test_batch_reads_cached_records():
    """A batch whose members all have cached records gives every member's
    single-problem result bitwise; a member's table freed afterwards makes
    the batch refuse to run."""
    gs = geoms()
    G = [cvp.Geometry(gs["pmax4"]), cvp.Geometry(gs["pmax8"])]
    xs = [torch.from_numpy(synth.uniform_volume(g.vol_shape, seed=94 + q)).cuda() for q, g in enumerate(G)]
    bs = [torch.from_numpy(synth.uniform_projections(g.proj_shape, seed=96 + q)).cuda() for q, g in enumerate(G)]
    opts = cvp.Options(variant="relaxed", ec=True)
    for g in G:
        g.cache_records()
    batch = cvp.Batch(G)
    pb = cvp.project_batched(xs, batch, opts)
    vb = cvp.backproject_batched(bs, batch, opts)
    for q, g in enumerate(G):
        assert torch.equal(pb[q], cvp.project(xs[q], g, opts))
        assert torch.equal(vb[q], cvp.backproject(bs[q], g, opts))
    G[1].cache_records(False)
    with pytest.raises(_lib.CVPError) as ei:
        cvp.project_batched(xs, batch, opts)
    assert ei.value.status == _lib.CVP_E_INVALID
