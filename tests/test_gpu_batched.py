"""Batched persistent launches over 16 uneven problems (volumes 96^3..320^3,
detectors 256x192..512x384, 60-400 views): every problem's result equals its
single-problem result bitwise; the batch is graph-capturable."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2110_09841_amd import cvp, synth

from gpu_util import assert_parity, needs_gpu, say

pytestmark = [pytest.mark.gpu, needs_gpu]


def test_batched_equals_single_problem_bitwise():
    params = synth.config_batch()
    geoms = [cvp.Geometry(p) for p in params]
    batch = cvp.Batch(geoms)
    xs = [torch.from_numpy(synth.ellipsoid_phantom(p["vol_dims"], p["voxel_mm"][0], 12, seed=100 + q)).cuda()
          for q, p in enumerate(params)]
    bs = [torch.from_numpy(synth.uniform_projections(g.proj_shape, seed=200 + q)).cuda()
          for q, g in enumerate(geoms)]
    for variant in ("relaxed", "exact"):
        opts = cvp.Options(variant=variant, ec=True)
        say("batched projection", variant)
        outs = cvp.project_batched(xs, batch, opts)
        say("batched backprojection", variant)
        vols = cvp.backproject_batched(bs, batch, opts)
        torch.cuda.synchronize()
        for q, g in enumerate(geoms):
            assert torch.equal(outs[q], cvp.project(xs[q], g, opts)), ("projection", variant, q)
            assert torch.equal(vols[q], cvp.backproject(bs[q], g, opts)), ("backprojection", variant, q)


def test_batched_member_against_oracle():
    """The smallest member checked against the FP64 oracle (one view and a
    voxel sample), through the batched path."""
    params = synth.config_batch()
    q = int(np.argmin([p["vol_dims"][0] ** 3 * len(p["angles_rad"]) for p in params]))
    geoms = [cvp.Geometry(p) for p in params]
    batch = cvp.Batch(geoms)
    p = params[q]
    xs = [torch.zeros(g.vol_shape, dtype=torch.float32, device="cuda") for g in geoms]
    xq = synth.ellipsoid_phantom(p["vol_dims"], p["voxel_mm"][0], 12, seed=7)
    xs[q] = torch.from_numpy(xq).cuda()
    bs = [torch.zeros(g.proj_shape, dtype=torch.float32, device="cuda") for g in geoms]
    bq = synth.uniform_projections(geoms[q].proj_shape, seed=8)
    bs[q] = torch.from_numpy(bq).cuda()
    opts = cvp.Options(variant="relaxed", ec=True)
    o = O.Options(exact=False, ec=True)
    say("batched member", q, p["vol_dims"])
    out = cvp.project_batched(xs, batch, opts)[q].cpu().numpy()
    assert_parity(out[3], O.project(p, o, xq, views=(3, 4))[0], "batched member A x view 3")
    vol = cvp.backproject_batched(bs, batch, opts)[q].cpu().numpy()
    idx = np.random.default_rng(0).integers(0, vol.size, 200)
    assert_parity(vol.ravel()[idx], O.backproject_voxels(p, o, bq, idx), "batched member A^T b")


def test_batched_graph_capture_replays():
    params = synth.config_batch()[:4]
    geoms = [cvp.Geometry(p) for p in params]
    batch = cvp.Batch(geoms)
    xs = [torch.from_numpy(synth.uniform_volume(g.vol_shape, seed=q)).cuda() for q, g in enumerate(geoms)]
    outs = [torch.empty(g.proj_shape, dtype=torch.float32, device="cuda") for g in geoms]
    opts = cvp.Options(variant="relaxed", ec=True)
    ref = [cvp.project(x, g, opts) for x, g in zip(xs, geoms)]
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            cvp.project_batched(xs, batch, opts, outs=outs)
    torch.cuda.current_stream().wait_stream(side)
    for rep in range(3):
        for o in outs:
            o.fill_(-1.0)
        say("batched graph replay", rep)
        graph.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            assert torch.equal(o, r)
