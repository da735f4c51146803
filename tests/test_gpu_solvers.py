"""View-subset operators, LSQR and OS-SART on the GPU (libcvp.so through the
C ABI) against the FP64 oracles (oracle/lsqr.py, oracle/sart.py) running on
the oracle's own CVP operators, on a ragged, offset 37 x 29 x 30 volume with
12 views; and graph-captured runs equal to eager ones bitwise."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle.lsqr import lsqr as lsqr_oracle
from oracle.sart import os_sart
from paper_2110_09841_amd import cvp, solvers, synth

from gpu_util import assert_parity, needs_gpu, rel_l2, say

pytestmark = [pytest.mark.gpu, needs_gpu]


def geom():
    return synth.geometry((37, 29, 30), (0.9, 1.1, 0.7), 53, 41, 1.3, 260.0, 430.0, 12, 360.0,
                          vol_offset_mm=(1.5, -2.0, 3.0))


def subset_geom(g, views):
    h = dict(g)
    h["angles_rad"] = np.asarray(g["angles_rad"])[views]
    return h


OPTS = [("relaxed", True), ("exact", False)]


@pytest.mark.parametrize("variant,ec", OPTS)
def test_view_subsets(variant, ec):
    g = geom()
    G = cvp.Geometry(g)
    x = torch.from_numpy(synth.ellipsoid_phantom((37, 29, 30), (0.9, 1.1, 0.7), 5, seed=71,
                                                 semi_axes_mm=(2.0, 9.0))).cuda()
    b = torch.from_numpy(synth.uniform_projections(G.proj_shape, seed=72)).cuda()
    opts = cvp.Options(variant=variant, ec=ec)
    o = O.Options(exact=variant == "exact", ec=ec)
    full = cvp.project(x, G, opts)
    for v0, st, n in ((1, 3, 4), (0, 1, 12), (11, 5, 1), (2, 4, 3)):
        say("views", v0, st, n, variant, ec)
        views = v0 + st * np.arange(n)
        out = torch.full(G.proj_shape, 7.0, device="cuda")
        solvers.project_views(x, G, v0, st, n, out, opts)
        mask = np.zeros(12, bool)
        mask[views] = True
        oc = out.cpu().numpy()
        assert np.all(oc[~mask] == 7.0)                       # other views untouched
        assert torch.equal(out[torch.from_numpy(mask).cuda()], full[torch.from_numpy(mask).cuda()])
        bt = solvers.backproject_views(b, G, v0, st, n, opts=opts).cpu().numpy()
        ref = O.backproject(subset_geom(g, views), o, b.cpu().numpy()[views])
        assert_parity(bt, ref, "A^T on views %d+%dk (%d)" % (v0, st, n))


def test_lsqr_iterates_match_oracle():
    g = geom()
    G = cvp.Geometry(g)
    opts = cvp.Options(variant="relaxed", ec=True)
    o = O.Options(exact=False, ec=True)
    xt = synth.ellipsoid_phantom((37, 29, 30), (0.9, 1.1, 0.7), 5, seed=73, semi_axes_mm=(2.0, 9.0))
    b = O.project(g, o, xt).astype(np.float32)
    n = 8
    x_ref, rn_ref, arn_ref = lsqr_oracle(lambda v: O.project(g, o, v), lambda v: O.backproject(g, o, v),
                                         b.astype(np.float64), n, np.zeros(xt.shape))
    L = solvers.LSQR(G, opts, torch.from_numpy(b).cuda())
    L.start()
    L.iterate(n)
    x = L.x.cpu().numpy()
    rn, arn = L.histories()
    e = rel_l2(x, x_ref)
    say("lsqr %d iterations: x rel L2 %.3e; |r| est %.6e vs %.6e" % (n, e, rn[-1], rn_ref[-1]))
    assert L.iterations() == n
    assert e < 1e-4
    assert np.allclose(rn, rn_ref, rtol=1e-4)
    assert np.allclose(arn, arn_ref, rtol=1e-3)


def test_lsqr_graph_replay_equals_eager():
    g = geom()
    G = cvp.Geometry(g)
    opts = cvp.Options(variant="relaxed", ec=True)
    b = torch.from_numpy(synth.uniform_projections(G.proj_shape, seed=74)).cuda()
    A = solvers.LSQR(G, opts, b)
    A.start()
    A.iterate(6)
    B = solvers.LSQR(G, opts, b)
    B.start()
    B.capture(3)
    for _ in range(2):
        B.replay()
        torch.cuda.synchronize()
    assert torch.equal(A.x, B.x)
    assert torch.equal(A.work[:16], B.work[:16])


@pytest.mark.parametrize("T,nonneg", [(4, False), (1, False), (3, True)])
def test_os_sart_matches_oracle(T, nonneg):
    g = geom()
    G = cvp.Geometry(g)
    opts = cvp.Options(variant="relaxed", ec=True)
    o = O.Options(exact=False, ec=True)
    xt = synth.ellipsoid_phantom((37, 29, 30), (0.9, 1.1, 0.7), 5, seed=75, semi_axes_mm=(2.0, 9.0))
    b = O.project(g, o, xt)
    b += synth.gaussian_noise(b.shape, 0.01 * float(np.sqrt(np.mean(b ** 2))), seed=76)
    b = b.astype(np.float32)
    sweeps = 3
    x_ref, res_ref = os_sart(lambda x, v: O.project(subset_geom(g, v), o, x),
                             lambda y, v: O.backproject(subset_geom(g, v), o, y),
                             b.astype(np.float64), 12, T, sweeps, np.zeros(xt.shape), lam=0.9, nonneg=nonneg)
    S = solvers.OSSART(G, opts, torch.from_numpy(b).cuda(), T, lam=0.9, nonneg=nonneg)
    S.setup()
    S.iterate(sweeps)
    x = S.x.cpu().numpy()
    e = rel_l2(x, x_ref)
    say("os-sart T=%d nonneg=%d %d sweeps: x rel L2 %.3e" % (T, nonneg, sweeps, e))
    assert e < 1e-4


def test_os_sart_graph_replay_equals_eager():
    g = geom()
    G = cvp.Geometry(g)
    opts = cvp.Options(variant="relaxed", ec=True)
    b = torch.from_numpy(synth.uniform_projections(G.proj_shape, seed=77)).cuda()
    A = solvers.OSSART(G, opts, b, 4)
    A.setup()
    A.iterate(4)
    B = solvers.OSSART(G, opts, b, 4)
    B.setup()
    B.capture(2)
    for _ in range(2):
        B.replay()
        torch.cuda.synchronize()
    assert torch.equal(A.x, B.x)
