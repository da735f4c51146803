"""GPU CGLS (device-side scalars, fused vector kernels, HIP graph) against
the FP64 oracle CGLS on the same data."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle.cgls import cgls as oracle_cgls
from paper_2110_09841_amd import cvp, synth
from paper_2110_09841_amd.cgls import CGLS

from gpu_util import needs_gpu, rel_l2, say

pytestmark = [pytest.mark.gpu, needs_gpu]


def setup():
    g = synth.config_small()
    xt = synth.ellipsoid_phantom(64, 1.0, 10, seed=11).astype(np.float64)
    o = O.Options(exact=False, ec=True)
    b = O.project(g, o, xt)
    return g, o, xt, b


def test_cgls_iterates_match_oracle():
    g, o, xt, b = setup()
    n = 10
    say("cgls oracle", n)
    xo, gam_o, rn_o = oracle_cgls(lambda v: O.project(g, o, v), lambda v: O.backproject(g, o, v), b, n,
                                  np.zeros_like(xt))
    G = cvp.Geometry(g)
    solver = CGLS(G, cvp.Options(variant="relaxed", ec=True), torch.from_numpy(b.astype(np.float32)).cuda())
    say("cgls gpu eager", n)
    solver.start()
    solver.iterate(n)
    x = solver.x.cpu().numpy()
    gam = solver.gamma_history()
    e = rel_l2(x, xo)
    eg = np.max(np.abs(gam - gam_o) / gam_o)
    say("cgls x rel L2 %.3e, gamma max rel %.3e" % (e, eg))
    assert e < 1e-4
    assert eg < 1e-3
    assert not solver.breakdown()


def test_cgls_graph_replay_equals_eager_and_converges():
    g, o, xt, b = setup()
    G = cvp.Geometry(g)
    bt = torch.from_numpy(b.astype(np.float32)).cuda()
    opts = cvp.Options(variant="relaxed", ec=True)
    eager = CGLS(G, opts, bt)
    eager.start()
    eager.iterate(15)
    graphed = CGLS(G, opts, bt)
    graphed.start()
    graphed.capture(5)
    for rep in range(3):
        say("graph replay", rep)
        graphed.replay()
        torch.cuda.synchronize()
        # eager work between replays
        _ = (bt * 2.0).sum().item()
    assert torch.equal(graphed.x, eager.x)
    assert np.array_equal(graphed.gamma_history(), eager.gamma_history())
    it, sec, rho = CGLS(G, opts, bt).run(tol=1e-3, max_iter=300, per_graph=10)
    say("cgls to 1e-3: %d iterations, %.3f s" % (it, sec))
    assert rho[it] <= 1e-3
    # the residual |b - A x_k| never increases
    rr = graphed.residual_history()
    assert np.all(np.diff(rr) <= 1e-6 * rr[0])


def _small_batch(n=3):
    """The n smallest members (voxels x views) of the 16-problem batch workload."""
    params = synth.config_batch()
    order = np.argsort([p["vol_dims"][0] ** 3 * len(p["angles_rad"]) for p in params], kind="stable")
    return [params[q] for q in order[:n]]


def test_batched_cgls_equals_single_problem_bitwise():
    params = _small_batch(3)
    geoms = [cvp.Geometry(p) for p in params]
    batch = cvp.Batch(geoms)
    opts = cvp.Options(variant="relaxed", ec=True)
    xs = [torch.from_numpy(synth.ellipsoid_phantom(p["vol_dims"], p["voxel_mm"][0], 12, seed=300 + q)).cuda()
          for q, p in enumerate(params)]
    bs = [cvp.project(x, g, opts) for x, g in zip(xs, geoms)]
    say("batched cgls: %s" % [p["vol_dims"][0] for p in params])
    bc = cvp.BatchedCGLS(batch, opts, bs)
    bc.start()
    bc.iterate(4)
    bc.capture(3)
    for rep in range(2):
        say("batched cgls graph replay", rep)
        bc.replay()
        torch.cuda.synchronize()
        _ = (bs[0] * 2.0).sum().item()     # eager work between replays
    for q, g in enumerate(geoms):
        single = CGLS(g, opts, bs[q])
        single.start()
        single.iterate(10)
        assert torch.equal(bc.x[q], single.x), q
        assert np.array_equal(bc.gamma_histories()[q], single.gamma_history()), q
    assert not any(bc.breakdown())


def test_batched_cgls_run_and_cgls_function():
    params = _small_batch(2)
    geoms = [cvp.Geometry(p) for p in params]
    opts = cvp.Options(variant="relaxed", ec=True)
    xs = [torch.from_numpy(synth.ellipsoid_phantom(p["vol_dims"], p["voxel_mm"][0], 12, seed=400 + q)).cuda()
          for q, p in enumerate(params)]
    bs = [cvp.project(x, g, opts) for x, g in zip(xs, geoms)]
    its, sec, rhos = cvp.BatchedCGLS(cvp.Batch(geoms), opts, bs).run(tol=1e-2, max_iter=100, per_graph=5)
    say("batched cgls to 1e-2: %s iterations, %.3f s" % (its, sec))
    for q in range(2):
        assert rhos[q][its[q]] <= 1e-2
        x, info = cvp.cgls(geoms[q], bs[q], opts, tol=1e-2, max_iter=100, per_graph=5)
        assert info["iterations"] == its[q]
        assert info["rho"][info["iterations"]] <= 1e-2 and not info["breakdown"]


def test_device_stop_flag_single_and_batched():
    """With a tolerance set on the device, CGLS stops at the first iteration
    whose rho <= tol: a graph replayed past that point leaves x, r, s and the
    counters as they were (bitwise equal to an eager run of exactly that many
    iterations), and in a batch each problem stops at its own iteration while
    the others run on."""
    params = _small_batch(3)
    geoms = [cvp.Geometry(p) for p in params]
    opts = cvp.Options(variant="relaxed", ec=True)
    xs = [torch.from_numpy(synth.ellipsoid_phantom(p["vol_dims"], p["voxel_mm"][0], 12, seed=500 + q)).cuda()
          for q, p in enumerate(params)]
    bs = [cvp.project(x, g, opts) for x, g in zip(xs, geoms)]
    tol = 3e-2
    stops = []
    for q, g in enumerate(geoms):
        s = CGLS(g, opts, bs[q])
        s.set_tolerance(tol)
        s.start()
        s.capture(4)
        for _ in range(6):
            s.replay()
        torch.cuda.synchronize()
        k = int(s.scalars()[6])
        rho = s.rho()
        say("problem %d stopped at %d (rho %.3e)" % (q, k, rho[-1]))
        assert s.stopped() and rho[-1] <= tol and np.all(rho[:-1] > tol), (k, rho)
        ref = CGLS(g, opts, bs[q])
        ref.start()
        ref.iterate(k)
        assert torch.equal(s.x, ref.x) and torch.equal(s.r, ref.r) and torch.equal(s.s, ref.s)
        stops.append(k)
    bc = cvp.BatchedCGLS(cvp.Batch(geoms), opts, bs)
    bc.set_tolerance(tol)
    bc.start()
    bc.capture(4)
    for _ in range(6):
        bc.replay()
    torch.cuda.synchronize()
    for q, g in enumerate(geoms):
        assert int(bc.work[q][6].item()) == stops[q], (q, stops)
        ref = CGLS(g, opts, bs[q])
        ref.start()
        ref.iterate(stops[q])
        assert torch.equal(bc.x[q], ref.x), q
    assert all(bc.stopped())
