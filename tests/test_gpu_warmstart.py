"""Learned warm start pipeline: the GPU input generators against their host
definitions, the two starting iterates against the FP64 oracle CGLS, and an
end-to-end train/evaluate pass on a small geometry."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
from oracle.cgls import cgls as oracle_cgls
from paper_2110_09841_amd import _lib, synth
from paper_2110_09841_amd.unet import UNet
from paper_2110_09841_amd.warmstart import Pipeline, evaluate_batched

from gpu_util import needs_gpu, rel_l2, say

pytestmark = [pytest.mark.gpu, needs_gpu]


def _s():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def small_params():
    """32^3 voxels of 1 mm, 64x48 pixels of 1.2 mm, 24 views over 360 degrees."""
    return synth.geometry(32, 1.0, 64, 48, 1.2, 750.0, 1200.0, 24, 360.0)


def test_ellipsoid_phantom_bitwise_equal_to_host():
    dims, vox = (40, 36, 28), (1.0, 0.8, 1.2)
    ells, _ = synth.draw_ellipsoids(dims, vox, 12, seed=5, semi_axes_mm=(2.0, 14.0))
    ref = synth.ellipsoid_phantom(dims, vox, 12, seed=5, semi_axes_mm=(2.0, 14.0))
    assert ref.max() > 0
    d = torch.from_numpy(ells).cuda()
    x = torch.empty((dims[2], dims[1], dims[0]), dtype=torch.float32, device="cuda")
    say("synth ellipsoids", dims)
    _lib.check(_lib.lib().cvp_synth_ellipsoids(ctypes.c_void_p(d.data_ptr()), len(ells), (ctypes.c_int32 * 3)(*dims),
                                               (ctypes.c_double * 3)(*vox), ctypes.c_void_p(x.data_ptr()), _s()))
    assert np.array_equal(x.cpu().numpy(), ref)


@pytest.mark.parametrize("n,seed", [(4003, 0x0123456789ABCDEF), (1, 7), (16, 2 ** 40 + 3)])
def test_gaussian_noise_matches_host_philox(n, seed):
    base = torch.full((n,), 0.5, dtype=torch.float32, device="cuda")
    say("synth gaussian", n, seed)
    _lib.check(_lib.lib().cvp_synth_add_gaussian(ctypes.c_void_p(base.data_ptr()), n, ctypes.c_float(2.0),
                                                 ctypes.c_uint64(seed), _s()))
    ref = 0.5 + 2.0 * synth.philox_gaussian(n, seed)
    err = np.abs(base.cpu().numpy().astype(np.float64) - ref)
    say("max abs err %.3e" % err.max())
    assert err.max() < 2e-5      # float32 log/sin/cos of the same float32 uniforms


def test_starting_iterates_match_oracle_cgls():
    p = small_params()
    pipe = Pipeline(params=p, n_ellipsoids=6, per_graph=3)
    b_h = synth.uniform_projections(pipe.geom.proj_shape, seed=9)
    say("warmstart iterates")
    x1, x2 = pipe.iterates(torch.from_numpy(b_h).cuda())
    o = O.Options(exact=False, ec=True)
    z = np.zeros(pipe.shape)
    A = lambda v: O.project(p, o, v)
    At = lambda v: O.backproject(p, o, v)
    xo1, _, _ = oracle_cgls(A, At, b_h.astype(np.float64), 1, z)
    xo2, _, _ = oracle_cgls(A, At, b_h.astype(np.float64), 2, z)
    e1, e2 = rel_l2(x1.cpu().numpy(), xo1), rel_l2(x2.cpu().numpy(), xo2)
    say("iterate rel L2: %.3e %.3e" % (e1, e2))
    assert e1 < 1e-5 and e2 < 1e-5


def test_train_and_evaluate_small():
    p = small_params()
    pipe = Pipeline(params=p, n_ellipsoids=6, per_graph=3)
    say("warmstart data")
    data = pipe.dataset(range(24))
    x1, x2, xt = data[0]
    assert x1.shape == xt.shape == pipe.shape and float(xt.max()) > 0
    net = UNet(pipe.shape, seed=1)
    say("warmstart train")
    losses = pipe.train(net, data, epochs=3, lr=2e-3)
    say("losses", losses)
    assert all(np.isfinite(losses))
    say("warmstart evaluate")
    r = pipe.evaluate(net, 100000, tol=1e-3, max_iter=300)
    say(r)
    assert r["reached_zero"] and r["reached_warm"]
    assert r["warm_iters"] >= 2 and r["rho0_warm"] > 0


def test_identity_warm_start_restarts_from_second_iterate():
    """With the network's output head zeroed, x0 = x2; the restarted CGLS
    then begins at rho = |A^T (b - A x2)| / |A^T b|, the zero run's rho_2."""
    p = small_params()
    pipe = Pipeline(params=p, n_ellipsoids=6, per_graph=3)
    net = UNet(pipe.shape, seed=1)
    net.hw.zero_()
    net.hb.zero_()
    r = pipe.evaluate(net, 100001, tol=1e-3, max_iter=300)
    x_true = pipe.phantom(100001)
    b = pipe.measure(x_true, 100001).clone()
    pipe.solver.reset(b)
    pipe.solver.start()
    pipe.solver.iterate(2)
    rho = pipe.solver.rho()
    say("rho2 %.6e warm rho0 %.6e" % (rho[2], r["rho0_warm"]))
    assert abs(r["rho0_warm"] - rho[2]) < 1e-3 * rho[2]


def test_trained_warm_start_beats_zero_start_in_batched_cgls():
    """What the trained network gains: trained on 400 phantoms (64^3 voxels
    of 1 mm, 128 x 128 pixels of 1 mm, 90 views; the 20th CGLS iterate as
    target, four epochs), it must bring 8 held-out phantoms, run as one batch
    through batched CGLS, to rho <= 1e-3 in at least 5 % fewer iterations in
    total than batched CGLS from zero (the warm count includes its two
    starting iterations), every problem reaching the tolerance and none
    taking more iterations than from zero."""
    p = synth.geometry(64, 1.0, 128, 128, 1.0, 750.0, 1200.0, 90, 360.0)
    pipe = Pipeline(params=p, n_ellipsoids=10, per_graph=5)
    say("warmstart gain: data")
    data = pipe.dataset(range(400))
    net = UNet(pipe.shape, seed=1)
    say("warmstart gain: train")
    pipe.train(net, data, epochs=4, lr=1e-3)
    del data
    say("warmstart gain: batched evaluation")
    r = evaluate_batched(pipe, net, [100000 + n for n in range(8)], tol=1e-3, max_iter=300)
    say("zero %s (%.3f s), warm %s (%.3f s), warm rho0 %s" % (r["zero_iters"], r["zero_s"], r["warm_iters"],
                                                            r["warm_s"], ["%.3f" % v for v in r["rho0_warm"]]))
    assert all(r["reached_zero"]) and all(r["reached_warm"])
    assert all(w <= z for w, z in zip(r["warm_iters"], r["zero_iters"]))
    assert sum(r["warm_iters"]) <= 0.95 * sum(r["zero_iters"])
