"""The differentiable operator: backward is the hand-written backprojector.
Checked by central finite differences of L = |A x - b|^2 (quadratic, so the
central difference is exact up to rounding) and by the dot-product test
through autograd."""
import numpy as np
import pytest
import torch

from paper_2110_09841_amd import autograd, cvp, synth

from gpu_util import needs_gpu, say

pytestmark = [pytest.mark.gpu, needs_gpu]


def geom128():
    return synth.geometry(128, 0.75, 256, 192, 1.05 * 1.6 * 128 * 0.75 * 2 ** 0.5 / 256, 750.0, 1200.0,
                          90, 200.0)


@pytest.mark.parametrize("variant", ["exact", "relaxed"])
def test_finite_differences(variant):
    g = geom128()
    G = cvp.Geometry(g)
    opts = cvp.Options(variant=variant, ec=True)
    x = torch.from_numpy(synth.ellipsoid_phantom(128, 0.75, 12, seed=3)).cuda().requires_grad_(True)
    b = cvp.project(torch.from_numpy(synth.ellipsoid_phantom(128, 0.75, 12, seed=4)).cuda(), G, opts)

    def loss(v):
        r = autograd.project(v, G, opts).double() - b.double()
        return (r * r).sum()

    L = loss(x)
    (grad,) = torch.autograd.grad(L, x)
    rng = np.random.default_rng(5)
    # L is quadratic, so the central difference has no truncation error at
    # any step; the step 1e-3 is per voxel (unit-RMS direction), large enough
    # that FP32 rounding of A x stays far below the signal 2 h <grad, d>.
    h = 1e-3
    for n in range(8):
        d = torch.from_numpy(rng.standard_normal(x.shape).astype(np.float32)).cuda()
        with torch.no_grad():
            fd = (loss(x + h * d) - loss(x - h * d)) / (2 * h)
        an = float((grad.double() * d.double()).sum())
        say("fd %s dir %d: fd %.6e analytic %.6e" % (variant, n, float(fd), an))
        assert abs(float(fd) - an) <= 1e-4 * abs(an) + 1e-6 * float(grad.double().norm())


def test_dot_product_through_autograd():
    g = geom128()
    G = cvp.Geometry(g)
    opts = cvp.Options(variant="relaxed", ec=True)
    x = torch.from_numpy(synth.uniform_volume(G.vol_shape, seed=6)).cuda().requires_grad_(True)
    y = torch.from_numpy(synth.uniform_projections(G.proj_shape, seed=7)).cuda()
    ip = (autograd.project(x, G, opts).double() * y.double()).sum()
    (gx,) = torch.autograd.grad(ip, x)
    ref = cvp.backproject(y, G, opts)
    assert torch.allclose(gx, ref, rtol=1e-6, atol=1e-6 * float(ref.abs().max()))
    lhs = float(ip)
    rhs = float((x.detach().double() * ref.double()).sum())
    assert abs(lhs - rhs) <= 1e-6 * abs(lhs)
    # and the adjoint of BackProject is the projector
    b = torch.from_numpy(synth.uniform_projections(G.proj_shape, seed=8)).cuda().requires_grad_(True)
    w = torch.from_numpy(synth.uniform_volume(G.vol_shape, seed=9)).cuda()
    (gb,) = torch.autograd.grad((autograd.backproject(b, G, opts) * w).sum(), b)
    assert torch.allclose(gb, cvp.project(w, G, opts), rtol=1e-6, atol=1e-6 * float(gb.abs().max()))
