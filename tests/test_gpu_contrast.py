"""GPU against the FP64 oracle on inputs of high dynamic range and of both
signs: a volume with one voxel a million times brighter than the rest, an
ellipsoid phantom with an insert of 1e4 times its largest attenuation, and
signed U[-1, 1) data (the search directions of CGLS and the inputs of the
autograd function are signed).

The projection sums in fixed point with one scale per work item, taken from
the largest |mu| its part of the volume holds, so these are the inputs that
could couple the precision of a pixel to a bright voxel elsewhere.  Errors
are therefore measured on the pixels the bright voxel does not reach, with
the denominator floored by the largest value of the pixel's own detector
column (or, for volumes, of the voxel's own x1 row), not by the global
maximum that the bright voxel sets."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2110_09841_amd import cvp, synth

from gpu_util import MAX_REL, REL_L2, needs_gpu, say

pytestmark = [pytest.mark.gpu, needs_gpu]

FLOOR = 1e-3


def local_errors(got, ref, axis, mask=None):
    """(relative L2, max relative error) over the elements where mask is
    True; each denominator is floored by FLOOR times the largest |ref| of the
    same line along `axis` (masked elements excluded from that maximum)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    if mask is None:
        mask = np.ones(ref.shape, bool)
    a = np.where(mask, np.abs(ref), 0.0)
    line = np.max(a, axis=axis, keepdims=True)
    den = np.maximum(np.abs(ref), FLOOR * line)
    err = np.abs(got - ref)
    sel = mask & (den > 0)
    e_max = float(np.max(err[sel] / den[sel])) if sel.any() else 0.0
    e_l2 = float(np.linalg.norm(err[mask]) / max(np.linalg.norm(ref[mask]), 1e-300))
    return e_l2, e_max


def check(got, ref, axis, what, mask=None):
    e2, em = local_errors(got, ref, axis, mask)
    say("%s: rel L2 %.3e, max rel (line floor) %.3e" % (what, e2, em))
    assert e2 <= REL_L2, (what, e2, em)
    assert em <= MAX_REL, (what, e2, em)


def ragged():
    return synth.geometry((37, 29, 70), (0.9, 1.1, 0.7), 53, 41, 1.3, 260.0, 430.0, 5, 200.0,
                          vol_offset_mm=(1.5, -2.0, 3.0), principal_px=(25.3, 21.8))


GEOMS = [("small", synth.config_small), ("ragged", ragged)]
VARIANTS = [("exact", True), ("relaxed", True), ("exact", False), ("relaxed", False)]


@pytest.mark.parametrize("gname,gfun", GEOMS)
@pytest.mark.parametrize("variant,ec", VARIANTS)
def test_hot_voxel_projection(gname, gfun, variant, ec):
    """U[0,1) volume with one voxel at 1e6: the pixels the hot voxel does not
    reach keep the bar, and so do the pixels it reaches."""
    g = gfun()
    G = cvp.Geometry(g)
    n3, n2, n1 = G.vol_shape
    x = synth.uniform_volume(G.vol_shape, seed=21)
    hot = (n3 // 2, min(3, n2 - 1), min(5, n1 - 1))
    x[hot] = 1e6
    say("hot voxel", gname, variant, "ec", ec, "at", hot)
    opts = cvp.Options(variant=variant, ec=ec)
    o = O.Options(exact=variant == "exact", ec=ec)
    got = cvp.project(torch.from_numpy(x).cuda(), G, opts).cpu().numpy()
    ref = O.project(g, o, x)
    only = np.zeros(G.vol_shape, np.float64)
    only[hot] = 1.0
    reach = O.project(g, o, only) != 0.0
    assert reach.any() and (~reach).any()
    check(got, ref, 1, "%s %s ec=%d hot voxel, pixels it does not reach" % (gname, variant, ec), ~reach)
    check(got, ref, 1, "%s %s ec=%d hot voxel, pixels it reaches" % (gname, variant, ec), reach)


@pytest.mark.parametrize("variant", ["exact", "relaxed"])
def test_high_contrast_phantom_projection(variant):
    """Ellipsoid phantom (64^3 workload) plus a ball of radius 3 voxels whose
    attenuation is 1e4 times the phantom's largest."""
    g = synth.config_small()
    G = cvp.Geometry(g)
    x = synth.ellipsoid_phantom(64, 1.0, 10, seed=11)
    k, j, i = np.meshgrid(np.arange(64), np.arange(64), np.arange(64), indexing="ij")
    ball = (i - 40) ** 2 + (j - 22) ** 2 + (k - 30) ** 2 <= 9
    x = x + np.where(ball, np.float32(1e4 * x.max()), np.float32(0.0)).astype(np.float32)
    opts = cvp.Options(variant=variant, ec=True)
    o = O.Options(exact=variant == "exact", ec=True)
    got = cvp.project(torch.from_numpy(x).cuda(), G, opts).cpu().numpy()
    ref = O.project(g, o, x)
    reach = O.project(g, o, ball.astype(np.float64)) != 0.0
    check(got, ref, 1, "contrast 1e4 %s, pixels the insert does not reach" % variant, ~reach)
    check(got, ref, 1, "contrast 1e4 %s, all pixels" % variant)


@pytest.mark.parametrize("gname,gfun", GEOMS)
@pytest.mark.parametrize("variant", ["exact", "relaxed"])
def test_signed_data_both_directions(gname, gfun, variant):
    """Signed U[-1, 1) volumes and projections."""
    g = gfun()
    G = cvp.Geometry(g)
    rng = np.random.default_rng(23)
    x = rng.uniform(-1.0, 1.0, G.vol_shape).astype(np.float32)
    b = rng.uniform(-1.0, 1.0, G.proj_shape).astype(np.float32)
    opts = cvp.Options(variant=variant, ec=True)
    o = O.Options(exact=variant == "exact", ec=True)
    say("signed", gname, variant)
    got_p = cvp.project(torch.from_numpy(x).cuda(), G, opts).cpu().numpy()
    got_b = cvp.backproject(torch.from_numpy(b).cuda(), G, opts).cpu().numpy()
    ref_p, ref_b = O.project(g, o, x), O.backproject(g, o, b)
    # Signed sums cancel: an element near zero carries the FP32 rounding of
    # terms far larger than itself.  Its error is therefore measured against
    # the sum of the absolute contributions (the oracle applied to |x| or
    # |b|), the scale of any floating-point sum, floored like the parity
    # metric at 1e-3 of the largest such sum; for data of one sign this is the
    # parity metric itself.
    abs_p, abs_b = O.project(g, o, np.abs(x)), O.backproject(g, o, np.abs(b))
    for got, ref, mag, what in ((got_p, ref_p, abs_p, "A x"), (got_b, ref_b, abs_b, "A^T b")):
        e2 = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        sel = mag > 0
        den = np.maximum(mag, FLOOR * mag.max())
        em = float(np.max(np.abs(got - ref)[sel] / den[sel]))
        assert np.all(got[~sel] == 0.0)
        say("%s %s signed %s: rel L2 %.3e, max |err| / floored sum |contributions| %.3e" % (gname, variant, what, e2,
                                                                                        em))
        assert e2 <= REL_L2, (what, e2, em)
        assert em <= MAX_REL, (what, e2, em)


@pytest.mark.parametrize("variant", ["exact", "relaxed"])
def test_hot_pixel_backprojection(variant):
    """U[0,1) projections with one pixel at 1e6: the voxels the hot pixel's
    rays do not reach keep the bar, and so do those they reach."""
    g = ragged()
    G = cvp.Geometry(g)
    b = synth.uniform_projections(G.proj_shape, seed=24)
    hot = (2, 20, 26)
    b[hot] = 1e6
    opts = cvp.Options(variant=variant, ec=True)
    o = O.Options(exact=variant == "exact", ec=True)
    got = cvp.backproject(torch.from_numpy(b).cuda(), G, opts).cpu().numpy()
    ref = O.backproject(g, o, b)
    only = np.zeros(G.proj_shape, np.float64)
    only[hot] = 1.0
    reach = O.backproject(g, o, only) != 0.0
    assert reach.any() and (~reach).any()
    check(got, ref, 2, "%s hot pixel, voxels it does not reach" % variant, ~reach)
    check(got, ref, 2, "%s hot pixel, voxels it reaches" % variant, reach)
