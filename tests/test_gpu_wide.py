"""Voxels whose base projects onto more than eight detector columns (fine
detectors): the single-voxel arrangements of the paper's accuracy comparison
(Sec. IV-B) and a small volume on the same fine detector, GPU against the
FP64 oracle element by element, every view, both forms, with and without
the elevation correction.  The projection serves such footprints with bands
of at most eight columns, the backprojection with four-column stacks that
keep up to 64 pieces per column."""
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
from paper_2110_09841_amd import cvp, synth

from gpu_util import assert_parity, needs_gpu, say

pytestmark = [pytest.mark.gpu, needs_gpu]

HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(HERE, "golden", "paper_setups.json")) as _f:
    SETUPS = json.load(_f)


def single_voxel_geometry(name, n_views=360):
    s = SETUPS[name]
    return synth.geometry((1, 1, 1), s["voxel_mm"], s["det_cols"], s["det_rows"], s["pitch_mm"],
                          s["sid_mm"], s["sdd_mm"], n_views, 360.0, vol_offset_mm=s["voxel_centre_mm"])


COMBOS = [("exact", True), ("relaxed", True), ("exact", False), ("relaxed", False)]


@pytest.mark.parametrize("name", ["accuracy_isocentre", "accuracy_shifted", "accuracy_large_cone"])
@pytest.mark.parametrize("variant,ec", COMBOS)
def test_single_voxel_setups(name, variant, ec):
    g = single_voxel_geometry(name)
    say("single voxel", name, variant, "ec", ec)
    G = cvp.Geometry(g)
    x = np.ones((1, 1, 1), np.float32)
    b = synth.uniform_projections(G.proj_shape, seed=51)
    opts = cvp.Options(variant=variant, ec=ec, scaling="cos")
    o = O.Options(exact=variant == "exact", ec=ec, scaling="cos")
    got = cvp.project(torch.from_numpy(x).cuda(), G, opts).cpu().numpy()
    assert_parity(got, O.project(g, o, x), "%s %s ec=%d A x" % (name, variant, ec))
    gotb = cvp.backproject(torch.from_numpy(b).cuda(), G, opts).cpu().numpy()
    assert_parity(gotb, O.backproject(g, o, b), "%s %s ec=%d A^T b" % (name, variant, ec))


@pytest.mark.parametrize("variant,ec", COMBOS[:2])
def test_small_volume_fine_detector(variant, ec):
    """14 x 11 x 9 voxels of 1 mm (ragged, offset) on the 616 x 480 detector
    of 0.154 mm pixels: about 15 columns per voxel, 12 views."""
    g = synth.geometry((14, 11, 9), 1.0, 616, 480, 0.154, 749.0, 1198.0, 12, 360.0,
                       vol_offset_mm=(1.3, -0.7, 2.1))
    say("fine detector volume", variant, "ec", ec)
    G = cvp.Geometry(g)
    assert G.launch[0] <= 8 and G.launch[1] == 4
    x = synth.ellipsoid_phantom((14, 11, 9), 1.0, 3, seed=52, semi_axes_mm=(2.0, 6.0))
    x += synth.uniform_volume(G.vol_shape, seed=53) * np.float32(0.01)
    b = synth.uniform_projections(G.proj_shape, seed=54)
    opts = cvp.Options(variant=variant, ec=ec)
    o = O.Options(exact=variant == "exact", ec=ec)
    got = cvp.project(torch.from_numpy(x).cuda(), G, opts).cpu().numpy()
    assert_parity(got, O.project(g, o, x), "fine %s ec=%d A x" % (variant, ec))
    gotb = cvp.backproject(torch.from_numpy(b).cuda(), G, opts).cpu().numpy()
    assert_parity(gotb, O.backproject(g, o, b), "fine %s ec=%d A^T b" % (variant, ec))
    # adjoint identity with FP64 dots of the FP32 results
    lhs = float(np.dot(got.astype(np.float64).ravel(), b.astype(np.float64).ravel()))
    rhs = float(np.dot(x.astype(np.float64).ravel(), gotb.astype(np.float64).ravel()))
    assert abs(lhs - rhs) <= 1e-6 * abs(lhs), (lhs, rhs)


def test_wide_band_plan_is_rejected():
    g = synth.geometry((4, 4, 4), 1.0, 616, 480, 0.154, 749.0, 1198.0, 2, 360.0)
    G = cvp.Geometry(g)
    with pytest.raises(Exception):
        G.set_launch(proj_band_cols=12)
    with pytest.raises(Exception):
        G.set_launch(bp_stack_cols=16)
    G.set_launch(proj_band_cols=6)
    assert G.launch[0] == 6
