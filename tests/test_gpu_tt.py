"""The TT separable-footprint projector (the comparator of Sec. I and IV,
Long, Fessler & Balter 2010) on the cutting voxel projector's work split
(Sec. V-C), through the C ABI, against its FP64 oracle (oracle/tt.py)
element by element: a ragged, offset, anisotropic volume on a cone
geometry, a camera-matrix trajectory, fine detectors whose voxel footprints
span up to ~15 columns, and the paper's single-voxel setups; plus the
adjoint identity on the GPU, CGLS on the TT operators, and the option
checks."""
import json
import os

import numpy as np
import pytest
import torch

import oracle.tt as T
from paper_2110_09841_amd import _lib, cvp, synth

from gpu_util import assert_parity, needs_gpu, say

pytestmark = [pytest.mark.gpu, needs_gpu]

HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(HERE, "golden", "paper_setups.json")) as _f:
    SETUPS = json.load(_f)


def cone_geom():
    # 37 x 29 x 30 voxels, about 9 degrees of cone half-angle, 12 views
    return synth.geometry((37, 29, 30), (0.9, 1.1, 0.7), 61, 47, 1.3, 160.0, 300.0, 12, 360.0,
                          vol_offset_mm=(1.5, -2.0, 3.0))


def check(g, x, b, what):
    G = cvp.Geometry(g)
    say(what)
    got = cvp.project(torch.from_numpy(x).cuda(), G, cvp.TT).cpu().numpy()
    assert_parity(got, T.project(g, x), what + " A x")
    gotb = cvp.backproject(torch.from_numpy(b).cuda(), G, cvp.TT).cpu().numpy()
    assert_parity(gotb, T.backproject(g, b), what + " A^T b")


def test_cone_volume():
    g = cone_geom()
    x = synth.uniform_volume((30, 29, 37), seed=81)
    b = synth.uniform_projections((12, 47, 61), seed=82)
    check(g, x, b, "TT cone 37x29x30, 12 views")


def test_signed_phantom():
    g = cone_geom()
    x = synth.ellipsoid_phantom((37, 29, 30), (0.9, 1.1, 0.7), 6, seed=83, semi_axes_mm=(2.0, 9.0))
    x = (x - 0.5 * x.max()).astype(np.float32)
    b = (synth.uniform_projections((12, 47, 61), seed=84) - 0.5).astype(np.float32)
    check(g, x, b, "TT signed phantom")


def test_camera_matrices():
    """A wobbling C-arm orbit given as per-view camera matrices (Sec. III-C)."""
    g = synth.matrix_geometry((37, 29, 30), (0.9, 1.1, 0.7), 61, 47, 1.3, 160.0, 300.0, 12, 360.0, seed=85,
                              vol_offset_mm=(1.5, -2.0, 3.0))
    x = synth.uniform_volume((30, 29, 37), seed=86)
    b = synth.uniform_projections((12, 47, 61), seed=87)
    check(g, x, b, "TT camera matrices")


def test_fine_detector_volume():
    """14 x 11 x 9 voxels of 1 mm on 616 x 480 pixels of 0.154 mm: about 15
    columns per voxel (the wide-footprint kernels)."""
    g = synth.geometry((14, 11, 9), 1.0, 616, 480, 0.154, 749.0, 1198.0, 6, 360.0, vol_offset_mm=(1.3, -0.7, 2.1))
    x = np.random.default_rng(88).uniform(0, 1, (9, 11, 14)).astype(np.float32)
    b = synth.uniform_projections((6, 480, 616), seed=89)
    check(g, x, b, "TT fine detector")


@pytest.mark.parametrize("name", ["accuracy_shifted", "accuracy_large_cone"])
def test_single_voxel_setups(name):
    s = SETUPS[name]
    g = synth.geometry((1, 1, 1), s["voxel_mm"], s["det_cols"], s["det_rows"], s["pitch_mm"], s["sid_mm"],
                       s["sdd_mm"], 24, 360.0, vol_offset_mm=s["voxel_centre_mm"])
    x = np.ones((1, 1, 1), np.float32)
    G = cvp.Geometry(g)
    got = cvp.project(torch.from_numpy(x).cuda(), G, cvp.TT).cpu().numpy()
    assert_parity(got, T.project(g, x), "TT single voxel " + name)


def test_adjoint_on_gpu():
    g = cone_geom()
    G = cvp.Geometry(g)
    x = torch.rand(G.vol_shape, device="cuda")
    b = torch.rand(G.proj_shape, device="cuda")
    lhs = float((cvp.project(x, G, cvp.TT).double() * b.double()).sum())
    rhs = float((x.double() * cvp.backproject(b, G, cvp.TT).double()).sum())
    say("TT <Ax,b> %.9e <x,A^T b> %.9e" % (lhs, rhs))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_cgls_on_tt_operators():
    g = cone_geom()
    G = cvp.Geometry(g)
    xt = torch.from_numpy(synth.ellipsoid_phantom((37, 29, 30), (0.9, 1.1, 0.7), 5, seed=90,
                                                  semi_axes_mm=(2.0, 9.0))).cuda()
    b = cvp.project(xt, G, cvp.TT)
    x, info = cvp.cgls(G, b, cvp.TT, tol=1e-3, max_iter=200, per_graph=5)
    its, rho = info["iterations"], info["rho"]
    say("TT CGLS %d iterations, rho %.2e" % (its, rho[its]))
    assert rho[its] <= 1e-3


def test_options_checked():
    g = cone_geom()
    G = cvp.Geometry(g)
    x = torch.rand(G.vol_shape, device="cuda")
    for bad in (cvp.Options(variant="tt", ec=False, scaling="solid_angle"),
                cvp.Options(variant="tt", ec=True, scaling="cos"),
                cvp.Options(variant="tt", ec=False, scaling="cos", raw_volume=True)):
        with pytest.raises(_lib.CVPError) as ei:
            cvp.project(x, G, bad)
        assert ei.value.status == _lib.CVP_E_INVALID
    batch = cvp.Batch([G, G])
    with pytest.raises(_lib.CVPError) as ei:
        cvp.project_batched([x, x.clone()], batch, cvp.TT)
    assert ei.value.status == _lib.CVP_E_UNSUPPORTED


@pytest.mark.parametrize("name", ["pfeiffer", "long"])
def test_paper_speed_benchmarks_sampled(name):
    """The TT projector at the sizes the paper times it (Sec. IV-A, Tables I
    and II; the same geometries bench.py times): the GPU computes the whole
    operator, the oracle full views of A x and sampled voxels of A^T b."""
    if name == "pfeiffer":
        g = synth.geometry(256, 0.5, 1280, 960, 0.25, 750.0, 1000.0, 100, 198.0)
        views, nvox = (61,), 1000
    else:
        g = synth.geometry((512, 512, 128), 0.5, 512, 512, 1.0, 541.0, 949.0, 720, 360.0)
        views, nvox = (397,), 500
    G = cvp.Geometry(g)
    n3, n2, n1 = G.vol_shape
    x = synth.uniform_volume(G.vol_shape, seed=97)
    say("TT", name, "projection")
    Ax = cvp.project(torch.from_numpy(x).cuda(), G, cvp.TT).cpu().numpy()
    for v in views:
        assert_parity(Ax[v], T.project(g, x, views=(v, v + 1))[0], "TT %s A x view %d" % (name, v))
    del Ax
    b = synth.uniform_projections(G.proj_shape, seed=98)
    say("TT", name, "backprojection")
    Atb = cvp.backproject(torch.from_numpy(b).cuda(), G, cvp.TT).cpu().numpy().ravel()
    rng = np.random.default_rng(99)
    idx = np.concatenate([[0, n1 - 1, n1 * n2 * n3 - 1], rng.integers(0, n1 * n2 * n3, size=nvox)])
    assert_parity(Atb[idx], T.backproject_voxels(g, b, idx), "TT %s A^T b sampled" % name)
