"""GPU (FP32, HIP) against the FP64 oracle, element by element, through the
C ABI.  Sizes span several column groups, bands and k-chunks with ragged
tails; the 512^3 / 248-view workload that bench.py times is checked on
sampled views and voxels the oracle computes one by one."""
import functools

import numpy as np
import pytest
import torch

import oracle as O
from paper_2110_09841_amd import cvp, synth

from gpu_util import assert_parity, needs_gpu, say

pytestmark = [pytest.mark.gpu, needs_gpu]

COMBOS = [("exact", True, "solid_angle"), ("exact", False, "solid_angle"),
          ("relaxed", True, "solid_angle"), ("relaxed", False, "solid_angle"),
          ("exact", True, "cos"), ("relaxed", True, "none")]


def oopts(variant, ec, scaling, raw=False):
    return O.Options(exact=variant == "exact", ec=ec, scaling=scaling, raw_volume=raw)


def gopts(variant, ec, scaling, raw=False):
    return cvp.Options(variant=variant, ec=ec, scaling=scaling, raw_volume=raw)


def run_pair(g, x, b, variant, ec, scaling, tag):
    say("%s %s ec=%d %s vol=%s det=%dx%d views=%d" % (tag, variant, ec, scaling, g["vol_dims"],
                                                      g["det_cols"], g["det_rows"], len(g["angles_rad"])))
    G = cvp.Geometry(g)
    Ax = cvp.project(torch.from_numpy(x).cuda(), G, gopts(variant, ec, scaling)).cpu().numpy()
    Atb = cvp.backproject(torch.from_numpy(b).cuda(), G, gopts(variant, ec, scaling)).cpu().numpy()
    torch.cuda.synchronize()
    o = oopts(variant, ec, scaling)
    assert_parity(Ax, O.project(g, o, x), tag + " A x")
    assert_parity(Atb, O.backproject(g, o, b), tag + " A^T b")


@pytest.mark.parametrize("variant,ec,scaling", COMBOS)
def test_small_workload_full(variant, ec, scaling):
    """64^3 / 96x96 / 32 views: every output compared."""
    g = synth.config_small()
    x = synth.ellipsoid_phantom(64, 1.0, 10, seed=11)
    b = synth.uniform_projections((32, 96, 96), seed=12)
    run_pair(g, x, b, variant, ec, scaling, "small")


def ragged():
    g = synth.geometry((37, 29, 70), (0.9, 1.1, 0.7), 53, 41, 1.3, 260.0, 430.0, 5, 200.0,
                       vol_offset_mm=(1.5, -2.0, 3.0), principal_px=(25.3, 21.8))
    return g


@pytest.mark.parametrize("variant,ec,scaling", COMBOS)
def test_ragged_offset_anisotropic(variant, ec, scaling):
    """Volume sizes that are not multiples of the column group (16) or the
    k-chunk (64), anisotropic voxels, an offset volume, an off-centre
    principal point and an odd detector."""
    g = ragged()
    x = synth.uniform_volume((70, 29, 37), seed=3)
    b = synth.uniform_projections((5, 41, 53), seed=4)
    run_pair(g, x, b, variant, ec, scaling, "ragged")


def test_volume_larger_than_field_of_view():
    """Voxels that project partly or wholly off the detector (dropped)."""
    g = synth.geometry((48, 48, 40), 1.0, 30, 24, 1.2, 200.0, 320.0, 7, 360.0)
    x = synth.uniform_volume((40, 48, 48), seed=5)
    b = synth.uniform_projections((7, 24, 30), seed=6)
    for variant in ("exact", "relaxed"):
        run_pair(g, x, b, variant, True, "solid_angle", "off-detector")


def test_large_voxels_many_pieces():
    """Voxels several pixels wide (up to 8 column pieces per voxel)."""
    g = synth.geometry((6, 7, 5), 2.0, 64, 48, 0.8, 150.0, 240.0, 9, 360.0)
    x = synth.uniform_volume((5, 7, 6), seed=7)
    b = synth.uniform_projections((9, 48, 64), seed=8)
    for variant in ("exact", "relaxed"):
        for ec in (True, False):
            run_pair(g, x, b, variant, ec, "solid_angle", "large-voxels")


def test_wide_elevation_boxes():
    """Large voxels close to the source on a tall detector, the volume
    shifted along x3: the EC depth boxes are wider than half a row, so the
    box average moves several row boundaries of a voxel edge."""
    g = synth.geometry((6, 7, 5), 2.0, 64, 160, 0.8, 150.0, 240.0, 9, 360.0, vol_offset_mm=(0.0, 0.0, 30.0))
    x = synth.uniform_volume((5, 7, 6), seed=17)
    b = synth.uniform_projections((9, 160, 64), seed=18)
    for variant in ("exact", "relaxed"):
        run_pair(g, x, b, variant, True, "solid_angle", "wide-EC")


def test_raw_volume_backprojection():
    """Raw cut volumes (no 1/r^2, no pixel factor) in both directions."""
    g = ragged()
    x = synth.uniform_volume((70, 29, 37), seed=19)
    b = synth.uniform_projections((5, 41, 53), seed=20)
    for variant in ("exact", "relaxed"):
        for ec in (True, False):
            say("raw", variant, ec)
            G = cvp.Geometry(g)
            opts = gopts(variant, ec, "none", raw=True)
            o = oopts(variant, ec, "none", raw=True)
            assert_parity(cvp.project(torch.from_numpy(x).cuda(), G, opts).cpu().numpy(), O.project(g, o, x),
                          "raw A x")
            assert_parity(cvp.backproject(torch.from_numpy(b).cuda(), G, opts).cpu().numpy(),
                          O.backproject(g, o, b), "raw A^T b")


def test_single_voxel_and_single_view():
    g = synth.geometry((1, 1, 1), 1.0, 5, 4, 0.9, 100.0, 170.0, 1, 360.0)
    x = np.ones((1, 1, 1), np.float32)
    b = synth.uniform_projections((1, 4, 5), seed=9)
    for variant in ("exact", "relaxed"):
        run_pair(g, x, b, variant, True, "solid_angle", "one-voxel")


def test_raw_volume_sums_to_voxel_volume():
    """With the raw-volume flag and no pixel scale, each fully projected
    voxel's cut volumes add up to a1 a2 a3 (eq. cutvolume)."""
    g = synth.config_small()
    G = cvp.Geometry(g)
    rng = np.random.default_rng(0)
    for _ in range(6):
        i, j, k = (int(t) for t in rng.integers(0, 64, size=3))
        x = torch.zeros((64, 64, 64), dtype=torch.float32, device="cuda")
        x[k, j, i] = 1.0
        for ec in (False, True):
            say("raw volume voxel", (i, j, k), "ec", ec)
            b = cvp.project(x, G, gopts("exact", ec, "none", raw=True))
            sums = b.double().sum(dim=(1, 2)).cpu().numpy()
            assert np.all(np.abs(sums - 1.0) < 2e-6), sums


@functools.lru_cache(maxsize=1)
def cone_inputs():
    x = synth.ellipsoid_phantom(256, 0.5, 40, seed=21)
    b = synth.uniform_projections((360, 384, 512), seed=22)
    return x, b


@pytest.mark.parametrize("variant", ["exact", "relaxed"])
def test_cone_workload_sampled(variant):
    """256^3 / 512x384 / 360 views (12-degree cone): the GPU computes the whole
    operator, the oracle eight full views spread over the orbit and 2000
    voxels (plus the eight corners of the volume)."""
    g = synth.config_cone()
    x, b = cone_inputs()
    G = cvp.Geometry(g)
    G.cache_records()          # the cut-piece records bench.py caches
    rng = np.random.default_rng(1)
    idx = np.concatenate([corner_indices(256, 256, 256), rng.integers(0, 256 ** 3, size=2000)])
    o = oopts(variant, True, "solid_angle")
    say("cone", variant)
    Ax = cvp.project(torch.from_numpy(x).cuda(), G, gopts(variant, True, "solid_angle")).cpu().numpy()
    for view in (0, 45, 97, 150, 203, 256, 301, 359):
        assert_parity(Ax[view], O.project(g, o, x, views=(view, view + 1))[0], "cone %s A x view %d" % (variant, view))
    del Ax
    Atb = cvp.backproject(torch.from_numpy(b).cuda(), G, gopts(variant, True, "solid_angle")).cpu().numpy()
    assert_parity(Atb.ravel()[idx], O.backproject_voxels(g, o, b, idx), "cone %s A^T b sampled" % variant)


def corner_indices(n1, n2, n3):
    return np.array([i + n1 * (j + n2 * k) for i in (0, n1 - 1) for j in (0, n2 - 1) for k in (0, n3 - 1)])


@functools.lru_cache(maxsize=1)
def carm_inputs():
    x = synth.ellipsoid_phantom(512, 0.25, 80, seed=31, noise_frac=0.01)
    b = synth.uniform_projections((248, 480, 616), seed=32)
    return x, b


@pytest.mark.parametrize("variant", ["relaxed", "exact"])
def test_carm_benchmark_workload_sampled(variant):
    """The benchmark workload (512^3 / 616x480 / 248 views over 200 degrees,
    elevation correction, cached cut-piece records as bench.py times it):
    the oracle checks
    eight full views of A x spread over the arc and 2000 voxels of A^T b plus
    the volume's corners, for the relaxed and the exact form."""
    g = synth.config_carm()
    x, b = carm_inputs()
    G = cvp.Geometry(g)
    G.cache_records()          # the cut-piece records bench.py caches
    o = oopts(variant, True, "solid_angle")
    say("carm projection", variant)
    Ax = cvp.project(torch.from_numpy(x).cuda(), G, gopts(variant, True, "solid_angle")).cpu().numpy()
    for view in (0, 31, 66, 99, 124, 171, 208, 247):
        assert_parity(Ax[view], O.project(g, o, x, views=(view, view + 1))[0],
                      "carm %s A x view %d" % (variant, view))
    del Ax
    say("carm backprojection", variant)
    Atb = cvp.backproject(torch.from_numpy(b).cuda(), G, gopts(variant, True, "solid_angle")).cpu().numpy()
    rng = np.random.default_rng(2)
    idx = np.concatenate([corner_indices(512, 512, 512), rng.integers(0, 512 ** 3, size=2000)])
    assert_parity(Atb.ravel()[idx], O.backproject_voxels(g, o, b, idx), "carm %s A^T b sampled" % variant)


def test_adjoint_and_determinism():
    """<A x, y> = <x, A^T y> (Sec. III-D) with FP64 dots of FP32 results, and
    bitwise-equal reruns (no float atomics across waves or workgroups)."""
    for g, tag in ((synth.config_small(), "small"), (ragged(), "ragged")):
        G = cvp.Geometry(g)
        n3, n2, n1 = G.vol_shape
        x = torch.from_numpy(synth.uniform_volume((n3, n2, n1), seed=13)).cuda()
        y = torch.from_numpy(synth.uniform_projections(G.proj_shape, seed=14)).cuda()
        for variant in ("exact", "relaxed"):
            say("adjoint", tag, variant)
            opts = gopts(variant, True, "solid_angle")
            Ax = cvp.project(x, G, opts)
            Aty = cvp.backproject(y, G, opts)
            lhs = float((Ax.double() * y.double()).sum())
            rhs = float((x.double() * Aty.double()).sum())
            assert abs(lhs - rhs) <= 1e-6 * abs(lhs), (lhs, rhs)
            assert torch.equal(Ax, cvp.project(x, G, opts))
            assert torch.equal(Aty, cvp.backproject(y, G, opts))


def _project_scanning(x, G, opts):
    """cvp_project without the workspace (the kernel reads its wedges for the scale)."""
    import ctypes
    from paper_2110_09841_amd import _lib
    out = torch.empty(G.proj_shape, dtype=torch.float32, device="cuda")
    o = opts.c()
    _lib.check(_lib.lib().cvp_project(G.handle, ctypes.byref(o), ctypes.c_void_p(x.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()),
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return out


def test_workspace_projection_equals_scanning_projection():
    """The per-group maxima path (cvp_project_ws, used by cvp.project) gives
    the same scales, hence bitwise the same projections, as the kernel's own
    wedge scan: ragged n1 (not a multiple of 16 or 4), an offset volume, a
    volume with a hot spot, and a non-finite voxel (its bands NaN in both)."""
    for g, tag in ((synth.config_small(), "small"), (ragged(), "ragged")):
        G = cvp.Geometry(g)
        x = torch.from_numpy(synth.uniform_volume(G.vol_shape, seed=21)).cuda()
        x[G.vol_shape[0] // 2, 3, 5] = 1e6       # hot spot: one wedge scale far above the rest
        for variant in ("exact", "relaxed"):
            opts = gopts(variant, True, "solid_angle")
            say("workspace projection", tag, variant)
            assert torch.equal(cvp.project(x, G, opts), _project_scanning(x, G, opts))
        xn = x.clone()
        xn[1, 2, 3] = float("nan")
        opts = gopts("relaxed", True, "solid_angle")
        a, b = cvp.project(xn, G, opts), _project_scanning(xn, G, opts)
        assert torch.equal(torch.isnan(a), torch.isnan(b)) and bool(torch.isnan(a).any())
        assert torch.equal(torch.nan_to_num(a), torch.nan_to_num(b))


def test_workspace_too_small_is_rejected():
    import ctypes
    from paper_2110_09841_amd import _lib
    G = cvp.Geometry(synth.config_small())
    x = torch.zeros(G.vol_shape, dtype=torch.float32, device="cuda")
    out = torch.empty(G.proj_shape, dtype=torch.float32, device="cuda")
    need = ctypes.c_int64()
    _lib.check(_lib.lib().cvp_project_workspace_size(G.handle, ctypes.byref(need)))
    work = torch.empty(need.value // 4, dtype=torch.int32, device="cuda")
    o = gopts("relaxed", True, "solid_angle").c()
    st = _lib.lib().cvp_project_ws(G.handle, ctypes.byref(o), ctypes.c_void_p(x.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(work.data_ptr()),
                                   need.value - 4, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.CVP_E_INVALID and "work_bytes" in _lib.last_error()
