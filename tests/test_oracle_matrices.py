"""Pins of the oracle on general trajectories given as one camera matrix per
view (Sec. III-C), under the convention of Sec. III-A (chi1 independent of
x3, chi2 opposite to x3).  The oracle takes each matrix apart (RQ) into a
frame and intrinsics; the pins come from the matrices themselves:

* a circular orbit written as matrices (any nonzero scale, either sign) gives
  the circular results;
* a point projects to the dehomogenised P [x; 1];
* the cut volumes of a fully projected voxel add up to the voxel's volume,
  and equal the exact volume of voxel n pixel pyramid (half-spaces taken
  from the matrix rows, definition.py) where no row plane crosses the top or
  bottom face over the base;
* 1 / the solid-angle factor equals the solid angle of the pyramid through
  the rays M^-1 (u +- 1/2, v +- 1/2, 1);
* <A x, y> = <x, A^T y>;
* a matrix that breaks the convention is refused.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import definition as D
from paper_2110_09841_amd import synth

RAW = O.Options(exact=True, ec=False, scaling="none", raw_volume=True)


def wobbly(seed=3, n_views=8):
    return synth.matrix_geometry((12, 10, 9), (0.9, 1.1, 0.8), 48, 40, 1.3, 200.0, 330.0, n_views, seed=seed,
                                 vol_offset_mm=(0.5, -0.3, 0.4))


def test_circular_orbit_as_matrices():
    g = synth.geometry((12, 10, 9), (0.9, 1.1, 0.8), 40, 32, 1.3, 200.0, 330.0, 6, 360.0,
                       vol_offset_mm=(0.5, -0.3, 0.4), principal_px=(20.2, 15.7))
    x = synth.uniform_volume((9, 10, 12), seed=1)
    y = synth.uniform_projections((6, 32, 40), seed=2)
    for scale in (1.0, -2.5):
        gm = dict(vol_dims=g["vol_dims"], voxel_mm=g["voxel_mm"], vol_offset_mm=g["vol_offset_mm"],
                  det_cols=40, det_rows=32, matrices=scale * synth.circular_matrices(g))
        for opts in (O.Options(exact=True, ec=True), O.Options(exact=False, ec=False, scaling="cos")):
            a, b = O.project(g, opts, x), O.project(gm, opts, x)
            assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a)
            a, b = O.backproject(g, opts, y), O.backproject(gm, opts, y)
            assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a)


def test_point_projection_is_the_matrix():
    g = wobbly()
    rng = np.random.default_rng(4)
    for view in range(8):
        P = np.asarray(g["matrices"][view])
        for _ in range(5):
            x = rng.uniform(-5, 5, 3)
            h = P @ np.append(x, 1.0)
            chi = O.project_point(g, view, x)
            assert np.allclose(chi, h[:2] / h[2], rtol=0, atol=1e-10), (view, chi, h[:2] / h[2])


def test_cut_volumes_partition_the_voxel():
    g = wobbly()
    a = np.prod(g["voxel_mm"])
    n1, n2, n3 = g["vol_dims"]
    rng = np.random.default_rng(5)
    for _ in range(60):
        i, j, k = int(rng.integers(0, n1)), int(rng.integers(0, n2)), int(rng.integers(0, n3))
        view = int(rng.integers(0, 8))
        for ec in (False, True):
            o = O.Options(exact=True, ec=ec, scaling="none", raw_volume=True)
            us, vs, ws = O.voxel_weights(g, o, view, i, j, k)
            assert abs(ws.sum() - a) < 1e-12 * a, (i, j, k, view, ec, ws.sum(), a)


def _row_planes_cross(g, view, ijk):
    """True if a row boundary chi2 = t plane crosses the voxel's top or bottom
    face over its base (from the matrix: chi2 over the four top/bottom corners)."""
    P = D.camera(g, view)
    lo, hi = D.voxel_box(g, *ijk)
    for z in (lo[2], hi[2]):
        chis = []
        for x in (lo[0], hi[0]):
            for y in (lo[1], hi[1]):
                h = P @ np.array([x, y, z, 1.0])
                chis.append(h[1] / h[2])
        if np.floor(min(chis) + 0.5) != np.floor(max(chis) + 0.5):
            return True
    return False


def test_cut_volume_equals_exact_polyhedron():
    g = wobbly()
    n1, n2, n3 = g["vol_dims"]
    rng = np.random.default_rng(6)
    checked = 0
    for _ in range(4000):
        ijk = (int(rng.integers(0, n1)), int(rng.integers(0, n2)), int(rng.integers(0, n3)))
        view = int(rng.integers(0, 8))
        if _row_planes_cross(g, view, ijk):
            continue
        us, vs, ws = O.voxel_weights(g, RAW, view, *ijk)
        for u, v, w in zip(us, vs, ws):
            vol = D.cut_integrals(g, view, ijk, u, v)[0]
            assert abs(w - vol) < 1e-9 * np.prod(g["voxel_mm"]), (ijk, view, u, v, w, vol)
        checked += 1
        if checked >= 25:
            break
    assert checked >= 25


def test_solid_angle_factor_from_corner_rays():
    g = wobbly()
    for view in (0, 3, 7):
        sig = O.pixel_scale(g, "solid_angle", view=view)
        for (u, v) in ((0, 0), (47, 39), (20, 17), (5, 33)):
            om = D.pixel_solid_angle_matrix(g, view, u, v)
            assert abs(1.0 / sig[v, u] - om) < 1e-9 * om, (view, u, v)


def test_adjoint_identity():
    g = wobbly()
    x = synth.uniform_volume((9, 10, 12), seed=7)
    y = synth.uniform_projections((8, 40, 48), seed=8)
    for opts in (O.Options(exact=True, ec=True), O.Options(exact=False, ec=True, scaling="cos")):
        lhs = float(np.vdot(O.project(g, opts, x), y))
        rhs = float(np.vdot(x, O.backproject(g, opts, y)))
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_convention_violations_refused():
    g = wobbly()
    P = np.array(g["matrices"])
    roll = math.radians(3.0)            # detector rolled about its principal ray
    Rz = np.array([[math.cos(roll), -math.sin(roll), 0.0], [math.sin(roll), math.cos(roll), 0.0], [0, 0, 1.0]])
    bad = dict(g)
    bad["matrices"] = np.einsum("ij,vjk->vik", Rz, P)
    with pytest.raises(ValueError):
        O.Geometry(bad)
    flip = dict(g)
    flip["matrices"] = P * np.array([1.0, -1.0, 1.0])[None, :, None]     # chi2 along +x3
    with pytest.raises(ValueError):
        O.Geometry(flip)
