"""Pins of the TT separable-footprint oracle (oracle/tt.py) against what the
mathematics and the paper fix, independently of its own formulas:

* the pixel integral of a trapezoid against midpoint quadrature;
* exactness in the parallel-beam limit (a square's chord profile across
  parallel rays is exactly the trapezoid of its corner projections, with the
  central chord as height, and the axial profile a rectangle): the single
  voxel's projection equals the exact area-averaged chord of the cut
  integrals (definition.voxel_definition) at four view angles;
* the paper's accuracy claims (Sec. I, Sec. III-B, Sec. IV-B): on the
  shifted and the large-cone single-voxel setups the cutting voxel projector
  with elevation correction is more accurate than TT at every view, and
  without it falls behind TT at some view of the large-cone setup;
* the published method's own claim that the trapezoid axial footprint beats
  the rectangle at a large cone angle (on average over views);
* A^T is the adjoint of A;
* four planted mistakes are caught.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import oracle.tt as T
from oracle import definition as D

HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(HERE, "golden", "paper_setups.json")) as _f:
    SETUPS = json.load(_f)


def single_voxel(sid, sdd, M, N, pitch, vox, centre, angles):
    return dict(vol_dims=(1, 1, 1), voxel_mm=tuple(vox), vol_offset_mm=tuple(centre), det_cols=M, det_rows=N,
                pitch_mm=(pitch, pitch), principal_px=None, sid_mm=sid, sdd_mm=sdd,
                angles_rad=np.asarray(angles, dtype=np.float64))


def paper_voxel(name, angles):
    s = SETUPS[name]
    return single_voxel(s["sid_mm"], s["sdd_mm"], s["det_cols"], s["det_rows"], s["pitch_mm"], s["voxel_mm"],
                        s["voxel_centre_mm"], angles)


def trapezoid_point(t, x):
    """Height-1 trapezoid with sorted vertices t at the points x."""
    t0, t1, t2, t3 = t
    y = np.zeros_like(x)
    if t1 > t0:
        y = np.where((x > t0) & (x < t1), (x - t0) / (t1 - t0), y)
    y = np.where((x >= t1) & (x <= t2), 1.0, y)
    if t3 > t2:
        y = np.where((x > t2) & (x < t3), (t3 - x) / (t3 - t2), y)
    return y


def test_trapezoid_integral_against_quadrature():
    rng = np.random.default_rng(3)
    cases = [np.sort(rng.uniform(-3, 3, 4)) for _ in range(40)]
    cases += [np.array([0.0, 0.0, 1.0, 1.0]), np.array([0.0, 1.0, 1.0, 2.0]), np.array([0.2, 0.2, 0.2, 0.9]),
              np.array([-1.0, 0.5, 0.5, 0.5])]
    for t in cases:
        for x0 in np.linspace(-3.5, 3.0, 14):
            x1 = x0 + 0.5 + rng.uniform(0, 1.0)
            n = 200000
            xs = x0 + (np.arange(n) + 0.5) * (x1 - x0) / n
            ref = trapezoid_point(t, xs).mean() * (x1 - x0)
            got = float(T.trapezoid_integral(t, x0, x1))
            # midpoint rule: exact on linear pieces, off by at most one cell width at a jump
            assert abs(got - ref) < 2.0 * (x1 - x0) / n + 1e-12, (t, x0, x1, got, ref)


def exact_area_average(g, view, pixels):
    return D.voxel_definition(g, view, (0, 0, 0), pixels, weighting="area")


def footprint_pixels(*projs):
    m = np.zeros_like(projs[0], dtype=bool)
    for p in projs:
        m |= p != 0
    v, u = np.nonzero(m)
    return m, list(zip(u, v))


PARALLEL_ANGLES = [0.0, 0.3, math.pi / 4, 1.1]


def parallel_limit():
    # the source a million mm away: rays through a 1 mm voxel are parallel to
    # about 1e-6, the magnification is 1.0003
    return single_voxel(1e6, 1e6 + 300.0, 24, 24, 0.25, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0), PARALLEL_ANGLES)


def test_parallel_beam_limit_is_exact():
    g = parallel_limit()
    b = T.project(g, np.ones(1))
    for view in range(len(PARALLEL_ANGLES)):
        m, pix = footprint_pixels(b[view])
        ex = exact_area_average(g, view, pix)
        e = np.linalg.norm(b[view][m] - ex) / np.linalg.norm(ex)
        assert e < 1e-6, (view, e)
        # nothing outside the footprint: the exact values there are 0 too
        assert abs(ex.sum() - b[view].sum()) < 1e-6 * ex.sum()


def view_errors(name, nv=12):
    ang = 2 * np.pi * np.arange(nv) / nv + 0.1
    g = paper_voxel(name, ang)
    one = np.ones(1)
    bt = T.project(g, one)
    bc = O.project(g, O.Options(exact=True, ec=True, scaling="cos"), one)
    bc0 = O.project(g, O.Options(exact=True, ec=False, scaling="cos"), one)
    br = T.project(g, one, axial="TR")
    err = {"tt": [], "tr": [], "cvp": [], "cvp_noec": []}
    for view in range(nv):
        m, pix = footprint_pixels(bt[view], bc[view])
        ex = exact_area_average(g, view, pix)
        n = np.linalg.norm(ex)
        for key, b in (("tt", bt), ("tr", br), ("cvp", bc), ("cvp_noec", bc0)):
            err[key].append(np.linalg.norm(b[view][m] - ex) / n)
    return {k: np.array(v) for k, v in err.items()}


@pytest.fixture(scope="module")
def errors():
    return {name: view_errors(name) for name in ("accuracy_large_cone", "accuracy_shifted")}


def test_cvp_with_ec_beats_tt_at_every_view(errors):
    for name, e in errors.items():
        assert np.all(e["cvp"] < e["tt"]), (name, e["cvp"], e["tt"])


def test_cvp_without_ec_falls_behind_tt_somewhere_at_large_cone(errors):
    e = errors["accuracy_large_cone"]
    assert np.any(e["cvp_noec"] > e["tt"]), (e["cvp_noec"], e["tt"])


def test_trapezoid_axial_footprint_beats_rectangle_at_large_cone(errors):
    e = errors["accuracy_large_cone"]
    assert e["tt"].mean() < e["tr"].mean()
    assert np.all(e["tt"] <= e["tr"] * (1 + 1e-9) + 1e-12) or e["tt"].max() < e["tr"].max()


def small_geom():
    return dict(vol_dims=(9, 7, 6), voxel_mm=(1.0, 1.2, 0.9), vol_offset_mm=(0.5, -1.0, 2.0), det_cols=23,
                det_rows=17, pitch_mm=(1.1, 1.3), principal_px=None, sid_mm=120.0, sdd_mm=210.0,
                angles_rad=np.linspace(0, 2 * np.pi, 5, endpoint=False) + 0.2)


def test_adjoint():
    g = small_geom()
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, (6, 7, 9))
    b = rng.uniform(-1, 1, (5, 17, 23))
    lhs = float(np.sum(T.project(g, x) * b))
    rhs = float(np.sum(x * T.backproject(g, b)))
    assert abs(lhs - rhs) < 1e-12 * max(abs(lhs), 1.0)


@pytest.mark.parametrize("mutation", [1, 2, 3, 4])
def test_planted_mistakes_are_caught(mutation):
    """1: amplitude from the longer side crossing; 2: axial rectangle at the
    centre depth (TR) under the TT name; 3: pixel windows shifted by half a
    pixel; 4: transaxial vertices in corner order, unsorted."""
    caught = False
    try:
        T.set_mutation(mutation)
        try:
            test_parallel_beam_limit_is_exact()
        except AssertionError:
            caught = True
        if not caught:
            e = {"accuracy_large_cone": view_errors("accuracy_large_cone", nv=6)}
            try:
                test_cvp_with_ec_beats_tt_at_every_view(e)
                test_trapezoid_axial_footprint_beats_rectangle_at_large_cone(e)
            except AssertionError:
                caught = True
    finally:
        T.set_mutation(0)
    assert caught
