"""Planted mistakes in the oracle (switched on in the C code by a test-only
flag, on the CPU) must each be caught by at least one pin: a mirrored
detector axis, a wrong pixel edge, the depth taken at the wrong point, a wrong
row plane, 1/r in place of 1/r^2, a shifted index in A^T, and three mistakes
at the detector's edges: the part of a voxel left or right of the detector
merged into its first or last column, the weights of a partly projected
voxel renormalised to the whole voxel, the rows above or below the detector
merged into its edge rows."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import definition as D
from paper_2110_09841_amd import synth

RAW = O.Options(exact=True, ec=False, scaling="none", raw_volume=True)
EX_EC = O.Options(exact=True, ec=True)


def pin_volume_partition():
    g = synth.config_small()
    rng = np.random.default_rng(0)
    for _ in range(20):
        i, j, k = (int(t) for t in rng.integers(0, 64, size=3))
        ws = O.voxel_weights(g, RAW, int(rng.integers(0, 32)), i, j, k)[2]
        assert abs(ws.sum() - 1.0) < 1e-12


def pin_exact_polyhedron():
    """A_u d_uv equals the exact cut volume when no row plane crosses the top
    or bottom face inside the base (same condition as in the pins)."""
    g = synth.config_cone()
    G = O.Geometry(g)
    rng = np.random.default_rng(7)
    f, b2, c2 = 900.0, 0.388, 191.5
    checked = 0
    while checked < 6:
        i, j, k = (int(t) for t in rng.integers(0, 256, size=3))
        view = int(rng.integers(0, 360))
        lo, hi = D.voxel_box(g, i, j, k)
        s, e1, e2, d = D.frame(g, view)
        dep = [d[0] * (x - s[0]) + d[1] * (y - s[1]) for x in (lo[0], hi[0]) for y in (lo[1], hi[1])]
        spans = [c2 - (z * f / b2) / np.array([min(dep), max(dep)]) for z in (lo[2], hi[2])]
        if any(np.floor(sp[0] + 0.5) != np.floor(sp[1] + 0.5) for sp in spans):
            continue
        us, vs, ws = O.voxel_weights(G, RAW, view, i, j, k)
        if not len(ws):
            continue
        for u, v, w in zip(us, vs, ws):
            assert abs(w - D.cut_integrals(g, view, (i, j, k), u, v)[0]) < 1e-9 * 0.125
        checked += 1


def pin_adjoint():
    g = synth.geometry((6, 5, 4), 1.0, 12, 10, 1.5, 200.0, 350.0, 3, 200.0)
    rng = np.random.default_rng(1)
    x, b = rng.random((4, 5, 6)), rng.random((3, 10, 12))
    lhs = float(np.sum(b * O.project(g, EX_EC, x)))
    rhs = float(np.sum(x * O.backproject(g, EX_EC, b)))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def pin_single_voxel_closed_form():
    g = synth.geometry(3, 0.1, 9, 9, 20.0, 700.0, 1100.0, 4, 360.0)
    G = O.Geometry(g)
    us, vs, ws = O.voxel_weights(G, EX_EC, 1, 1, 1, 1)
    sig = O.pixel_scale(G, "solid_angle")[4, 4]
    ref = 1e-3 / (700.0 ** 2 * D.pixel_solid_angle_arctan(1100.0, -10, 10, -10, 10))
    assert len(ws) == 1 and abs(ws[0] * sig - ref) < 1e-12 * ref


def pin_pixel_ray():
    g = synth.config_cone()
    rng = np.random.default_rng(2)
    for _ in range(5):
        view = int(rng.integers(0, 360))
        u, v = rng.uniform(0, 511), rng.uniform(0, 383)
        P = D.detector_point(g, view, u, v)[0]
        s = D.frame(g, view)[0]
        chi = O.project_point(g, view, s + 0.5 * (P - s))
        assert np.allclose(chi, [u, v], atol=1e-9)


def pin_parallel_limit():
    lam = math.radians(30.0)
    g = synth.geometry((5, 5, 5), 1.0, 21, 21, 2.0, 1e6, 2e6, 1, 360.0)
    g["angles_rad"] = np.array([lam])
    G = O.Geometry(g)
    opts = O.Options(exact=True, ec=True, scaling="cos")
    us, vs, ws = O.voxel_weights(G, opts, 0, 2, 2, 2)
    sig = O.pixel_scale(G, "cos")
    tot = sum(w * sig[v, u] for u, v, w in zip(us, vs, ws))
    assert abs(tot - 1.0) < 2e-5     # unit voxel volume over unit object pixels


def pin_off_detector():
    """Voxels straddling the detector's edges keep exactly the cut volumes of
    their on-detector pixels (the identity of pin_exact_polyhedron); the rest
    is dropped."""
    from test_oracle_pins import edge_geometry, straddling_cases
    g = edge_geometry()
    G = O.Geometry(g)
    cases, _ = straddling_cases(g, 3, 10, 11, need_no_crossing=True)
    for ijk, view in cases:
        us, vs, ws = O.voxel_weights(G, RAW, view, *ijk)
        assert np.all((us >= 0) & (us < g["det_cols"]) & (vs >= 0) & (vs < g["det_rows"]))
        for u, v, w in zip(us, vs, ws):
            assert abs(w - D.cut_integrals(g, view, ijk, int(u), int(v))[0]) < 1e-9


PINS = [pin_volume_partition, pin_exact_polyhedron, pin_adjoint,
        pin_single_voxel_closed_form, pin_pixel_ray, pin_parallel_limit, pin_off_detector]


def _failing(pins):
    out = []
    for p in pins:
        try:
            p()
        except AssertionError:
            out.append(p.__name__)
    return out


def test_pins_hold_without_mutation():
    O.set_mutation(0)
    assert _failing(PINS) == []


@pytest.mark.parametrize("mutation", [1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_planted_mistake_is_caught(mutation):
    O.set_mutation(mutation)
    try:
        failing = _failing(PINS)
    finally:
        O.set_mutation(0)
    assert failing, "mutation %d went unnoticed" % mutation
