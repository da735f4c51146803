"""Launch plans: every band width and stack width computes the same operator
(parity with the FP64 oracle for each), invalid plans are rejected without
changing the plan in use, and the autotuner picks, applies and caches a plan."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2110_09841_amd import _lib, cvp, synth
from paper_2110_09841_amd.autotune import autotune

from gpu_util import assert_parity, needs_gpu, rel_l2, say

pytestmark = [pytest.mark.gpu, needs_gpu]


def geometry():
    """Ragged sizes, an offset volume and 7 views: several bands and column
    groups for every band width."""
    return synth.geometry((45, 38, 70), (0.9, 1.0, 0.8), 61, 47, 1.2, 300.0, 480.0, 7, 200.0,
                          vol_offset_mm=(1.0, -1.5, 2.0))


def test_every_plan_matches_the_oracle():
    g = geometry()
    x = synth.ellipsoid_phantom(g["vol_dims"], g["voxel_mm"], 8, seed=3)
    b = synth.uniform_projections((7, 47, 61), seed=4)
    o = O.Options(exact=False, ec=True)
    ref_p, ref_b = O.project(g, o, x), O.backproject(g, o, b)
    G = cvp.Geometry(g)
    opts = cvp.Options(variant="relaxed", ec=True)
    xd, bd = torch.from_numpy(x).cuda(), torch.from_numpy(b).cuda()
    default = G.launch
    outs = []
    for u in (1, 3, 7, 16, 32):
        say("plan band", u)
        G.set_launch(u, 0)
        assert G.launch == (u,) + default[1:]
        p = cvp.project(xd, G, opts).cpu().numpy()
        assert_parity(p, ref_p, "A x, band %d" % u)
        outs.append(p)
    for p in outs[1:]:
        assert rel_l2(p, outs[0]) < 1e-6
    backs = []
    for gw in (4, 8, 16):
        for kp in (1, 2):
            say("plan stack", gw, "passes", kp)
            G.set_launch(0, gw, kp)
            assert G.launch == (default[0], gw, kp)
            backs.append(cvp.backproject(bd, G, opts).cpu().numpy())
            assert_parity(backs[-1], ref_b, "A^T b, stack %d, %d passes" % (gw, kp))
    # the backprojection's sums do not depend on the plan
    for v in backs[1:]:
        assert np.array_equal(v, backs[0])
    G.set_launch(0, 0)
    assert G.launch == default


def test_invalid_plans_are_rejected_and_leave_the_plan():
    g = synth.geometry(16, 1.0, 32, 3000, 0.5, 750.0, 1200.0, 2, 360.0)
    G = cvp.Geometry(g)
    before = G.launch
    wpc_before = G.bp_workgroups_per_cu
    for u, gw, kp, wpc, status in ((33, 0, 0, 0, _lib.CVP_E_INVALID), (-1, 0, 0, 0, _lib.CVP_E_INVALID),
                                   (0, 5, 0, 0, _lib.CVP_E_INVALID), (0, 0, 3, 0, _lib.CVP_E_INVALID),
                                   (0, 0, 0, 2, _lib.CVP_E_INVALID), (0, 0, 0, 5, _lib.CVP_E_INVALID),
                                   (32, 0, 0, 0, _lib.CVP_E_UNSUPPORTED)):
        with pytest.raises(_lib.CVPError) as ei:
            G.set_launch(u, gw, kp, wpc)
        assert ei.value.status == status, (u, gw, kp, wpc, ei.value)
        assert G.launch == before and G.bp_workgroups_per_cu == wpc_before


def test_autotune_chooses_the_backprojection_budget_with_cached_records(tmp_path):
    g = synth.config_small()
    G = cvp.Geometry(g)
    G.cache_records()
    opts = cvp.Options(variant="relaxed", ec=True)
    cache = str(tmp_path / "plans.json")
    say("autotune, cached records")
    rec = autotune(G, opts, bands=(8,), stacks=(16,), passes=(2,), reps=1, cache=cache)
    assert rec["bp_workgroups_per_cu"] in (3, 4)
    assert set(rec["backproject_ms"]) == {"16/2/4", "16/2/3", "16/2/4/s", "16/2/3/s"}
    assert G.bp_workgroups_per_cu == rec["bp_workgroups_per_cu"]
    G2 = cvp.Geometry(g)
    G2.cache_records()
    rec2 = autotune(G2, opts, cache=cache)
    assert rec2["cached"] and G2.launch == G.launch and G2.bp_workgroups_per_cu == G.bp_workgroups_per_cu
    b = torch.from_numpy(synth.uniform_projections(G.proj_shape, seed=95)).cuda()
    G3 = cvp.Geometry(g)
    assert torch.equal(cvp.backproject(b, G2, opts), cvp.backproject(b, G3, opts))


def test_autotune_sets_and_caches_a_plan(tmp_path):
    g = synth.config_small()
    G = cvp.Geometry(g)
    opts = cvp.Options(variant="relaxed", ec=True)
    cache = str(tmp_path / "plans.json")
    say("autotune")
    rec = autotune(G, opts, bands=(4, 8, 16), stacks=(16, 8), reps=1, cache=cache)
    assert not rec["cached"]
    assert G.launch == (rec["proj_band_cols"], rec["bp_stack_cols"], rec["bp_passes"])
    assert rec["proj_band_cols"] in (4, 8, 16) and rec["bp_stack_cols"] in (16, 8) and rec["bp_passes"] in (1, 2)
    G2 = cvp.Geometry(g)
    rec2 = autotune(G2, opts, cache=cache)
    assert rec2["cached"] and G2.launch == G.launch
    # a tuned plan still computes the operator
    x = synth.ellipsoid_phantom(64, 1.0, 10, seed=11)
    o = O.Options(exact=False, ec=True)
    assert_parity(cvp.project(torch.from_numpy(x).cuda(), G2, opts).cpu().numpy(), O.project(g, o, x),
                  "A x, tuned plan")
