"""The GPU SiddonK projector (cvp_project_siddon) against the oracle's
brute-force definition (oracle/definition.py: every ray against every voxel
box by the slab method, no traversal), element by element: a ragged, offset,
anisotropic volume on a small detector for several K, and the paper's
single voxel at the isocentre on a cropped fine detector."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import definition as D
from paper_2110_09841_amd import cvp, synth

from gpu_util import assert_parity, needs_gpu, say

pytestmark = [pytest.mark.gpu, needs_gpu]

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("K", [1, 2, 3, 5])
def test_siddon_ragged_volume(K):
    g = synth.geometry((6, 5, 7), (0.9, 1.1, 0.7), 17, 13, 1.3, 60.0, 100.0, 3, 200.0,
                       vol_offset_mm=(0.7, -0.4, 0.9), principal_px=(8.3, 6.1))
    x = synth.uniform_volume((7, 5, 6), seed=61)
    say("siddon ragged K", K)
    G = cvp.Geometry(g)
    got = cvp.project_siddon(torch.from_numpy(x).cuda(), G, K).cpu().numpy()
    ref = D.siddon_project(g, x, K)
    assert_parity(got, ref, "siddon K=%d" % K)
    # pixels outside the volume's shadow are exactly zero on both sides
    assert np.array_equal(got == 0.0, ref == 0.0)


def test_siddon_isocentre_voxel_cropped_detector():
    s = json.load(open(os.path.join(HERE, "golden", "paper_setups.json")))["accuracy_isocentre"]
    # the paper's 1 x 1 x 5 mm voxel at the isocentre, detector cropped to the
    # 24 x 64 pixels around the principal point (same pitch and distances)
    g = synth.geometry((1, 1, 1), s["voxel_mm"], 24, 64, s["pitch_mm"], s["sid_mm"], s["sdd_mm"], 360, 360.0)
    g["angles_rad"] = g["angles_rad"][[0, 17, 45]]
    x = np.ones((1, 1, 1), np.float32)
    G = cvp.Geometry(g)
    for K in (4, 16):
        say("siddon isocentre voxel K", K)
        got = cvp.project_siddon(torch.from_numpy(x).cuda(), G, K).cpu().numpy()
        assert_parity(got, D.siddon_project(g, x, K), "siddon isocentre K=%d" % K)


def test_siddon_rejects_bad_K():
    from paper_2110_09841_amd import _lib
    G = cvp.Geometry(synth.config_small())
    x = torch.zeros(G.vol_shape, dtype=torch.float32, device="cuda")
    for K in (0, 1025):
        with pytest.raises(_lib.CVPError):
            cvp.project_siddon(x, G, K)
