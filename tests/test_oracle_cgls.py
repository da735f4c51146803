"""Pins of the FP64 CGLS oracle: on an explicit full-rank matrix it reaches
the least-squares solution (numpy.linalg.lstsq) in n iterations, and the
residual norm |b - A x_k| never increases (CGLS minimises it over growing
Krylov spaces)."""
import numpy as np

import oracle as O
from oracle.cgls import cgls
from paper_2110_09841_amd import synth


def test_cgls_matches_lstsq_on_explicit_matrix():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((40, 12))
    b = rng.standard_normal(40)
    x, gam, rn = cgls(lambda v: A @ v, lambda v: A.T @ v, b, 12, np.zeros(12))
    ref = np.linalg.lstsq(A, b, rcond=None)[0]
    assert np.linalg.norm(x - ref) < 1e-8 * np.linalg.norm(ref)
    assert np.all(np.diff(rn) <= 1e-12 * rn[0])


def test_cgls_on_cvp_oracle_monotone():
    g = synth.geometry((10, 9, 8), 1.0, 16, 14, 1.4, 200.0, 330.0, 6, 360.0)
    opts = O.Options(exact=False, ec=True)
    xt = synth.uniform_volume((8, 9, 10), seed=1).astype(np.float64)
    b = O.project(g, opts, xt)
    x, gam, rn = cgls(lambda v: O.project(g, opts, v), lambda v: O.backproject(g, opts, v), b, 15,
                      np.zeros_like(xt))
    assert np.all(np.diff(rn) <= 1e-12 * rn[0])
    assert np.sqrt(gam[-1] / gam[0]) < 1e-2
