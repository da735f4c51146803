"""Helpers shared by the GPU tests (comparison metrics, case logging)."""
import sys

import numpy as np
import pytest
import torch

# Parity bar for FP32 GPU results against the FP64 oracle:
#   relative L2 <= 1e-5, max per-element relative error <= 1e-4 with the
#   denominator floored at 1e-3 * max|oracle| (elements that are ~0 would
#   otherwise turn rounding noise into huge ratios).
REL_L2 = 1e-5
MAX_REL = 1e-4
FLOOR = 1e-3

needs_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def rel_l2(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def max_rel(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.maximum(np.abs(ref), FLOOR * np.abs(ref).max())
    return float(np.max(np.abs(got - ref) / np.maximum(den, 1e-300)))


def assert_parity(got, ref, what):
    e2, em = rel_l2(got, ref), max_rel(got, ref)
    say("%s: rel L2 %.3e, max rel %.3e" % (what, e2, em))
    assert e2 <= REL_L2, (what, e2, em)
    assert em <= MAX_REL, (what, e2, em)
