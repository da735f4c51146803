"""Textbook CGLS (Hestenes & Stiefel 1952, the CG method applied to the normal
equations; see Bjorck, Numerical Methods for Least Squares Problems) in FP64.

TEST INFRASTRUCTURE (see the package docstring).  A and At are callables, so
the same routine runs on an explicit matrix (to pin it) and on the oracle's
CVP operators.
"""
import numpy as np


def cgls(A, At, b, n_iter, x0):
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - A(x)
    s = At(r)
    p = s.copy()
    gamma = float(np.vdot(s, s))
    gammas = [gamma]
    rnorms = []
    for _ in range(n_iter):
        q = A(p)
        qq = float(np.vdot(q, q))
        if qq == 0.0 or gamma == 0.0:
            break
        alpha = gamma / qq
        x = x + alpha * p
        r = r - alpha * q
        s = At(r)
        gamma_new = float(np.vdot(s, s))
        p = s + (gamma_new / gamma) * p
        gamma = gamma_new
        gammas.append(gamma)
        rnorms.append(float(np.vdot(r, r)))
    return x, np.array(gammas), np.array(rnorms)
