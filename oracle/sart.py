"""OS-SART: the simultaneous algebraic reconstruction technique (Andersen &
Kak, Ultrasonic Imaging 6, 1984) over ordered subsets of the views (Jiang &
Wang, IEEE TMI 22(11), 2003), in FP64.  The paper's framework offers it with
a subset count (Sec. V-E, OS-SART with --os-subset-count).

TEST INFRASTRUCTURE (see the package docstring).

The views are split into T subsets S_t = {t, t + T, t + 2T, ...}.  With the
row sums R = A 1 (one per detector pixel and view) and the column sums of
each subset C_t = A_t^T 1 (one per voxel), one sweep visits t = 0 .. T-1:
  x <- x + lam * A_t^T ((b_t - A_t x) / R_t) / C_t
where a quotient with a zero denominator is 0 (pixels no voxel reaches and
voxels no ray of the subset reaches are left alone); with nonneg, x is then
clipped at 0.  A_t, A_t^T: the operator restricted to the views of S_t.
"""
import numpy as np


def subsets(n_views, n_subsets):
    return [np.arange(t, n_views, n_subsets) for t in range(n_subsets)]


def _safe_div(a, d):
    out = np.zeros_like(a)
    nz = d != 0
    out[nz] = a[nz] / d[nz]
    return out


def os_sart(project, backproject, b, n_views, n_subsets, n_sweeps, x0, lam=1.0, nonneg=False):
    """project(x, views) -> b restricted to `views` ([len(views), ...]);
    backproject(y, views) -> volume from data on `views`; b: [n_views, ...].
    Returns x after n_sweeps sweeps and the residual norm |b - A x| after
    each sweep."""
    x = np.array(x0, dtype=np.float64, copy=True)
    all_views = np.arange(n_views)
    R = project(np.ones_like(x), all_views)
    S = subsets(n_views, n_subsets)
    C = [backproject(np.ones_like(b[v]), v) for v in S]
    res = []
    for _ in range(n_sweeps):
        for t, v in enumerate(S):
            r = _safe_div(b[v] - project(x, v), R[v])
            x = x + lam * _safe_div(backproject(r, v), C[t])
            if nonneg:
                x = np.maximum(x, 0.0)
        res.append(float(np.linalg.norm(b - project(x, all_views))))
    return x, np.array(res)
