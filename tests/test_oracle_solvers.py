"""Pins of the FP64 LSQR and OS-SART oracles against what the mathematics
fixes, on explicit matrices:

* LSQR reaches the least-squares solution (numpy.linalg.lstsq) and its two
  residual estimates equal the true |b - A x| and |A^T (b - A x)|; its
  iterates equal those of CGLS (both minimise |b - A x| over the same
  Krylov spaces), an independent algorithm;
* SART with one subset and lam = 1 on a positive diagonal matrix solves the
  system in one step (row and column sums are the diagonal); with one subset
  it converges to the solution of the row-sum-weighted least-squares
  problem min |R^-1/2 (A x - b)| (its fixed point solves A^T R^-1 (b - A x)
  = 0), and with several subsets on consistent data to the exact solution;
  the column sums of the subsets add up to A^T 1.
"""
import numpy as np

from oracle.cgls import cgls
from oracle.lsqr import lsqr
from oracle.sart import os_sart, subsets


def _mat(m, n, seed):
    return np.random.default_rng(seed).standard_normal((m, n))


def test_lsqr_reaches_lstsq_and_estimates_are_true():
    A = _mat(40, 12, 0)
    b = np.random.default_rng(1).standard_normal(40)
    x, rn, arn = lsqr(lambda v: A @ v, lambda v: A.T @ v, b, 30, np.zeros(12))
    ref = np.linalg.lstsq(A, b, rcond=None)[0]
    assert np.linalg.norm(x - ref) < 1e-10 * np.linalg.norm(ref)
    for n in (1, 3, 7):
        xn, rnn, arnn = lsqr(lambda v: A @ v, lambda v: A.T @ v, b, n, np.zeros(12))
        r = b - A @ xn
        assert abs(rnn[-1] - np.linalg.norm(r)) < 1e-10 * np.linalg.norm(b)
        assert abs(arnn[-1] - np.linalg.norm(A.T @ r)) < 1e-9 * np.linalg.norm(A.T @ b)


def test_lsqr_iterates_equal_cgls_iterates():
    A = _mat(30, 10, 2)
    b = np.random.default_rng(3).standard_normal(30)
    x0 = np.random.default_rng(4).standard_normal(10)
    for n in range(1, 7):
        xl = lsqr(lambda v: A @ v, lambda v: A.T @ v, b, n, x0)[0]
        xc = cgls(lambda v: A @ v, lambda v: A.T @ v, b, n, x0)[0]
        assert np.linalg.norm(xl - xc) < 1e-9 * np.linalg.norm(xc), n


def _views_ops(A, n_views, rows):
    """An explicit matrix whose rows are grouped in views of `rows` rows."""
    def project(x, views):
        return np.stack([A[v * rows:(v + 1) * rows] @ x for v in views])

    def backproject(y, views):
        out = np.zeros(A.shape[1])
        for k, v in enumerate(views):
            out += A[v * rows:(v + 1) * rows].T @ y[k]
        return out
    return project, backproject


def test_sart_diagonal_one_step():
    d = np.random.default_rng(5).uniform(0.5, 2.0, 6)
    A = np.diag(d)
    b = np.random.default_rng(6).uniform(-1, 1, 6)
    P, B = _views_ops(A, 6, 1)
    x, _ = os_sart(P, B, b.reshape(6, 1), 6, 1, 1, np.full(6, 0.3))
    assert np.allclose(x, b / d, rtol=0, atol=1e-14)


def test_sart_one_subset_converges_to_weighted_least_squares():
    rng = np.random.default_rng(7)
    A = rng.uniform(0.0, 1.0, (24, 8))          # nonnegative, like a projector
    b = rng.uniform(0.0, 1.0, 24)               # inconsistent
    P, B = _views_ops(A, 6, 4)
    x, res = os_sart(P, B, b.reshape(6, 4), 6, 1, 3000, np.zeros(8))
    R = A @ np.ones(8)
    W = 1.0 / np.sqrt(R)
    ref = np.linalg.lstsq(A * W[:, None], b * W, rcond=None)[0]
    assert np.linalg.norm(x - ref) < 1e-8 * np.linalg.norm(ref)


def test_os_sart_consistent_data_converges_to_solution():
    rng = np.random.default_rng(8)
    A = rng.uniform(0.0, 1.0, (30, 9))
    xt = rng.uniform(0.0, 1.0, 9)
    P, B = _views_ops(A, 10, 3)
    b = (A @ xt).reshape(10, 3)
    x, res = os_sart(P, B, b, 10, 5, 400, np.zeros(9))
    assert np.linalg.norm(x - xt) < 1e-8 * np.linalg.norm(xt)
    assert res[-1] < 1e-8 * np.linalg.norm(b)


def test_subset_column_sums_partition():
    rng = np.random.default_rng(9)
    A = rng.uniform(0.0, 1.0, (21, 5))
    P, B = _views_ops(A, 7, 3)
    S = subsets(7, 3)
    assert sorted(np.concatenate(S).tolist()) == list(range(7))
    tot = sum(B(np.ones((len(v), 3)), v) for v in S)
    assert np.allclose(tot, A.T @ np.ones(21), rtol=1e-14)
