"""LSQR (Paige & Saunders, ACM TOMS 8(1), 1982: bidiagonalisation of A by the
Golub-Kahan process and a QR update of the bidiagonal least-squares problem)
in FP64.  One of the paper's Krylov solvers on the same operators (Sec. V-E
names LSQR next to CGLS).

TEST INFRASTRUCTURE (see the package docstring).  A and At are callables.

Recurrences (x0 given; the solver works on the correction):
  beta1 u1 = b - A x0,  alpha1 v1 = At u1,  w1 = v1,
  phibar1 = beta1,  rhobar1 = alpha1;
  for i = 1, 2, ...:
    beta_{i+1} u_{i+1} = A v_i - alpha_i u_i
    alpha_{i+1} v_{i+1} = At u_{i+1} - beta_{i+1} v_i
    rho_i = sqrt(rhobar_i^2 + beta_{i+1}^2);  c_i = rhobar_i / rho_i;
    s_i = beta_{i+1} / rho_i;  theta_{i+1} = s_i alpha_{i+1};
    rhobar_{i+1} = -c_i alpha_{i+1};  phi_i = c_i phibar_i;
    phibar_{i+1} = s_i phibar_i
    x_i = x_{i-1} + (phi_i / rho_i) w_i
    w_{i+1} = v_{i+1} - (theta_{i+1} / rho_i) w_i
Estimates: |b - A x_i| = phibar_{i+1};  |At (b - A x_i)| = phibar_{i+1}
alpha_{i+1} |c_i|.
"""
import math

import numpy as np


def lsqr(A, At, b, n_iter, x0):
    """Returns (x, rnorm_est, arnorm_est): x after n_iter iterations (fewer
    if the bidiagonalisation ends), and per iteration i = 0..n the estimates
    of |b - A x_i| and |At (b - A x_i)| (entry 0: the start)."""
    x = np.array(x0, dtype=np.float64, copy=True)
    u = b - A(x)
    beta = float(np.linalg.norm(u))
    if beta > 0:
        u = u / beta
    v = At(u)
    alpha = float(np.linalg.norm(v))
    if alpha > 0:
        v = v / alpha
    w = v.copy()
    phibar, rhobar = beta, alpha
    rn = [beta]
    arn = [alpha * beta]
    for _ in range(n_iter):
        if alpha == 0.0 or beta == 0.0:
            break
        u = A(v) - alpha * u
        beta = float(np.linalg.norm(u))
        if beta > 0:
            u = u / beta
        v = At(u) - beta * v
        alpha = float(np.linalg.norm(v))
        if alpha > 0:
            v = v / alpha
        rho = math.hypot(rhobar, beta)
        c, s = rhobar / rho, beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = s * phibar
        x = x + (phi / rho) * w
        w = v - (theta / rho) * w
        rn.append(phibar)
        arn.append(phibar * alpha * abs(c))
    return x, np.array(rn), np.array(arn)
