"""Closed forms of the discrete problem with k = 1 (test helper; no oracle code).

With k = 1 every face coefficient is 1, so the scaled 7-point operator is
A' = T (+) T (+) T with T = tridiag(-1, 2, -1) of order m = n - 2, whose
eigenvectors are the sine modes phi_p(i) = sqrt(2/(m+1)) sin(pi p i/(m+1)),
lambda_p = 2 - 2 cos(pi p/(m+1)).  For f = 1 (b' = h^2) the discrete QoI
Q = h^3 sum u = h^5 1^T A'^-1 1 = h^5 sum_{p,q,r} w_p w_q w_r / (lambda_p +
lambda_q + lambda_r), w_p = <phi_p, 1>^2 = (2/(m+1)) cot^2(pi p/(2(m+1))) for
odd p and 0 for even p (the sum of sin(i theta) over i = 1..m in closed form).
"""
import math

import numpy as np


def q_const_modes(n):
    """h^3 sum_interior u for k = 1, f = 1 on an n^3 grid, by the mode sum."""
    m = n - 2
    h = 1.0 / (n - 1)
    p = np.arange(1, m + 1, 2, dtype=np.float64)  # odd modes only
    th = np.pi * p / (m + 1)
    lam = 2.0 - 2.0 * np.cos(th)
    w = (2.0 / (m + 1)) / np.tan(th / 2.0) ** 2
    wqr = w[:, None] * w[None, :]
    lqr = lam[:, None] + lam[None, :]
    parts = [float(np.sum(w[i] * wqr / (lam[i] + lqr))) for i in range(p.size)]
    return h**5 * math.fsum(parts)
