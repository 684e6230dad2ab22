"""The numerical example: Eq. 4 (source), Eq. 5 (exact solution), Eq. 6 (error)
and the rounding experiment reported in Table 1.

Procedure (section "Numerical example"): build the full Fig. 3-style matrix
for n_x = n_y = n grid points on [0,1]^2 (h = 1/(n-1), Eq. 2), invert it, round
every entry of the inverse to d digits after the decimal point, multiply by the
right-hand-side vector (boundary values and scaled source) and compare with
Eq. 5 using Eq. 6.
"""

import numpy as np

from . import grid, inverse, metrics


def eq4_source(x, y):
    """Right side of Eq. 4: (12x^2 - 6x)(y^3 - y^2) + (x^4 - x^3)(6y - 2)."""
    return (12 * x ** 2 - 6 * x) * (y ** 3 - y ** 2) + (x ** 4 - x ** 3) * (6 * y - 2)


def eq5_solution(x, y):
    """Eq. 5: u = (x^4 - x^3)(y^3 - y^2)."""
    return (x ** 4 - x ** 3) * (y ** 3 - y ** 2)


def node_coords(n):
    """Eq. 2: x_j = h*j, y_i = h*i (0-based), h = 1/(n-1); arrays [n_y][n_x]."""
    h = 1.0 / (n - 1)
    i = np.arange(n, dtype=np.float64)
    Y, X = np.meshgrid(i * h, i * h, indexing='ij')
    return X, Y, h


def full_inverse(n):
    """Inverse of the full unit-diagonal Fig. 3 matrix for an n x n grid."""
    return inverse.lu_inverse(grid.paper_full_matrix(n, n))


def round_decimals(A, digits):
    """Round every entry to ``digits`` places after the decimal point, ties to even."""
    return np.round(A, digits)


def experiment(n, digits_list, Ainv=None):
    """Eq. 6 error of the rounded-inverse solution for each entry of digits_list
    (None = no rounding).  Returns {digits: error}."""
    X, Y, h = node_coords(n)
    rho = eq4_source(X, Y)
    u_exact = eq5_solution(X, Y)
    rhs = grid.paper_full_rhs(n, n, h, rho, np.zeros((n, n)))
    if Ainv is None:
        Ainv = full_inverse(n)
    out = {}
    for d in digits_list:
        M = Ainv if d is None else round_decimals(Ainv, d)
        u = (M @ rhs).reshape(n, n)
        out[d] = metrics.eq6_error(u, u_exact)
    return out
