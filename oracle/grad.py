"""Derivatives of the solve (not in the paper).

Forward: u_r = K(eps)^{-1} b_r(eps),  b_r = -h^2 rho_r + b_B(eps), for every
right-hand side r.  For a loss with dLoss/du_r = g_r, let mu_r = K^{-T} g_r.

* dLoss/drho_r = -h^2 mu_r =: lambda_r (the adjoint output).
* K and b_B are sums over faces f = (p, q) of
      eps_f (e_p - e_q)(e_p - e_q)^T        (both p, q interior),
      eps_f e_p e_p^T and eps_f u_B(q) e_p  (q on the boundary),
  so  dLoss/deps_f = sum_r mu_r^T (db_r/deps_f - dK/deps_f u_r)
                   = -sum_r (mu_p - mu_q)(u_p - u_q)
  with mu_q = 0 and u_q = u_B(q) when q is a boundary node.  In terms of the
  adjoint output: dLoss/deps_f = (1/h^2) sum_r (lambda_p - lambda_q)(u_p - u_q).
* eps_f = (eps_p + eps_q)/2, so the nodal gradient is half the sum over the
  faces that touch the node (boundary nodes included; faces that join two
  boundary nodes do not enter K and contribute nothing).

The finite-difference reference re-solves the system from scratch in float64
(banded Cholesky) at eps +- delta*v.
"""

import numpy as np
import scipy.linalg as sla

from . import grid as _grid


def adjoint(G, g, h):
    """lambda = -h^2 G^T g (float64)."""
    return -(h * h) * (np.asarray(G, dtype=np.float64).T @ np.asarray(g, dtype=np.float64))


def grad_eps_nodes(nx, ny, h, u_int, lam_int, ub_nodes=None):
    """Nodal dLoss/deps from forward solutions u and adjoint outputs lambda.

    u_int, lam_int: [N, R] (interior, p order).  Returns [n_y][n_x].
    Loops over faces of the full grid, one face at a time.
    """
    my, mx = ny - 2, nx - 2
    u_int = np.asarray(u_int, dtype=np.float64).reshape(my * mx, -1)
    lam_int = np.asarray(lam_int, dtype=np.float64).reshape(my * mx, -1)
    R = u_int.shape[1]
    U = np.zeros((ny, nx, R))
    if ub_nodes is not None:
        U[:, :, :] = np.asarray(ub_nodes, dtype=np.float64)[:, :, None]
    U[1:ny - 1, 1:nx - 1, :] = u_int.reshape(my, mx, R)
    L = np.zeros((ny, nx, R))
    L[1:ny - 1, 1:nx - 1, :] = lam_int.reshape(my, mx, R)
    out = np.zeros((ny, nx))
    inv_h2 = 1.0 / (h * h)
    # horizontal faces (i, j)-(i, j+1) and vertical faces (i, j)-(i+1, j)
    for (di, dj) in ((0, 1), (1, 0)):
        for i in range(ny - di):
            for j in range(nx - dj):
                k, l = i + di, j + dj
                if _grid.is_boundary(nx, ny, i, j) and _grid.is_boundary(nx, ny, k, l):
                    continue
                gf = inv_h2 * float(np.sum((L[i, j] - L[k, l]) * (U[i, j] - U[k, l])))
                out[i, j] += 0.5 * gf
                out[k, l] += 0.5 * gf
    return out


def banded_solve(nx, ny, h, eps_nodes, rho, ub_nodes=None):
    """u = K^{-1}(-h^2 rho + b_B) by banded Cholesky (scipy solveh_banded)."""
    ab = _grid.conservative_operator_banded(nx, ny, eps_nodes)
    rhs = -(h * h) * np.asarray(rho, dtype=np.float64)
    if ub_nodes is not None:
        bB = _grid.boundary_term(nx, ny, eps_nodes, ub_nodes)
        rhs = rhs + (bB[:, None] if rhs.ndim == 2 else bB)
    return sla.solveh_banded(ab, rhs, lower=True)


def sampling_loss(nx, ny, h, eps_nodes, rho, sample_idx, d, ub_nodes=None):
    """Source-reconstruction loss sum_r ||C u_r - d_r||^2 with C selecting the
    interior unknowns ``sample_idx``; u from a fresh float64 banded solve."""
    u = banded_solve(nx, ny, h, eps_nodes, rho, ub_nodes)
    r = u[np.asarray(sample_idx)] - d
    return float(np.sum(r * r))


def sampling_loss_grad_u(u, sample_idx, d):
    """g = dLoss/du = 2 C^T (C u - d)."""
    g = np.zeros_like(u)
    g[np.asarray(sample_idx)] = 2.0 * (u[np.asarray(sample_idx)] - d)
    return g


def central_difference(fun, x, v, delta):
    """[fun(x + delta v) - fun(x - delta v)] / (2 delta)."""
    return (fun(x + delta * v) - fun(x - delta * v)) / (2.0 * delta)
