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


def apply_operator_extended(nx, ny, eps_nodes, u_int):
    """K u for interior values u (columns), accumulated in numpy longdouble
    (80-bit extended on x86): K's entries are formed in float64 exactly as in
    :func:`grid.conservative_operator`, then every product and sum is carried in
    extended precision."""
    my, mx = ny - 2, nx - 2
    eps = np.asarray(eps_nodes, dtype=np.float64)
    ex = (0.5 * (eps[:, :-1] + eps[:, 1:])).astype(np.longdouble)     # face (i, j)-(i, j+1)
    ey = (0.5 * (eps[:-1, :] + eps[1:, :])).astype(np.longdouble)     # face (i, j)-(i+1, j)
    u = np.asarray(u_int).astype(np.longdouble).reshape(my, mx, -1)
    U = np.zeros((ny, nx, u.shape[2]), dtype=np.longdouble)
    U[1:-1, 1:-1] = u
    c = U[1:-1, 1:-1]
    out = (ex[1:-1, :-1, None] * (c - U[1:-1, :-2]) + ex[1:-1, 1:, None] * (c - U[1:-1, 2:])
           + ey[:-1, 1:-1, None] * (c - U[:-2, 1:-1]) + ey[1:, 1:-1, None] * (c - U[2:, 1:-1]))
    return out.reshape(my * mx, -1)


def banded_solve_refined(nx, ny, h, eps_nodes, rho, ub_nodes=None):
    """:func:`banded_solve` followed by one step of iterative refinement whose
    residual b - K u is accumulated in extended precision.  The float64 solve
    alone is accurate to about cond(K) * eps_mach; the refined solution to about
    eps_mach, which is what a finite-difference quotient with a small step needs."""
    rho = np.asarray(rho, dtype=np.float64)
    vec = rho.ndim == 1
    R = rho.reshape(rho.shape[0], -1)
    rhs = (-(h * h)) * R.astype(np.longdouble)
    if ub_nodes is not None:
        rhs = rhs + _grid.boundary_term(nx, ny, eps_nodes, ub_nodes).astype(np.longdouble)[:, None]
    ab = _grid.conservative_operator_banded(nx, ny, eps_nodes)
    u0 = sla.solveh_banded(ab, rhs.astype(np.float64), lower=True)
    r = rhs - apply_operator_extended(nx, ny, eps_nodes, u0)
    du = sla.solveh_banded(ab, r.astype(np.float64), lower=True)
    u = (u0.astype(np.longdouble) + du).astype(np.float64)
    return u[:, 0] if vec else u


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


def sampling_loss_central_difference(nx, ny, h, eps_nodes, rho, sample, d, v_eps=None, v_rho=None,
                                     delta=1e-6, ub_nodes=None):
    """Central difference of :func:`sampling_loss` along (v_eps, v_rho) with step
    delta, each side re-solved from scratch in float64.

    Same quantity as [L(+) - L(-)] / (2 delta), evaluated as
    sum (r+ - r-)(r+ + r-) / (2 delta) with r = C u - d: the difference of the two
    squared-residual sums is formed term by term instead of subtracting two
    large sums, which removes the cancellation that otherwise limits the
    difference quotient to about eps_mach * L / delta.  Each side is solved with
    :func:`banded_solve_refined`, so the solver's own error (about
    cond(K) * eps_mach) does not enter the quotient either.
    """
    e_p = eps_nodes if v_eps is None else eps_nodes + delta * v_eps
    e_m = eps_nodes if v_eps is None else eps_nodes - delta * v_eps
    r_p_src = rho if v_rho is None else rho + delta * v_rho
    r_m_src = rho if v_rho is None else rho - delta * v_rho
    idx = np.asarray(sample)
    rp = banded_solve_refined(nx, ny, h, e_p, r_p_src, ub_nodes)[idx] - d
    rm = banded_solve_refined(nx, ny, h, e_m, r_m_src, ub_nodes)[idx] - d
    return float(np.sum((rp - rm) * (rp + rm))) / (2.0 * delta)


def grad_eps_nodes_3d(nx, ny, nz, h, u_int, lam_int, ub_nodes=None):
    """Nodal dLoss/deps for the 3-D operator (same face rule as
    :func:`grad_eps_nodes` over the 6 face directions): for every face f = (p, q)
    that is not between two boundary nodes,
        g_f = (1/h^2) sum_r (lambda_p - lambda_q)(u_p - u_q)
    (lambda = 0 and u = u_B on boundary nodes), half of it to each end node.
    u_int, lam_int: [N, R] in the interior order of
    :func:`grid.conservative_operator_3d`.  Returns [n_z][n_y][n_x]."""
    mz, my, mx = nz - 2, ny - 2, nx - 2
    u_int = np.asarray(u_int, dtype=np.float64).reshape(mz * my * mx, -1)
    lam_int = np.asarray(lam_int, dtype=np.float64).reshape(mz * my * mx, -1)
    R = u_int.shape[1]
    U = np.zeros((nz, ny, nx, R))
    if ub_nodes is not None:
        U[:] = np.asarray(ub_nodes, dtype=np.float64)[..., None]
    U[1:-1, 1:-1, 1:-1] = u_int.reshape(mz, my, mx, R)
    L = np.zeros((nz, ny, nx, R))
    L[1:-1, 1:-1, 1:-1] = lam_int.reshape(mz, my, mx, R)
    out = np.zeros((nz, ny, nx))

    def bnd(k, i, j):
        return k in (0, nz - 1) or i in (0, ny - 1) or j in (0, nx - 1)

    for (dk, di, dj) in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
        for k in range(nz - dk):
            for i in range(ny - di):
                for j in range(nx - dj):
                    a, b, c = k + dk, i + di, j + dj
                    if bnd(k, i, j) and bnd(a, b, c):
                        continue
                    gf = float(np.sum((L[k, i, j] - L[a, b, c]) * (U[k, i, j] - U[a, b, c]))) / (h * h)
                    out[k, i, j] += 0.5 * gf
                    out[a, b, c] += 0.5 * gf
    return out


def grad_eps_general(x, y, u_int, lam_int, ub_nodes=None):
    """dLoss/deps_x and dLoss/deps_y (nodal, [n_y][n_x] each) for the
    finite-volume operator of :func:`grid.conservative_operator_general`.

    There the solve is K u = -A rho + b_B with the stored inverse
    G' = K^{-1} diag(A), so the adjoint output lambda = -G'^T g gives
    mu = K^{-1} g = -lambda / A (per interior node).  Face f = (p, q) carries
    c_f = eps_f * s_f with the geometric factor s_f = (cell height at the face's
    row) / |x_q - x_p| for an x-face and (cell width at its column) / |y_q - y_p|
    for a y-face, so, as for the uniform grid,
        dLoss/dc_f = -sum_r (mu_p - mu_q)(u_p - u_q)
                   = sum_r (lambda_p/A_p - lambda_q/A_q)(u_p - u_q)
    (lambda = 0 and u = u_B on boundary nodes), and each end node of an x-face
    receives s_f/2 of it in the x gradient (y-faces: the y gradient).
    u_int, lam_int: [N, R] in interior order.  Returns (grad_x, grad_y)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    nx, ny = x.size, y.size
    my, mx = ny - 2, nx - 2
    u_int = np.asarray(u_int, dtype=np.float64).reshape(my * mx, -1)
    lam_int = np.asarray(lam_int, dtype=np.float64).reshape(my * mx, -1)
    R = u_int.shape[1]
    U = np.zeros((ny, nx, R))
    if ub_nodes is not None:
        U[:, :, :] = np.asarray(ub_nodes, dtype=np.float64)[:, :, None]
    U[1:-1, 1:-1, :] = u_int.reshape(my, mx, R)
    M = np.zeros((ny, nx, R))       # lambda / A on interior nodes, 0 on the boundary
    for i in range(1, ny - 1):
        for j in range(1, nx - 1):
            area = 0.5 * (x[j + 1] - x[j - 1]) * 0.5 * (y[i + 1] - y[i - 1])
            M[i, j] = lam_int[(i - 1) * mx + (j - 1)] / area
    gx = np.zeros((ny, nx))
    gy = np.zeros((ny, nx))
    for i in range(ny):
        for j in range(nx - 1):           # x-faces (i, j)-(i, j+1)
            if _grid.is_boundary(nx, ny, i, j) and _grid.is_boundary(nx, ny, i, j + 1):
                continue
            s = 0.5 * (y[i + 1] - y[i - 1]) / (x[j + 1] - x[j])
            gf = s * float(np.sum((M[i, j] - M[i, j + 1]) * (U[i, j] - U[i, j + 1])))
            gx[i, j] += 0.5 * gf
            gx[i, j + 1] += 0.5 * gf
    for i in range(ny - 1):               # y-faces (i, j)-(i+1, j)
        for j in range(nx):
            if _grid.is_boundary(nx, ny, i, j) and _grid.is_boundary(nx, ny, i + 1, j):
                continue
            s = 0.5 * (x[j + 1] - x[j - 1]) / (y[i + 1] - y[i])
            gf = s * float(np.sum((M[i, j] - M[i + 1, j]) * (U[i, j] - U[i + 1, j])))
            gy[i, j] += 0.5 * gf
            gy[i + 1, j] += 0.5 * gf
    return gx, gy


def grad_beta(nx, ny, u_int, lam_int, ub_nodes=None):
    """dLoss/dbeta for Eq. 3's operator (:func:`grid.beta_operator`), where
    u = A^{-1}(rho + b_B), A[p,q_d] = -beta_d(p)/4 and b_B[p] carries
    beta_d(p)/4 u_B(q_d) for boundary neighbours.  With lambda = dLoss/drho =
    A^{-T} g (the adjoint output), dLoss/dbeta_d(p) = lambda^T (db/dbeta -
    dA/dbeta u) = (1/4) sum_r lambda_p U_{q_d}, U_q = u_q at interior q and
    u_B(q) on the boundary.  Returns [4][n_y][n_x] (zero off the interior)."""
    my, mx = ny - 2, nx - 2
    u_int = np.asarray(u_int, dtype=np.float64).reshape(my * mx, -1)
    lam_int = np.asarray(lam_int, dtype=np.float64).reshape(my * mx, -1)
    R = u_int.shape[1]
    U = np.zeros((ny, nx, R))
    if ub_nodes is not None:
        U[:, :, :] = np.asarray(ub_nodes, dtype=np.float64)[:, :, None]
    U[1:-1, 1:-1, :] = u_int.reshape(my, mx, R)
    out = np.zeros((4, ny, nx))
    for i in range(1, ny - 1):
        for j in range(1, nx - 1):
            lp = lam_int[(i - 1) * mx + (j - 1)]
            for d, (di, dj) in enumerate(_grid.BETA_DIRECTIONS):
                out[d, i, j] = 0.25 * float(np.sum(lp * U[i + di, j + dj]))
    return out
