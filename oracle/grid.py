"""Grid, node order and the two forms of the discrete operator.

Node order follows Fig. 3: for n_x = 3, n_y = 5 the unknown vector is
u_{1,1}, u_{1,2}, u_{1,3}, u_{2,1}, ... so the FIRST subscript is the slow axis
with n_y points and the second subscript the fast axis with n_x points.  Here
both are 0-based: node (i, j), i in [0, n_y), j in [0, n_x), full index
P = i*n_x + j.  Boundary nodes are i in {0, n_y-1} or j in {0, n_x-1}.
Interior unknowns are numbered row-major over (i-1, j-1):
p = (i-1)*(n_x-2) + (j-1).  Uniform step h (Eq. 2: h = L/(n-1)).
"""

import numpy as np


def interior_shape(nx, ny):
    """(m_y, m_x) = number of interior rows / columns (Fig. 2: crosses are boundary)."""
    return ny - 2, nx - 2


def interior_count(nx, ny):
    """N = number of interior unknowns."""
    my, mx = interior_shape(nx, ny)
    return my * mx


def is_boundary(nx, ny, i, j):
    return i == 0 or i == ny - 1 or j == 0 or j == nx - 1


def paper_full_matrix(nx, ny):
    """The full unit-diagonal system of Fig. 3 (eps = 1, Eq. 2).

    One row per grid node, in Fig. 3's order.  A boundary node's row is an
    identity row (its value is the prescribed Dirichlet datum).  An interior
    node's row is Eq. 2: 1 on the diagonal and -0.25 on the four neighbours.
    Returned as a dense float64 (nx*ny) x (nx*ny) array.
    """
    n_tot = nx * ny
    A = np.zeros((n_tot, n_tot), dtype=np.float64)
    for i in range(ny):
        for j in range(nx):
            P = i * nx + j
            A[P, P] = 1.0
            if is_boundary(nx, ny, i, j):
                continue
            A[P, P - 1] = -0.25
            A[P, P + 1] = -0.25
            A[P, P - nx] = -0.25
            A[P, P + nx] = -0.25
    return A


def paper_full_rhs(nx, ny, h, rho_nodes, ub_nodes):
    """Right-hand side vector of the Fig. 3 system.

    Boundary entries carry the Dirichlet value u_B.  Interior entries carry the
    source term of Eq. 2.  Eq. 2 prints the source as -rho*h^2; with the
    operator of Eq. 1 (Laplacian = rho for eps = 1) and the unit-diagonal row
    u - 0.25*(sum of 4 neighbours), the consistent source is -(h^2/4)*rho.
    That reading is the one that reproduces Table 1 (see the Table 1 tests),
    so it is the one used here.
    """
    rhs = np.empty(nx * ny, dtype=np.float64)
    for i in range(ny):
        for j in range(nx):
            P = i * nx + j
            if is_boundary(nx, ny, i, j):
                rhs[P] = ub_nodes[i, j]
            else:
                rhs[P] = -0.25 * h * h * rho_nodes[i, j]
    return rhs


def face_eps(eps_nodes, i, j, k, l):
    """Permittivity on the face between nodes (i,j) and (k,l): nodal arithmetic mean.

    Eq. 1 is in divergence form, d/dx_i eps_i du/dx_i; the flux through a face
    uses the permittivity on that face, taken as the mean of the two nodal
    values it joins (the text after Eq. 2 allows eps = eps(x_i)).
    """
    return 0.5 * (eps_nodes[i, j] + eps_nodes[k, l])


def neighbours(i, j):
    """The four 5-point neighbours of node (i, j) (Eq. 2 / Fig. 1)."""
    return ((i - 1, j), (i + 1, j), (i, j - 1), (i, j + 1))


def conservative_operator(nx, ny, eps_nodes=None, ub_nodes=None):
    """Interior operator K (SPD) and the boundary data term b_B.

    Multiplying Eq. 1 by h^2 and summing the four face fluxes of the 5-point
    stencil gives, for every interior node p,
        sum_f eps_f * (u_p - u_q) = -h^2 * rho_p ,
    where f runs over the 4 faces of p and q is the node across f.  Moving the
    known Dirichlet values u_B(q) of boundary neighbours to the right:
        K[p,p] = sum_f eps_f,  K[p,q] = -eps_f  (q interior),
        b_B[p] = sum over boundary faces of eps_f * u_B(q).
    With eps = 1, K = 4 * (interior block of the Fig. 3 matrix).
    The solve is u_I = K^{-1} (-h^2 rho + b_B).
    """
    if eps_nodes is None:
        eps_nodes = np.ones((ny, nx), dtype=np.float64)
    if ub_nodes is None:
        ub_nodes = np.zeros((ny, nx), dtype=np.float64)
    my, mx = interior_shape(nx, ny)
    N = my * mx
    K = np.zeros((N, N), dtype=np.float64)
    bB = np.zeros(N, dtype=np.float64)
    for i in range(1, ny - 1):
        for j in range(1, nx - 1):
            p = (i - 1) * mx + (j - 1)
            for (k, l) in neighbours(i, j):
                ef = face_eps(eps_nodes, i, j, k, l)
                K[p, p] += ef
                if is_boundary(nx, ny, k, l):
                    bB[p] += ef * ub_nodes[k, l]
                else:
                    q = (k - 1) * mx + (l - 1)
                    K[p, q] -= ef
    return K, bB


def conservative_operator_banded(nx, ny, eps_nodes):
    """K in LAPACK lower symmetric band storage (bandwidth m_x), for the banded
    Cholesky used by the finite-difference checks at sizes where a dense LU is
    too slow.  Same entries as :func:`conservative_operator`.
    """
    my, mx = interior_shape(nx, ny)
    N = my * mx
    ab = np.zeros((mx + 1, N), dtype=np.float64)
    for i in range(1, ny - 1):
        for j in range(1, nx - 1):
            p = (i - 1) * mx + (j - 1)
            for (k, l) in neighbours(i, j):
                ef = face_eps(eps_nodes, i, j, k, l)
                ab[0, p] += ef
                if not is_boundary(nx, ny, k, l):
                    q = (k - 1) * mx + (l - 1)
                    if q > p:
                        ab[q - p, p] -= ef
    return ab


def boundary_term(nx, ny, eps_nodes, ub_nodes):
    """b_B alone (see :func:`conservative_operator`), without building K."""
    my, mx = interior_shape(nx, ny)
    bB = np.zeros(my * mx, dtype=np.float64)
    for i in range(1, ny - 1):
        for j in range(1, nx - 1):
            p = (i - 1) * mx + (j - 1)
            for (k, l) in neighbours(i, j):
                if is_boundary(nx, ny, k, l):
                    bB[p] += face_eps(eps_nodes, i, j, k, l) * ub_nodes[k, l]
    return bB


def interior_to_nodes(nx, ny, u_int, ub_nodes=None):
    """Scatter interior values (length N, p order) into a [n_y][n_x] nodal array
    holding u_B on the boundary."""
    my, mx = interior_shape(nx, ny)
    out = np.zeros((ny, nx), dtype=np.float64) if ub_nodes is None else np.array(ub_nodes, dtype=np.float64)
    out[1:ny - 1, 1:nx - 1] = np.asarray(u_int).reshape(my, mx)
    return out


def nodes_to_interior(nx, ny, nodal):
    """Gather the interior values of a [n_y][n_x] array in p order."""
    return np.ascontiguousarray(np.asarray(nodal)[1:ny - 1, 1:nx - 1]).reshape(-1)


# --- three dimensions (the paper's N = n_x n_y n_z, "Statement of the problem") ---

def conservative_operator_3d(nx, ny, nz, eps_nodes=None, ub_nodes=None):
    """7-point conservative operator on an n_z x n_y x n_x grid (nodal arrays
    [n_z][n_y][n_x], slowest axis z; interior index
    p = ((k-1)(n_y-2) + (i-1))(n_x-2) + (j-1)), built exactly as the 2-D form:
    for every interior node p and each of its 6 faces f to node q,
        K[p,p] += eps_f,  K[p,q] -= eps_f (q interior),
        b_B[p] += eps_f * u_B(q) (q on the boundary),
    with eps_f the mean of the two nodal values.  With eps = 1, K is 6 I minus
    the interior adjacency (the 7-point Laplacian times -h^2)."""
    if eps_nodes is None:
        eps_nodes = np.ones((nz, ny, nx), dtype=np.float64)
    if ub_nodes is None:
        ub_nodes = np.zeros((nz, ny, nx), dtype=np.float64)
    mz, my, mx = nz - 2, ny - 2, nx - 2
    N = mz * my * mx
    K = np.zeros((N, N), dtype=np.float64)
    bB = np.zeros(N, dtype=np.float64)

    def bnd(k, i, j):
        return k in (0, nz - 1) or i in (0, ny - 1) or j in (0, nx - 1)

    for k in range(1, nz - 1):
        for i in range(1, ny - 1):
            for j in range(1, nx - 1):
                p = ((k - 1) * my + (i - 1)) * mx + (j - 1)
                for (a, b, c) in ((k - 1, i, j), (k + 1, i, j), (k, i - 1, j), (k, i + 1, j), (k, i, j - 1),
                                  (k, i, j + 1)):
                    ef = 0.5 * (eps_nodes[k, i, j] + eps_nodes[a, b, c])
                    K[p, p] += ef
                    if bnd(a, b, c):
                        bB[p] += ef * ub_nodes[a, b, c]
                    else:
                        K[p, ((a - 1) * my + (b - 1)) * mx + (c - 1)] -= ef
    return K, bB


# --- non-uniform tensor grids and per-direction permittivity (Eq. 1's eps_i) ---

def conservative_operator_general(x, y, eps_x=None, eps_y=None, ub_nodes=None):
    """Finite-volume form of Eq. 1 with eps_i per direction on a tensor grid with
    node coordinates x[0..n_x-1], y[0..n_y-1] (strictly increasing).

    Interior node p = (i, j) owns the control volume
        A_p = (x_{j+1} - x_{j-1}) / 2 * (y_{i+1} - y_{i-1}) / 2.
    The face towards its x-neighbour q = (i, j +- 1) carries
        c = eps_x,f * ((y_{i+1} - y_{i-1}) / 2) / |x_q - x_j|,
    towards a y-neighbour c = eps_y,f * ((x_{j+1} - x_{j-1}) / 2) / |y_q - y_i|,
    with eps_f the mean of the two nodal values of that direction's field.
    Summing the face fluxes of Eq. 1 over the control volume:
        K[p,p] = sum c,  K[p,q] = -c (q interior),  b_B[p] = sum c * u_B(q) (q on the boundary),
        K u = -A rho + b_B.
    On a uniform grid (spacing h) with eps_x = eps_y = eps this is
    :func:`conservative_operator` with A = h^2.  Returns (K, b_B, A)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    nx, ny = x.size, y.size
    if eps_x is None:
        eps_x = np.ones((ny, nx), dtype=np.float64)
    if eps_y is None:
        eps_y = eps_x
    if ub_nodes is None:
        ub_nodes = np.zeros((ny, nx), dtype=np.float64)
    my, mx = interior_shape(nx, ny)
    N = my * mx
    K = np.zeros((N, N), dtype=np.float64)
    bB = np.zeros(N, dtype=np.float64)
    A = np.zeros(N, dtype=np.float64)
    for i in range(1, ny - 1):
        for j in range(1, nx - 1):
            p = (i - 1) * mx + (j - 1)
            wx = 0.5 * (x[j + 1] - x[j - 1])
            wy = 0.5 * (y[i + 1] - y[i - 1])
            A[p] = wx * wy
            for (k, l) in neighbours(i, j):
                if k == i:
                    c = 0.5 * (eps_x[i, j] + eps_x[k, l]) * wy / abs(x[l] - x[j])
                else:
                    c = 0.5 * (eps_y[i, j] + eps_y[k, l]) * wx / abs(y[k] - y[i])
                K[p, p] += c
                if is_boundary(nx, ny, k, l):
                    bB[p] += c * ub_nodes[k, l]
                else:
                    K[p, (k - 1) * mx + (l - 1)] -= c
    return K, bB, A


# --- Eq. 3: the unit-diagonal system with arbitrary neighbour coefficients ---

BETA_DIRECTIONS = ((-1, 0), (1, 0), (0, -1), (0, 1))   # (i-1, j), (i+1, j), (i, j-1), (i, j+1)


def beta_operator(nx, ny, beta, ub_nodes=None):
    """Eq. 3 restricted to the interior unknowns: row p = (i, j) reads
        u_p - 0.25 * sum_d beta[d][i, j] * u_{q_d} = rho_p,
    with q_d the neighbour in direction d (BETA_DIRECTIONS).  Boundary
    neighbours carry their Dirichlet value, moved to the right-hand side:
        A[p,p] = 1,  A[p,q_d] = -0.25 beta[d][i, j] (q_d interior),
        b_B[p] = 0.25 * sum over boundary q_d of beta[d][i, j] * u_B(q_d),
        u = A^{-1} (rho + b_B).
    beta: [4][n_y][n_x] (one coefficient per row and direction, arbitrary
    numbers).  With beta = 1 this is the interior part of Fig. 3's system.
    Returns (A, b_B)."""
    beta = np.asarray(beta, dtype=np.float64)
    if ub_nodes is None:
        ub_nodes = np.zeros((ny, nx), dtype=np.float64)
    my, mx = interior_shape(nx, ny)
    N = my * mx
    A = np.eye(N, dtype=np.float64)
    bB = np.zeros(N, dtype=np.float64)
    for i in range(1, ny - 1):
        for j in range(1, nx - 1):
            p = (i - 1) * mx + (j - 1)
            for d, (di, dj) in enumerate(BETA_DIRECTIONS):
                k, l = i + di, j + dj
                c = 0.25 * beta[d, i, j]
                if is_boundary(nx, ny, k, l):
                    bB[p] += c * ub_nodes[k, l]
                else:
                    A[p, (k - 1) * mx + (l - 1)] -= c
    return A, bB
