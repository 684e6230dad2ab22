"""Step 2 of "The solution steps": invert the operator by a standard method.

The oracle inverts with dense LU factorisation with partial pivoting followed by
one forward/back substitution per column of the identity (LAPACK getrf/getrs
through scipy, used as a library primitive).  The result is not symmetrised:
symmetry of K^{-1} is checked as an invariant instead.

:func:`dst_inverse` is the closed form for eps = 1 (eigen-decomposition of the
5-point Laplacian by the type-I discrete sine transform); it is independent of
the LU route and pins it.
"""

import numpy as np
import scipy.linalg as sla


def lu_inverse(A):
    """A^{-1} by LU with partial pivoting and N substitutions (step 2)."""
    A = np.asarray(A, dtype=np.float64)
    lu, piv = sla.lu_factor(A, check_finite=True)
    return sla.lu_solve((lu, piv), np.eye(A.shape[0]), check_finite=False)


def dst_basis(m):
    """Orthonormal DST-I basis S[a, i] = sqrt(2/(m+1)) sin((a+1)(i+1) pi/(m+1))
    and eigenvalues lam[a] = 4 sin^2((a+1) pi / (2(m+1))) of tridiag(-1, 2, -1)."""
    a = np.arange(1, m + 1, dtype=np.float64)
    S = np.sqrt(2.0 / (m + 1)) * np.sin(np.outer(a, a) * np.pi / (m + 1))
    lam = 4.0 * np.sin(a * np.pi / (2.0 * (m + 1))) ** 2
    return S, lam


def dst_inverse(nx, ny):
    """Closed-form K^{-1} for eps = 1 (K = 4*I - adjacency on the interior grid).

    K = T_y (x) I + I (x) T_x with T = tridiag(-1, 2, -1), so
    K^{-1}[(i,j),(k,l)] = sum_{a,b} Sy[a,i] Sy[a,k] Sx[b,j] Sx[b,l] / (ly[a] + lx[b]).
    Evaluated as one (my^2 x my) @ (my x mx^2) matrix product per the
    separable structure.
    """
    my, mx = ny - 2, nx - 2
    Sy, ly = dst_basis(my)
    Sx, lx = dst_basis(mx)
    # T[a, j, l] = sum_b Sx[b,j] Sx[b,l] / (ly[a] + lx[b])
    inv = 1.0 / (ly[:, None] + lx[None, :])                     # [a, b]
    T = np.einsum('bj,bl,ab->ajl', Sx, Sx, inv, optimize=True)   # [a, j, l]
    Y = np.einsum('ai,ak->ika', Sy, Sy, optimize=True)           # [i, k, a]
    G = Y.reshape(my * my, my) @ T.reshape(my, mx * mx)          # [(i,k), (j,l)]
    G = G.reshape(my, my, mx, mx).transpose(0, 2, 1, 3).reshape(my * mx, my * mx)
    return np.ascontiguousarray(G)


def dst_inverse_rows(nx, ny, rows):
    """Selected rows of the closed-form K^{-1} (eps = 1), for sampled checks at
    sizes where the full N x N matrix is not wanted."""
    my, mx = ny - 2, nx - 2
    Sy, ly = dst_basis(my)
    Sx, lx = dst_basis(mx)
    inv = 1.0 / (ly[:, None] + lx[None, :])                     # [a, b]
    out = np.empty((len(rows), my * mx), dtype=np.float64)
    for t, p in enumerate(rows):
        i, j = divmod(int(p), mx)
        # row[(k,l)] = sum_{a,b} Sy[a,i] Sy[a,k] Sx[b,j] Sx[b,l] inv[a,b]
        C = (Sy[:, i][:, None] * Sx[:, j][None, :]) * inv        # [a, b]
        out[t] = (Sy.T @ C @ Sx).reshape(-1)                     # [k, l]
    return out


def dst_inverse_3d(nx, ny, nz):
    """Closed-form K^{-1} for the 7-point operator with eps = 1:
    K = T_z (x) I (x) I + I (x) T_y (x) I + I (x) I (x) T_x with T = tridiag(-1, 2, -1),
    so K = V diag(lz_a + ly_b + lx_c) V^T with V = S_z (x) S_y (x) S_x (the
    orthonormal DST-I bases), and K^{-1} = V diag(1 / (lz_a + ly_b + lx_c)) V^T."""
    Sz, lz = dst_basis(nz - 2)
    Sy, ly = dst_basis(ny - 2)
    Sx, lx = dst_basis(nx - 2)
    V = np.kron(Sz, np.kron(Sy, Sx))
    lam = (lz[:, None, None] + ly[None, :, None] + lx[None, None, :]).reshape(-1)
    return (V / lam[None, :]) @ V.T
