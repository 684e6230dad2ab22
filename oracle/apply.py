"""Step 3 of "The solution steps": multiply the (rounded) inverse by the RHS.

The product the paper's method repeats "at every time moment" is
u = L^{-1} rho.  With the conservative interior operator K of ``grid`` this is
    u = K^{-1} (-h^2 rho + b_B) = -h^2 * G rho + w,   G = K^{-1},  w = G b_B.
Right-hand sides are the columns of rho [N, R].
"""

import numpy as np

from .quant import max_mag


def lift(G, bB):
    """w = G b_B: the part of u due to the Dirichlet data."""
    return np.asarray(G, dtype=np.float64) @ np.asarray(bB, dtype=np.float64)


def plain_apply(G, rho, h, w=None):
    """u = -h^2 G rho + w in float64 (library matmul)."""
    u = (-(h * h)) * (np.asarray(G, dtype=np.float64) @ np.asarray(rho, dtype=np.float64))
    if w is not None:
        u = u + np.asarray(w, dtype=np.float64)[:, None]
    return u


def integer_product(qG, qR):
    """acc[i, r] = sum_k qG[i, k] * qR[k, r], exact in int64."""
    return np.asarray(qG, dtype=np.int64) @ np.asarray(qR, dtype=np.int64)


def scale_constant(h, S, Sr):
    """c = -h^2 / (M_S * M_Sr), computed once in float64."""
    return -(h * h) / (float(max_mag(S)) * float(max_mag(Sr)))


def integer_apply(qG, e, S, qR, f, Sr, h, w=None, row_exponent=True):
    """Quantised solve: u[i, r] = double(acc[i, r]) * 2^(e_i + f_r) * c + w_i.

    acc is the exact integer product, converted to float64 once (exact while
    |acc| < 2^53, round-half-even beyond), multiplied by the power-of-two-scaled
    constant c = -h^2/(M_S M_Sr) (one rounding) and then added to w_i (one
    rounding).  With ``row_exponent=False`` e is ignored (its scales were
    already folded into qR, as in the adjoint).
    Returns (u float64 [N, R], acc int64 [N, R]).
    """
    acc = integer_product(qG, qR)
    c = scale_constant(h, S, Sr)
    ee = np.asarray(e, dtype=np.int64)[:, None] if row_exponent else np.zeros((acc.shape[0], 1), np.int64)
    scale = np.ldexp(np.full(acc.shape, c), ee + np.asarray(f, dtype=np.int64)[None, :])
    u = acc.astype(np.float64) * scale
    if w is not None:
        u = u + np.asarray(w, dtype=np.float64)[:, None]
    return u, acc


def slice_pair_products(dG, dR):
    """Per slice-pair integer partial products P[s, t] = dG[s] @ dR[t] (int64),
    for debugging the slice decomposition.  sum_{s,t} P[s,t] * 256^(S-1-s + Sr-1-t)
    equals the full integer product."""
    S, Sr = dG.shape[0], dR.shape[0]
    return np.stack([np.stack([dG[s] @ dR[t] for t in range(Sr)]) for s in range(S)])


def tile_apply(q, e, S, tile, rho, h, w=None):
    """Solve with 2-D tile scales (the rounding of Table 1 with one exponent
    per tile x tile block of G instead of one per row):
        u_i = -h^2 / M_S * sum_b 2^(e_ab) * sum_(k in tile b) q_ik rho_k + w_i,
    a = the row's tile.  Each tile's product is a float64 matmul of the stored
    integers with rho; the tile sums are scaled by their power of two (exact)
    and added over b in increasing order.  Returns float64 [N, R]."""
    q = np.asarray(q, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    e = np.asarray(e, dtype=np.int64)
    N, K = q.shape
    acc = np.zeros((N, rho.shape[1]))
    for a in range(e.shape[0]):
        rows = slice(a * tile, min(N, (a + 1) * tile))
        for b in range(e.shape[1]):
            cols = slice(b * tile, min(K, (b + 1) * tile))
            acc[rows] += np.ldexp(q[rows, cols] @ rho[cols], int(e[a, b]))
    u = (-(h * h) / float(max_mag(S))) * acc
    if w is not None:
        u = u + np.asarray(w, dtype=np.float64)[:, None]
    return u
