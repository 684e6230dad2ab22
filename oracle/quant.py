"""Rounding of the inverse's entries, in binary fixed point.

The paper's experiment behind Table 1 rounds every entry of the inverse to a
fixed number of decimal places and multiplies the rounded matrix by the
right-hand side.  Here the same idea is stated in base 2 with one scale per
row, so that the product becomes an exact integer product:

* b = 8*S bits per entry, S in {1, 2, 3}.  The largest magnitude is
  M_S = 127 * (256^S - 1) / 255  (127, 32639, 8355711): the largest integer
  whose balanced base-256 expansion has S digits in [-128, 127] with a top
  digit in [-127, 127].
* e_i = the binary exponent of max_k |G_ik| as returned by frexp, so that
  max_k |G_ik| < 2^e_i (an all-zero row gets e_i = 0).
* q_ik = round-half-even( (G_ik * 2^-e_i) * M_S ): one exact power-of-two scaling,
  one rounded float64 multiply, one rint.  |q_ik| <= M_S.
* The represented value is G^_ik = q_ik * 2^e_i / M_S.

The right-hand side is quantised the same way with one exponent per column
(per right-hand side) and S_r digits.
"""

import numpy as np


def max_mag(S):
    """M_S = 127 * (256^S - 1) / 255."""
    if S not in (1, 2, 3):
        raise ValueError("S must be 1, 2 or 3")
    return 127 * (256 ** S - 1) // 255


def frexp_exponent(x):
    """Exponent e with |x| < 2^e (frexp convention), 0 for x == 0."""
    _, e = np.frexp(np.asarray(x, dtype=np.float64))
    return np.asarray(e, dtype=np.int64)


def quantize_rows(G, S):
    """Per-row fixed point: returns (q int64 [N, K], e int64 [N])."""
    G = np.asarray(G, dtype=np.float64)
    M = float(max_mag(S))
    e = frexp_exponent(np.max(np.abs(G), axis=1))
    scaled = np.ldexp(G, -e[:, None])          # exact (power of two)
    q = np.rint(scaled * M)                     # one rounded multiply, then half-even
    return q.astype(np.int64), e


def quantize_cols(X, S, pre_exponent=None):
    """Per-column fixed point of X [K, R] (one exponent per right-hand side).

    If ``pre_exponent`` (int [K]) is given, row k of X is first multiplied by
    2^pre_exponent[k] (exact); the adjoint uses this to carry the row scales of
    the quantised inverse over to its transpose.
    Returns (q int64 [K, R], f int64 [R]).
    """
    X = np.asarray(X, dtype=np.float64)
    if pre_exponent is not None:
        X = np.ldexp(X, np.asarray(pre_exponent, dtype=np.int64)[:, None])
    M = float(max_mag(S))
    f = frexp_exponent(np.max(np.abs(X), axis=0)) if X.shape[0] > 0 else np.zeros(X.shape[1], np.int64)
    scaled = np.ldexp(X, -f[None, :])
    q = np.rint(scaled * M)
    return q.astype(np.int64), f


def dequantize_rows(q, e, S):
    """G^ = q * 2^e / M_S (float64; exact when |q| < 2^53)."""
    return np.ldexp(np.asarray(q, dtype=np.float64) / float(max_mag(S)), np.asarray(e)[:, None])


def balanced_digits(q, S):
    """Balanced base-256 digits of integers q, most significant first.

    Repeatedly take d = ((q + 128) mod 256) - 128 (in [-128, 127]) off the low
    end and divide the rest by 256.  Returns int64 [S, ...] with
    q = sum_s digits[s] * 256^(S-1-s).
    """
    q = np.array(q, dtype=np.int64, copy=True)
    out = np.empty((S,) + q.shape, dtype=np.int64)
    for s in range(S - 1, -1, -1):
        d = np.mod(q + 128, 256) - 128
        out[s] = d
        q = (q - d) // 256
    if np.any(q != 0):
        raise ValueError("value does not fit in S balanced digits")
    return out


def quantize_tiles(G, S, tile):
    """2-D tile scales: one exponent per tile x tile block of G.

    Returns (q int64 [N, K], e int64 [ceil(N/tile), ceil(K/tile)]).
    """
    G = np.asarray(G, dtype=np.float64)
    N, K = G.shape
    tn, tk = -(-N // tile), -(-K // tile)
    e = np.zeros((tn, tk), dtype=np.int64)
    q = np.zeros((N, K), dtype=np.int64)
    M = float(max_mag(S))
    for a in range(tn):
        for b in range(tk):
            blk = G[a * tile:(a + 1) * tile, b * tile:(b + 1) * tile]
            ee = int(frexp_exponent(np.max(np.abs(blk))))
            e[a, b] = ee
            q[a * tile:(a + 1) * tile, b * tile:(b + 1) * tile] = np.rint(np.ldexp(blk, -ee) * M).astype(np.int64)
    return q, e


def dequantize_tiles(q, e, S, tile):
    """G^ = q * 2^e_ab / M_S with e_ab the exponent of the entry's tile (float64)."""
    q = np.asarray(q, dtype=np.float64)
    N, K = q.shape
    E = np.repeat(np.repeat(np.asarray(e, dtype=np.int64), tile, axis=0), tile, axis=1)[:N, :K]
    return np.ldexp(q / float(max_mag(S)), E)
