"""Pins of the quantiser and the integer apply: brute force with exact rational
arithmetic (Python Fraction) on small inputs, digit identities and bounds."""

from fractions import Fraction
import math

import numpy as np
import pytest

from oracle import apply, grid, inverse, metrics, quant


def _frexp_exp_exact(x):
    """Smallest e with |x| < 2^e, by exact comparison (0 -> 0)."""
    x = abs(Fraction(x))
    if x == 0:
        return 0
    e = 0
    while x >= Fraction(2) ** e:
        e += 1
    while x < Fraction(2) ** (e - 1):
        e -= 1
    return e


def _round_half_even(fr):
    fl = math.floor(fr)
    rem = fr - fl
    if rem > Fraction(1, 2):
        return fl + 1
    if rem < Fraction(1, 2):
        return fl
    return fl if fl % 2 == 0 else fl + 1


def _brute_quantize_row(row, S):
    M = 127 * (256 ** S - 1) // 255
    e = _frexp_exp_exact(max(abs(float(v)) for v in row))
    out = []
    for v in row:
        # one float64 multiply (correctly rounded) of the exactly scaled value
        prod = Fraction(float(Fraction(v) / Fraction(2) ** e * M))
        out.append(_round_half_even(prod))
    return out, e


def test_max_mag():
    assert [quant.max_mag(s) for s in (1, 2, 3)] == [127, 32639, 8355711]
    for s in (1, 2, 3):
        # the largest value with s balanced digits, top digit <= 127
        assert quant.max_mag(s) == sum(127 * 256 ** k for k in range(s))


@pytest.mark.parametrize("S", [1, 2, 3])
def test_quantize_rows_brute_force(S):
    g = np.random.default_rng(S)
    G = g.standard_normal((6, 9)) * np.exp(g.uniform(-8, 3, (6, 1)))
    G[2, :] = 0.0
    G[3, 4] = 0.75  # an exact power-of-two-scaled value
    q, e = quant.quantize_rows(G, S)
    for i in range(G.shape[0]):
        qb, eb = _brute_quantize_row(G[i], S)
        assert e[i] == eb
        assert list(q[i]) == qb
    assert e[2] == 0 and np.all(q[2] == 0)
    assert np.all(np.abs(q) <= quant.max_mag(S))


def test_quantize_ties_to_even():
    """Products that land exactly on k + 1/2 round to the even neighbour."""
    S, M = 1, quant.max_mag(1)
    xs = [(2 * k + 1) / (2.0 * M) for k in range(50)]
    row = np.array([0.5] + xs + [-x for x in xs])      # max 0.5 -> e = 0
    q, e = quant.quantize_rows(row[None, :], S)
    assert e[0] == 0
    ties = 0
    for idx, x in enumerate(row[1:], start=1):
        p = x * M
        if abs(p - np.trunc(p)) == 0.5:
            ties += 1
            assert q[0, idx] % 2 == 0
            assert abs(q[0, idx] - p) == 0.5
    assert ties >= 20


@pytest.mark.parametrize("S", [1, 2, 3])
def test_balanced_digits_identity_and_range(S):
    M = quant.max_mag(S)
    g = np.random.default_rng(10 + S)
    extra = np.array([M, -M, 0, 127, -127, 128, -128, 255, -255, 32767, -32768])
    q = np.concatenate([g.integers(-M, M + 1, 5000), extra[np.abs(extra) <= M]])
    d = quant.balanced_digits(q, S)
    rec = sum(d[s] * 256 ** (S - 1 - s) for s in range(S))
    assert np.array_equal(rec, q)
    assert d.min() >= -128 and d.max() <= 127
    assert np.all(np.abs(d[0]) <= 127)


def test_balanced_digits_reject_overflow():
    with pytest.raises(ValueError):
        quant.balanced_digits(np.array([quant.max_mag(1) + 200]), 1)


@pytest.mark.parametrize("S", [1, 2, 3])
def test_quantisation_error_bound(S):
    """|G^ - G| <= 2^e / (2 M_S) per entry, with equality impossible beyond it."""
    g = np.random.default_rng(20 + S)
    G = g.standard_normal((40, 50))
    q, e = quant.quantize_rows(G, S)
    Gh = quant.dequantize_rows(q, e, S)
    bound = np.ldexp(np.ones((40, 1)) / (2 * quant.max_mag(S)), e[:, None])
    assert np.all(np.abs(Gh - G) <= bound * (1 + 1e-12))


def _brute_quantize_col(col, S, pre=None):
    """One right-hand side by exact rationals: the optional row pre-scaling
    2^pre[k] (exact), the frexp exponent of the column's largest magnitude,
    then per entry one correctly rounded float64 multiply of the exactly
    scaled value by M_S and a round-half-even."""
    M = 127 * (256 ** S - 1) // 255
    vals = [Fraction(v) * (Fraction(2) ** int(pre[k]) if pre is not None else 1) for k, v in enumerate(col)]
    f = _frexp_exp_exact(max(abs(v) for v in vals))
    out = [_round_half_even(Fraction(float(v / Fraction(2) ** f * M))) for v in vals]
    return out, f


@pytest.mark.parametrize("S", [1, 2, 3])
def test_quantize_cols_brute_force(S):
    """Per-column exponents and digits against exact rationals: columns of
    magnitudes spread over 2^-12 .. 2^4, an all-zero column (exponent 0,
    digits 0), a column whose largest magnitude is an exact power of two (its
    exponent is one more than that power's), and a column with one negative
    extreme."""
    g = np.random.default_rng(30 + S)
    K, R = 11, 7
    X = g.standard_normal((K, R)) * np.exp2(g.uniform(-12, 4, (1, R)))
    X[:, 2] = 0.0
    X[:, 4] = g.uniform(-0.25, 0.25, K)
    X[3, 4] = 0.5                      # max |x| = 2^-1 exactly -> f = 0
    X[5, 6] = -40.0 * np.max(np.abs(X[:, 6]))
    q, f = quant.quantize_cols(X, S)
    for r in range(R):
        qb, fb = _brute_quantize_col(X[:, r], S)
        assert f[r] == fb, r
        assert list(q[:, r]) == qb, r
    assert f[2] == 0 and np.all(q[:, 2] == 0)
    M = quant.max_mag(S)                 # odd, so 0.5 M is a tie: the even neighbour
    assert f[4] == 0 and q[3, 4] == ((M + 1) // 2 if (M + 1) // 2 % 2 == 0 else (M - 1) // 2)
    assert -M <= q[5, 6] <= -(M // 2)    # the column's extreme scales into [-1, -1/2)
    assert np.all(np.abs(q) <= quant.max_mag(S))


@pytest.mark.parametrize("S", [1, 2])
def test_quantize_cols_pre_exponent_brute_force(S):
    """The adjoint's path: row k of X scaled by 2^pre[k] before the column
    exponent is taken, checked against exact rationals (pre-scalings that move
    a column's maximum to another row included)."""
    g = np.random.default_rng(40 + S)
    K, R = 9, 5
    X = g.standard_normal((K, R))
    pre = g.integers(-6, 7, K)
    pre[0] = 12                         # row 0 dominates every column after scaling
    q, f = quant.quantize_cols(X, S, pre_exponent=pre)
    for r in range(R):
        qb, fb = _brute_quantize_col(X[:, r], S, pre)
        assert f[r] == fb, r
        assert list(q[:, r]) == qb, r


def test_quantize_cols_ties_to_even():
    """Entries whose scaled product lands exactly on k + 1/2 round to the even
    neighbour, per column (a column of max 0.5 has exponent 0)."""
    S, M = 1, quant.max_mag(1)
    xs = [(2 * k + 1) / (2.0 * M) for k in range(50)]
    col = np.array([0.5] + xs + [-x for x in xs])
    X = np.stack([col, col * 0.5], axis=1)          # second column: exponent -1, same digits
    q, f = quant.quantize_cols(X, S)
    assert list(f) == [0, -1]
    assert np.array_equal(q[:, 0], q[:, 1])
    ties = 0
    for idx, x in enumerate(col[1:], start=1):
        p = x * M
        if abs(p - np.trunc(p)) == 0.5:
            ties += 1
            assert q[idx, 0] % 2 == 0
            assert abs(q[idx, 0] - p) == 0.5
    assert ties >= 20


def test_quantize_cols_pre_exponent_is_exact_scaling():
    g = np.random.default_rng(4)
    X = g.standard_normal((30, 5))
    pe = g.integers(-4, 4, 30)
    q1, f1 = quant.quantize_cols(X, 2, pre_exponent=pe)
    q2, f2 = quant.quantize_cols(np.ldexp(X, pe[:, None]), 2)
    assert np.array_equal(q1, q2) and np.array_equal(f1, f2)


def test_integer_apply_brute_force():
    """acc is the exact integer product; u = RNE(RNE(acc * scale) + w)."""
    g = np.random.default_rng(9)
    N, R, S, Sr, h = 7, 3, 3, 2, 0.125
    G = g.standard_normal((N, N))
    rho = g.standard_normal((N, R))
    w = g.standard_normal(N)
    qG, e = quant.quantize_rows(G, S)
    qR, f = quant.quantize_cols(rho, Sr)
    u, acc = apply.integer_apply(qG, e, S, qR, f, Sr, h, w)
    c = Fraction(-(h * h) / (quant.max_mag(S) * quant.max_mag(Sr)))
    cf = float(c)  # the constant is computed once in float64
    for i in range(N):
        for r in range(R):
            a = sum(int(qG[i, k]) * int(qR[k, r]) for k in range(N))
            assert acc[i, r] == a
            scale = Fraction(cf) * Fraction(2) ** (int(e[i]) + int(f[r]))
            v = float(Fraction(float(Fraction(a) * scale)) + Fraction(float(w[i])))
            assert u[i, r] == v


def test_slice_pairs_recombine_to_integer_product():
    g = np.random.default_rng(12)
    S, Sr, N = 3, 2, 33
    qG = g.integers(-quant.max_mag(S), quant.max_mag(S) + 1, (N, N))
    qR = g.integers(-quant.max_mag(Sr), quant.max_mag(Sr) + 1, (N, 4))
    P = apply.slice_pair_products(quant.balanced_digits(qG, S), quant.balanced_digits(qR, Sr))
    tot = sum(P[s, t] * 256 ** ((S - 1 - s) + (Sr - 1 - t)) for s in range(S) for t in range(Sr))
    assert np.array_equal(tot, apply.integer_product(qG, qR))


def test_quantised_solve_error_envelope():
    """The quantised solve tracks the FP64 solve within the rounding envelope,
    and the 24x16-bit variant is within 1e-4 relative L2 on uniform RHS."""
    n = 40
    K, _ = grid.conservative_operator(n, n)
    G = inverse.lu_inverse(K)
    h = 1.0 / (n - 1)
    rho = np.random.default_rng(1).uniform(-1, 1, (G.shape[0], 8))
    ref = apply.plain_apply(G, rho, h)
    errs = {}
    for S in (1, 2, 3):
        qG, e = quant.quantize_rows(G, S)
        qR, f = quant.quantize_cols(rho, 2)
        u, _ = apply.integer_apply(qG, e, S, qR, f, 2, h)
        errs[S] = np.max(metrics.rel_l2_per_rhs(u, ref))
    assert errs[1] > errs[2] > errs[3]
    assert errs[3] < 1e-4


@pytest.mark.parametrize("S,tile", [(1, 3), (2, 4), (3, 5)])
def test_quantize_tiles_brute_force(S, tile):
    """2-D tile scales (one exponent per tile x tile block, ragged edge tiles):
    every block quantised exactly like one row holding all of the block's
    entries; an all-zero block gets exponent 0."""
    g = np.random.default_rng(10 + S)
    G = g.standard_normal((11, 13)) * np.exp(g.uniform(-6, 2, (11, 13)))
    G[:tile, :tile] = 0.0
    q, e = quant.quantize_tiles(G, S, tile)
    tn, tk = -(-11 // tile), -(-13 // tile)
    assert e.shape == (tn, tk)
    for a in range(tn):
        for b in range(tk):
            blk = G[a * tile:(a + 1) * tile, b * tile:(b + 1) * tile]
            qb, eb = _brute_quantize_row(blk.reshape(-1), S)
            assert e[a, b] == eb
            assert list(q[a * tile:(a + 1) * tile, b * tile:(b + 1) * tile].reshape(-1)) == qb
    assert e[0, 0] == 0 and np.all(q[:tile, :tile] == 0)
    # a tile as large as the matrix is one exponent for all of it
    q1, e1 = quant.quantize_tiles(G, S, 16)
    qb, eb = _brute_quantize_row(G.reshape(-1), S)
    assert e1.shape == (1, 1) and e1[0, 0] == eb and list(q1.reshape(-1)) == qb


def test_tile_apply_against_exact_rationals():
    """The tile-scaled solve against the same sum evaluated exactly in rational
    arithmetic, entry by entry (q / M_S * 2^e * rho summed with Fractions, times
    -h^2, plus w): a wrong tile index (a transposed exponent table), a dropped
    scale or sign, or a wrong M_S fails by far more than float64 rounding."""
    from fractions import Fraction
    g = np.random.default_rng(61)
    N, R, tile, S, h = 11, 3, 4, 2, 0.3
    G = g.standard_normal((N, N)) * np.exp(-np.abs(np.subtract.outer(np.arange(N), np.arange(N))))
    q, e = quant.quantize_tiles(G, S, tile)
    assert not np.all(e == e[0, 0])                      # tiles really differ in exponent
    rho = g.standard_normal((N, R))
    w = g.standard_normal(N)
    u = apply.tile_apply(q, e, S, tile, rho, h, w)
    M = quant.max_mag(S)
    for i in range(N):
        for r in range(R):
            s = Fraction(0)
            for k in range(N):
                s += Fraction(int(q[i, k])) / M * Fraction(2) ** int(e[i // tile, k // tile]) * Fraction(float(rho[k, r]))
            exact = -Fraction(h) * Fraction(h) * s + Fraction(float(w[i]))
            assert abs(float(exact) - u[i, r]) <= 1e-14 * (abs(float(exact)) + 1.0)


def test_tile_dequantisation_error_bound_and_transposed_tiles():
    """|G^ - G| <= 2^e_ab / (2 M) entry by entry (round to nearest), and a
    transposed exponent table does not satisfy it on a matrix whose tiles'
    magnitudes are not symmetric."""
    g = np.random.default_rng(62)
    N, tile, S = 24, 8, 2
    G = g.standard_normal((N, N))
    G[:8, 8:] *= 1e-3                                    # upper-right tiles small
    q, e = quant.quantize_tiles(G, S, tile)
    Gh = quant.dequantize_tiles(q, e, S, tile)
    E = np.repeat(np.repeat(e, tile, 0), tile, 1)
    M = quant.max_mag(S)
    assert np.all(np.abs(Gh - G) <= np.ldexp(1.0, E) / (2 * M) * (1 + 1e-12))
    bad = quant.dequantize_tiles(q, e.T, S, tile)
    assert np.max(np.abs(bad - G)) > 1.0


def test_tile_scales_meet_the_accuracy_bound_per_row_scales_miss():
    """At 16 bits on the 62^2 Poisson inverse with uniform rho, 64 x 64 tile
    scales keep the relative L2 error below 1e-4 where one exponent per row
    does not (the reason for the storage variant)."""
    from oracle import grid
    K, _ = grid.conservative_operator(64, 64)
    G = np.linalg.inv(K)
    N = G.shape[0]
    g = np.random.default_rng(63)
    rho = g.uniform(-1, 1, (N, 16))
    ref = G @ rho
    qr, er = quant.quantize_rows(G, 2)
    ur = quant.dequantize_rows(qr, er, 2) @ rho
    qt, et = quant.quantize_tiles(G, 2, 64)
    ut = apply.tile_apply(qt, et, 2, 64, rho, 1.0) * -1.0
    rel = lambda u: np.max(np.linalg.norm(u - ref, axis=0) / np.linalg.norm(ref, axis=0))
    assert rel(ut) < 1e-4 < rel(ur)
