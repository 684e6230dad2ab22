"""Pins of the oracle to values the paper prints: Fig. 3 and Table 1."""

import os

import numpy as np
import pytest

from oracle import grid, table1


def _load_fig3(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "fig3_matrix.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([float(t) for t in line.split()])
    return np.array(rows)


def test_fig3_matrix_bit_exact(golden_dir):
    """Fig. 3: node order, identity rows at the boundary, -0.25 stencil."""
    A = grid.paper_full_matrix(3, 5)
    ref = _load_fig3(golden_dir)
    assert A.shape == (15, 15)
    assert np.array_equal(A, ref)


def test_fig3_rhs_layout(golden_dir):
    """Fig. 3 RHS: boundary values at the identity rows, the source at rows 5, 8, 11."""
    with open(os.path.join(golden_dir, "fig3_rhs.txt")) as f:
        tokens = [t for line in f if not line.startswith("#") for t in line.split()]
    nx, ny, h = 3, 5, 0.5
    ub = np.arange(15, dtype=np.float64).reshape(5, 3) + 100.0
    rho = np.full((5, 3), 8.0)
    rhs = grid.paper_full_rhs(nx, ny, h, rho, ub)
    for P, tok in enumerate(tokens):
        i, j = divmod(P, nx)
        if tok == "B":
            assert rhs[P] == ub[i, j]
        else:
            # source term of Eq. 2 in the unit-diagonal form: -(h^2/4) rho
            assert rhs[P] == -0.25 * h * h * 8.0
    assert grid.interior_count(nx, ny) == 3


def test_fig3_interior_block_is_quarter_K():
    """With eps = 1 the conservative interior operator is 4x the interior block of Fig. 3."""
    for nx, ny in ((3, 5), (6, 4), (7, 7)):
        A = grid.paper_full_matrix(nx, ny)
        interior = [i * nx + j for i in range(1, ny - 1) for j in range(1, nx - 1)]
        K, bB = grid.conservative_operator(nx, ny)
        assert np.array_equal(K, 4.0 * A[np.ix_(interior, interior)])
        assert np.all(bB == 0)


def _load_table1(golden_dir):
    out = {}
    with open(os.path.join(golden_dir, "table1.txt")) as f:
        lines = [l for l in f if not l.startswith("#") and l.strip()]
    sizes = [int(t) for t in lines[0].split()[1:]]
    for l in lines[1:]:
        t = l.split()
        d = None if t[0] == "none" else int(t[0])
        for n, v in zip(sizes, t[1:]):
            out[(d, n)] = v
    return sizes, out


def _matches_printed(value, printed):
    """Same value at the printed number of decimals (half-up display rounding)."""
    dec = len(printed.split(".")[1])
    return abs(value - float(printed)) <= 0.5 * 10.0 ** (-dec) + 1e-12


@pytest.mark.parametrize("n", [5, 11, 21, 41, pytest.param(81, marks=pytest.mark.slow)])
def test_table1_column(golden_dir, n):
    """Table 1: every cell except (1 digit, n=5) reproduces to the printed digits.

    The (1 digit, n=5) cell depends on how exact decimal ties are rounded and
    no tie rule reproduces the printed 0.0569; it is parity-unpinned and only
    checked to lie in the range spanned by the tie rules (half-up 0.0566 to
    half-even 0.0632).  The text says 6 digits where the table says 5; both are
    checked against the 5-digit row.
    """
    sizes, ref = _load_table1(golden_dir)
    errs = table1.experiment(n, [1, 2, 3, 5, 6, None])
    for d in (1, 2, 3, 5, None):
        if d == 1 and n == 5:
            assert 0.0566 <= errs[d] <= 0.0633
            continue
        assert _matches_printed(errs[d], ref[(d, n)]), (d, n, errs[d], ref[(d, n)])
    assert _matches_printed(errs[6], ref[(5, n)])


def test_table1_printed_rhs_reading_fails():
    """The RHS printed in Eq. 2 (-rho h^2 with the unit-diagonal row) does not
    reproduce Table 1, so the -(h^2/4) rho reading is the one pinned."""
    n = 11
    X, Y, h = table1.node_coords(n)
    rho = table1.eq4_source(X, Y)
    rhs = grid.paper_full_rhs(n, n, h, 4.0 * rho, np.zeros((n, n)))   # = -rho h^2
    u = (table1.full_inverse(n) @ rhs).reshape(n, n)
    err = float(np.max(np.abs(u - table1.eq5_solution(X, Y))) / np.max(np.abs(table1.eq5_solution(X, Y))))
    assert err > 1.0


def test_eq5_solves_eq4():
    """Eq. 5 is the exact solution of Eq. 4: check the Laplacian symbolically via
    a high-order finite difference at random interior points."""
    g = np.random.default_rng(7)
    x, y = g.uniform(0.1, 0.9, 20), g.uniform(0.1, 0.9, 20)
    d = 1e-3
    u = table1.eq5_solution
    lap = (u(x + d, y) + u(x - d, y) + u(x, y + d) + u(x, y - d) - 4 * u(x, y)) / d ** 2
    # u is a polynomial of degree 4 in each variable: the 5-point error is
    # d^2/12 (u_xxxx + u_yyyy), tiny here.
    assert np.allclose(lap, table1.eq4_source(x, y), atol=1e-5)
