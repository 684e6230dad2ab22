"""CPU oracle for the dense-inverse Poisson solve.  TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call or execute anything in this package.  The product
path (the HIP library and its Python binding) never touches it, and the two
share no code: no kernels, headers, helpers, tables or constant generators.

What it computes, written from the paper (Dourbal & Pekker, "A New Numerical
Method for Fast Solution of Partial Integro-Differential Equations"):

* ``grid``     -- the 5-point discretisation of Eq. 1 / Eq. 2 with Dirichlet
                  identity rows in the node order of Fig. 3, and the
                  conservative variable-eps interior operator.
* ``inverse``  -- step 2 of "The solution steps": invert the matrix by a
                  standard method (dense LU with partial pivoting), plus the
                  closed-form DST inverse used to pin it.
* ``quant``    -- the rounding of the inverse's entries (the rounding experiment
                  behind Table 1), restated in binary fixed point with one
                  exponent per row or per 2-D tile.
* ``apply``    -- step 3: multiply the (rounded) inverse by the right-hand side,
                  in FP64, as an exact integer product, and with 2-D tile
                  scales.
* ``split``    -- BF16/FP32 split-precision emulation with exact products.
* ``grad``     -- adjoint, eps-gradients (2-D, 3-D, per direction on
                  non-uniform grids), Eq. 3 coefficient gradient and central
                  finite differences (not in the paper; the derivative of the
                  step-3 map).
* ``table1``   -- Eq. 4-6 and the Table 1 experiment.
* ``metrics``  -- relative L2 per right-hand side and the Eq. 6 error.

Everything is plain numpy/scipy in float64 (int64 / Python int for the
integer work), unblocked and unfused beyond what a library primitive does.
"""

from . import grid, inverse, quant, apply, split, grad, table1, metrics  # noqa: F401
