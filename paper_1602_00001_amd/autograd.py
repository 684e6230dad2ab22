"""torch.autograd.Function around the solve: forward = step 3 (u = L^{-1} rho),
backward = adjoint apply + permittivity gradient, both in the HIP library."""

import torch


class PinvSolve(torch.autograd.Function):
    """u = PinvSolve.apply(rho, eps, op, mode, bits).

    rho: [nrhs, N] float64 CUDA tensor.  eps: the nodal permittivity tensor
    [n_y, n_x] ([n_z, n_y, n_x] for a 3-D op) the op was built from (only its
    gradient is produced here; the op is not rebuilt).  op: a PoissonInverse
    built on a uniform grid.  Returns u [nrhs, N].
    Gradients: drho = lambda = -h^2 G^T g, deps = nodal eps-gradient.
    """

    @staticmethod
    def forward(ctx, rho, eps, op, mode="fp64", bits=16):
        u = op.apply(rho.contiguous(), mode=mode, rho_bits=bits)
        ctx.op, ctx.mode, ctx.bits = op, mode, bits
        ctx.save_for_backward(u)
        ctx.eps_shape = None if eps is None else tuple(eps.shape)
        return u

    @staticmethod
    def backward(ctx, g):
        (u,) = ctx.saved_tensors
        op = ctx.op
        lam = op.apply_adjoint(g.contiguous(), mode=ctx.mode, g_bits=ctx.bits)
        deps = None
        if ctx.needs_input_grad[1]:
            deps = op.grad_eps(u, lam)
        return lam, deps, None, None, None


class PinvSolveGeneral(torch.autograd.Function):
    """u = PinvSolveGeneral.apply(rho, eps_x, eps_y, op, mode, bits) for an op
    from PoissonInverse.build_general (non-uniform grid, permittivity per
    direction).  eps_y may be None when the op was built with one field for
    both directions; eps_x then receives the whole gradient.
    Gradients: drho = lambda = -(K^{-1} diag(A))^T g; deps_x, deps_y from the
    x- and y-faces (pinv_grad_eps_general)."""

    @staticmethod
    def forward(ctx, rho, eps_x, eps_y, op, mode="fp64", bits=16):
        u = op.apply(rho.contiguous(), mode=mode, rho_bits=bits)
        ctx.op, ctx.mode, ctx.bits = op, mode, bits
        ctx.split = eps_y is not None
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, g):
        (u,) = ctx.saved_tensors
        op = ctx.op
        lam = op.apply_adjoint(g.contiguous(), mode=ctx.mode, g_bits=ctx.bits)
        gx = gy = None
        if ctx.needs_input_grad[1] or ctx.needs_input_grad[2]:
            if ctx.split:
                gx, gy = op.grad_eps_general(u, lam, split=True)
            else:
                gx = op.grad_eps_general(u, lam, split=False)
        return lam, gx, gy, None, None, None


class PinvSolveBeta(torch.autograd.Function):
    """u = PinvSolveBeta.apply(rho, beta, op, mode, bits) for an op from
    PoissonInverse.build_beta (Eq. 3 with arbitrary neighbour coefficients,
    u = A^{-1}(rho + b_B)).  beta: the [4, n_y, n_x] tensor the op was built
    from (only its gradient is produced here).
    Gradients: drho = lambda = A^{-T} g; dbeta = (1/4) sum_r lambda_p U_q
    (pinv_grad_beta)."""

    @staticmethod
    def forward(ctx, rho, beta, op, mode="fp64", bits=16):
        u = op.apply(rho.contiguous(), mode=mode, rho_bits=bits)
        ctx.op, ctx.mode, ctx.bits = op, mode, bits
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, g):
        (u,) = ctx.saved_tensors
        op = ctx.op
        lam = op.apply_adjoint(g.contiguous(), mode=ctx.mode, g_bits=ctx.bits)
        dbeta = op.grad_beta(u, lam) if ctx.needs_input_grad[1] else None
        return lam, dbeta, None, None, None
