"""Seeded synthetic inputs for the Poisson-inverse workloads.

This module only draws inputs (permittivity fields, charge densities, request
lists).  It holds none of the solver's arithmetic, and both the HIP path and
the CPU reference receive the very same arrays from it.  Seeds follow
seed = 1000 * workload + stream.

Node coordinates follow Eq. 2 on the unit square: x_j = j*h, y_i = i*h with
h = 1/(n-1); arrays are [n_y][n_x] (slow axis y, fast axis x, as in Fig. 3).
Interior arrays are [R][N] with N = (n_y-2)*(n_x-2) in row-major interior order.
"""

import numpy as np

WORKLOADS = {
    # name: (grid points per side, number of right-hand sides)
    "plain_32": (32, 1),
    "vareps_64": (64, 256),
    "quant_128": (128, 1024),
    "grad_192": (192, 256),
}


def rng(workload, stream):
    return np.random.default_rng(1000 * int(workload) + int(stream))


def coords(n):
    h = 1.0 / (n - 1)
    t = np.arange(n, dtype=np.float64) * h
    Y, X = np.meshgrid(t, t, indexing="ij")
    return X, Y, h


def interior(a):
    """Interior part of a nodal [n_y][n_x] array (or a stack [..., n_y, n_x]), flattened."""
    a = np.asarray(a)
    sub = a[..., 1:-1, 1:-1]
    return np.ascontiguousarray(sub.reshape(sub.shape[:-2] + (-1,)))


def blob_params(g, count=4):
    """Gaussian blob parameters: amplitude ~ N(0,1), width ~ U[0.05, 0.15],
    centre ~ U[0.1, 0.9]^2."""
    amp = g.standard_normal(count)
    width = g.uniform(0.05, 0.15, count)
    cx = g.uniform(0.1, 0.9, count)
    cy = g.uniform(0.1, 0.9, count)
    return amp, width, cx, cy


def blobs(n, amp, width, cx, cy):
    """Nodal field sum_b amp_b * exp(-r_b^2 / (2 width_b^2))."""
    X, Y, _ = coords(n)
    f = np.zeros_like(X)
    for a, w, x0, y0 in zip(amp, width, cx, cy):
        f += a * np.exp(-((X - x0) ** 2 + (Y - y0) ** 2) / (2.0 * w * w))
    return f


def blob_rhs(n, nrhs, g, drift_steps=None):
    """[nrhs][N] interior charge densities made of 4 Gaussian blobs.

    With ``drift_steps`` the blobs are drawn once and move with seeded
    velocities v ~ U[-1,1]^2: centre(t) = c + v * t / drift_steps, t = 0..nrhs-1
    (time steps of one drifting field).  Without it every RHS has its own blobs.
    """
    out = np.empty((nrhs, (n - 2) * (n - 2)), dtype=np.float64)
    if drift_steps is not None:
        amp, width, cx, cy = blob_params(g)
        vx = g.uniform(-1.0, 1.0, 4)
        vy = g.uniform(-1.0, 1.0, 4)
        for t in range(nrhs):
            out[t] = interior(blobs(n, amp, width, cx + vx * t / drift_steps, cy + vy * t / drift_steps))
    else:
        for r in range(nrhs):
            out[r] = interior(blobs(n, *blob_params(g)))
    return out


def eps_sincos(n):
    """eps(x, y) = 1 + 0.5 sin(2 pi x) cos(2 pi y) at the nodes."""
    X, Y, _ = coords(n)
    return 1.0 + 0.5 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)


def eps_lognormal(n, g, sigma=0.3, box=5):
    """Log-normal field smoothed by a box filter: Z ~ N(0,1) iid on an
    (n+box-1)^2 array, eps = exp(sigma * Z), then the mean over each valid
    box x box window gives the n x n nodal field."""
    pad = box - 1
    Z = g.standard_normal((n + pad, n + pad))
    E = np.exp(sigma * Z)
    c = np.cumsum(np.cumsum(np.pad(E, ((1, 0), (1, 0))), axis=0), axis=1)
    S = c[box:, box:] - c[:-box, box:] - c[box:, :-box] + c[:-box, :-box]
    return S / float(box * box)


def uniform_rhs(n, nrhs, g):
    """[nrhs][N] iid uniform[-1, 1] charge densities."""
    return g.uniform(-1.0, 1.0, (nrhs, (n - 2) * (n - 2)))


def uniform_rhs_n(N, nrhs, g):
    """[nrhs][N] iid uniform[-1, 1] values for N unknowns (any dimension)."""
    return g.uniform(-1.0, 1.0, (nrhs, N))


# --- the five workloads -----------------------------------------------------

def plain_32():
    """32x32 grid (900 unknowns), eps = 1, zero Dirichlet data, one blob RHS."""
    n = 32
    return dict(n=n, h=1.0 / (n - 1), eps=None, ub=None, rho=blob_rhs(n, 1, rng(1, 0)))


def coupled_32(steps=64, tau=4.0):
    """Time-coupled stepping on the 32x32 grid: rho_{t+1} = rho_t + tau * u_t
    with u_t the solution for rho_t (one right-hand side per step, each step
    depending on the previous one); rho_0 is the plain_32 blob field."""
    n = 32
    return dict(n=n, h=1.0 / (n - 1), rho0=blob_rhs(n, 1, rng(1, 0)), tau=tau, steps=steps)


def vareps_64(nrhs=256):
    """64x64 grid, eps = 1 + 0.5 sin(2 pi x) cos(2 pi y), 256 drifting-blob time steps."""
    n = 64
    return dict(n=n, h=1.0 / (n - 1), eps=eps_sincos(n), ub=None,
                rho=blob_rhs(n, nrhs, rng(2, 0), drift_steps=512))


def quant_128(nrhs=1024):
    """128x128 grid (15876 unknowns), eps = 1, nrhs uniform[-1,1] RHS."""
    n = 128
    return dict(n=n, h=1.0 / (n - 1), eps=None, ub=None, rho=uniform_rhs(n, nrhs, rng(3, 0)))


BATCH_SIZES = (32, 64, 96, 128, 160)


def batched_requests(nreq=4096, pool=4, sizes=BATCH_SIZES, max_rhs=64, seed_stream=0):
    """Request list for the batched uneven workload.

    Returns (operators, requests): operators is a list of dicts (n, eps) with
    ``pool`` log-normal eps fields per grid size; every request names an
    operator index and a number of blob right-hand sides ~ U{1..max_rhs}.
    Right-hand sides are drawn lazily by :func:`request_rhs`.
    """
    g = rng(4, seed_stream)
    ops = []
    for n in sizes:
        for k in range(pool):
            ops.append(dict(n=n, eps=eps_lognormal(n, g)))
    reqs = []
    for r in range(nreq):
        n = sizes[int(g.integers(0, len(sizes)))]
        k = int(g.integers(0, pool))
        op = sizes.index(n) * pool + k
        nrhs = int(g.integers(1, max_rhs + 1))
        reqs.append(dict(op=op, nrhs=nrhs, seed=int(g.integers(0, 2 ** 31))))
    return ops, reqs


def request_rhs(n, nrhs, seed):
    return blob_rhs(n, nrhs, np.random.default_rng(seed))


def grad_192(nrhs=256, nsample=512):
    """192x192 grid (36100 unknowns), eps as vareps_64, 256 blob RHS, 512 sampled
    interior points; also a separately seeded true source for the data d."""
    n = 192
    g = rng(5, 0)
    N = (n - 2) * (n - 2)
    sample = np.sort(g.choice(N, nsample, replace=False))
    rho = blob_rhs(n, nrhs, rng(5, 1))
    rho_true = blob_rhs(n, nrhs, rng(5, 2))
    return dict(n=n, h=1.0 / (n - 1), eps=eps_sincos(n), ub=None, rho=rho,
                rho_true=rho_true, sample=sample)


def random_eps(nx, ny, g, lo=0.5, hi=2.0):
    """Generic positive eps field for tests: iid uniform in [lo, hi], [n_y][n_x]."""
    return g.uniform(lo, hi, (ny, nx))


def blob_params_batch(g, nrhs, count=4):
    """Blob parameters for nrhs independent right-hand sides: arrays [nrhs, count]."""
    return (g.standard_normal((nrhs, count)), g.uniform(0.05, 0.15, (nrhs, count)),
            g.uniform(0.1, 0.9, (nrhs, count)), g.uniform(0.1, 0.9, (nrhs, count)))


def blob_rhs_device(n, params, device="cuda"):
    """The blob fields of :func:`blob_rhs` evaluated with torch on a device, for
    workloads too large to draw on the host: params from :func:`blob_params_batch`;
    returns a float64 tensor [nrhs, (n-2)^2]."""
    import torch
    amp, width, cx, cy = (torch.as_tensor(a, dtype=torch.float64, device=device) for a in params)
    t = torch.arange(1, n - 1, dtype=torch.float64, device=device) / (n - 1)
    Y, X = torch.meshgrid(t, t, indexing="ij")
    X = X.reshape(1, 1, -1)
    Y = Y.reshape(1, 1, -1)
    r2 = (X - cx[:, :, None]) ** 2 + (Y - cy[:, :, None]) ** 2
    return (amp[:, :, None] * torch.exp(-r2 / (2.0 * width[:, :, None] ** 2))).sum(dim=1)
