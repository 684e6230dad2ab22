"""Error measures: relative L2 per right-hand side and the Eq. 6 error."""

import numpy as np


def rel_l2_per_rhs(u, ref):
    """||u_r - ref_r||_2 / ||ref_r||_2 for every column r (0 for a zero column
    that is matched exactly, inf if the reference column is zero and u is not)."""
    u = np.asarray(u, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if u.ndim == 1:
        u, ref = u[:, None], ref[:, None]
    num = np.sqrt(np.sum((u - ref) ** 2, axis=0))
    den = np.sqrt(np.sum(ref ** 2, axis=0))
    with np.errstate(divide='ignore', invalid='ignore'):
        out = np.where(den > 0, num / np.where(den > 0, den, 1.0), np.where(num > 0, np.inf, 0.0))
    return out


def eq6_error(u_num, u_anal):
    """Eq. 6: max |u_anal - u_num| over grid points / max |u_anal| over grid points."""
    u_num = np.asarray(u_num, dtype=np.float64)
    u_anal = np.asarray(u_anal, dtype=np.float64)
    return float(np.max(np.abs(u_anal - u_num)) / np.max(np.abs(u_anal)))
