"""Split-precision emulation of the inverse-times-RHS product (not in the paper).

A float64 value x is written as a sum of bfloat16 parts, each the
round-to-nearest-even bfloat16 of what the earlier parts left over:
    x0 = bf16(x), x1 = bf16(x - x0), x2 = bf16(x - x0 - x1).
The residuals are exact in float64.  BF16x3 keeps the products
a0*b0 + a0*b1 + a1*b0; BF16x6 adds a0*b2 + a1*b1 + a2*b0 (the published BF16
split scheme of Henry, Tang and Heinecke, ARITH 2019).  Products of bfloat16
values are exact in float64, and the emulation sums them in float64, so the
only rounding is the split itself.  FP32 mode rounds both operands to float32.
"""

import numpy as np


def round_bf16(x):
    """Round float64 -> bfloat16 (as float64), round-half-even, via float32.

    Rounding first to float32 and then to bfloat16 can double-round; to avoid
    that the float64 value is rounded directly: take the float64 bits, keep the
    top 1+8+7 bits of the float32-equivalent mantissa with half-even on the rest.
    Implemented exactly with frexp/ldexp on the float64 value.
    """
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                       # x = m * 2^e, 0.5 <= |m| < 1
    # bfloat16 keeps 8 significant bits: m * 2^8 rounded half-even.
    r = np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)
    return np.where(x == 0, 0.0, r)


def round_f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def split_bf16(x, parts):
    """Return a list of ``parts`` bfloat16-valued float64 arrays summing to ~x."""
    x = np.asarray(x, dtype=np.float64)
    out, rest = [], x.copy()
    for _ in range(parts):
        p = round_bf16(rest)
        out.append(p)
        rest = rest - p                      # exact
    return out


def split_apply(G, rho, h, mode, w=None):
    """Emulated u = -h^2 * G rho + w for mode in {'fp32', 'bf16x3', 'bf16x6'}."""
    G = np.asarray(G, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    if mode == 'fp32':
        acc = round_f32(G) @ round_f32(rho)
    elif mode == 'bf16x3':
        a, b = split_bf16(G, 2), split_bf16(rho, 2)
        acc = a[0] @ b[0] + (a[0] @ b[1] + a[1] @ b[0])
    elif mode == 'bf16x6':
        a, b = split_bf16(G, 3), split_bf16(rho, 3)
        acc = a[0] @ b[0] + (a[0] @ b[1] + a[1] @ b[0]) + (a[0] @ b[2] + a[1] @ b[1] + a[2] @ b[0])
    else:
        raise ValueError(mode)
    u = -(h * h) * acc
    if w is not None:
        u = u + np.asarray(w, dtype=np.float64)[:, None]
    return u
