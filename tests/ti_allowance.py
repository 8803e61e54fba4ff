"""The smallest value a float32 LB_TI kernel may return for a pair, from the
oracle's float64 per-cell triangle bounds (test helper)."""
import numpy as np

import oracle as O


def ti_lower_allowance(q, c, W, P, top):
    """The smallest value the float32 LB_TI may return for (q, c): per band
    cell the oracle's float64 triangle bounds (L, U) with L lowered by twice
    the kernel's allowance s U (the allowance it subtracts, plus at most as
    much float32 drift of the recursion in its (V = L + U, U) form),
    s = (1.5 D + 20 + r_max) u 1.02 with r_max the longest chain of
    recursion steps since an exact value; the
    column minima of max(0, .) squared and summed, then lowered by the
    float32 summation error and the kernel's final deflation, 2 (n + 5) u."""
    m, D = q.shape
    n = c.shape[0]
    u = 2.0 ** -24
    if P > 0:
        rmax = P - 1 if top else 2 * (P - 1) + 1
    else:
        rmax = m if top else 2 * m + 1
    s = (1.5 * D + 20.0 + rmax) * u * 1.02
    Lo, Hi = O.ti_cells(q, c, W, P=P, top=top)
    cell = np.maximum(Lo - 2.0 * 1.01 * s * Hi, 0.0)
    col = np.nanmin(np.where(np.isnan(Lo), np.inf, cell), axis=0)
    return float(np.sum(col * col)) * (1.0 - 2.0 * (n + 5) * u * 1.01)
