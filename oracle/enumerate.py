"""Exhaustive enumeration over {0,1}^n for small n.

* ``all_binary(n)``: every binary vector, in counting order (bit i of the index
  is x_i).
* ``brute_force(objective, n)``: min over {0,1}^n of any exact objective, with
  the first minimiser in counting order.
* ``multilinear_by_definition(F_all, x)``: f(x) = sum_xi P_x(xi) F(xi) with
  P_x(xi) = prod_i x_i^xi_i (1-x_i)^(1-xi_i) (Def. 2.2).
"""
from __future__ import annotations

import numpy as np

__all__ = ["all_binary", "brute_force", "multilinear_by_definition"]


def all_binary(n: int, start: int = 0, stop=None) -> np.ndarray:
    stop = (1 << n) if stop is None else stop
    idx = np.arange(start, stop, dtype=np.int64)
    return ((idx[:, None] >> np.arange(n, dtype=np.int64)[None, :]) & 1).astype(np.uint8)


def brute_force(objective, n: int, chunk: int = 1 << 16):
    """(F*, first minimiser) of objective over {0,1}^n; objective maps a (N, n)
    binary array to N exact values."""
    if n > 22:
        raise ValueError("brute force is for n <= 22")
    best, arg = None, None
    for s in range(0, 1 << n, chunk):
        Xb = all_binary(n, s, min(s + chunk, 1 << n))
        F = objective(Xb)
        i = int(np.argmin(F))
        if best is None or F[i] < best:
            best, arg = F[i].item(), Xb[i].copy()
    return best, arg


def multilinear_by_definition(F_all, x) -> float:
    """Def. 2.2: sum over all xi of P_x(xi) F(xi); F_all[idx] is F at all_binary(n)[idx]."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    Xi = all_binary(n).astype(np.float64)
    P = np.prod(np.where(Xi == 1.0, x[None, :], 1.0 - x[None, :]), axis=1)
    return float(np.sum(P * np.asarray(F_all, dtype=np.float64)))
