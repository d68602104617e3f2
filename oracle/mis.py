"""Maximum independent set as a penalised QUBO (App. D, Experiments on MIS).

Test infrastructure (oracle): plain, slow, obviously correct.

The paper maximises sum_i x_i subject to x_i x_j = 0 on every edge, through
the penalised form max sum_i x_i - lam sum_{(i,j) in E} x_i x_j with lam = 4,
i.e. it minimises F(x) = -sum_i x_i + lam sum_{(i,j) in E} x_i x_j, and reports
the set size only for vectors that satisfy every constraint.

* ``objective(edges, x, lam)``: F by the definition above, per row of x.
* ``set_size(edges, x)``: (|S|, number of edges inside S) of each row: the size
  counts only when no edge lies inside (an independent set).
* ``independence_number(n, edges)``: the largest independent set by
  enumeration of all subsets (small n).
"""
from __future__ import annotations

import numpy as np

__all__ = ["objective", "set_size", "independence_number"]


def objective(edges, X, lam: int = 4) -> np.ndarray:
    X = np.atleast_2d(np.asarray(X)).astype(np.int64)
    E = np.asarray(edges)
    inside = np.sum(X[:, E[:, 0]] * X[:, E[:, 1]], axis=1)
    return -np.sum(X, axis=1) + lam * inside


def set_size(edges, X):
    X = np.atleast_2d(np.asarray(X)).astype(np.int64)
    E = np.asarray(edges)
    return np.sum(X, axis=1), np.sum(X[:, E[:, 0]] * X[:, E[:, 1]], axis=1)


def independence_number(n: int, edges) -> int:
    """max |S| over S with no edge inside, over all 2^n subsets (plain loops)."""
    adj = [0] * n
    for i, j in np.asarray(edges).tolist():
        adj[i] |= 1 << j
        adj[j] |= 1 << i
    best = 0
    for S in range(1 << n):
        ok = True
        T = S
        while T:
            i = (T & -T).bit_length() - 1
            if adj[i] & S:
                ok = False
                break
            T &= T - 1
        if ok:
            best = max(best, bin(S).count("1"))
    return best
