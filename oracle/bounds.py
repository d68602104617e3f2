"""Quantities from the convergence analysis (Sec. 3.2.2).

* Prop. 3.3: with Theta = max over the box of ||grad f||_1, every dual iterate
  satisfies y_i^t >= b = (1 + Theta) / g'(1/2 - delta)
                         + (2 + ceil(1 / (2 alpha))) * beta * g(1/2).
  Any upper bound on Theta gives a (weaker) valid bound, since g'(1/2-delta) < 0.
* Proof of Thm. 3.7: y_i^0 - y_i^T = -beta * sum_{t<T} g(x_i^t), so
  sum_i (y_i^0 - y_i^T) = -beta * sum_{t<T} sum_i g(x_i^t).
* Def. 3.6: x is epsilon-binary when -sum_i g(x_i) <= epsilon.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["prop33_lower_bound", "telescoping_gap", "binarity_gap"]


def prop33_lower_bound(theta: float, alpha: float, beta: float, delta: float, g) -> float:
    gp = float(g.deriv(np.array(0.5 - delta)))
    ghalf = float(g.value(np.array(0.5)))
    return (1.0 + theta) / gp + (2 + math.ceil(1.0 / (2.0 * alpha))) * beta * ghalf


def telescoping_gap(Y0, YT, sum_g_per_step, beta) -> np.ndarray:
    """Per restart: sum_i (y_i^0 - y_i^T) + beta * sum_t sum_i g(x_i^t) (zero up to rounding)."""
    lhs = np.sum(np.asarray(Y0) - np.asarray(YT), axis=1)
    rhs = -beta * np.sum(np.asarray(sum_g_per_step), axis=0)
    return lhs - rhs


def binarity_gap(X, g) -> np.ndarray:
    """-sum_i g(x_i) per restart (Def. 3.6)."""
    return -np.sum(g.value(np.asarray(X, dtype=np.float64)), axis=1)
