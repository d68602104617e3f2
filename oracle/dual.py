"""Dual certificate (App. D, Dual Certificate): a lower bound on min F.

Test infrastructure (oracle): plain float64, no blocking or reordering.

For any y, min over the box [0,1]^n of L(x, y) = f(x)/s + sum_i y_i g(x_i) is at
most min over {0,1}^n of L(x, y) = min F / s, since g vanishes on binary points
(the weak duality in the proof of Thm. 3.2).  With the quadratic g and
y = ybar * 1, L(., y) is convex when A/s + 2 ybar I is positive semidefinite;
then at any box point x the linearisation gives
    min_box L >= L(x) + sum_i min(-d_i x_i, d_i (1 - x_i)),  d = grad_x L(x),
since a convex function lies above its tangent plane and the linear term is
minimised over the box coordinate by coordinate.  The paper minimises L(., y^0)
by gradient descent; here projected gradient descent, x <- clip(x - alpha d),
which is Alg. 1 with beta = 0 (y stays positive, so the perturbation never
applies).
"""
from __future__ import annotations

import numpy as np

__all__ = ["lagrangian", "grad_lagrangian", "certificate", "projected_descent"]


def lagrangian(prob, x, ybar: float) -> float:
    """L(x, ybar 1) = f(x)/s + ybar sum_i (x_i^2 - x_i)."""
    x = np.asarray(x, dtype=np.float64)
    return float(prob.f(x[None])[0]) + ybar * float(np.sum(x * x - x))


def grad_lagrangian(prob, x, ybar: float) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    return prob.grad(x[None])[0] + ybar * (2.0 * x - 1.0)


def certificate(prob, x, ybar: float):
    """(lower bound on min F, s L(x), Frank-Wolfe gap in objective units) at x."""
    x = np.asarray(x, dtype=np.float64)
    d = grad_lagrangian(prob, x, ybar)
    L = lagrangian(prob, x, ybar)
    lin = float(np.sum(np.minimum(-d * x, d * (1.0 - x))))
    return prob.s * (L + lin), prob.s * L, -prob.s * lin


def projected_descent(prob, ybar: float, alpha: float, iters: int, x0=None) -> np.ndarray:
    x = np.full(prob.q.n, 0.5) if x0 is None else np.array(x0, dtype=np.float64)
    for _ in range(iters):
        x = np.clip(x - alpha * grad_lagrangian(prob, x, ybar), 0.0, 1.0)
    return x
