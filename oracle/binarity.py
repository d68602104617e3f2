"""Binarity constraint functions g and their derivatives (Sec. 3.1).

The paper requires g to be convex and continuous on [0,1] with g(0)=g(1)=0,
differentiable on (0,1) with g'(x)=0 only at x=1/2, and symmetric about 1/2.
It names three choices: the quadratic x^2 - x (its default, Sec. 4.2 Model
Settings, and the Max-Cut example of Sec. 3.2.1), the entropy
x log x + (1-x) log(1-x) extended continuously to the end points (used for
Max-k-SAT), and the even-degree polynomial (2x-1)^(2d) - 1.

Reading: the entropy's derivative log(x/(1-x)) is unbounded at 0 and 1; it is
evaluated at x clipped to [eps, 1-eps] with eps = 2**-20.
"""
from __future__ import annotations

import numpy as np

__all__ = ["Quadratic", "Entropy", "Polynomial", "by_name"]


class Quadratic:
    """g(x) = x^2 - x,  g'(x) = 2x - 1."""
    name = "quad"

    @staticmethod
    def value(x):
        return x * x - x

    @staticmethod
    def deriv(x):
        return 2.0 * x - 1.0


class Entropy:
    """g(x) = x log x + (1-x) log(1-x) with 0 log 0 := 0,
    g'(x) = log(x~) - log(1 - x~),  x~ = clip(x, eps, 1-eps)."""
    name = "entropy"

    def __init__(self, eps: float = 2.0 ** -20):
        self.eps = eps

    @staticmethod
    def _xlogx(x):
        x = np.asarray(x, dtype=np.float64)
        out = np.zeros_like(x)
        pos = x > 0
        out[pos] = x[pos] * np.log(x[pos])
        return out

    def value(self, x):
        x = np.asarray(x, dtype=np.float64)
        return self._xlogx(x) + self._xlogx(1.0 - x)

    def deriv(self, x):
        xc = np.clip(np.asarray(x, dtype=np.float64), self.eps, 1.0 - self.eps)
        return np.log(xc) - np.log(1.0 - xc)


class Polynomial:
    """g(x) = (2x-1)^(2d) - 1,  g'(x) = 4d (2x-1)^(2d-1)."""
    name = "poly"

    def __init__(self, d: int = 1):
        self.d = int(d)

    def value(self, x):
        return (2.0 * x - 1.0) ** (2 * self.d) - 1.0

    def deriv(self, x):
        return 4.0 * self.d * (2.0 * x - 1.0) ** (2 * self.d - 1)


def by_name(name: str, **kw):
    if name in ("quad", "quadratic"):
        return Quadratic()
    if name == "entropy":
        return Entropy(**kw)
    if name in ("poly", "polynomial"):
        return Polynomial(**kw)
    raise ValueError(f"unknown constraint function {name!r}")
