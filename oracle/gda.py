"""Algorithm 1 (PDBO): simultaneous projected gradient descent-ascent on
L(x, y) = f(x) + sum_i y_i g(x_i), with the perturbation away from 1/2.

For every coordinate i, from (x^t, y^t) (Alg. 1; Eq. 6):
  * if |x_i - 1/2| <= delta and |dL/dx_i| <= 2 delta and y_i <= 0, x_i moves to
    1/2 - delta when x_i <= 1/2 and to 1/2 + delta otherwise;
  * else x_i takes the projected gradient step clip(x_i - alpha dL/dx_i, 0, 1);
  * in both cases y_i gains beta g(x_i^t), evaluated at the OLD x (the update is
    simultaneous).
B independent restarts run side by side and the best rounded solution over all
restarts is retained (Sec. 4.2 Model Settings).

Readings where the paper is silent:
  * rounding: x_r = [x > 1/2] (ties go to 0, like the x <= 1/2 branch);
  * tracking: round(x^t) is evaluated exactly after every iteration t = 1..T;
    the incumbent is the lexicographic minimum of (F, t, b): the first restart
    attaining the best value of an iteration, replaced only on strict
    improvement, so the earliest iteration wins ties.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .binarity import by_name

__all__ = ["alg1_update", "constraint_fn", "round_half", "Incumbent", "RunResult", "run", "step"]


def alg1_update(X, Y, grad_f, alpha, beta, delta, g, dual="vector"):
    """One iteration of Alg. 1 for all coordinates of all restarts.

    X, grad_f: arrays of shape (B, n); grad_f is the gradient of f at X.
    Y: shape (B, n), one dual variable per constraint g(x_i) = 0 (Alg. 1), or
    with dual="scalar" shape (B, 1), one per restart for the single constraint
    sum_i g(x_i) = 0 (the PDBO-s variant, Sec. 4.5): the same primal step with
    y in place of every y_i, and the dual ascent along the constraint's value,
    y + beta * sum_i g(x_i).
    Returns (X^{t+1}, Y^{t+1}, dL/dx)."""
    dL = grad_f + Y * g.deriv(X)
    near_half = np.abs(X - 0.5) <= delta
    flat = np.abs(dL) <= 2.0 * delta
    nonpos = Y <= 0.0
    perturb = near_half & flat & nonpos
    x_pert = np.where(X <= 0.5, 0.5 - delta, 0.5 + delta)
    x_step = np.clip(X - alpha * dL, 0.0, 1.0)
    X_new = np.where(perturb, x_pert, x_step)
    if dual == "scalar":
        Y_new = Y + beta * np.sum(g.value(X), axis=1, keepdims=True)
    else:
        Y_new = Y + beta * g.value(X)
    return X_new, Y_new, dL


def constraint_fn(p):
    """The g named by the parameters (with its degree for the polynomial)."""
    name = p.get("g", "quad")
    if name in ("poly", "polynomial"):
        return by_name(name, d=int(p.get("g_degree", 1)))
    return by_name(name)


def round_half(X):
    return np.asarray(X) > 0.5


@dataclass
class Incumbent:
    F: Optional[int] = None
    t: int = -1
    b: int = -1
    x: Optional[np.ndarray] = None

    def offer(self, F_all, t, Xr):
        b = int(np.argmin(F_all))                    # first index of the minimum
        if self.F is None or F_all[b] < self.F:
            F = F_all[b]
            self.F, self.t, self.b = (F.item() if hasattr(F, "item") else F), t, b
            self.x = np.array(Xr[b], dtype=np.uint8)
            return True
        return False


@dataclass
class RunResult:
    inc: Incumbent
    X: np.ndarray
    Y: np.ndarray
    steps: int
    F_last: Optional[np.ndarray] = None
    sum_g: list = field(default_factory=list)        # per step: sum_i g(x_i^t) per restart
    y_min: list = field(default_factory=list)
    f_values: list = field(default_factory=list)     # per step: f(x^t) per restart
    trace: list = field(default_factory=list)        # (t, F, b) at each improvement


def step(problem, X, Y, p):
    """One Alg. 1 iteration from (X, Y); returns (X+, Y+, grad f, dL/dx)."""
    g = constraint_fn(p)
    G = problem.grad(X)
    Xn, Yn, dL = alg1_update(X, Y, G, p["alpha"], p["beta"], p["delta"], g,
                             p.get("dual", "vector"))
    return Xn, Yn, G, dL


def run(problem, x0, p, T=None, Y0=None, record=False, eval_every=1) -> RunResult:
    """Alg. 1 for T iterations over the restarts given by the rows of x0
    (p["dual"] == "scalar": the single-constraint variant, Y of shape (B, 1))."""
    g = constraint_fn(p)
    dual = p.get("dual", "vector")
    T = p["T"] if T is None else T
    X = np.array(x0, dtype=np.float64, copy=True)
    if Y0 is not None:
        Y = np.array(Y0, dtype=np.float64, copy=True)
    elif dual == "scalar":
        Y = np.full((X.shape[0], 1), float(p["y0"]))
    else:
        Y = np.full_like(X, p["y0"])
    res = RunResult(inc=Incumbent(), X=X, Y=Y, steps=0)
    for t in range(T):
        G = problem.grad(X)
        if record:
            res.sum_g.append(np.sum(g.value(X), axis=1))
            res.y_min.append(float(Y.min()))
            res.f_values.append(problem.f(X))
        X, Y, _ = alg1_update(X, Y, G, p["alpha"], p["beta"], p["delta"], g, dual)
        if (t + 1) % eval_every == 0:
            Xr = round_half(X)
            F = problem.objective(Xr)
            res.F_last = F
            if res.inc.offer(F, t + 1, Xr):
                res.trace.append((t + 1, res.inc.F, res.inc.b))
        res.steps = t + 1
    res.X, res.Y = X, Y
    return res
