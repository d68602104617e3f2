"""Weighted Max-k-SAT as binary optimisation (Sec. 4.1, Max-k-SAT).

A clause C_j is a set of literals; x_v = 1 means variable v is true.  With
p(x) = x for a negated literal and p(x) = 1 - x for a plain one, the product
prod_{l in C_j} p(x_l) is 1 exactly when every literal of C_j is false, i.e.
when the clause is unsatisfied, and 0 otherwise.  The paper minimises the count
of unsatisfied clauses; this build weights clause j by w_j (reading), so

    F(x) = sum_j w_j [C_j unsatisfied],   f(x) = sum_j w_j prod_{l in C_j} p(x_l),

and by Prop. 2.4 this f is already the multilinear extension of F (the k
variables of a clause are distinct).

Literals use the DIMACS convention: +v is x_v, -v is not x_v, v is 1-based.
Arrays of iterates have shape (B, n).
"""
from __future__ import annotations

import numpy as np

__all__ = ["split_literals", "literal_probs", "objective", "f_multilinear",
           "grad_f", "MaxSatProblem"]


def split_literals(lits):
    """(variable index 0-based, negated flag) for an (m, k) DIMACS literal array."""
    lits = np.asarray(lits)
    if np.any(lits == 0):
        raise ValueError("literal 0 is not a DIMACS literal")
    return np.abs(lits) - 1, lits < 0


def literal_probs(lits, X):
    """p(x_l) for every literal of every clause: shape (B, m, k)."""
    var, neg = split_literals(lits)
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    xv = X[:, var]                                   # (B, m, k)
    return np.where(neg[None], xv, 1.0 - xv)


def objective(inst, Xr) -> np.ndarray:
    """Exact weighted count of unsatisfied clauses of each binary row of Xr (int64)."""
    var, neg = split_literals(inst.lits)
    Xr = np.atleast_2d(np.asarray(Xr)).astype(bool)
    true_lit = Xr[:, var] != neg[None]               # literal value: x_v, or not x_v
    unsat = ~np.any(true_lit, axis=2)                # (B, m)
    return unsat.astype(np.int64) @ np.asarray(inst.w, dtype=np.int64)


def f_multilinear(inst, X) -> np.ndarray:
    """f(x) = sum_j w_j prod_l p(x_l) for each row of X."""
    P = literal_probs(inst.lits, X)
    return np.prod(P, axis=2) @ np.asarray(inst.w, dtype=np.float64)


def grad_f(inst, X, s: float = 1.0) -> np.ndarray:
    """Gradient of f/s: for each occurrence of variable i at position l of
    clause j, add w_j * p'(x_l) * prod_{l' != l} p(x_l'), with p' = +1 for a
    negated literal and -1 otherwise."""
    var, neg = split_literals(inst.lits)
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    B, n = X.shape
    P = literal_probs(inst.lits, X)                  # (B, m, k)
    w = np.asarray(inst.w, dtype=np.float64)
    k = P.shape[2]
    G = np.zeros((B, n), dtype=np.float64)
    GT = G.T                                         # (n, B) view for scatter-add
    for l in range(k):
        others = np.ones(P.shape[:2])
        for l2 in range(k):
            if l2 != l:
                others = others * P[:, :, l2]
        dp = np.where(neg[:, l], 1.0, -1.0)          # (m,)
        contrib = others * (w * dp)[None, :]          # (B, m)
        np.add.at(GT, var[:, l], contrib.T)
    return G / s


class MaxSatProblem:
    """Adapter giving Alg. 1 the gradient of f/s and the exact objective."""

    def __init__(self, inst, s: float = 1.0):
        self.inst = inst
        self.s = float(s)
        self.n = inst.n

    def grad(self, X):
        return grad_f(self.inst, X, self.s)

    def objective(self, Xr):
        return objective(self.inst, Xr)

    def f(self, X):
        return f_multilinear(self.inst, X) / self.s

    def theta_upper(self) -> float:
        """Upper bound on max over the box of ||grad(f/s)||_1: each occurrence
        contributes at most w_j."""
        return float(self.inst.k * np.sum(np.asarray(self.inst.w, dtype=np.float64)) / self.s)
