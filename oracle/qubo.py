"""QUBO objective, its multilinear extension and gradient.

Problem (Eq. 1 with a quadratic F): minimise F(x) = sum_ij Q_ij x_i x_j +
sum_i c_i x_i over x in {0,1}^n.  Q may be asymmetric and may carry a diagonal.

Canonical form (Prop. 2.4): on binary points x_i^2 = x_i, so the multilinear
extension drops the exponent of every diagonal term:
    f(x) = sum_{i != j} Q_ij x_i x_j + sum_i (c_i + Q_ii) x_i
         = 1/2 x^T A x + c'^T x,   A = offdiag(Q + Q^T),  c' = c + diag(Q).
Its gradient is A x + c'.  The method runs on (f/s) for a scale s > 0, so the
gradient used by Alg. 1 is (A x + c') / s.

Arrays of iterates have shape (B, n): one row per restart.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

__all__ = ["dense_Q", "canonicalize", "objective", "objective_fsum", "objective_exact",
           "f_multilinear", "grad_f", "QuboProblem", "RealQuboProblem"]

_EXACT = 2.0 ** 53


def dense_Q(q) -> np.ndarray:
    """The coupling matrix of a workloads.Qubo as a dense int64 array."""
    if q.Q is not None:
        return q.Q.astype(np.int64)
    out = np.zeros((q.n, q.n), dtype=np.int64)
    rows = np.repeat(np.arange(q.n), np.diff(q.row_ptr))
    np.add.at(out, (rows, q.col_idx), q.vals.astype(np.int64))
    return out


def _sparse_Q(q) -> sp.csr_matrix:
    return sp.csr_matrix((q.vals.astype(np.float64), q.col_idx, q.row_ptr), shape=(q.n, q.n))


def _c(q) -> np.ndarray:
    return np.zeros(q.n, dtype=np.float64) if q.c is None else np.asarray(q.c, dtype=np.float64)


def canonicalize(q):
    """(A, c') of Prop. 2.4: A = offdiag(Q + Q^T) (dense ndarray or scipy CSR,
    float64) and c' = c + diag(Q) (float64)."""
    if q.Q is not None:
        Qf = q.Q.astype(np.float64)
        A = Qf + Qf.T
        np.fill_diagonal(A, 0.0)
        cp = _c(q) + np.diag(Qf)
        return A, cp
    S = _sparse_Q(q)
    A = (S + S.T).tolil()
    A.setdiag(0.0)
    A = A.tocsr()
    A.eliminate_zeros()
    cp = _c(q) + S.diagonal()
    return A, cp


def objective(q, Xr) -> np.ndarray:
    """Exact F(x) = x^T Q x + c^T x of each row of the binary array Xr, from the
    original (uncanonicalised) Q and c.  Returns int64 of shape (B,).

    Integer data are summed in float64 only under the guard that the sum of
    |Q_ij| and |c_i| stays below 2**53, so that every partial sum is an exactly
    representable integer whatever the summation order."""
    Xr = np.atleast_2d(np.asarray(Xr)).astype(np.float64)
    if not np.all((Xr == 0.0) | (Xr == 1.0)):
        raise ValueError("objective() takes binary vectors")
    c = _c(q)
    if q.Q is not None:
        bound = float(np.abs(q.Q.astype(np.float64)).sum()) + float(np.abs(c).sum())
        if not bound < _EXACT:
            raise OverflowError("weights too large for the exact float64 path")
        XQ = Xr @ q.Q.astype(np.float64)                # (B, n): sum_i x_i Q_ij
    else:
        bound = float(np.abs(q.vals.astype(np.float64)).sum()) + float(np.abs(c).sum())
        if not bound < _EXACT:
            raise OverflowError("weights too large for the exact float64 path")
        XQ = (_sparse_Q(q).T @ Xr.T).T
    quad = np.sum(XQ * Xr, axis=1)
    lin = Xr @ c
    return np.rint(quad + lin).astype(np.int64)


def objective_fsum(Q, c, x) -> float:
    """F(x) for real weights, correctly rounded (math.fsum of every selected term)."""
    x = np.asarray(x).astype(bool)
    S = np.nonzero(x)[0]
    terms = [float(Q[i, j]) for i in S for j in S]
    if c is not None:
        terms += [float(c[i]) for i in S]
    return math.fsum(terms)


_SCALE_BITS = 1074   # every finite float64 is an integer multiple of 2**-1074


def _exact_int(v) -> int:
    """v * 2**1074 as a Python int (exact for every finite float64)."""
    num, den = float(v).as_integer_ratio()
    return num * ((1 << _SCALE_BITS) // den)


def objective_exact(q, Xr) -> np.ndarray:
    """Exact F(x) = sum_ij Q_ij x_i x_j + sum_i c_i x_i (Eq. 1) for real
    (float64) weights, one value per row of the binary array Xr, as
    fractions.Fraction in an object array.  Each selected term is taken as the
    integer v * 2**1074 and the integers are added exactly, so the value is the
    exact real sum; float() of it is the correctly rounded float64.  q is a
    workloads.Qubo whose Q or vals (and c) hold float64."""
    from fractions import Fraction
    Xr = np.atleast_2d(np.asarray(Xr)).astype(bool)
    n = q.n
    c = [0] * n if q.c is None else [_exact_int(v) for v in np.asarray(q.c, dtype=np.float64)]
    if q.Q is not None:
        rows, cols = np.nonzero(np.asarray(q.Q) != 0)
        vals = [_exact_int(q.Q[i, j]) for i, j in zip(rows, cols)]
    else:
        rows = np.repeat(np.arange(n), np.diff(q.row_ptr))
        cols = np.asarray(q.col_idx)
        vals = [_exact_int(v) for v in np.asarray(q.vals, dtype=np.float64)]
    out = np.empty(Xr.shape[0], dtype=object)
    for b in range(Xr.shape[0]):
        x = Xr[b]
        sel = np.nonzero(x[rows] & x[cols])[0]
        total = sum(vals[k] for k in sel) + sum(c[i] for i in np.nonzero(x)[0])
        out[b] = Fraction(total, 1 << _SCALE_BITS)
    return out


def f_multilinear(A, cp, X) -> np.ndarray:
    """f(x) = 1/2 x^T A x + c'^T x for each row of X (Prop. 2.4)."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    AX = (A @ X.T).T
    return 0.5 * np.sum(AX * X, axis=1) + X @ cp


def grad_f(A, cp, X, s: float = 1.0) -> np.ndarray:
    """Gradient of f/s at each row of X: (A x + c') / s."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    return ((A @ X.T).T + cp[None, :]) / s


class QuboProblem:
    """Adapter giving Alg. 1 the gradient of f/s and the exact objective."""

    def __init__(self, q, s: float = 1.0):
        self.q = q
        self.s = float(s)
        self.A, self.cp = canonicalize(q)
        self.n = q.n

    def grad(self, X):
        return grad_f(self.A, self.cp, X, self.s)

    def objective(self, Xr):
        return objective(self.q, Xr)

    def f(self, X):
        return f_multilinear(self.A, self.cp, X) / self.s

    def theta_upper(self) -> float:
        """Upper bound on max over the box of ||grad(f/s)||_1 (used by Prop. 3.3)."""
        absA = abs(self.A)
        rows = np.asarray(absA.sum(axis=1)).ravel()
        return float(np.sum(rows + np.abs(self.cp)) / self.s)


class RealQuboProblem(QuboProblem):
    """QuboProblem for float64 weights: the gradient as for integers (float64),
    the objective exact (Fractions), so that the incumbent's comparisons of
    Alg. 1's best-of-B are exact."""

    def objective(self, Xr):
        return objective_exact(self.q, Xr)
