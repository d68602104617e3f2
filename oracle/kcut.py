"""Max-k-Cut through the softmax reparametrisation (App. B).

Test infrastructure (oracle): plain float64 NumPy/SciPy, one step at a time.

Node i has logits Z_{:,i} in R^k and probabilities X_{:,i} = softmax(Z_{:,i}).
Here arrays are restart-major with the category last: Z, X of shape (B, n, k).
The objective Tr(X W X^T) = sum_{i,j} W_ij X_{:,i}.X_{:,j} is minimised; on
one-hot X it is twice the weight of the edges inside the parts.  With g
quadratic (sum_c X_ci^2 - 1) or entropy (sum_c X_ci log X_ci) the Lagrangian is
L(Z, y) = Tr(X W X^T)/s + sum_i y_i g(X_{:,i}), and simultaneous gradient
descent-ascent moves Z by -alpha dL/dZ and y by +beta g(X) at the old X.

Readings: Z is unconstrained, so Alg. 1's projection and perturbation (defined
for the box) are not applied; the entropy's log is taken at X clipped below at
2^-20; the rounded assignment of node i is argmax_c X_ci, the lowest c on ties;
F is the weight of the edges whose ends share a category, each edge once.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

__all__ = ["Graph", "softmax", "objective", "cut_weight", "lagrangian", "grad_Z", "step", "run"]

EPS = 2.0 ** -20


class Graph:
    """Symmetric weighted graph from CSR arrays holding both directions."""

    def __init__(self, g):
        self.n, self.k = int(g.n), int(g.k)
        self.W = sp.csr_matrix((np.asarray(g.w, np.float64), g.col_idx, g.row_ptr),
                               shape=(self.n, self.n))
        iu = sp.triu(self.W, 1).tocoo()
        self.ei, self.ej, self.ew = iu.row, iu.col, iu.data.astype(np.int64)
        self.total = int(self.ew.sum())


def softmax(Z):
    Z = np.asarray(Z)
    e = np.exp(Z - np.max(Z.real, axis=-1, keepdims=True))
    return e / np.sum(e, axis=-1, keepdims=True)


def objective(G: Graph, cats) -> np.ndarray:
    """Weight of the edges inside the parts, each edge once (int64), per row of
    the category array (B, n)."""
    cats = np.atleast_2d(np.asarray(cats))
    same = cats[:, G.ei] == cats[:, G.ej]
    return same.astype(np.int64) @ G.ew


def cut_weight(G: Graph, cats) -> np.ndarray:
    return G.total - objective(G, cats)


def _g(X, kind):
    if kind == "quad":
        return np.sum(X * X, axis=-1) - 1.0
    return np.sum(np.where(X.real > 0, X * np.log(np.where(X.real > 0, X, 1.0)), 0.0), axis=-1)


def _dg(X, kind):
    if kind == "quad":
        return 2.0 * X
    return np.log(np.maximum(X.real, EPS) if not np.iscomplexobj(X) else X) + 1.0


def lagrangian(G: Graph, Z, Y, s: float, kind: str):
    """L(Z, y) per restart (accepts complex Z for complex-step derivatives)."""
    X = softmax(Z)
    XW = np.stack([G.W @ X[b] for b in range(X.shape[0])])
    return np.sum(X * XW, axis=(1, 2)) / s + np.sum(Y * _g(X, kind), axis=1)


def grad_Z(G: Graph, Z, Y, s: float, kind: str):
    """dL/dZ (B, n, k): the gradient with respect to X, then the softmax Jacobian
    X_c (G_c - sum_c' X_c' G_c') of each node."""
    X = softmax(Z)
    XW = np.stack([G.W @ X[b] for b in range(X.shape[0])])
    GX = 2.0 * XW / s + Y[:, :, None] * _dg(X, kind)
    return X * (GX - np.sum(X * GX, axis=-1, keepdims=True))


def step(G: Graph, Z, Y, p):
    kind = p.get("g", "quad")
    X = softmax(Z)
    Zn = Z - p["alpha"] * grad_Z(G, Z, Y, p["scale"], kind)
    Yn = Y + p["beta"] * _g(X, kind)
    return Zn, Yn


def run(G: Graph, Z0, p, T: int):
    """T iterations; after each, the rounded assignment of every restart is
    evaluated and the incumbent (lexicographic minimum of (F, t, b)) kept."""
    Z = np.array(Z0, dtype=np.float64)
    Y = np.full(Z.shape[:2], float(p["y0"]))
    best = (None, -1, -1)
    for t in range(T):
        Z, Y = step(G, Z, Y, p)
        F = objective(G, np.argmax(softmax(Z), axis=-1))
        b = int(np.argmin(F))
        if best[0] is None or F[b] < best[0]:
            best = (int(F[b]), t + 1, b)
    return Z, Y, best
