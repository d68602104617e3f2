"""Hyper-parameters: the paper's table (Appendix C, tab:hyper_parameters) and
the readings this build adopts where the paper is silent.

``delta``: Alg. 1 only asks for delta > 0 and never prints a value; 2**-7 is used
so that 1/2 +- delta and the test |x - 1/2| <= delta are exact in fp64, fp32 and
bf16 alike.

``scale``: the table was tuned on +-1 Gset graphs and unweighted CNF formulas.
For larger integer weights the method is run on (Q/s, c/s), with s chosen so
that the paper's convexity threshold for the initial dual (Sec. 4.4: y_bar at
least -lambda_min of the quadratic form's matrix makes L(., y^0) convex) sits at
2/3 of y_bar = 6, as it does on Gset.  For a QUBO this is
s = -lambda_min(offdiag(Q + Q^T)/2) / 4; +-1 graphs use s = 1; weighted MaxSAT
uses s = mean clause weight.  The objective is always reported on the original
integers.
"""
from __future__ import annotations

import numpy as np

__all__ = ["PAPER_HYPER", "DELTA", "EPS_ENTROPY", "gda_params", "qubo_scale",
           "mis_scale", "maxsat_scale"]

# tab:hyper_parameters (Appendix C): B, y_bar, alpha, beta per problem class.
PAPER_HYPER = {
    "maxcut": dict(B=100, y0=6.0, alpha=0.025, beta=0.025),
    "mis": dict(B=10, y0=5.0, alpha=0.02, beta=0.02),
    "maxsat": dict(B=10, y0=2.0, alpha=0.01, beta=0.005),
    "maxkcut": dict(B=100, y0=6.0, alpha=0.01, beta=0.01),
}

DELTA = 2.0 ** -7          # perturbation tolerance delta of Alg. 1 (reading)
EPS_ENTROPY = 2.0 ** -20   # clip for the entropy derivative (reading)


def gda_params(kind: str, B: int, T: int, scale: float = 1.0, **over) -> dict:
    """Parameter dict shared by the oracle and the library bindings."""
    base = PAPER_HYPER["maxsat" if kind == "maxsat" else "maxcut"]
    p = dict(B=B, T=T, alpha=base["alpha"], beta=base["beta"], y0=base["y0"],
             delta=DELTA, scale=float(scale),
             g="entropy" if kind == "maxsat" else "quad")
    p.update(over)
    return p


def _qubo_scale(q) -> float:
    """s = -lambda_min(offdiag(Q+Q^T)/2) / 4, floored at 1 (ARPACK, fixed start)."""
    import scipy.sparse as sp
    from scipy.sparse.linalg import LinearOperator, eigsh

    n = q.n
    if q.Q is not None:
        M = q.Q.astype(np.float32)
        d = np.diag(q.Q).astype(np.float64)

        def mv(v):
            v32 = np.asarray(v, dtype=np.float32).ravel()
            return 0.5 * (M @ v32 + v32 @ M).astype(np.float64) - d * np.asarray(v).ravel()
    else:
        S = sp.csr_matrix((q.vals.astype(np.float64), q.col_idx, q.row_ptr), shape=(n, n))
        d = S.diagonal()

        def mv(v):
            v = np.asarray(v).ravel()
            return 0.5 * (S @ v + S.T @ v) - d * v
    op = LinearOperator((n, n), matvec=mv, dtype=np.float64)
    lam = eigsh(op, k=1, which="SA", tol=1e-3, v0=np.ones(n), return_eigenvectors=False)[0]
    return max(1.0, float(-lam / 4.0))


_SCALES = {}


def qubo_scale(q) -> float:
    """s = -lambda_min(offdiag(Q+Q^T)/2) / 4, floored at 1, computed once per
    instance in a process: ARPACK keeps a random seed between calls, so a
    second call can end in different last bits, and runs compared bit for bit
    must share s."""
    import hashlib
    h = hashlib.sha1(str(q.n).encode())
    for a in (q.Q, q.row_ptr, q.col_idx, q.vals, q.c):
        h.update(b"|" if a is None else np.ascontiguousarray(a).view(np.uint8).ravel())
    key = h.hexdigest()
    if key not in _SCALES:
        _SCALES[key] = _qubo_scale(q)
    return _SCALES[key]


def mis_scale(q) -> float:
    """Scale s of the MIS workloads (the penalised QUBO of App. D with lam = 4,
    y_bar = 5, alpha = beta = 0.02).  Graphs of degree d < 50 take qubo_scale.
    For d = 100 the paper's route to hyper-parameters, a grid search (App. C),
    was run over s on the n = 10^4 graph (rep 0, T = 40,000): s = 3, 4, 5, 6,
    8 and qubo_scale's 9.9 gave independent sets of 0, 507, 517, 497, 439 and
    340 nodes (n = 5*10^4: 0, 2497, 2569, 2447, 2166), so half of qubo_scale
    is taken there."""
    d = int(q.meta.get("d", 0))
    s = qubo_scale(q)
    return s / 2 if d >= 50 else s


def maxsat_scale(inst) -> float:
    return float(np.mean(inst.w))
