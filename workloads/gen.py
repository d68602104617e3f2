"""Seeded instance generators.

Every draw comes from ``numpy.random.default_rng([cfg_id, rep, stream, ...])``
with stream 0 the instance and stream 1 the starting points, so the oracle and
the HIP path see bit-identical inputs.  The shapes and distributions stand in
for the paper's benchmarks (Gset graphs for Max-Cut, random k-CNF formulas for
Max-k-SAT, Sec. 4.2), which are not reproduced here.

Conventions
-----------
* A QUBO instance is ``min_x  x^T Q x + c^T x`` over ``x in {0,1}^n`` (Eq. 1
  with a quadratic F).  ``Q`` is int32, dense row-major ``(n, n)`` or CSR
  (``row_ptr``, ``col_idx``, ``vals``); ``c`` is int64 ``(n,)`` or ``None``.
* A MaxSAT instance stores ``lits`` as an ``(m, k)`` int32 array with the DIMACS
  sign convention (``+v`` is the literal ``x_v``, ``-v`` its negation, 1-based)
  and ``w`` as ``(m,)`` int32 clause weights.
* Starting points are float64 arrays of shape ``(B, n)``: one row per restart.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "Qubo", "MaxSat", "rng_for", "x0_uniform",
    "gnp_pm1", "qubo_c1", "qubo_c1_twin", "maxcut_c2", "qubo_c3", "batch_c4",
    "maxsat_c5", "random_dense_qubo", "random_asym_qubo", "random_maxsat",
    "random_regular_graph", "mis_qubo", "real_qubo", "Kcut", "kcut_graph",
]


def rng_for(cfg_id: int, rep: int, stream: int, *extra: int) -> np.random.Generator:
    return np.random.default_rng([cfg_id, rep, stream, *extra])


@dataclass
class Qubo:
    n: int
    Q: Optional[np.ndarray] = None          # dense (n, n) int32
    row_ptr: Optional[np.ndarray] = None    # CSR int32 (n+1,)
    col_idx: Optional[np.ndarray] = None    # CSR int32 (nnz,)
    vals: Optional[np.ndarray] = None       # CSR int32 (nnz,)
    c: Optional[np.ndarray] = None          # int64 (n,) or None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def is_csr(self) -> bool:
        return self.Q is None

    def dense(self) -> np.ndarray:
        if self.Q is not None:
            return self.Q
        out = np.zeros((self.n, self.n), dtype=np.int32)
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        np.add.at(out, (rows, self.col_idx), self.vals)
        return out


@dataclass
class MaxSat:
    n: int
    lits: np.ndarray                        # (m, k) int32, DIMACS signs, 1-based
    w: np.ndarray                           # (m,) int32
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.lits.shape[0])

    @property
    def k(self) -> int:
        return int(self.lits.shape[1])


def x0_uniform(cfg_id: int, rep: int, B: int, n: int, *extra: int) -> np.ndarray:
    """Starting points x^0 ~ U([0,1]^n), one row per restart (Appendix C)."""
    return rng_for(cfg_id, rep, 1, *extra).random((B, n))


def _pairs_from_linear(n: int, lin: np.ndarray):
    iu, ju = np.triu_indices(n, 1)
    return iu[lin], ju[lin]


def _csr_from_upper(n: int, i: np.ndarray, j: np.ndarray, w: np.ndarray, diag=None):
    """Symmetric CSR holding w at (i,j) and (j,i) for i<j, plus an optional diagonal."""
    ii = [i, j]
    jj = [j, i]
    ww = [w, w]
    if diag is not None:
        nz = np.nonzero(diag)[0]
        ii.append(nz)
        jj.append(nz)
        ww.append(diag[nz])
    ii = np.concatenate(ii)
    jj = np.concatenate(jj)
    ww = np.concatenate(ww).astype(np.int32)
    order = np.lexsort((jj, ii))
    ii, jj, ww = ii[order], jj[order], ww[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, ii + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    return row_ptr, jj.astype(np.int32), ww


def gnp_pm1(n: int, p: float, rng: np.random.Generator) -> np.ndarray:
    """Dense symmetric adjacency of an Erdos-Renyi G(n,p) graph with weights
    +1/-1 drawn with probability 1/2 each; zero diagonal."""
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.shape[0]) < p
    sign = np.where(rng.random(iu.shape[0]) < 0.5, 1, -1).astype(np.int32)
    W = np.zeros((n, n), dtype=np.int32)
    W[iu[keep], ju[keep]] = sign[keep]
    W[ju[keep], iu[keep]] = sign[keep]
    return W


def qubo_c1(rep: int = 0, n: int = 200) -> Qubo:
    """G(n, 0.05) with +-1 weights, read as the literal QUBO Q=W, c=0."""
    W = gnp_pm1(n, 0.05, rng_for(1, rep, 0, n))
    return Qubo(n=n, Q=W, c=None, name=f"gnp_pm1_n{n}")


def qubo_c1_twin(rep: int = 0) -> Qubo:
    """The n=18 instance of the same generator, small enough for brute force."""
    return qubo_c1(rep, n=18)


def maxcut_c2(rep: int = 0, n: int = 2000, M: int = 6000) -> Qubo:
    """Max-Cut on G(n, M) (M distinct edges, mean degree 2M/n) with +-1 weights.

    As a QUBO: Q = W (symmetric CSR, both directions stored) and c = -W 1, so that
    F(x) = x^T W x - 1^T W x equals minus the cut weight (Sec. 4.1 Max-Cut)."""
    g = rng_for(2, rep, 0, n, M)
    lin = g.choice(n * (n - 1) // 2, size=M, replace=False)
    i, j = _pairs_from_linear(n, np.sort(lin))
    w = np.where(g.random(M) < 0.5, 1, -1).astype(np.int32)
    row_ptr, col_idx, vals = _csr_from_upper(n, i, j, w)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    c = -np.bincount(rows, weights=vals, minlength=n).astype(np.int64)
    return Qubo(n=n, row_ptr=row_ptr, col_idx=col_idx, vals=vals, c=c,
                name=f"maxcut_gnm_n{n}_m{M}")


def random_dense_qubo(n: int, lo: int, hi: int, rng: np.random.Generator,
                      with_c: bool = True) -> Qubo:
    """Symmetric dense Q with Q_ij = Q_ji ~ U{lo..hi} (diagonal included) and
    c ~ U{lo..hi}."""
    Q = rng.integers(lo, hi + 1, size=(n, n), dtype=np.int32)
    # mirror the upper triangle (diagonal included) into the lower one, blockwise
    bs = 1024
    for bi in range(0, n, bs):
        blk = Q[bi:bi + bs, bi:bi + bs]
        Q[bi:bi + bs, bi:bi + bs] = np.triu(blk) + np.triu(blk, 1).T
        for bj in range(bi + bs, n, bs):
            Q[bj:bj + bs, bi:bi + bs] = Q[bi:bi + bs, bj:bj + bs].T
    c = rng.integers(lo, hi + 1, size=n).astype(np.int64) if with_c else None
    return Qubo(n=n, Q=Q, c=c, name=f"dense_u{lo}_{hi}_n{n}")


def random_asym_qubo(n: int, lo: int, hi: int, rng: np.random.Generator) -> Qubo:
    """Dense Q with independent entries U{lo..hi} (asymmetric, diagonal
    included) and c ~ U{lo..hi}."""
    Q = rng.integers(lo, hi + 1, size=(n, n), dtype=np.int64).astype(np.int32)
    c = rng.integers(lo, hi + 1, size=n).astype(np.int64)
    return Qubo(n=n, Q=Q, c=c, name=f"asym_u{lo}_{hi}_n{n}")


def random_regular_graph(n: int, d: int, rng: np.random.Generator) -> np.ndarray:
    """Edges (i < j), shape (n d / 2, 2), of a simple d-regular graph on n
    vertices: a uniform random pairing of the n d half-edges (configuration
    model), after which every loop or repeated edge is replaced through a
    degree-preserving switch with a random other edge."""
    if (n * d) % 2 or not 0 <= d < n:
        raise ValueError("need n d even and d < n")
    stubs = np.repeat(np.arange(n, dtype=np.int64), d)
    rng.shuffle(stubs)
    E = np.sort(stubs.reshape(-1, 2), axis=1)
    key = E[:, 0] * n + E[:, 1]
    order = np.argsort(key, kind="stable")
    dup = np.zeros(len(E), dtype=bool)
    dup[order[1:]] = key[order[1:]] == key[order[:-1]]
    bad = np.flatnonzero((E[:, 0] == E[:, 1]) | dup)
    good = set(key[~((E[:, 0] == E[:, 1]) | dup)].tolist())
    for e in bad:
        while True:
            f = int(rng.integers(len(E)))
            if f == e or E[f, 0] * n + E[f, 1] not in good:
                continue
            u, v = int(E[e, 0]), int(E[e, 1])
            x, y = (int(E[f, 0]), int(E[f, 1])) if rng.random() < 0.5 else (int(E[f, 1]), int(E[f, 0]))
            a, b = min(u, x), max(u, x)
            c, dd = min(v, y), max(v, y)
            if a == b or c == dd or a * n + b in good or c * n + dd in good or (a, b) == (c, dd):
                continue
            good.discard(E[f, 0] * n + E[f, 1])
            E[e] = (a, b)
            E[f] = (c, dd)
            good.add(a * n + b)
            good.add(c * n + dd)
            break
    return E[np.lexsort((E[:, 1], E[:, 0]))]


def mis_qubo(n: int, d: int, rep: int = 0, lam: int = 4) -> Qubo:
    """Maximum independent set on a random d-regular graph as the penalised
    QUBO of App. D: minimise -sum_i x_i + lam sum_{(i,j) in E} x_i x_j (CSR
    holding lam/2 at (i,j) and (j,i) for every edge, c = -1)."""
    if lam % 2:
        raise ValueError("lam must be even: Q holds lam/2 at (i,j) and (j,i)")
    E = random_regular_graph(n, d, rng_for(6, rep, 0, n, d))
    rp, col, val = _csr_from_upper(n, E[:, 0], E[:, 1], np.full(len(E), lam // 2, dtype=np.int64))
    return Qubo(n=n, row_ptr=rp, col_idx=col, vals=val, c=np.full(n, -1, dtype=np.int64),
                name=f"mis_d{d}_n{n}", meta=dict(edges=E, d=d, lam=lam))


def real_qubo(n: int, M: int, rep: int = 0, spread: int = 0, dense: bool = False) -> Qubo:
    """QUBO with float64 weights (Eq. 1 with real Q, c): M distinct random
    off-diagonal positions (i, j), i != j, each stored once (Q asymmetric),
    plus a diagonal; values N(0, 1) times 2^U{-spread..spread}, c likewise times
    10.  dense: the (n, n) array instead of CSR."""
    g = rng_for(8, rep, 0, n, M, spread)
    lin = g.choice(n * (n - 1), size=M, replace=False)
    i = lin // (n - 1)
    j = lin % (n - 1)
    j = j + (j >= i)                                  # skip the diagonal
    scale = lambda k: np.exp2(g.integers(-spread, spread + 1, size=k)) if spread else 1.0
    w = g.standard_normal(M) * scale(M)
    diag = g.standard_normal(n) * scale(n)
    c = 10.0 * g.standard_normal(n) * scale(n)
    ii = np.concatenate([i, np.arange(n)])
    jj = np.concatenate([j, np.arange(n)])
    ww = np.concatenate([w, diag])
    if dense:
        Q = np.zeros((n, n))
        Q[ii, jj] = ww
        return Qubo(n=n, Q=Q, c=c, name=f"real_dense_n{n}_m{M}_s{spread}")
    order = np.lexsort((jj, ii))
    ii, jj, ww = ii[order], jj[order], ww[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, ii + 1, 1)
    return Qubo(n=n, row_ptr=np.cumsum(row_ptr).astype(np.int32), col_idx=jj.astype(np.int32),
                vals=ww, c=c, name=f"real_csr_n{n}_m{M}_s{spread}")


@dataclass
class Kcut:
    n: int
    k: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    w: np.ndarray
    name: str = ""


def kcut_graph(n: int, M: int, k: int, rep: int = 0, signed: bool = True) -> Kcut:
    """Max-k-Cut instance on G(n, M): M distinct edges, weights +-1 with
    probability 1/2 (or all 1), symmetric CSR with both directions."""
    rng = rng_for(7, rep, 0, n, M, k)
    keys = np.zeros(0, dtype=np.int64)
    while len(keys) < M:  # distinct unordered pairs, drawn uniformly
        a = rng.integers(0, n, size=2 * (M - len(keys)) + 16)
        b = rng.integers(0, n, size=a.shape[0])
        ok = a != b
        new = np.minimum(a, b)[ok] * n + np.maximum(a, b)[ok]
        keys = np.concatenate([keys, new])
        _, first = np.unique(keys, return_index=True)
        keys = keys[np.sort(first)][:M]
    i, j = keys // n, keys % n
    w = np.where(rng.random(M) < 0.5, 1, -1) if signed else np.ones(M, dtype=np.int64)
    rp, col, val = _csr_from_upper(n, i, j, w.astype(np.int64))
    return Kcut(n=n, k=k, row_ptr=rp, col_idx=col, w=val, name=f"kcut{k}_n{n}_m{M}")


def qubo_c3(rep: int = 0, n: int = 10000) -> Qubo:
    """Dense QUBO, Q symmetric with entries U{-100..100}, c ~ U{-100..100}."""
    return random_dense_qubo(n, -100, 100, rng_for(3, rep, 0, n))


def batch_c4(rep: int = 0, k: int = 64, n_lo: int = 500, n_hi: int = 5000,
             rho_lo: float = 0.01, rho_hi: float = 0.10, wmax: int = 10):
    """k QUBOs of uneven size: n ~ U{n_lo..n_hi}, density rho ~ U[rho_lo, rho_hi];
    each pair i<j and each diagonal entry is present with probability rho and
    carries a weight U{-wmax..wmax}; c = 0.  Returned in CSR form."""
    g = rng_for(4, rep, 0)
    sizes = g.integers(n_lo, n_hi + 1, size=k)
    rhos = g.uniform(rho_lo, rho_hi, size=k)
    out = []
    for idx in range(k):
        gi = rng_for(4, rep, 0, idx)
        n = int(sizes[idx])
        rho = float(rhos[idx])
        npairs = n * (n - 1) // 2
        cnt = gi.binomial(npairs, rho)
        lin = np.sort(gi.choice(npairs, size=cnt, replace=False))
        i, j = _pairs_from_linear(n, lin)
        w = gi.integers(-wmax, wmax + 1, size=cnt).astype(np.int32)
        dmask = gi.random(n) < rho
        diag = np.where(dmask, gi.integers(-wmax, wmax + 1, size=n), 0).astype(np.int32)
        keep = w != 0
        row_ptr, col_idx, vals = _csr_from_upper(n, i[keep], j[keep], w[keep], diag)
        out.append(Qubo(n=n, row_ptr=row_ptr, col_idx=col_idx, vals=vals, c=None,
                        name=f"batch{idx}_n{n}_rho{rho:.3f}", meta={"rho": rho}))
    return out


def random_maxsat(n: int, m: int, k: int, wlo: int, whi: int,
                  rng: np.random.Generator) -> MaxSat:
    """Random weighted k-SAT: k distinct variables per clause drawn uniformly,
    each negated with probability 1/2, weights U{wlo..whi}."""
    v = rng.integers(0, n, size=(m, k))
    while True:
        srt = np.sort(v, axis=1)
        bad = np.any(srt[:, 1:] == srt[:, :-1], axis=1)
        if not bad.any():
            break
        v[bad] = rng.integers(0, n, size=(int(bad.sum()), k))
    neg = rng.random((m, k)) < 0.5
    lits = np.where(neg, -(v + 1), v + 1).astype(np.int32)
    w = rng.integers(wlo, whi + 1, size=m).astype(np.int32)
    return MaxSat(n=n, lits=lits, w=w, name=f"wsat{k}_n{n}_m{m}")


def maxsat_c5(rep: int = 0, n: int = 20000, m: int = 84000) -> MaxSat:
    """Weighted random 3-SAT at clause ratio 4.2, weights U{1..10}."""
    return random_maxsat(n, m, 3, 1, 10, rng_for(5, rep, 0, n, m))
