"""Max-k-Cut oracle (App. B) against Max-Cut for k = 2, brute force over all
assignments, the one-hot identity of the objective, and complex-step
derivatives of the Lagrangian through the softmax."""
import itertools

import numpy as np

import workloads as W
from oracle import enumerate as en
from oracle import kcut as ok
from oracle import qubo as oq


def test_k2_is_maxcut():
    g = W.kcut_graph(30, 90, 2, rep=1)
    G = ok.Graph(g)
    X = en.all_binary(12)
    g12 = W.kcut_graph(12, 30, 2, rep=2)
    G12 = ok.Graph(g12)
    # Max-Cut as a QUBO: Q = W (both directions), c = -W 1, F = -cut
    q = W.Qubo(n=12, row_ptr=g12.row_ptr, col_idx=g12.col_idx, vals=g12.w,
               c=-np.asarray(G12.W.sum(axis=1)).ravel().astype(np.int64))
    assert np.array_equal(ok.cut_weight(G12, X), -oq.objective(q, X))
    assert G.total == int(np.sum(g.w)) // 2


def test_brute_force_k3():
    g = W.kcut_graph(8, 16, 3, rep=3)
    G = ok.Graph(g)
    E = [(int(a), int(b), int(c)) for a, b, c in zip(G.ei, G.ej, G.ew)]
    best = None
    for cats in itertools.product(range(3), repeat=8):
        F = sum(w for a, b, w in E if cats[a] == cats[b])
        best = F if best is None else min(best, F)
        assert ok.objective(G, np.array(cats)[None])[0] == F
    allc = np.array(list(itertools.product(range(3), repeat=8)))
    assert ok.objective(G, allc).min() == best


def test_one_hot_identity():
    g = W.kcut_graph(40, 120, 4, rep=4)
    G = ok.Graph(g)
    cats = np.random.default_rng(0).integers(0, 4, size=(5, 40))
    X = np.eye(4)[cats]
    XW = np.stack([G.W @ X[b] for b in range(5)])
    assert np.array_equal(np.sum(X * XW, axis=(1, 2)), 2.0 * ok.objective(G, cats))


def test_grad_complex_step():
    """dL/dZ (softmax Jacobian applied to the X-gradient, with the y g term)
    equals the complex-step derivative of L, for both kinds of g."""
    g = W.kcut_graph(15, 40, 3, rep=5)
    G = ok.Graph(g)
    rng = np.random.default_rng(1)
    Z = rng.normal(size=(2, 15, 3))
    Y = rng.normal(size=(2, 15))
    s, h = 1.7, 1e-30
    for kind in ("quad", "entropy"):
        D = ok.grad_Z(G, Z, Y, s, kind)
        for b, i, c in [(0, 0, 0), (1, 7, 2), (0, 14, 1), (1, 3, 0)]:
            Zc = Z.astype(np.complex128)
            Zc[b, i, c] += 1j * h
            d = ok.lagrangian(G, Zc, Y, s, kind)[b].imag / h
            assert abs(d - D[b, i, c]) <= 1e-12 * max(1.0, abs(d)), (kind, b, i, c)
