"""Oracle pins of the variants of Alg. 1: the single-constraint dual (PDBO-s,
Sec. 4.5) and the polynomial g of Sec. 3.1 as the parameters name it."""
import numpy as np

import workloads as W
from oracle import gda
from oracle import qubo as oq
from oracle.binarity import Polynomial


def _zero_problem(n):
    Q = np.zeros((n, n), dtype=np.int32)
    return oq.QuboProblem(W.Qubo(n=n, Q=Q, c=None), 1.0)


def test_scalar_dual_one_step_by_hand():
    """f = 0, quadratic g: dL/dx_i = y (2 x_i - 1), so with y > 0 and no clipping
    d_i = x_i - 1/2 becomes d_i (1 - 2 alpha y), and the single dual variable
    gains beta sum_i (d_i^2 - 1/4).  x0 = (1/4, 3/4, 5/8), y = 2, alpha = 1/10,
    beta = 1/20: d = (-1/4, 1/4, 1/8) -> 0.6 d, x+ = (0.35, 0.65, 0.575);
    y+ = 2 + (1/20)(1/16 + 1/16 + 1/64 - 3/4) = 1.96953125."""
    prob = _zero_problem(3)
    p = dict(alpha=0.1, beta=0.05, delta=2.0 ** -7, y0=2.0, g="quad", dual="scalar")
    X = np.array([[0.25, 0.75, 0.625]])
    Xn, Yn, _, _ = gda.step(prob, X, np.array([[2.0]]), p)
    assert np.allclose(Xn, [[0.35, 0.65, 0.575]], rtol=0, atol=1e-15)
    assert Yn.shape == (1, 1) and abs(Yn[0, 0] - 1.96953125) < 1e-15


def test_scalar_dual_equals_vector_dual_on_identical_coordinates():
    """With f = 0 and every coordinate of a restart equal, the n per-coordinate
    duals stay equal, and the vector dual with step n*beta moves exactly like
    the single dual with step beta (its ascent is beta * n * g(x)).  The run
    crosses y <= 0, so the perturbation branch is reached."""
    n, B, T = 6, 4, 60
    prob = _zero_problem(n)
    x0 = np.repeat(np.array([[0.1], [0.45], [0.5], [0.93]]), n, axis=1)
    ps = dict(alpha=0.2, beta=0.02, delta=2.0 ** -7, y0=0.3, g="quad", dual="scalar")
    pv = dict(ps, beta=0.02 * n, dual="vector")
    rs = gda.run(prob, x0, ps, T=T, record=True)
    rv = gda.run(prob, x0, pv, T=T, record=True)
    assert np.allclose(rs.X, rv.X, rtol=0, atol=1e-12)
    assert np.allclose(np.broadcast_to(rs.Y, rv.Y.shape), rv.Y, rtol=0, atol=1e-12)
    assert min(rv.y_min) <= 0.0


def test_constraint_fn_degree():
    g = gda.constraint_fn(dict(g="poly", g_degree=3))
    assert isinstance(g, Polynomial) and g.d == 3
    x = np.array([0.0, 0.25, 0.5, 1.0])
    assert np.array_equal(g.value(x), (2 * x - 1) ** 6 - 1)
    assert gda.constraint_fn(dict(g="quad")).name == "quad"
