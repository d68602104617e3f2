"""Dual certificate oracle (App. D, Dual Certificate) against a closed form
(separable case), brute force (weak duality at every box point when the
Lagrangian is convex) and the descent's convergence (gap to zero)."""
import numpy as np

import workloads as W
from oracle import dual
from oracle import enumerate as en
from oracle import qubo as oq


def test_separable_closed_form():
    """Q diagonal (A = 0): L = c'^T x / s + ybar sum (x_i^2 - x_i) separates;
    coordinate i is minimised at clip(1/2 - c'_i / (2 s ybar), 0, 1).  The
    descent reaches it, the bound there equals s min L, and min F is the sum
    of min(0, c'_i)."""
    n = 7
    Q = np.diag(np.array([3, -5, 0, 12, -1, 7, -9], dtype=np.int32))
    c = np.array([-4, 2, 1, -20, 0, 3, 8], dtype=np.int64)
    q = W.Qubo(n=n, Q=Q, c=c)
    s, ybar = 2.0, 3.0
    prob = oq.QuboProblem(q, s)
    cp = c + np.diag(Q)
    xs = np.clip(0.5 - cp / (2 * s * ybar), 0, 1)
    Lmin = float(np.sum(cp * xs) / s + ybar * np.sum(xs * xs - xs))
    x = dual.projected_descent(prob, ybar, alpha=0.05, iters=2000)
    assert np.allclose(x, xs, atol=1e-12)
    lb, val, gap = dual.certificate(prob, x, ybar)
    assert abs(val - s * Lmin) < 1e-9 and abs(gap) < 1e-9 and abs(lb - s * Lmin) < 1e-9
    assert lb <= np.sum(np.minimum(0, cp)) + 1e-12   # min F over {0,1}^n


def test_weak_duality_brute_force_and_tightness():
    """Random dense QUBOs (n <= 14) with ybar at or above the convexity
    threshold -lambda_min(A)/(2 s): the bound at ANY box point (random points
    and the descent's end point) is <= min F, it never exceeds s L(x), and at
    the descent's end point the Frank-Wolfe gap vanishes."""
    rng = np.random.default_rng(4)
    for n in (6, 10, 14):
        q = W.random_dense_qubo(n, -20, 20, rng)
        s = 3.0
        prob = oq.QuboProblem(q, s)
        A, _ = oq.canonicalize(q)
        thr = -np.linalg.eigvalsh(A / s).min() / 2
        Fstar, _ = en.brute_force(lambda Xb: oq.objective(q, Xb), n)
        for ybar in (thr, 1.5 * thr + 0.1):
            assert np.linalg.eigvalsh(A / s + 2 * ybar * np.eye(n)).min() >= -1e-9
            for x in list(rng.random((5, n))) + [np.zeros(n), np.ones(n)]:
                lb, val, gap = dual.certificate(prob, x, ybar)
                assert lb <= Fstar + 1e-9 and gap >= -1e-12 and lb <= val + 1e-12
            L = np.abs(np.linalg.eigvalsh(A / s + 2 * ybar * np.eye(n))).max()
            x = dual.projected_descent(prob, ybar, alpha=1.0 / L, iters=20000)
            lb, val, gap = dual.certificate(prob, x, ybar)
            assert lb <= Fstar + 1e-9 and gap < 1e-6 * max(1.0, abs(val))


def test_bound_fails_below_convexity_as_expected():
    """Below the threshold the tangent plane need not lie below L: some box
    point then gives a value above min F (the certificate needs convexity,
    which the caller provides)."""
    rng = np.random.default_rng(5)
    q = W.random_dense_qubo(10, -20, 20, rng)
    prob = oq.QuboProblem(q, 1.0)
    Fstar, xstar = en.brute_force(lambda Xb: oq.objective(q, Xb), 10)
    # at a binary minimiser with ybar tiny the bound is F* plus a nonnegative
    # linear term; away from it, some point overshoots
    over = [dual.certificate(prob, x, 1e-3)[0] > Fstar + 1e-9 for x in rng.random((200, 10))]
    assert any(over)
