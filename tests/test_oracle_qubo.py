"""Pins of the oracle's QUBO parts against definitions, identities and brute
force (CPU only).  Each test names the passage it pins."""
import itertools
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import enumerate as en
from oracle import qubo as oq
from oracle.binarity import Quadratic

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_qubo(n, seed, lo=-5, hi=5, asym=True, with_c=True):
    g = np.random.default_rng(seed)
    Q = g.integers(lo, hi + 1, size=(n, n)).astype(np.int32)
    if not asym:
        Q = np.triu(Q) + np.triu(Q, 1).T
    c = g.integers(lo, hi + 1, size=n).astype(np.int64) if with_c else None
    return W.Qubo(n=n, Q=Q, c=c)


def _loop_F(Q, c, x):
    """F(x) = sum_ij Q_ij x_i x_j + sum_i c_i x_i by plain Python loops (Eq. 1)."""
    n = len(x)
    tot = 0
    for i in range(n):
        for j in range(n):
            tot += int(Q[i][j]) * int(x[i]) * int(x[j])
        if c is not None:
            tot += int(c[i]) * int(x[i])
    return tot


def test_maxcut_edge_identity():
    # Sec. 4.1 Max-Cut: x_i + x_j - 2 x_i x_j equals 1 iff x_i != x_j on {0,1}^2
    for xi, xj in itertools.product((0, 1), repeat=2):
        assert xi + xj - 2 * xi * xj == int(xi != xj)


def test_objective_matches_loops():
    q = _rand_qubo(9, 1)
    g = np.random.default_rng(2)
    X = g.integers(0, 2, size=(20, 9))
    F = oq.objective(q, X)
    for b in range(20):
        assert F[b] == _loop_F(q.Q, q.c, X[b])


def test_objective_csr_equals_dense_and_minus_cut():
    q = W.maxcut_c2(rep=0, n=60, M=150)
    g = np.random.default_rng(3)
    X = g.integers(0, 2, size=(12, q.n))
    F_csr = oq.objective(q, X)
    qd = W.Qubo(n=q.n, Q=q.dense().astype(np.int32), c=q.c)
    F_dense = oq.objective(qd, X)
    assert np.array_equal(F_csr, F_dense)
    # cut(x) = sum over edges i<j of W_ij [x_i != x_j]; F = -cut (Sec. 4.1, Sec. 3.2.1 example)
    Wd = q.dense()
    for b in range(12):
        cut = 0
        for i in range(q.n):
            for j in range(i + 1, q.n):
                if Wd[i, j] != 0 and X[b, i] != X[b, j]:
                    cut += int(Wd[i, j])
        assert F_csr[b] == -cut


def test_objective_rejects_fractional():
    q = _rand_qubo(4, 0)
    with pytest.raises(ValueError):
        oq.objective(q, np.array([[0.5, 0, 1, 0]]))


def test_brute_force_matches_itertools():
    q = _rand_qubo(10, 5)
    Fstar, xstar = en.brute_force(lambda X: oq.objective(q, X), q.n, chunk=100)
    best = min(_loop_F(q.Q, q.c, x) for x in itertools.product((0, 1), repeat=q.n))
    assert Fstar == best
    assert _loop_F(q.Q, q.c, xstar) == best


def test_brute_force_gray_code_n18_twin():
    # independent incremental Gray-code enumeration of the n=18 instance
    q = W.qubo_c1_twin(0)
    Fstar, _ = en.brute_force(lambda X: oq.objective(q, X), q.n)
    Qd = q.Q.astype(np.int64)
    S = Qd + Qd.T
    x = np.zeros(q.n, dtype=np.int64)
    F = 0
    best = 0
    for k in range(1, 1 << q.n):
        i = (k & -k).bit_length() - 1          # bit flipped by the Gray code
        d = 1 - 2 * x[i]
        F += d * (int(S[i] @ x) - 2 * Qd[i, i] * x[i] + Qd[i, i])
        x[i] += d
        best = min(best, F)
    assert Fstar == best


def test_canonical_f_equals_definition_bit_exact():
    # Def. 2.2 enumeration vs the Prop. 2.4 closed form, at dyadic points k/8
    q = _rand_qubo(8, 7)
    F_all = oq.objective(q, en.all_binary(q.n))
    A, cp = oq.canonicalize(q)
    g = np.random.default_rng(8)
    for _ in range(10):
        x = g.integers(0, 9, size=q.n) / 8.0
        assert oq.f_multilinear(A, cp, x[None])[0] == en.multilinear_by_definition(F_all, x)


def test_f_is_extension():
    # Def. 2.1: f = F on {0,1}^n
    q = _rand_qubo(7, 11)
    A, cp = oq.canonicalize(q)
    Xb = en.all_binary(q.n)
    assert np.array_equal(oq.f_multilinear(A, cp, Xb), oq.objective(q, Xb).astype(np.float64))


def test_canonical_csr_equals_dense():
    q = W.batch_c4(rep=0, k=2, n_lo=30, n_hi=40, rho_lo=0.2, rho_hi=0.3)[0]
    A_s, cp_s = oq.canonicalize(q)
    A_d, cp_d = oq.canonicalize(W.Qubo(n=q.n, Q=q.dense(), c=q.c))
    assert np.array_equal(A_s.toarray(), A_d)
    assert np.array_equal(cp_s, cp_d)
    assert np.all(np.diag(A_d) == 0)


def test_gradient_forward_difference_exact():
    # f is affine in each coordinate (Sec. 2), so a forward difference with a
    # dyadic step is exact at dyadic points
    q = _rand_qubo(6, 13)
    A, cp = oq.canonicalize(q)
    g = np.random.default_rng(14)
    h = 2.0 ** -10
    for s in (1.0, 4.0):
        x = g.integers(0, 9, size=q.n) / 8.0
        G = oq.grad_f(A, cp, x[None], s)[0]
        for i in range(q.n):
            e = np.zeros(q.n)
            e[i] = h
            fd = (oq.f_multilinear(A, cp, (x + e)[None])[0] - oq.f_multilinear(A, cp, x[None])[0]) / h / s
            assert fd == G[i]


def test_maxcut_example_gradient_vanishes_at_half():
    # Sec. 3.2.1 Max-Cut example: f = x^T W x - 1^T W x, g = x^2 - x, x = 1/2 gives
    # grad_x L = 0 for every y
    q = W.maxcut_c2(rep=1, n=40, M=90)
    P = oq.QuboProblem(q, 1.0)
    x = np.full((1, q.n), 0.5)
    G = P.grad(x)
    for y in (-3.0, 0.0, 6.0):
        dL = G + y * Quadratic.deriv(x)
        assert np.all(dL == 0.0)


def test_scale_gives_convex_start():
    # Sec. 4.4: L(., y0) convex when the Hessian A/s + 2 y_bar I is PSD; the
    # scale recipe places the threshold at 2/3 of y_bar = 6
    for q in (W.qubo_c1(0), W.random_dense_qubo(300, -100, 100, W.rng_for(3, 0, 0, 300))):
        s = W.qubo_scale(q)
        A, _ = oq.canonicalize(q)
        lam = np.linalg.eigvalsh(A / s).min()
        assert lam + 2 * 6.0 >= 0
        if q.n == 300:
            assert abs(-lam / 2 - 4.0) < 0.05


def test_hyperparameter_table():
    with open(os.path.join(GOLDEN, "hyperparameters.json")) as fh:
        tab = json.load(fh)
    for k, v in W.PAPER_HYPER.items():
        for name in ("B", "y0", "alpha", "beta"):
            assert v[name] == tab[k][name]


def test_real_weight_objective_fsum():
    g = np.random.default_rng(21)
    Q = g.standard_normal((6, 6)) * 1e3
    c = g.standard_normal(6)
    x = np.array([1, 0, 1, 1, 0, 1])
    import math
    from fractions import Fraction
    S = [i for i in range(6) if x[i]]
    exact = sum(Fraction(Q[i, j]) for i in S for j in S) + sum(Fraction(c[i]) for i in S)
    assert oq.objective_fsum(Q, c, x) == float(exact)
    assert math.isfinite(oq.objective_fsum(Q, None, x))


def _real_instance(g, n, wide):
    """Dense float64 Q and c; wide: magnitudes spread over 2^-60 .. 2^40 with
    subnormal and cancelling entries."""
    Q = g.standard_normal((n, n))
    c = g.standard_normal(n)
    if wide:
        Q = Q * np.exp2(g.integers(-60, 41, size=(n, n)))
        c = c * np.exp2(g.integers(-60, 41, size=n))
        Q[0, 1], Q[1, 0] = 1e300, -1e300          # cancel when x_0 = x_1 = 1
        Q[2, 2] = 5e-324                          # smallest subnormal
        c[3] = -3.0 * 2.0 ** -1070
    return Q, c


@pytest.mark.parametrize("wide", [False, True])
def test_real_weight_objective_exact(wide):
    """objective_exact against Fraction sums of every selected term (the
    definition of Eq. 1 in exact rationals) and against math.fsum (a correctly
    rounded library sum); dense and CSR storage of the same Q agree."""
    import math
    from fractions import Fraction
    g = np.random.default_rng(5 + wide)
    n = 9
    Q, c = _real_instance(g, n, wide)
    X = g.integers(0, 2, size=(12, n)).astype(np.uint8)
    X[0] = 1
    X[1] = 0
    X[2, :4] = 1
    qd = W.Qubo(n=n, Q=Q, c=c)
    rp = np.arange(0, n * n + 1, n, dtype=np.int32)
    col = np.tile(np.arange(n, dtype=np.int32), n)
    qs = W.Qubo(n=n, row_ptr=rp, col_idx=col, vals=Q.ravel().copy(), c=c)
    Fd = oq.objective_exact(qd, X)
    Fs = oq.objective_exact(qs, X)
    for b in range(X.shape[0]):
        S = [i for i in range(n) if X[b, i]]
        exact = sum((Fraction(Q[i, j]) for i in S for j in S), Fraction(0)) + \
            sum((Fraction(c[i]) for i in S), Fraction(0))
        assert Fd[b] == exact and Fs[b] == exact
        assert float(Fd[b]) == oq.objective_fsum(Q, c, X[b]) == math.fsum(
            [Q[i, j] for i in S for j in S] + [c[i] for i in S])
    assert Fd[1] == 0


def test_real_weight_objective_exact_integers():
    """Integer-valued float64 weights give the int64 objective of the same
    integers."""
    g = np.random.default_rng(8)
    n = 30
    Qi = g.integers(-1000, 1001, size=(n, n)).astype(np.int32)
    ci = g.integers(-5000, 5001, size=n).astype(np.int64)
    X = g.integers(0, 2, size=(16, n)).astype(np.uint8)
    Fi = oq.objective(W.Qubo(n=n, Q=Qi, c=ci), X)
    Fr = oq.objective_exact(W.Qubo(n=n, Q=Qi.astype(np.float64), c=ci.astype(np.float64)), X)
    assert [int(v) for v in Fr] == Fi.tolist()
    assert all(v.denominator == 1 for v in Fr)


def test_real_weight_incumbent_exact_comparison():
    """Two restarts whose objectives round to the same float64 (1 + 2^-60 and
    1): the incumbent of Alg. 1's best of B takes the exactly smaller one, not
    the first index."""
    from oracle.gda import Incumbent
    Q = np.zeros((3, 3))
    c = np.array([1.0, 2.0 ** -60, 0.0])
    q = W.Qubo(n=3, Q=Q, c=c)
    X = np.array([[1, 1, 0], [1, 0, 1]], dtype=np.uint8)
    F = oq.objective_exact(q, X)
    assert float(F[0]) == float(F[1]) == 1.0 and F[1] < F[0]
    inc = Incumbent()
    assert inc.offer(F, 1, X) and inc.b == 1 and inc.F == 1


@pytest.mark.parametrize("even", [False, True])
def test_incremental_difference_identity(even):
    """The identity behind the incremental evaluation: for x' = x + d (d = +-1 on
    a set D of changed coordinates) and A = offdiag(Q + Q^T) = kappa Ahat,
    F(x') - F(x) = sum_{i in D} d_i (c'_i + kappa (Ahat x')_i)
                   - kappa sum_{i < j in D} d_i d_j Ahat_ij,
    checked against the objective computed from scratch (Eq. 1), with an
    asymmetric Q and a diagonal, and with all couplings even (kappa = 2)."""
    g = np.random.default_rng(11 + even)
    n = 40
    Q = g.integers(-9, 10, size=(n, n)).astype(np.int64)
    if even:
        Q = 2 * Q
        np.fill_diagonal(Q, g.integers(-9, 10, n))
    q = W.Qubo(n=n, Q=Q, c=g.integers(-20, 21, n).astype(np.int64))
    A, cp = oq.canonicalize(q)
    kappa = 2 if np.all(A.astype(np.int64) % 2 == 0) else 1
    assert kappa == (2 if even else 1)
    Ah = (A / kappa).astype(np.int64)
    for trial in range(30):
        x = (g.random(n) < 0.5).astype(np.int64)
        D = g.choice(n, size=int(g.integers(1, 9)), replace=False)
        xn = x.copy()
        xn[D] = 1 - xn[D]
        d = xn - x
        Ax = Ah @ xn
        lin = sum(int(d[i]) * (int(cp[i]) + kappa * int(Ax[i])) for i in D)
        quad = sum(int(d[i]) * int(d[j]) * int(Ah[i, j]) for i in D for j in D if i < j)
        F = oq.objective(q, np.stack([x, xn]).astype(np.uint8))
        assert F[1] - F[0] == lin - kappa * quad
