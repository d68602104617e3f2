"""Pins of the oracle's Alg. 1 and constraint functions (CPU only)."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import bounds as ob
from oracle import enumerate as en
from oracle import gda
from oracle import maxsat as om
from oracle import qubo as oq
from oracle.binarity import Entropy, Polynomial, Quadratic

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
DELTA = W.DELTA


@pytest.mark.parametrize("g", [Quadratic(), Entropy(), Polynomial(2)])
def test_constraint_function_conditions(g):
    # Sec. 3.1: convex, g(0)=g(1)=0, g'(x)=0 only at 1/2, symmetric, g<0 inside
    x = np.linspace(0.0, 1.0, 2049)
    v = g.value(x)
    assert v[0] == 0.0 and v[-1] == 0.0
    assert np.all(v[1:-1] < 0)
    assert np.allclose(v, g.value(1.0 - x), atol=1e-15)
    assert np.all(np.diff(v, 2) >= -1e-15)
    d = g.deriv(x[1:-1])
    assert g.deriv(np.array(0.5)) == 0.0
    assert np.all(d[x[1:-1] < 0.5] < 0) and np.all(d[x[1:-1] > 0.5] > 0)


def test_entropy_closed_forms_and_derivative():
    g = Entropy()
    assert g.value(np.array(0.5)) == pytest.approx(-math.log(2.0), abs=1e-16)
    assert g.deriv(np.array(0.25)) == pytest.approx(math.log(1.0 / 3.0), abs=1e-15)
    x = np.linspace(0.05, 0.95, 19)
    h = 1e-6
    fd = (g.value(x + h) - g.value(x - h)) / (2 * h)
    assert np.allclose(fd, g.deriv(x), atol=1e-8)
    # the clip reading: derivative at the end points equals the one at eps
    assert g.deriv(np.array(0.0)) == pytest.approx(math.log(2.0 ** -20 / (1 - 2.0 ** -20)))


def test_quadratic_derivative_central_difference_exact():
    x = np.arange(0, 257) / 256.0
    h = 2.0 ** -12
    assert np.array_equal((Quadratic.value(x + h) - Quadratic.value(x - h)) / (2 * h), Quadratic.deriv(x))


@pytest.mark.parametrize("d", [1, 2, 3, 5])
def test_polynomial_derivative_complex_step_and_expanded(d):
    """g(x) = (2x-1)^(2d) - 1 (Sec. 3.1): the derivative agrees with the complex
    step Im g(x + ih)/h, which has no cancellation and is exact to rounding for
    a polynomial, and with numpy.polynomial's derivative of the expanded
    coefficients; d = 1 is four times the quadratic g."""
    from numpy.polynomial import polynomial as npp
    g = Polynomial(d)
    x = np.linspace(0.0, 1.0, 129)
    h = 1e-30
    cs = np.imag(g.value(x + 1j * h)) / h
    assert np.allclose(g.deriv(x), cs, rtol=1e-13, atol=1e-13)
    coef = npp.polysub(npp.polypow([-1.0, 2.0], 2 * d), [1.0])
    assert np.allclose(g.value(x), npp.polyval(x, coef), rtol=0, atol=1e-12)
    assert np.allclose(g.deriv(x), npp.polyval(x, npp.polyder(coef)), rtol=1e-12, atol=1e-12)
    if d == 1:
        assert np.array_equal(g.deriv(x), 4.0 * Quadratic.deriv(x))


def test_prop33_lower_bound_golden():
    """Prop. 3.3 bound b on hand-worked values (tests/golden/prop33_lower_bound.json)."""
    with open(os.path.join(GOLDEN, "prop33_lower_bound.json")) as fh:
        gold = json.load(fh)
    kinds = {"quad": Quadratic(), "entropy": Entropy(), "poly2": Polynomial(2)}
    for case in gold["cases"]:
        b = ob.prop33_lower_bound(case["theta"], case["alpha"], case["beta"], case["delta"],
                                  kinds[case["g"]])
        assert b == pytest.approx(case["b"], rel=1e-12, abs=1e-9), case["name"]


def _one_var(c, s):
    return oq.QuboProblem(W.Qubo(n=1, Q=np.zeros((1, 1), np.int32), c=None), s), c


def test_alg1_worked_examples():
    with open(os.path.join(GOLDEN, "alg1_worked_examples.json")) as fh:
        gold = json.load(fh)
    assert gold["delta"] == DELTA
    for case in gold["cases"]:
        G = np.array([[case["c"] / case["s"]]])
        X = np.array([[case["x"]]])
        Y = np.array([[case["y"]]])
        Xn, Yn, _ = gda.alg1_update(X, Y, G, case["alpha"], case["beta"], DELTA, Quadratic())
        assert Xn[0, 0] == pytest.approx(case["x_next"], abs=1e-15), case["name"]
        assert Yn[0, 0] == pytest.approx(case["y_next"], abs=1e-12), case["name"]


def test_maxcut_example_step_at_half():
    # Sec. 3.2.1 example: at x = 1/2 the gradient vanishes; with y <= 0 every
    # coordinate is perturbed to 1/2 - delta, with y > 0 it stays at 1/2
    q = W.maxcut_c2(rep=2, n=50, M=120)
    P = oq.QuboProblem(q, 1.0)
    X = np.full((2, q.n), 0.5)
    Y = np.stack([np.full(q.n, -0.5), np.full(q.n, 0.5)])
    p = dict(alpha=0.025, beta=0.025, delta=DELTA, g="quad")
    Xn, Yn, _, _ = gda.step(P, X, Y, p)
    assert np.all(Xn[0] == 0.5 - DELTA)
    assert np.all(Xn[1] == 0.5)
    assert np.all(Yn == Y - 0.025 * 0.25)


def test_zero_objective_scalar_recurrence():
    # Q = 0, c = 0: with d = x - 1/2, Alg. 1 reduces to
    #   d+ = clip(d (1 - 2 alpha y), -1/2, 1/2)   (or +-delta when perturbed)
    #   y+ = y + beta (d^2 - 1/4)
    n, B = 5, 3
    q = W.Qubo(n=n, Q=np.zeros((n, n), np.int32), c=None)
    P = oq.QuboProblem(q, 1.0)
    g = np.random.default_rng(0)
    X = g.random((B, n))
    Y = np.stack([np.full(n, 6.0), np.full(n, 0.3), np.full(n, -0.2)])
    alpha, beta = 0.025, 0.025
    p = dict(alpha=alpha, beta=beta, delta=DELTA, g="quad")
    d = X - 0.5
    y = Y.copy()
    for _ in range(400):
        X, Y, _, _ = gda.step(P, X, Y, p)
        d_new = np.empty_like(d)
        for b in range(B):
            for i in range(n):
                grad = y[b, i] * 2.0 * d[b, i]
                if abs(d[b, i]) <= DELTA and abs(grad) <= 2 * DELTA and y[b, i] <= 0:
                    d_new[b, i] = -DELTA if d[b, i] <= 0 else DELTA
                else:
                    d_new[b, i] = min(max(d[b, i] * (1.0 - 2.0 * alpha * y[b, i]), -0.5), 0.5)
        y = y + beta * (d * d - 0.25)
        d = d_new
        assert np.allclose(X - 0.5, d, atol=1e-14, rtol=0)
        assert np.allclose(Y, y, atol=1e-13, rtol=0)


def _invariants(problem, x0, p, T, Fstar=None):
    g = Quadratic() if p["g"] == "quad" else Entropy()
    res = gda.run(problem, x0, p, T=T, record=True)
    # box (Alg. 1 projection) after the run
    assert np.all((res.X >= 0) & (res.X <= 1))
    # y non-increasing: each increment beta*g(x) <= 0 (Sec. 3.2.1)
    Y0 = np.full_like(x0, p["y0"])
    assert np.all(res.Y <= Y0)
    # telescoping identity (proof of Thm. 3.7)
    gap = ob.telescoping_gap(Y0, res.Y, res.sum_g, p["beta"])
    scale = np.sum(np.abs(Y0 - res.Y), axis=1) + 1.0
    assert np.all(np.abs(gap) <= 1e-12 * scale)
    # Prop. 3.3 lower bound with an upper bound on Theta
    b = ob.prop33_lower_bound(problem.theta_upper(), p["alpha"], p["beta"], p["delta"], g)
    assert min(res.y_min) >= b and res.Y.min() >= b
    if Fstar is not None:
        # Lemma 2.3: f(x) >= min F on the box (f is the multilinear extension)
        assert min(float(np.min(v)) for v in res.f_values) * problem.s >= Fstar - 1e-9
        assert res.inc.F >= Fstar
    # incumbent is consistent with its own vector
    assert problem.objective(res.inc.x[None])[0] == res.inc.F
    return res


def test_invariants_qubo_twin_and_hits_optimum():
    q = W.qubo_c1_twin(0)
    P = oq.QuboProblem(q, 1.0)
    Fstar, _ = en.brute_force(lambda X: oq.objective(q, X), q.n)
    x0 = W.x0_uniform(1, 0, 16, q.n, 18)
    p = W.gda_params("maxcut", B=16, T=1000)
    res = _invariants(P, x0, p, 1000, Fstar)
    assert res.inc.F == Fstar


def test_invariants_dense_weighted():
    q = W.random_dense_qubo(16, -100, 100, W.rng_for(3, 0, 0, 16))
    s = W.qubo_scale(q)
    P = oq.QuboProblem(q, s)
    Fstar, _ = en.brute_force(lambda X: oq.objective(q, X), q.n)
    x0 = W.x0_uniform(3, 0, 32, q.n, 16)
    p = W.gda_params("qubo", B=32, T=600, scale=s)
    res = _invariants(P, x0, p, 600, Fstar)
    assert res.inc.F >= Fstar


def test_invariants_maxsat_entropy():
    inst = W.random_maxsat(14, 60, 3, 1, 10, W.rng_for(5, 0, 0, 14, 60))
    s = W.maxsat_scale(inst)
    P = om.MaxSatProblem(inst, s)
    Fstar, _ = en.brute_force(lambda X: om.objective(inst, X), inst.n)
    x0 = W.x0_uniform(5, 0, 8, inst.n, 14)
    p = W.gda_params("maxsat", B=8, T=500, scale=s)
    res = _invariants(P, x0, p, 500, Fstar)
    assert res.inc.F >= Fstar


def test_incumbent_tie_rules():
    inc = gda.Incumbent()
    Xr = np.eye(3, dtype=bool)
    assert inc.offer(np.array([5, 3, 3]), 1, Xr) and (inc.F, inc.t, inc.b) == (3, 1, 1)
    assert not inc.offer(np.array([3, 9, 9]), 2, Xr) and (inc.t, inc.b) == (1, 1)
    assert inc.offer(np.array([9, 9, 2]), 3, Xr) and (inc.F, inc.t, inc.b) == (2, 3, 2)


def test_binarity_of_long_run():
    # Cor. 3.5 / Def. 3.6: -sum g(x) shrinks towards 0 as y decreases
    q = W.qubo_c1(0, n=60)
    P = oq.QuboProblem(q, 1.0)
    x0 = W.x0_uniform(1, 0, 4, q.n, 60)
    p = W.gda_params("maxcut", B=4, T=3000)
    gaps = [ob.binarity_gap(gda.run(P, x0, p, T=T).X, Quadratic()) for T in (300, 1000, 3000)]
    assert np.all(gaps[1] < gaps[0]) and np.all(gaps[2] < gaps[1])
    assert np.all(gaps[2] < 1e-3)
