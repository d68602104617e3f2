"""Pins of the oracle's weighted Max-k-SAT parts (CPU only)."""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import enumerate as en
from oracle import maxsat as om


def _loop_unsat(lits, w, x):
    """Weighted unsatisfied count by plain loops over clauses and literals."""
    tot = 0
    for j, clause in enumerate(lits):
        sat = False
        for lit in clause:
            v = abs(int(lit)) - 1
            val = bool(x[v]) if lit > 0 else not bool(x[v])
            sat = sat or val
        if not sat:
            tot += int(w[j])
    return tot


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_clause_product_is_unsat_indicator(k):
    # Sec. 4.1 Max-k-SAT: prod_l p(x_l) = 1 iff the clause is unsatisfied
    for signs in itertools.product((1, -1), repeat=k):
        lits = np.array([[s * (i + 1) for i, s in enumerate(signs)]], dtype=np.int32)
        inst = W.MaxSat(n=k, lits=lits, w=np.array([1], np.int32))
        for x in itertools.product((0, 1), repeat=k):
            f = om.f_multilinear(inst, np.array([x], dtype=float))[0]
            assert f == _loop_unsat(lits, [1], x)


def test_objective_matches_loops():
    inst = W.random_maxsat(12, 50, 3, 1, 10, np.random.default_rng(4))
    X = np.random.default_rng(5).integers(0, 2, size=(30, inst.n))
    F = om.objective(inst, X)
    for b in range(30):
        assert F[b] == _loop_unsat(inst.lits, inst.w, X[b])


def test_multilinear_equals_definition_bit_exact():
    inst = W.random_maxsat(9, 30, 3, 1, 10, np.random.default_rng(6))
    F_all = om.objective(inst, en.all_binary(inst.n))
    g = np.random.default_rng(7)
    for _ in range(8):
        x = g.integers(0, 9, size=inst.n) / 8.0
        assert om.f_multilinear(inst, x[None])[0] == en.multilinear_by_definition(F_all, x)


def test_gradient_forward_difference_exact():
    inst = W.random_maxsat(10, 40, 3, 1, 10, np.random.default_rng(8))
    g = np.random.default_rng(9)
    h = 2.0 ** -10
    x = g.integers(0, 9, size=inst.n) / 8.0
    for s in (1.0, 2.0):
        G = om.grad_f(inst, x[None], s)[0]
        for i in range(inst.n):
            e = np.zeros(inst.n)
            e[i] = h
            fd = (om.f_multilinear(inst, (x + e)[None])[0] - om.f_multilinear(inst, x[None])[0]) / h / s
            assert fd == G[i]


def test_gradient_batched_rows_independent():
    inst = W.random_maxsat(15, 60, 3, 1, 10, np.random.default_rng(10))
    X = np.random.default_rng(11).random((5, inst.n))
    G = om.grad_f(inst, X, 3.0)
    for b in range(5):
        assert np.array_equal(G[b], om.grad_f(inst, X[b:b + 1], 3.0)[0])


def test_brute_force_matches_itertools():
    inst = W.random_maxsat(10, 45, 3, 1, 10, np.random.default_rng(12))
    Fstar, xs = en.brute_force(lambda X: om.objective(inst, X), inst.n, chunk=64)
    best = min(_loop_unsat(inst.lits, inst.w, x) for x in itertools.product((0, 1), repeat=inst.n))
    assert Fstar == best == _loop_unsat(inst.lits, inst.w, xs)


def test_generator_shape_c5_small():
    inst = W.random_maxsat(50, 210, 3, 1, 10, W.rng_for(5, 0, 0, 50, 210))
    var, neg = om.split_literals(inst.lits)
    assert inst.lits.shape == (210, 3)
    assert np.all(np.sort(var, axis=1)[:, 1:] != np.sort(var, axis=1)[:, :-1])
    assert inst.w.min() >= 1 and inst.w.max() <= 10
    assert 0.3 < neg.mean() < 0.7
