"""MIS oracle (App. D) against textbook independence numbers and the QUBO
objective of the generated CSR instance; the penalised minimum equals the
independence number for lam = 4."""
import itertools

import numpy as np

import workloads as W
from oracle import enumerate as en
from oracle import mis
from oracle import qubo as oq


def _cycle(n):
    return np.array([(i, (i + 1) % n) if i < (i + 1) % n else ((i + 1) % n, i) for i in range(n)])


PETERSEN = np.array([(0, 1), (1, 2), (2, 3), (3, 4), (0, 4), (0, 5), (1, 6), (2, 7), (3, 8),
                     (4, 9), (5, 7), (7, 9), (6, 9), (6, 8), (5, 8)])


def test_textbook_independence_numbers():
    for n in (5, 6, 7, 10):
        assert mis.independence_number(n, _cycle(n)) == n // 2
    assert mis.independence_number(10, PETERSEN) == 4
    K5 = np.array(list(itertools.combinations(range(5), 2)))
    assert mis.independence_number(5, K5) == 1


def test_feasible_vectors_objective_is_minus_size():
    E = PETERSEN
    X = en.all_binary(10)
    size, inside = mis.set_size(E, X)
    F = mis.objective(E, X)
    feas = inside == 0
    assert np.array_equal(-F[feas], size[feas])
    assert np.all(F[~feas] > -size[~feas])  # every infeasible vector is penalised


def test_penalised_minimum_is_independence_number_and_matches_qubo():
    """On generated d-regular graphs the CSR QUBO's exact objective equals the
    MIS objective on every vector, and -min F = alpha(G) (lam = 4 > 1: removing
    a vertex with a neighbour inside S lowers F)."""
    for n, d, rep in ((12, 3, 0), (14, 3, 1), (16, 4, 2), (10, 3, 3)):
        q = W.mis_qubo(n, d, rep)
        E = q.meta["edges"]
        X = en.all_binary(n)
        Fq = oq.objective(q, X)
        assert np.array_equal(Fq, mis.objective(E, X))
        Fstar, _ = en.brute_force(lambda Xb: oq.objective(q, Xb), n)
        assert -Fstar == mis.independence_number(n, E)


def test_generator_is_simple_and_regular():
    for n, d in ((20, 3), (500, 7), (2000, 100)):
        E = W.random_regular_graph(n, d, np.random.default_rng(n + d))
        assert np.all(np.bincount(E.ravel(), minlength=n) == d)
        assert np.all(E[:, 0] < E[:, 1])
        assert len(np.unique(E[:, 0] * n + E[:, 1])) == len(E)
