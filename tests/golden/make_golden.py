"""Writes the stored expected values under tests/golden/ by calling only the
oracle (brute force over {0,1}^n) on the seeded generators.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import enumerate as en  # noqa: E402
from oracle import qubo as oq  # noqa: E402


def main():
    out = {"_source": "min over {0,1}^18 of x^T Q x (Q from the n=18 G(n,0.05) +-1 generator, "
                      "literal QUBO with c=0) and of the Max-Cut form (c = -W 1) on the same graph; "
                      "brute force by oracle/enumerate.py",
           "reps": {}}
    for rep in range(10):
        q = W.qubo_c1_twin(rep)
        F_q, _ = en.brute_force(lambda X: oq.objective(q, X), q.n)
        qc = W.Qubo(n=q.n, Q=q.Q, c=-q.Q.sum(axis=1).astype("int64"))
        F_c, _ = en.brute_force(lambda X: oq.objective(qc, X), q.n)
        out["reps"][str(rep)] = {"qubo_Fstar": int(F_q), "maxcut_Fstar": int(F_c)}
    dense = {}
    for rep in range(3):
        q = W.random_dense_qubo(20, -100, 100, W.rng_for(3, rep, 0, 20))
        F, _ = en.brute_force(lambda X: oq.objective(q, X), q.n)
        dense[str(rep)] = int(F)
    out["dense_u100_n20"] = dense
    with open(os.path.join(HERE, "c1_twin_optima.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
