"""Plain FP64 CPU oracle for the PDBO hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute this package: only ``tests/``, the smoke check in
``__graft_entry__.py`` and the ``cpu_baseline`` leg of ``bench.py`` use it.  It
shares no code with the HIP library (no kernels, headers, helpers, tables or
pre/post-processing); the only common inputs come from the seeded generators in
``workloads/``.

Modules
-------
``qubo``       exact QUBO objective, canonical multilinear extension and its
               gradient (Eq. 1, Def. 2.2, Prop. 2.2)
``maxsat``     weighted Max-k-SAT objective, multilinear extension and gradient
               (Sec. 5.1 Max-k-SAT)
``binarity``   the constraint functions g and their derivatives (Sec. 3.1)
``gda``        Algorithm 1 (PDBO) over B independent restarts, keeping the best
               rounded solution (Sec. 5.2 Model Settings)
``enumerate``  brute force over {0,1}^n and the multilinear extension by its
               definition (Def. 2.2), for small n
``bounds``     the dual lower bound of Prop. 4.1 and the telescoping identity in
               the proof of Thm. 4.2

Every function works in float64 (objectives of integer instances in int64).
Parity is pinned for every function by the CPU tests under ``tests/`` (see
``test_oracle_*.py``); none is "parity unpinned".
"""
from . import binarity, bounds, enumerate, gda, maxsat, qubo  # noqa: F401
