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
               gradient (Eq. 1, Def. 2.2, Prop. 2.4)
``maxsat``     weighted Max-k-SAT objective, multilinear extension and gradient
               (Sec. 4.1 Max-k-SAT)
``binarity``   the constraint functions g and their derivatives (Sec. 3.1)
``gda``        Algorithm 1 (PDBO) over B independent restarts, keeping the best
               rounded solution (Sec. 4.2 Model Settings)
``enumerate``  brute force over {0,1}^n and the multilinear extension by its
               definition (Def. 2.2), for small n
``bounds``     the dual lower bound of Prop. 3.3 and the telescoping identity in
               the proof of Thm. 3.7
``philox``     Philox4x32-10 and the starting points the library draws when the
               caller passes none (App. C: x^0 uniform on [0,1]^n)
``dual``       the dual certificate of App. D: a lower bound on min F from the
               Lagrangian at a fixed y, and projected descent to reach it
``kcut``       Max-k-Cut through the softmax reparametrisation (App. B): exact
               objective, Lagrangian, its gradient in the logits, GDA steps
``mis``        maximum independent set as the penalised QUBO of App. D, set
               size of feasible vectors, independence number by enumeration

Every function works in float64 (objectives of integer instances in int64).
Each function is pinned by a CPU test under ``tests/`` against something other
than itself: plain-loop and brute-force definitions, the paper's worked
examples and identities, hand-worked golden values under ``tests/golden/``,
closed forms, exact finite or complex-step differences, library routines
(numpy.polynomial) and the published known-answer vectors of Philox4x32-10.
Which test pins which function is listed in the design notes; no function here
is "parity unpinned".
"""
from . import binarity, bounds, dual, enumerate, gda, kcut, maxsat, mis, philox, qubo  # noqa: F401
