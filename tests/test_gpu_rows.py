"""The row-parallel CSR path (one launch per iteration over all rows,
node-major iterates; tile = PDBO_CSR_ROWS) against the oracle: gradient,
iterations from the GPU's own state with exact objectives at every step,
graph replay and split calls bit for bit, and the MIS workload of App. D
(d-regular graphs, lam = 4) up to n = 5*10^4, d = 100."""
import numpy as np
import pytest

import workloads as W
from gpu_util import amb_limit, lockstep_compare, normwise, require_gpu, say
from oracle import mis
from oracle import qubo as oq

pytestmark = pytest.mark.gpu
ROWS = 2

CASES = {
    # (instance, B): B = 10 (paper's MIS setting, 6 lane groups per wave),
    # 70 (a full and a ragged slice of 64), 1, 256
    "mis_d3_n2000_B10": (lambda: W.mis_qubo(2000, 3, 5), 10),
    "mis_d100_n3000_B70": (lambda: W.mis_qubo(3000, 100, 6), 70),
    "maxcut_n2000_B256": (lambda: W.maxcut_c2(0), 256),
    "mis_d7_n40001_B1": (lambda: W.mis_qubo(40000, 7, 7), 1),
}


_SCALE = {}


def _ctx(P, q, B, **over):
    # the scale is computed once per instance: ARPACK over threaded BLAS can
    # differ in its last bits from call to call, and runs compared bit for bit
    # must share every parameter
    if id(q) not in _SCALE:
        _SCALE[id(q)] = (q, W.qubo_scale(q))
    p = W.gda_params("qubo", B=B, T=1, scale=_SCALE[id(q)][1], tile=ROWS, **over)
    if q.name.startswith("mis"):
        p.update(alpha=0.02, beta=0.02, y0=5.0)  # tab:hyper_parameters, MIS column
    return P.qubo_gda_init(q, p, W.x0_uniform(6, 1, B, q.n)), p


@pytest.mark.parametrize("name", list(CASES))
def test_rows_gradient_and_steps(name):
    P = require_gpu()
    make, B = CASES[name]
    q = make()
    A, cp = oq.canonicalize(q)
    ctx, p = _ctx(P, q, B)
    s = p["scale"]
    say(f"[rows] {name} n={q.n} B={B}")
    X = np.random.default_rng(1).random((B, q.n)).astype(np.float32)
    G64 = oq.grad_f(A, cp, X.astype(np.float64), s)
    err = normwise(ctx.grad(X), G64)
    say(f"   gradient normwise error {err:.3e}")
    assert err <= 1e-5
    X, Y, _ = ctx.get_state()
    for step in range(1, 4):
        ctx.step(1)
        Xn, Yn, t = ctx.get_state()
        assert t == step
        X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
        G64 = oq.grad_f(A, cp, X64, s)
        gabs = 1e-5 * float(np.max(np.abs(G64))) + 1e-6
        dx, dy, namb, _, _ = lockstep_compare(X64, Y64, G64, Xn, Yn, p, gabs)
        say(f"   t={step}: max|dX|={dx:.3e} max|dY|={dy:.3e} excluded={namb}")
        assert dx <= p["alpha"] * gabs + 2e-6
        assert dy <= 2e-6 * (1 + np.max(np.abs(Y64)))
        assert namb <= amb_limit("fp32", X.size)
        assert np.array_equal(ctx.objectives(), oq.objective(q, Xn > 0.5)), step
        X, Y = Xn, Yn
    xr = np.random.default_rng(2).integers(0, 2, size=(B, q.n), dtype=np.uint8)
    assert np.array_equal(ctx.eval(xr), oq.objective(q, xr.astype(bool)))
    ctx.destroy()


def test_rows_graph_split_and_trace():
    """Graph replay (chunks of 8) and split step calls reproduce one eager
    call bit for bit; the incumbent is the oracle's rule over the objectives of
    every iteration; the trace is strictly improving."""
    P = require_gpu()
    q = W.mis_qubo(5000, 3, 8)
    B, T = 10, 60
    out = []
    for gc, parts in ((0, [T]), (8, [T]), (0, [7, 30, 23])):
        ctx, p = _ctx(P, q, B, graph_chunk=gc)
        for k in parts:
            ctx.step(k)
        r = ctx.result()
        X, Y, t = ctx.get_state()
        out.append((r, X, Y, ctx.trace()))
        assert t == T
        ctx.destroy()
    r0, X0, Y0, tr0 = out[0]
    for r, X, Y, tr in out[1:]:
        assert (r["best_obj"], r["best_iter"], r["best_restart"]) == \
            (r0["best_obj"], r0["best_iter"], r0["best_restart"])
        assert np.array_equal(X, X0) and np.array_equal(Y, Y0)
        assert np.array_equal(r["best_x"], r0["best_x"])
    assert r0["best_obj"] == oq.objective(q, r0["best_x"][None])[0]
    assert np.all(np.diff(tr0["F"]) < 0) and tr0["F"][-1] == r0["best_obj"]
    # the same run, objectives of every iteration replayed through the oracle's rule
    from oracle.gda import Incumbent
    ctx, p = _ctx(P, q, B)
    inc = Incumbent()
    for t in range(1, T + 1):
        ctx.step(1)
        X, _, _ = ctx.get_state()
        F = ctx.objectives()
        assert np.array_equal(F, oq.objective(q, X > 0.5))
        inc.offer(F, t, X > 0.5)
    r = ctx.result()
    assert (r["best_obj"], r["best_iter"], r["best_restart"]) == (inc.F, inc.t, inc.b)
    ctx.destroy()


@pytest.mark.parametrize("n,d", [(10000, 3), (10000, 100), (50000, 3), (50000, 100)])
def test_mis_workload(n, d):
    """The MIS configurations of App. D (B = 10, y0 = 5, alpha = beta = 0.02,
    lam = 4): every objective of the last iteration exact, one iteration in
    lockstep on sampled restarts, the incumbent re-evaluated, and the set size
    of the incumbent reported when it is independent."""
    P = require_gpu()
    q = W.mis_qubo(n, d, 0)
    B = 10
    ctx, p = _ctx(P, q, B)
    A, cp = oq.canonicalize(q)
    s = p["scale"]
    say(f"[mis] n={n} d={d} s={s:.3f}")
    ctx.step(200)
    X, Y, _ = ctx.get_state()
    assert np.array_equal(ctx.objectives(), oq.objective(q, X > 0.5))
    ctx.step(1)
    Xn, Yn, _ = ctx.get_state()
    G64 = oq.grad_f(A, cp, X.astype(np.float64), s)
    gabs = 1e-5 * float(np.max(np.abs(G64))) + 1e-6
    dx, dy, namb, _, _ = lockstep_compare(X.astype(np.float64), Y.astype(np.float64), G64, Xn, Yn,
                                          p, gabs)
    say(f"   lockstep max|dX|={dx:.3e} max|dY|={dy:.3e} excluded={namb}")
    assert dx <= p["alpha"] * gabs + 2e-6 and namb <= amb_limit("fp32", X.size)
    ctx.step(300)
    r = ctx.result()
    E = q.meta["edges"]
    size, inside = mis.set_size(E, r["best_x"][None])
    assert r["best_obj"] == oq.objective(q, r["best_x"][None])[0] == mis.objective(E, r["best_x"][None])[0]
    say(f"   best F {r['best_obj']} at t={r['best_iter']}: |S| = {size[0]}, edges inside {inside[0]}")
    if inside[0] == 0:
        assert -r["best_obj"] == size[0]
    ctx.destroy()
