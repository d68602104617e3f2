"""Float64 weights (Eq. 1 with real Q and c) on the row-parallel CSR path
against the oracle: gradient and iterations from the GPU's own state, the
objective of every rounded iterate equal to the correctly rounded exact real
sum (bit for bit), exact incumbent comparisons replayed through the oracle's
rule, ties of the final rounding, and integer-valued weights agreeing with the
int32 path."""
import numpy as np
import pytest

import workloads as W
from gpu_util import amb_limit, lockstep_compare, normwise, require_gpu, say
from oracle import qubo as oq
from oracle.gda import Incumbent

pytestmark = pytest.mark.gpu

CASES = {
    # (instance, B)
    "dense_n300_normal_B16": (lambda: W.real_qubo(300, 6000, 0, dense=True), 16),
    "csr_n3000_spread30_B70": (lambda: W.real_qubo(3000, 9000, 1, spread=30), 70),
    # binary exponents over 2^-116 .. 2^62: eight 24-bit digits
    "csr_n800_spread60_B10": (lambda: W.real_qubo(800, 2400, 2, spread=60), 10),
}


def _exact_f64(q, Xr):
    return np.array([float(v) for v in oq.objective_exact(q, Xr)])


def _ctx(P, q, B, **over):
    p = W.gda_params("qubo", B=B, T=1, scale=1.0, **over)
    return P.qubo_gda_init(q, p, W.x0_uniform(9, 1, B, q.n)), p


@pytest.mark.parametrize("name", list(CASES))
def test_real_gradient_steps_objectives(name):
    P = require_gpu()
    make, B = CASES[name]
    q = make()
    A, cp = oq.canonicalize(q)
    ctx, p = _ctx(P, q, B)
    say(f"[real] {name} n={q.n} B={B}")
    X = np.random.default_rng(1).random((B, q.n)).astype(np.float32)
    G64 = oq.grad_f(A, cp, X.astype(np.float64), 1.0)
    err = normwise(ctx.grad(X), G64)
    say(f"   gradient normwise error {err:.3e}")
    assert err <= 1e-5
    X, Y, _ = ctx.get_state()
    for step in range(1, 4):
        ctx.step(1)
        Xn, Yn, t = ctx.get_state()
        assert t == step
        X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
        G64 = oq.grad_f(A, cp, X64, 1.0)
        gabs = 1e-5 * float(np.max(np.abs(G64))) + 1e-6
        dx, dy, namb, _, _ = lockstep_compare(X64, Y64, G64, Xn, Yn, p, gabs)
        say(f"   t={step}: max|dX|={dx:.3e} max|dY|={dy:.3e} excluded={namb}")
        assert dx <= p["alpha"] * gabs + 2e-6
        assert dy <= 2e-6 * (1 + np.max(np.abs(Y64)))
        assert namb <= amb_limit("fp32", X.size)
        assert np.array_equal(ctx.objectives_f64(), _exact_f64(q, Xn > 0.5)), step
        X, Y = Xn, Yn
    xr = np.random.default_rng(2).integers(0, 2, size=(B, q.n), dtype=np.uint8)
    xr[0] = 1
    xr[1] = 0
    assert np.array_equal(ctx.eval_f64(xr), _exact_f64(q, xr.astype(bool)))
    assert np.array_equal(ctx.eval_f64(xr[:3]), _exact_f64(q, xr[:3].astype(bool)))
    with pytest.raises(P.PdboError):
        ctx.objectives()        # int64 objectives do not exist for real weights
    ctx.destroy()


def test_real_incumbent_replay_and_trace():
    """Every iteration's objectives through the oracle's exact incumbent rule;
    graph replay and split calls reproduce the eager run bit for bit."""
    P = require_gpu()
    q = W.real_qubo(2000, 8000, 3, spread=8)
    B, T = 12, 40
    ctx, p = _ctx(P, q, B)
    inc = Incumbent()
    for t in range(1, T + 1):
        ctx.step(1)
        X, _, _ = ctx.get_state()
        Fx = oq.objective_exact(q, X > 0.5)
        assert np.array_equal(ctx.objectives_f64(), np.array([float(v) for v in Fx])), t
        inc.offer(Fx, t, X > 0.5)
    r = ctx.result()
    say(f"[real] incumbent F={r['best_obj_f64']!r} t={r['best_iter']} b={r['best_restart']}")
    assert (r["best_obj_f64"], r["best_iter"], r["best_restart"]) == (float(inc.F), inc.t, inc.b)
    assert np.array_equal(r["best_x"], inc.x)
    tr = ctx.trace_f64()
    assert len(tr["F"]) >= 1 and np.all(np.diff(tr["F"]) <= 0) and tr["F"][-1] == r["best_obj_f64"]
    X0, Y0 = ctx.get_state()[:2]
    ctx.destroy()
    for gc, parts in ((8, [T]), (0, [7, 33])):
        c2, _ = _ctx(P, q, B, graph_chunk=gc)
        for k in parts:
            c2.step(k)
        r2 = c2.result()
        X2, Y2, _ = c2.get_state()
        assert (r2["best_obj_f64"], r2["best_iter"], r2["best_restart"]) == \
            (r["best_obj_f64"], r["best_iter"], r["best_restart"])
        assert np.array_equal(X2, X0) and np.array_equal(Y2, Y0)
        c2.destroy()


def test_real_rounding_ties_and_cancellation():
    """Exact sums halfway between two float64 values round to even; terms that
    cancel exactly (2^100 + 2^48 against its negative, 160 bits above the
    smallest weight) leave the small ones intact."""
    P = require_gpu()
    n = 6
    Q = np.zeros((n, n))
    big = 2.0 ** 100 + 2.0 ** 48
    Q[0, 1], Q[1, 0] = big, -big
    c = np.array([1.0, 2.0 ** -53, 1.0 + 2.0 ** -52, 2.0 ** -53, 3.0 * 2.0 ** -60, -1.0])
    q = W.Qubo(n=n, Q=Q, c=c)
    ctx, _ = _ctx(P, q, 8)
    xr = np.array([[1, 1, 0, 0, 0, 0],     # 1 + 2^-53: tie, even is 1
                   [0, 0, 1, 1, 0, 0],     # 1 + 3 2^-53: tie, even is 1 + 2^-51
                   [1, 1, 0, 0, 1, 0],     # just above the tie: rounds up
                   [1, 1, 0, 0, 0, 1],     # 2^-53 after the cancellation of 1 - 1
                   [0, 0, 0, 0, 0, 0]], dtype=np.uint8)
    F = ctx.eval_f64(xr)
    want = _exact_f64(q, xr.astype(bool))
    say(f"[real] ties {F.tolist()}")
    assert np.array_equal(F, want)
    assert F[0] == 1.0 and F[1] == 1.0 + 2.0 ** -51 and F[2] == 1.0 + 2.0 ** -52
    assert F[3] == 2.0 ** -53 and F[4] == 0.0
    ctx.destroy()


def test_real_integer_valued_matches_int_path():
    """Integer-valued float64 weights give the objectives, iterates and
    incumbent of the same int32 instance on the row-parallel path."""
    P = require_gpu()
    qi = W.maxcut_c2(0, n=1500, M=5000)
    qr = W.Qubo(n=qi.n, row_ptr=qi.row_ptr, col_idx=qi.col_idx, vals=qi.vals.astype(np.float64),
                c=qi.c.astype(np.float64))
    B, T = 32, 25
    out = []
    for q in (qi, qr):
        p = W.gda_params("maxcut", B=B, T=T, tile=2)
        ctx = P.qubo_gda_init(q, p, W.x0_uniform(9, 2, B, q.n))
        ctx.step(T)
        r = ctx.result()
        X, Y, _ = ctx.get_state()
        out.append((r, X, Y, ctx.objectives_f64()))
        ctx.destroy()
    (ri, Xi, Yi, Fi), (rr, Xr, Yr, Fr) = out
    assert np.array_equal(Fi, Fr)
    assert rr["best_obj_f64"] == float(ri["best_obj"]) == ri["best_obj_f64"]
    assert (rr["best_iter"], rr["best_restart"]) == (ri["best_iter"], ri["best_restart"])
    # A/s = (Q_ij + Q_ji) / s is the same float32 in both forms (integers, s = 1)
    assert np.array_equal(Xi, Xr) and np.array_equal(Yi, Yr)
