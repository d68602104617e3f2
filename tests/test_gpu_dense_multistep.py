"""Dense path over several iterations, each compared with the oracle's Alg. 1
iteration taken from the GPU's own iterate (no set_state in between), so that
the second and later gradient products read the operand shadow that the step
epilogue wrote (int8 code, e4m3 or bf16 copy of x^{t+1}, ping-pong buffers);
a short float32 trajectory against the float64 one; the batched path replayed
through hipGraphs; and the incumbent replayed through the oracle's rule."""
import numpy as np
import pytest

import workloads as W
from gpu_util import amb_limit, lockstep_compare, normwise, require_gpu, say
from oracle import gda
from oracle import qubo as oq
from oracle.binarity import by_name

pytestmark = pytest.mark.gpu

GTOL = {"fp32": 1e-5, "bf16": 1e-2, "fp8": 1e-1, "i8": 1e-2}


def _recovered_gradient(X, Y, Xn, p, mask_out):
    """The gradient the GPU used, read back from its own update where the plain
    projected step applied strictly inside the box: x+ = x - alpha (G + y g'(x))."""
    g = by_name(p.get("g", "quad"))
    G = (X - Xn) / p["alpha"] - Y * g.deriv(X)
    ok = (Xn > 0.0) & (Xn < 1.0) & ~mask_out
    return G, ok


@pytest.mark.parametrize("tile", [0, 8])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8", "i8"])
def test_multistep_lockstep_from_own_state(prec, tile):
    P = require_gpu()
    n, B = 517, 150
    q = W.random_dense_qubo(n, -100, 100, W.rng_for(3, 4, 0, n))
    s = W.qubo_scale(q)
    A, cp = oq.canonicalize(q)
    x0 = W.x0_uniform(3, 4, B, n)
    # y0 small enough that y crosses zero within the steps below: the
    # perturbation branch is reached from the GPU's own state
    p = W.gda_params("qubo", B=B, T=1, scale=s, precision=prec, tile=tile, y0=0.01, beta=0.05)
    say(f"[dense multistep] prec={prec} tile={tile} n={n} B={B}")
    ctx = P.qubo_gda_init(q, p, x0)
    X, Y, t = ctx.get_state()
    assert t == 0
    for step in range(1, 5):
        ctx.step(1)
        Xn, Yn, t = ctx.get_state()
        assert t == step
        X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
        G64 = oq.grad_f(A, cp, X64, s)
        gabs = GTOL[prec] * float(np.max(np.abs(G64))) + 1e-6
        dx, dy, namb, _, _ = lockstep_compare(X64, Y64, G64, Xn, Yn, p, gabs)
        pert = (np.abs(X64 - 0.5) <= p["delta"]) & (Y64 <= 0)
        Gr, ok = _recovered_gradient(X64, Y64, Xn.astype(np.float64), p, pert)
        # (x - x+)/alpha carries the float32 rounding of x and x+ divided by alpha
        err = float(np.max(np.abs(Gr - G64)[ok])) / float(np.max(np.abs(G64)))
        say(f"   t={step}: max|dX|={dx:.3e} max|dY|={dy:.3e} excluded={namb} "
            f"recovered-gradient error {err:.3e} on {int(ok.sum())} coordinates, "
            f"perturbation-eligible {int(pert.sum())}")
        assert dx <= p["alpha"] * gabs + 2e-6
        assert dy <= 2e-6 * (1 + np.max(np.abs(Y64)))
        assert namb <= amb_limit(prec, X.size)
        assert err <= GTOL[prec] + 4e-7 / p["alpha"] / float(np.max(np.abs(G64)))
        assert np.all((Xn >= 0) & (Xn <= 1))
        assert np.array_equal(ctx.objectives(), oq.objective(q, Xn > 0.5)), step
        X, Y = Xn, Yn
    assert np.any(Y <= 0), "the run never reached y <= 0"


def test_fp32_trajectory_short_horizon():
    """Five float32 iterations from x0 track the oracle's float64 trajectory."""
    P = require_gpu()
    n, B = 300, 16
    q = W.random_dense_qubo(n, -100, 100, W.rng_for(3, 5, 0, n))
    s = W.qubo_scale(q)
    x0 = W.x0_uniform(3, 5, B, n)
    p = W.gda_params("qubo", B=B, T=5, scale=s, precision="fp32")
    say(f"[dense fp32 trajectory] n={n} B={B} T=5")
    ctx = P.qubo_gda_init(q, p, x0)
    ctx.step(5)
    X, Y, _ = ctx.get_state()
    ref = gda.run(oq.QuboProblem(q, s), x0, p, T=5)
    dx, dy = float(np.max(np.abs(X - ref.X))), float(np.max(np.abs(Y - ref.Y)))
    say(f"   max|dX|={dx:.3e} max|dY|={dy:.3e}")
    assert dx < 1e-4 and dy < 1e-5
    assert np.array_equal(ctx.objectives(), oq.objective(q, X > 0.5))
    near = np.abs(ref.X - 0.5) < 1e-4
    assert np.array_equal((X > 0.5)[~near], (ref.X > 0.5)[~near])


@pytest.mark.parametrize("grouped", [1, 0])
def test_batched_graph_replay_equals_eager(grouped):
    """A batch stepped through hipGraph replays (after the evaluation GEMM's
    transient of 64 eager iterations) equals the same batch stepped eagerly,
    bit for bit; every incumbent is re-evaluated by the oracle."""
    P = require_gpu()
    qs = W.batch_c4(rep=1, k=4, n_lo=80, n_hi=500)
    B, T = 48, 100
    say(f"[dense batch graph] 4 instances, grouped={grouped}, T={T}, graph chunk 8")
    x0s = [W.x0_uniform(4, 1, B, q.n, i) for i, q in enumerate(qs)]
    out = {}
    for gc in (0, 8):
        ps = [W.gda_params("qubo", B=B, T=T, scale=W.qubo_scale(q), precision="bf16", graph_chunk=gc)
              for q in qs]
        ctx = P.qubo_gda_batch_init(qs, ps, x0s, grouped=bool(grouped))
        ctx.step(37)
        ctx.step(63)
        out[gc] = [P.qubo_gda_batch_result(ctx, i) for i in range(len(qs))]
        ctx.destroy()
    for i, q in enumerate(qs):
        a, b = out[0][i], out[8][i]
        assert (a["best_obj"], a["best_iter"], a["best_restart"]) == \
            (b["best_obj"], b["best_iter"], b["best_restart"]), i
        assert np.array_equal(a["best_x"], b["best_x"])
        assert a["best_obj"] == oq.objective(q, a["best_x"][None])[0]


def test_incumbent_replayed_through_oracle_rule():
    """The objectives of every iteration (bit-exact with the oracle's) fed to
    the oracle's incumbent rule (first restart of the minimum, strict
    improvement, earliest iteration) give the GPU's incumbent: value,
    iteration, restart and vector."""
    P = require_gpu()
    n, B = 300, 200
    q = W.random_dense_qubo(n, -30, 30, W.rng_for(7, 3, 0, n))
    s = W.qubo_scale(q)
    x0 = W.x0_uniform(7, 3, B, n)
    p = W.gda_params("qubo", B=B, T=1, scale=s, precision="i8")
    say(f"[incumbent replay] n={n} B={B} 90 iterations")
    ctx = P.qubo_gda_init(q, p, x0)
    inc = gda.Incumbent()
    ties = 0
    for t in range(1, 91):
        ctx.step(1)
        Xg, _, _ = ctx.get_state()
        xr = Xg > 0.5
        F = oq.objective(q, xr)
        assert np.array_equal(ctx.objectives(), F), t
        ties += int(np.sum(F == F.min()) > 1) + int(inc.F is not None and F.min() == inc.F)
        inc.offer(F, t, xr)
    r = ctx.result()
    say(f"   incumbent F={inc.F} t={inc.t} b={inc.b}; iterations with ties {ties}")
    assert (r["best_obj"], r["best_iter"], r["best_restart"]) == (inc.F, inc.t, inc.b)
    assert np.array_equal(r["best_x"], inc.x)
    tr = ctx.trace()
    assert tr["t"][-1] == inc.t and tr["F"][-1] == inc.F


@pytest.mark.parametrize("kind", ["dense_i8", "dense_fp32", "csr", "maxsat"])
def test_restart_equals_fresh_context(kind):
    """qubo_gda_restart on a used context reproduces a fresh context's run bit
    for bit (iterate, incumbent, iteration of the best)."""
    P = require_gpu()
    B, T = 40, 90
    if kind.startswith("dense"):
        q = W.random_dense_qubo(230, -100, 100, W.rng_for(3, 6, 0, 230))
        p = W.gda_params("qubo", B=B, T=T, scale=W.qubo_scale(q), precision=kind.split("_")[1])
        init = lambda x: P.qubo_gda_init(q, p, x)  # noqa: E731
        n = q.n
    elif kind == "csr":
        q = W.maxcut_c2(2, n=400, M=1200)
        p = W.gda_params("maxcut", B=B, T=T)
        init = lambda x: P.qubo_gda_init(q, p, x)  # noqa: E731
        n = q.n
    else:
        f = W.random_maxsat(300, 1200, 3, 1, 10, W.rng_for(5, 6, 0, 300))
        p = W.gda_params("maxsat", B=B, T=T, scale=W.maxsat_scale(f))
        init = lambda x: P.maxsat_gda_init(f, p, x)  # noqa: E731
        n = f.n
    xa, xb = W.x0_uniform(9, 0, B, n), W.x0_uniform(9, 1, B, n)
    say(f"[restart] {kind} n={n} B={B} T={T}")
    ctx = init(xa)
    ctx.step(T)
    ctx.restart(xb)
    ctx.step(T)
    X1, Y1, t1 = ctx.get_state()
    r1 = ctx.result()
    ref = init(xb)
    ref.step(T)
    X2, Y2, t2 = ref.get_state()
    r2 = ref.result()
    assert t1 == t2 == T
    assert np.array_equal(X1, X2) and np.array_equal(Y1, Y2)
    assert (r1["best_obj"], r1["best_iter"], r1["best_restart"]) == \
        (r2["best_obj"], r2["best_iter"], r2["best_restart"])
    assert np.array_equal(r1["best_x"], r2["best_x"])
