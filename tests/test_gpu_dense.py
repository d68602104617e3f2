"""Dense QUBO path on the GPU against the oracle (P1-P5 of the parity plan).

Sizes span several tiles and ragged tails in n and in B."""
import numpy as np
import pytest

import workloads as W
from gpu_util import amb_limit, lockstep_compare, normwise, require_gpu, say
from oracle import enumerate as en
from oracle import gda
from oracle import qubo as oq

pytestmark = pytest.mark.gpu

# normwise gradient tolerances: 1e-5 (fp32) and 1e-2 (bf16) as required for
# the hot path; fp8 (3 mantissa bits on both operands) is measured and held to
# a loose bound
GTOL = {"fp32": 1e-5, "bf16": 1e-2, "fp8": 1e-1, "i8": 1e-2}


def _cases():
    return {
        "gnp_n200": (W.qubo_c1(0), 16, 1.0),
        "gnp_n333_B40": (W.qubo_c1(1, n=333), 40, 1.0),
        "dense_u100_n700": (W.random_dense_qubo(700, -100, 100, W.rng_for(3, 0, 0, 700)), 100, None),
        "asym_diag_n150": (W.Qubo(n=150, Q=np.random.default_rng(5).integers(-20, 21, (150, 150)).astype(np.int32),
                                  c=np.random.default_rng(6).integers(-50, 51, 150).astype(np.int64)), 24, None),
        "tiny_n1_B1": (W.Qubo(n=1, Q=np.array([[3]], np.int32), c=np.array([-5], np.int64)), 1, 1.0),
        "n7_B3": (W.qubo_c1(2, n=7), 3, 1.0),
    }


CASES = _cases()


def _scale(q, s):
    return W.qubo_scale(q) if s is None else s


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8", "i8"])
@pytest.mark.parametrize("name", list(CASES))
def test_gradient_parity(name, prec):
    P = require_gpu()
    q, B, s = CASES[name]
    s = _scale(q, s)
    say(f"[dense grad] case={name} prec={prec} n={q.n} B={B}")
    x = W.x0_uniform(7, 0, B, q.n).astype(np.float32)
    p = W.gda_params("qubo", B=B, T=1, scale=s, precision=prec)
    ctx = P.qubo_gda_init(q, p, x.astype(np.float64))
    G = ctx.grad(x)
    G64 = oq.grad_f(*oq.canonicalize(q), x.astype(np.float64), s)
    err = normwise(G, G64)
    say(f"   normwise gradient error {err:.3e} (tile {ctx.tile_name})")
    assert err <= GTOL[prec], err


@pytest.mark.parametrize("tile", list(range(1, 11)))
def test_gradient_parity_every_tile(tile):
    P = require_gpu()
    q = W.random_dense_qubo(517, -100, 100, W.rng_for(3, 1, 0, 517))
    s = W.qubo_scale(q)
    B = 150
    say(f"[dense grad tile] tile={tile} n={q.n} B={B}")
    x = W.x0_uniform(7, 1, B, q.n).astype(np.float32)
    for prec in ("fp32", "bf16", "i8"):
        ctx = P.qubo_gda_init(q, W.gda_params("qubo", B=B, T=1, scale=s, precision=prec, tile=tile),
                              x.astype(np.float64))
        err = normwise(ctx.grad(x), oq.grad_f(*oq.canonicalize(q), x.astype(np.float64), s))
        assert err <= GTOL[prec], (tile, prec, err)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8", "i8"])
@pytest.mark.parametrize("name", ["gnp_n200", "dense_u100_n700", "asym_diag_n150", "n7_B3"])
def test_lockstep_iteration(name, prec):
    P = require_gpu()
    q, B, s = CASES[name]
    s = _scale(q, s)
    say(f"[dense lockstep] case={name} prec={prec}")
    g = np.random.default_rng(11)
    X = g.random((B, q.n)).astype(np.float32)
    # include exact perturbation cases: points at 1/2 and 1/2 +- delta
    X[:, ::7] = 0.5
    X[:, 3::11] = np.float32(0.5 + W.DELTA)
    Y = g.uniform(-2.0, 6.0, (B, q.n)).astype(np.float32)
    p = W.gda_params("qubo", B=B, T=1, scale=s, precision=prec)
    ctx = P.qubo_gda_init(q, p, X.astype(np.float64))
    ctx.set_state(X, Y, 0)
    Gg = ctx.grad(X)
    ctx.step(1)
    Xg, Yg, t = ctx.get_state()
    assert t == 1
    G64 = oq.grad_f(*oq.canonicalize(q), X.astype(np.float64), s)
    gabs = GTOL[prec] * float(np.max(np.abs(G64))) + 1e-6
    dx, dy, namb, _, _ = lockstep_compare(X.astype(np.float64), Y.astype(np.float64), G64, Xg, Yg, p, gabs)
    say(f"   max|dX|={dx:.3e} max|dY|={dy:.3e} excluded={namb}/{X.size}")
    assert dx <= p["alpha"] * gabs + 2e-6
    assert dy <= 2e-6 * (1 + np.max(np.abs(Y)))
    assert namb <= amb_limit(prec, X.size)
    assert np.all((Xg >= 0) & (Xg <= 1))
    # P1: objectives of the rounded iterate, bit-exact
    F = ctx.objectives()
    assert np.array_equal(F, oq.objective(q, Xg > 0.5))
    assert np.max(np.abs(Gg - G64)) <= gabs


@pytest.mark.parametrize("prec", ["fp32", "bf16", "i8"])
@pytest.mark.parametrize("name", ["gnp_n200", "dense_u100_n700"])
def test_lockstep_iteration_entropy_g(name, prec):
    """The dense step with the entropy g (a separate step kernel variant):
    one iteration against the oracle, including x at 0, 1/2 and 1, where g'
    is taken at the clipped point."""
    P = require_gpu()
    q, B, s = CASES[name]
    s = _scale(q, s)
    say(f"[dense lockstep entropy] case={name} prec={prec}")
    g = np.random.default_rng(12)
    X = g.random((B, q.n)).astype(np.float32)
    X[:, ::7] = 0.5
    X[:, 3::11] = np.float32(0.5 + W.DELTA)
    X[:, 5::13] = 0.0
    X[:, 6::17] = 1.0
    Y = g.uniform(-2.0, 6.0, (B, q.n)).astype(np.float32)
    p = W.gda_params("qubo", B=B, T=1, scale=s, precision=prec, g="entropy")
    ctx = P.qubo_gda_init(q, p, X.astype(np.float64))
    ctx.set_state(X, Y, 0)
    ctx.step(1)
    Xg, Yg, t = ctx.get_state()
    assert t == 1
    G64 = oq.grad_f(*oq.canonicalize(q), X.astype(np.float64), s)
    # float32 logarithms of g' near the clip: up to |y| * 2e-6 in dL
    gabs = GTOL[prec] * float(np.max(np.abs(G64))) + 2e-6 * float(np.max(np.abs(Y))) + 1e-6
    dx, dy, namb, _, _ = lockstep_compare(X.astype(np.float64), Y.astype(np.float64), G64, Xg, Yg, p, gabs)
    say(f"   max|dX|={dx:.3e} max|dY|={dy:.3e} excluded={namb}/{X.size}")
    assert dx <= p["alpha"] * gabs + 2e-6
    assert dy <= 2e-6 * (1 + np.max(np.abs(Y)))
    assert namb <= amb_limit(prec, X.size)
    assert np.all((Xg >= 0) & (Xg <= 1))
    F = ctx.objectives()
    assert np.array_equal(F, oq.objective(q, Xg > 0.5))


@pytest.mark.parametrize("name", list(CASES))
def test_eval_exact_random_vectors(name):
    P = require_gpu()
    q, B, s = CASES[name]
    say(f"[dense eval] case={name}")
    ctx = P.qubo_gda_init(q, W.gda_params("qubo", B=B, T=1, scale=_scale(q, s)),
                          W.x0_uniform(7, 2, B, q.n))
    g = np.random.default_rng(3)
    xr = (g.random((B, q.n)) < g.random((B, 1))).astype(np.uint8)
    xr[0] = 0
    if B > 1:
        xr[1] = 1
    assert np.array_equal(ctx.eval(xr), oq.objective(q, xr))


def test_full_run_invariants_and_optimum():
    P = require_gpu()
    q = W.qubo_c1(0)
    B, T = 16, 1000
    x0 = W.x0_uniform(1, 0, B, q.n, q.n)
    p = W.gda_params("maxcut", B=B, T=T, precision="fp32")
    say("[dense run] C1 n=200 B=16 T=1000 fp32")
    ctx = P.qubo_gda_init(q, p, x0)
    ctx.step(T // 2)
    _, Yh, _ = ctx.get_state()
    ctx.step(T - T // 2)
    X, Y, t = ctx.get_state()
    assert t == T
    assert np.all((X >= 0) & (X <= 1))
    assert np.all(Y <= Yh) and np.all(Yh <= p["y0"])
    r = ctx.result()
    assert r["best_obj"] == oq.objective(q, r["best_x"][None])[0]
    assert 1 <= r["best_iter"] <= T and 0 <= r["best_restart"] < B
    ref = gda.run(oq.QuboProblem(q, 1.0), x0, p, T=T)
    say(f"   GPU fp32 best {r['best_obj']} at t={r['best_iter']}; oracle fp64 best {ref.inc.F}")
    # trajectories diverge at the discontinuous branch; quality must agree closely
    assert r["best_obj"] <= ref.inc.F + max(2, abs(ref.inc.F) // 50)


@pytest.mark.parametrize("rep", range(4))
def test_twin_reaches_brute_force_optimum(rep):
    P = require_gpu()
    q = W.qubo_c1_twin(rep)
    Fstar, _ = en.brute_force(lambda X: oq.objective(q, X), q.n)
    for prec in ("fp32", "bf16", "i8"):
        r = P.qubo_gda_solve(q, W.gda_params("maxcut", B=16, T=1000, precision=prec),
                             W.x0_uniform(1, rep, 16, q.n, q.n), 1000)
        assert r["best_obj"] == Fstar, (rep, prec)


def test_determinism_resume_graph():
    """Bit-identical iterates and incumbents with and without hipGraph replays
    (graphs start after the evaluation GEMM's transient of 64 iterations), and
    through get/set_state into a fresh context, whose transient restarts at
    the resumed iteration."""
    P = require_gpu()
    q = W.random_dense_qubo(300, -100, 100, W.rng_for(3, 2, 0, 300))
    s = W.qubo_scale(q)
    B = 64
    x0 = W.x0_uniform(3, 2, B, q.n)
    say("[dense determinism/resume/graph]")
    outs = []
    for gc in (0, 0, 8):
        ctx = P.qubo_gda_init(q, W.gda_params("qubo", B=B, T=100, scale=s, precision="bf16", graph_chunk=gc), x0)
        ctx.step(17)
        ctx.step(23)
        ctx.step(60)
        X, Y, t = ctx.get_state()
        outs.append((X, Y, ctx.result()))
    for X, Y, r in outs[1:]:
        assert np.array_equal(X, outs[0][0]) and np.array_equal(Y, outs[0][1])
        assert r["best_obj"] == outs[0][2]["best_obj"] and r["best_iter"] == outs[0][2]["best_iter"]
    # resume through get/set_state into a fresh context
    ctx = P.qubo_gda_init(q, W.gda_params("qubo", B=B, T=100, scale=s, precision="bf16"), x0)
    ctx.step(17)
    X17, Y17, _ = ctx.get_state()
    ctx2 = P.qubo_gda_init(q, W.gda_params("qubo", B=B, T=100, scale=s, precision="bf16", graph_chunk=8), x0)
    ctx2.set_state(X17, Y17, 17)
    ctx2.step(83)
    X, Y, t = ctx2.get_state()
    assert t == 100 and np.array_equal(X, outs[0][0]) and np.array_equal(Y, outs[0][1])
    F = ctx2.objectives()
    assert np.array_equal(F, oq.objective(q, X > 0.5))


@pytest.mark.parametrize("full_iters", ["0", "2"])
def test_objectives_by_rows_after_transient(full_iters, monkeypatch):
    """Past the transient (PDBO_FULL_EVAL_ITERS iterations after init) the
    evaluation GEMM no longer runs: restarts with more than 32 rounding changes,
    and with 0 the first evaluation, are evaluated by rows of Ahat in the
    incremental kernel.  The objectives equal the oracle's at every step, and
    the incumbent equals that of a context that runs the GEMM throughout."""
    P = require_gpu()
    monkeypatch.setenv("PDBO_FULL_EVAL_ITERS", full_iters)
    n, B = 517, 96
    q = W.random_dense_qubo(n, -50, 50, W.rng_for(7, 1, 0, n))
    s = W.qubo_scale(q)
    x0 = W.x0_uniform(7, 1, B, n)
    p = W.gda_params("qubo", B=B, T=30, scale=s, precision="i8")
    say(f"[objectives by rows] n={n} B={B} transient={full_iters}")
    ctx = P.qubo_gda_init(q, p, x0)
    prev = None
    many = 0
    for t in range(30):
        ctx.step(1)
        Xg, _, _ = ctx.get_state()
        xr = Xg > 0.5
        assert np.array_equal(ctx.objectives(), oq.objective(q, xr)), t
        if prev is not None and t >= int(full_iters):
            many += int(np.sum(np.sum(xr != prev, axis=1) > 32))
        prev = xr
    say(f"   restarts evaluated by rows after the transient: {many}")
    assert many > 0
    r = ctx.result()
    assert r["best_obj"] == oq.objective(q, r["best_x"][None])[0]
    monkeypatch.setenv("PDBO_FULL_EVAL_ITERS", "1000")
    ref = P.qubo_gda_init(q, p, x0)
    ref.step(30)
    r2 = ref.result()
    assert (r["best_obj"], r["best_iter"], r["best_restart"]) == \
        (r2["best_obj"], r2["best_iter"], r2["best_restart"])
    assert np.array_equal(r["best_x"], r2["best_x"])


@pytest.mark.parametrize("T", [30, 100])
def test_batched_grouped_equals_per_instance_and_single(T):
    """Grouped, per-instance and single-instance runs agree bit for bit; T = 100
    runs past the evaluation GEMM's transient (by-rows evaluation, best of B in
    the step launches of each instance)."""
    P = require_gpu()
    qs = W.batch_c4(rep=0, k=5, n_lo=60, n_hi=400)
    B = 32
    ps = [W.gda_params("qubo", B=B, T=T, scale=W.qubo_scale(q), precision="bf16", tile=2) for q in qs]
    x0s = [W.x0_uniform(4, 0, B, q.n, i) for i, q in enumerate(qs)]
    say(f"[dense batch] 5 instances grouped vs per-instance vs single, T={T}")
    rg = P.qubo_gda_batch_solve(qs, ps, x0s, T, grouped=True)
    ri = P.qubo_gda_batch_solve(qs, ps, x0s, T, grouped=False)
    for i, q in enumerate(qs):
        rs = P.qubo_gda_solve(W.Qubo(n=q.n, Q=q.dense(), c=q.c), ps[i], x0s[i], T)
        for r in (ri[i], rs):
            assert r["best_obj"] == rg[i]["best_obj"] and r["best_iter"] == rg[i]["best_iter"]
            assert np.array_equal(r["best_x"], rg[i]["best_x"])
        assert rg[i]["best_obj"] == oq.objective(q, rg[i]["best_x"][None])[0]


@pytest.mark.parametrize("tile", [0, 1, 8])
def test_incremental_objectives_every_step(tile):
    """The objectives the in-loop evaluation keeps (a full product first, then
    exact differences from the recorded rounding changes, or a full product for
    column blocks where some restart changed many coordinates) equal the
    oracle's at every step; the run passes through both regimes."""
    P = require_gpu()
    n, B = 600, 300
    q = W.random_dense_qubo(n, -50, 50, W.rng_for(7, 0, 0, n))
    s = W.qubo_scale(q)
    x0 = W.x0_uniform(7, 0, B, n)
    p = W.gda_params("qubo", B=B, T=1, scale=s, precision="i8", tile=tile)
    say(f"[incremental eval] n={n} B={B} tile={tile}")
    ctx = P.qubo_gda_init(q, p, x0)
    prev = None
    few = many = 0
    for t in range(80):
        ctx.step(1)
        Xg, _, _ = ctx.get_state()
        xr = Xg > 0.5
        assert np.array_equal(ctx.objectives(), oq.objective(q, xr)), t
        if prev is not None:
            k = np.sum(xr != prev, axis=1)
            few += int(np.sum((k >= 1) & (k <= 32)))
            many += int(np.sum(k > 32))
        prev = xr
    say(f"   (restart, step) pairs with 1..32 changes {few}, with more {many}")
    assert few > 0 and many > 0
    r = ctx.result()
    assert r["best_obj"] == oq.objective(q, r["best_x"][None])[0]


def test_timing_classes_and_trace():
    """Per-class timing counts exactly the launches of the classes asked for;
    an unknown class is rejected; the incumbent trace improves strictly and ends
    at the result."""
    P = require_gpu()
    q = W.qubo_c1(0)
    B = 64
    x0 = W.x0_uniform(1, 0, B, q.n)
    p = W.gda_params("qubo", B=B, T=1, scale=W.qubo_scale(q), precision="i8")
    ctx = P.qubo_gda_init(q, p, x0)
    ctx.timing(True, classes=[P.PDBO_K_STEP])
    ctx.step(7)
    ms, cnt = ctx.kernel_time(P.PDBO_K_STEP)
    assert cnt == 7 and ms > 0
    for k in (P.PDBO_K_EVAL, P.PDBO_K_INCR, P.PDBO_K_ARGMIN):
        assert ctx.kernel_time(k)[1] == 0
    ctx.timing(True)
    ctx.step(3)
    for k in (P.PDBO_K_STEP, P.PDBO_K_EVAL, P.PDBO_K_INCR):
        assert ctx.kernel_time(k)[1] == 3, k
    # the best of B of the first two iterations runs inside the next step
    # launch; only the last one has a launch of its own
    assert ctx.kernel_time(P.PDBO_K_ARGMIN)[1] == 1
    with pytest.raises(P.PdboError):
        ctx.timing(True, classes=[7])
    # every third launch: launches 0, 3 and 6 of seven
    ctx.timing(True, classes=[P.PDBO_K_STEP], stride=3)
    ctx.step(7)
    assert ctx.kernel_time(P.PDBO_K_STEP)[1] == 3
    with pytest.raises(P.PdboError):
        ctx.timing(True, classes=[P.PDBO_K_STEP], stride=0)
    ctx.timing(False)
    ctx.step(40)
    tr = ctx.trace()
    r = ctx.result()
    assert len(tr["F"]) >= 1
    assert np.all(np.diff(tr["F"]) < 0) and np.all(np.diff(tr["t"]) > 0)
    assert tr["F"][-1] == r["best_obj"] and tr["t"][-1] == r["best_iter"]
    assert r["best_obj"] == oq.objective(q, r["best_x"][None])[0]
