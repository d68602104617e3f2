"""Parity at the workloads' full sizes, in the launch configuration bench.py
times (autotuned tiles), on outputs the oracle computes restart by restart:
sampled gradients and one lockstep iteration, plus the exact objectives of
every restart's rounded iterate."""
import numpy as np
import pytest

import workloads as W
from gpu_util import amb_limit, lockstep_compare, require_gpu, say
from oracle import maxsat as om
from oracle import qubo as oq

pytestmark = pytest.mark.gpu

GTOL = {"fp32": 1e-5, "bf16": 1e-2, "i8": 1e-2, "fp8": 1e-1}
SAMPLE = [0, 1, 317, 511, 1022, 1023]


@pytest.fixture(scope="module")
def c3():
    q = W.qubo_c3(0)
    s = W.qubo_scale(q)
    x0 = W.x0_uniform(3, 0, 1024, q.n)
    A, cp = oq.canonicalize(q)
    return q, s, x0, A, cp


@pytest.mark.parametrize("prec", ["i8", "fp8", "bf16", "fp32"])
def test_c3_dense_n10000_B1024(c3, prec):
    P = require_gpu()
    q, s, x0, A, cp = c3
    B = 1024
    say(f"[fullsize c3] n={q.n} B={B} prec={prec}")
    p = W.gda_params("qubo", B=B, T=1, scale=s, precision=prec)
    ctx = P.qubo_gda_init(q, p, x0)
    say(f"   tile {ctx.tile_name}")
    X = x0.astype(np.float32)
    G = ctx.grad(X)
    ctx.step(1)
    Xg, Yg, t = ctx.get_state()
    # sampled restarts, one matrix-vector product each
    Xs = X[SAMPLE].astype(np.float64)
    G64 = (Xs @ A + cp[None, :]) / s          # A is symmetric
    err = np.max(np.abs(G[SAMPLE] - G64)) / np.max(np.abs(G64))
    say(f"   normwise gradient error on sampled restarts {err:.3e}")
    assert err <= GTOL[prec]
    gabs = GTOL[prec] * float(np.max(np.abs(G64))) + 1e-6
    Y0 = np.full_like(Xs, p["y0"])
    dx, dy, namb, _, _ = lockstep_compare(Xs, Y0, G64, Xg[SAMPLE], Yg[SAMPLE], p, gabs)
    say(f"   lockstep max|dX|={dx:.3e} max|dY|={dy:.3e} excluded={namb}")
    assert dx <= p["alpha"] * gabs + 2e-6 and dy <= 1e-5
    # exact objectives of all 1024 rounded restarts, bit for bit
    F = ctx.objectives()
    assert np.array_equal(F, oq.objective(q, Xg > 0.5))
    r = ctx.result()
    assert r["best_obj"] == F.min() and r["best_iter"] == 1 and r["best_restart"] == int(np.argmin(F))
    assert r["best_obj"] == oq.objective(q, r["best_x"][None])[0]
    # two more iterations from the GPU's own iterate: these gradient products
    # read the operand shadow the step epilogue wrote
    for step in (2, 3):
        Xs, Ys = Xg[SAMPLE].astype(np.float64), Yg[SAMPLE].astype(np.float64)
        ctx.step(1)
        Xg, Yg, t = ctx.get_state()
        assert t == step
        G64 = (Xs @ A + cp[None, :]) / s
        gabs = GTOL[prec] * float(np.max(np.abs(G64))) + 1e-6
        dx, dy, namb, _, _ = lockstep_compare(Xs, Ys, G64, Xg[SAMPLE], Yg[SAMPLE], p, gabs)
        say(f"   t={step} lockstep max|dX|={dx:.3e} max|dY|={dy:.3e} excluded={namb}")
        assert dx <= p["alpha"] * gabs + 2e-6 and dy <= 1e-5
        assert namb <= amb_limit(prec, Xs.size)
        assert np.array_equal(ctx.objectives(), oq.objective(q, Xg > 0.5))


def test_c5_maxsat_n20000_m84000_B256():
    P = require_gpu()
    f = W.maxsat_c5(0)
    s = W.maxsat_scale(f)
    B = 256
    x0 = W.x0_uniform(5, 0, B, f.n)
    p = W.gda_params("maxsat", B=B, T=1, scale=s)
    say(f"[fullsize c5] n={f.n} m={f.m} B={B}")
    ctx = P.maxsat_gda_init(f, p, x0)
    X = x0.astype(np.float32)
    G = ctx.grad(X)
    smp = [0, 1, 128, 255]
    G64 = om.grad_f(f, X[smp].astype(np.float64), s)
    assert np.max(np.abs(G[smp] - G64)) / np.max(np.abs(G64)) <= 1e-5
    ctx.step(1)
    Xg, Yg, _ = ctx.get_state()
    gabs = 1e-5 * float(np.max(np.abs(G64))) + 1e-6
    Xs = X[smp].astype(np.float64)
    dx, dy, namb, _, _ = lockstep_compare(Xs, np.full_like(Xs, p["y0"]), G64, Xg[smp],
                                          Yg[smp], p, gabs)
    say(f"   lockstep max|dX|={dx:.3e} max|dY|={dy:.3e} excluded={namb}")
    assert dx <= p["alpha"] * (gabs + 1e-5) + 2e-6 and dy <= 1e-5
    assert np.array_equal(ctx.objectives(), om.objective(f, Xg > 0.5))


def test_c4_batch_64_instances():
    P = require_gpu()
    qs = W.batch_c4(0)
    B, T = 128, 20
    ps = [W.gda_params("qubo", B=B, T=T, scale=W.qubo_scale(q), precision="bf16") for q in qs]
    x0s = [W.x0_uniform(4, 0, B, q.n, i) for i, q in enumerate(qs)]
    say(f"[fullsize c4] 64 instances, n in [{min(q.n for q in qs)}, {max(q.n for q in qs)}], B={B}")
    rg = P.qubo_gda_batch_solve(qs, ps, x0s, T, grouped=True)
    ri = P.qubo_gda_batch_solve(qs, ps, x0s, T, grouped=False)
    for i, q in enumerate(qs):
        assert (rg[i]["best_obj"], rg[i]["best_iter"], rg[i]["best_restart"]) == \
            (ri[i]["best_obj"], ri[i]["best_iter"], ri[i]["best_restart"])
        assert rg[i]["best_obj"] == oq.objective(q, rg[i]["best_x"][None])[0]


@pytest.mark.parametrize("full_iters", ["0", "64"])
def test_dense_n13000_objectives_multi_pass(full_iters, monkeypatch):
    """Rows longer than one pass of the incremental kernel (n = 13,000: each
    thread holds three 16-byte chunks of a row, 12,288 bytes per pass): with
    the evaluation GEMM kept (64) the incremental differences run over two
    passes once few coordinates change; with 0 every restart is evaluated by
    rows over two passes.  Objectives of every step against the oracle."""
    P = require_gpu()
    monkeypatch.setenv("PDBO_FULL_EVAL_ITERS", full_iters)
    n, B = 13000, 8
    q = W.random_dense_qubo(n, -50, 50, W.rng_for(8, 0, 0, n))
    s = W.qubo_scale(q)
    x0 = W.x0_uniform(8, 0, B, n)
    p = W.gda_params("qubo", B=B, T=40, scale=s, precision="i8")
    steps = 40 if full_iters == "64" else 3
    say(f"[fullsize multi-pass] n={n} B={B} transient={full_iters} steps={steps}")
    ctx = P.qubo_gda_init(q, p, x0)
    xs, Fs = [], []
    for _ in range(steps):
        ctx.step(1)
        Xg, _, _ = ctx.get_state()
        xs.append(Xg > 0.5)
        Fs.append(ctx.objectives())
    X = np.concatenate(xs)
    assert np.array_equal(np.concatenate(Fs), oq.objective(q, X))
    if full_iters == "64":
        k = np.sum(xs[-1] != xs[-2], axis=1)
        few = sum(int(np.sum((np.sum(a != b, axis=1) >= 1) & (np.sum(a != b, axis=1) <= 32)))
                  for a, b in zip(xs[1:], xs[:-1]))
        say(f"   (restart, step) pairs with 1..32 changes {few}; last step {k.tolist()}")
        assert few > 0
    r = ctx.result()
    assert r["best_obj"] == oq.objective(q, r["best_x"][None])[0]
