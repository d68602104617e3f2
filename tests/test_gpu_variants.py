"""Variants of Alg. 1 on the dense path, through the C ABI: the polynomial g
(2x - 1)^(2d) - 1 of Sec. 3.1 and the single-constraint dual (PDBO-s,
Sec. 4.5), each stepped from the GPU's own iterate and compared with the
oracle's iteration from the same state, with exact objectives every step."""
import numpy as np
import pytest

import workloads as W
from gpu_util import amb_limit, lockstep_compare, require_gpu, say
from oracle import gda
from oracle import qubo as oq

pytestmark = pytest.mark.gpu

GTOL = {"fp32": 1e-5, "bf16": 1e-2, "fp8": 1e-1, "i8": 1e-2}


def _multistep(P, q, p, x0, steps, prec):
    s = p["scale"]
    A, cp = oq.canonicalize(q)
    ctx = P.qubo_gda_init(q, p, x0)
    X, Y, _ = ctx.get_state()
    for step in range(1, steps + 1):
        ctx.step(1)
        Xn, Yn, t = ctx.get_state()
        assert t == step
        X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
        G64 = oq.grad_f(A, cp, X64, s)
        gabs = GTOL[prec] * float(np.max(np.abs(G64))) + 1e-6
        dx, dy, namb, _, _ = lockstep_compare(X64, Y64, G64, Xn, Yn, p, gabs)
        say(f"   t={step}: max|dX|={dx:.3e} max|dY|={dy:.3e} excluded={namb}")
        assert dx <= p["alpha"] * gabs + 2e-6
        assert dy <= 2e-6 * (1 + np.max(np.abs(Y64)))
        assert namb <= amb_limit(prec, X.size)
        assert np.all((Xn >= 0) & (Xn <= 1))
        assert np.array_equal(ctx.objectives(), oq.objective(q, Xn > 0.5)), step
        X, Y = Xn, Yn
    return ctx, X, Y


@pytest.mark.parametrize("deg", [1, 2, 3])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_poly_g_multistep(prec, deg):
    P = require_gpu()
    n, B = 517, 150
    q = W.random_dense_qubo(n, -100, 100, W.rng_for(3, 40, 0, n))
    p = W.gda_params("qubo", B=B, T=1, scale=W.qubo_scale(q), precision=prec, g="poly",
                     g_degree=deg, y0=0.01, beta=0.05)
    say(f"[poly g] d={deg} prec={prec}")
    ctx, X, Y = _multistep(P, q, p, W.x0_uniform(3, 40, B, n), 4, prec)
    assert np.any(Y <= 0), "the run never reached y <= 0"
    ctx.destroy()


@pytest.mark.parametrize("prec", ["fp32", "i8"])
def test_scalar_dual_multistep(prec):
    P = require_gpu()
    n, B = 517, 150
    q = W.random_dense_qubo(n, -100, 100, W.rng_for(3, 41, 0, n))
    # beta small enough that y = y0 + beta * sum_i g stays of order one
    p = W.gda_params("qubo", B=B, T=1, scale=W.qubo_scale(q), precision=prec, dual="scalar",
                     y0=0.5, beta=0.004)
    say(f"[scalar dual] prec={prec}")
    ctx, X, Y = _multistep(P, q, p, W.x0_uniform(3, 41, B, n), 5, prec)
    assert np.all(Y == Y[:, :1]), "one dual value per restart"
    assert np.any(Y[:, 0] <= 0), "the run never reached y <= 0"
    ctx.destroy()


def test_scalar_dual_fp32_trajectory_and_batch():
    """Five float32 iterations of the scalar-dual run track the float64
    oracle; a grouped batch of two instances equals the single runs bit for
    bit."""
    P = require_gpu()
    n, B = 300, 16
    q = W.random_dense_qubo(n, -100, 100, W.rng_for(3, 42, 0, n))
    s = W.qubo_scale(q)
    x0 = W.x0_uniform(3, 42, B, n)
    p = W.gda_params("qubo", B=B, T=5, scale=s, precision="fp32", dual="scalar", y0=0.5, beta=0.004)
    ctx = P.qubo_gda_init(q, p, x0)
    ctx.step(5)
    X, Y, _ = ctx.get_state()
    ref = gda.run(oq.QuboProblem(q, s), x0, p, T=5)
    dx = float(np.max(np.abs(X - ref.X)))
    dy = float(np.max(np.abs(Y[:, 0] - ref.Y[:, 0])))
    say(f"[scalar dual trajectory] max|dX|={dx:.3e} max|dy|={dy:.3e}")
    assert dx < 1e-4 and dy < 1e-5
    ctx.destroy()
    q2 = W.random_dense_qubo(211, -100, 100, W.rng_for(3, 43, 0, 211))
    qs = [q, q2]
    ps = [dict(p, scale=W.qubo_scale(x), T=40) for x in qs]
    x0s = [x0, W.x0_uniform(3, 43, B, 211)]
    rg = P.qubo_gda_batch_solve(qs, ps, x0s, 40, grouped=True)
    for i, qq in enumerate(qs):
        r = P.qubo_gda_solve(qq, ps[i], x0s[i], 40)
        assert (r["best_obj"], r["best_iter"]) == (rg[i]["best_obj"], rg[i]["best_iter"])
        assert r["best_obj"] == oq.objective(qq, r["best_x"][None])[0]


def test_variants_on_the_sparse_paths():
    """The restart-resident CSR and MaxSAT kernels take neither variant
    (EUNSUPPORTED); the row-parallel CSR path takes the polynomial g (chosen
    automatically for it), not the scalar dual."""
    P = require_gpu()
    q = W.maxcut_c2(0, n=300, M=900)
    x0 = W.x0_uniform(2, 4, 8, q.n)
    for over in (dict(g="poly", g_degree=2, tile=1), dict(dual="scalar", tile=1),
                 dict(dual="scalar", tile=2), dict(dual="scalar")):
        with pytest.raises(P.PdboError) as ei:
            P.qubo_gda_init(q, W.gda_params("maxcut", B=8, T=1, **over), x0)
        assert ei.value.status == 6, over
    f = W.random_maxsat(100, 400, 3, 1, 5, W.rng_for(5, 45, 0))
    with pytest.raises(P.PdboError) as ei:
        P.maxsat_gda_init(f, W.gda_params("maxsat", B=8, T=1, g="poly"), W.x0_uniform(5, 45, 8, 100))
    assert ei.value.status == 6
    p = W.gda_params("maxcut", B=8, T=1, g="poly", g_degree=2, y0=0.01, beta=0.05)
    ctx = P.qubo_gda_init(q, p, x0)
    A, cp = oq.canonicalize(q)
    X, Y, _ = ctx.get_state()
    for step in range(3):
        ctx.step(1)
        Xn, Yn, _ = ctx.get_state()
        G64 = oq.grad_f(A, cp, X.astype(np.float64), 1.0)
        gabs = 1e-5 * float(np.max(np.abs(G64))) + 1e-6
        dx, dy, namb, _, _ = lockstep_compare(X.astype(np.float64), Y.astype(np.float64), G64, Xn,
                                              Yn, p, gabs)
        assert dx <= p["alpha"] * gabs + 2e-6 and dy <= 2e-6 * (1 + np.max(np.abs(Y)))
        assert np.array_equal(ctx.objectives(), oq.objective(q, Xn > 0.5))
        X, Y = Xn, Yn
    ctx.destroy()


@pytest.mark.parametrize("kind", ["dense", "csr", "maxsat"])
def test_enomem_injection_frees_everything(kind, monkeypatch):
    """A device allocation failing part-way through init returns PDBO_ENOMEM
    and leaves no device memory behind; a later init succeeds."""
    import torch
    P = require_gpu()
    if kind == "dense":
        q = W.random_dense_qubo(300, -50, 50, W.rng_for(3, 44, 0, 300))
        mk = lambda: P.qubo_gda_init(q, W.gda_params("qubo", B=64, T=1, scale=50.0), None)
    elif kind == "csr":
        q = W.maxcut_c2(0, n=400, M=1200)
        mk = lambda: P.qubo_gda_init(q, W.gda_params("maxcut", B=32, T=1), None)
    else:
        f = W.random_maxsat(300, 1200, 3, 1, 10, W.rng_for(5, 44, 0))
        mk = lambda: P.maxsat_gda_init(f, W.gda_params("maxsat", B=16, T=1, scale=5.5), None)
    mk().destroy()  # modules loaded, caches warm
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    failures = 0
    for k in (1, 2, 3, 5, 8, 13, 21, 34):
        monkeypatch.setenv("PDBO_FAIL_ALLOC_AT", str(k))
        try:
            mk().destroy()
        except P.PdboError as e:
            assert e.status == 2, e
            failures += 1
        monkeypatch.setenv("PDBO_FAIL_ALLOC_AT", "0")
        free1 = torch.cuda.mem_get_info()[0]
        say(f"[enomem] {kind} k={k}: free {free0 - free1} bytes below the start")
        assert free1 >= free0 - (2 << 20), k
    assert failures >= 3
    mk().destroy()
