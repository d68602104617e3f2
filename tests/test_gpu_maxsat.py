"""Weighted MaxSAT path on the GPU: adjoint kernel, autograd.Function, fused
exact evaluation and the persistent solver, against the oracle."""
import numpy as np
import pytest

import workloads as W
from gpu_util import lockstep_compare, normwise, require_gpu, say
from oracle import gda
from oracle import maxsat as om
from oracle.binarity import Entropy

pytestmark = pytest.mark.gpu

# The larger cases reach the other variants of the persistent kernel: up to 8
# variables per thread in registers (n6000), up to 20 with y in LDS (n12345,
# and the general-k form n9001), and 512 threads with 64 variables each
# (n25000).
CASES = {
    "3sat_n500": (lambda: W.random_maxsat(500, 2100, 3, 1, 10, W.rng_for(5, 0, 0, 500, 2100)), 16),
    "4sat_n333": (lambda: W.random_maxsat(333, 2000, 4, 1, 10, W.rng_for(5, 1, 0, 333, 2000)), 7),
    "2sat_n65": (lambda: W.random_maxsat(65, 150, 2, 0, 3, W.rng_for(5, 2, 0, 65, 150)), 3),
    "3sat_n6000": (lambda: W.random_maxsat(6000, 25200, 3, 1, 10, W.rng_for(5, 3, 0, 6000, 25200)), 8),
    "3sat_n12345": (lambda: W.random_maxsat(12345, 51849, 3, 1, 10, W.rng_for(5, 4, 0, 12345, 51849)), 6),
    "4sat_n9001": (lambda: W.random_maxsat(9001, 80000, 4, 1, 10, W.rng_for(5, 5, 0, 9001, 80000)), 4),
    "3sat_n25000": (lambda: W.random_maxsat(25000, 105000, 3, 1, 10, W.rng_for(5, 6, 0, 25000, 105000)), 4),
}


@pytest.mark.parametrize("name", list(CASES))
def test_gradient_lockstep_eval(name):
    P = require_gpu()
    mk, B = CASES[name]
    f = mk()
    s = W.maxsat_scale(f)
    say(f"[sat lockstep] case={name} n={f.n} m={f.m} k={f.k} B={B}")
    g = np.random.default_rng(3)
    X = g.random((B, f.n)).astype(np.float32)
    X[:, ::13] = 0.0
    X[:, 5::17] = 1.0
    Y = g.uniform(-1.0, 2.0, (B, f.n)).astype(np.float32)
    p = W.gda_params("maxsat", B=B, T=1, scale=s)
    ctx = P.maxsat_gda_init(f, p, X.astype(np.float64))
    G64 = om.grad_f(f, X.astype(np.float64), s)
    assert normwise(ctx.grad(X), G64) <= 1e-5
    ctx.set_state(X, Y, 0)
    ctx.step(1)
    Xg, Yg, _ = ctx.get_state()
    gabs = 1e-5 * float(np.max(np.abs(G64))) + 1e-6
    dx, dy, namb, _, _ = lockstep_compare(X.astype(np.float64), Y.astype(np.float64), G64, Xg, Yg, p, gabs)
    say(f"   max|dX|={dx:.3e} max|dY|={dy:.3e} excluded={namb}/{X.size}")
    # entropy derivative near the clip adds up to |y| * 2e-6 of float32 log error
    assert dx <= p["alpha"] * (gabs + 4e-6 * 2) + 2e-6
    assert dy <= 1e-5
    assert np.array_equal(ctx.objectives(), om.objective(f, Xg > 0.5))
    xr = (g.random((B, f.n)) < 0.5).astype(np.uint8)
    assert np.array_equal(ctx.eval(xr), om.objective(f, xr))


@pytest.mark.parametrize("name", ["3sat_n500", "3sat_n6000", "3sat_n12345", "4sat_n9001"])
def test_lockstep_quadratic_g(name):
    """The persistent kernel's variant for the quadratic g (the MaxSAT workloads
    use the entropy one): one iteration against the oracle."""
    P = require_gpu()
    mk, B = CASES[name]
    f = mk()
    s = W.maxsat_scale(f)
    say(f"[sat lockstep quad] case={name} n={f.n} m={f.m} k={f.k} B={B}")
    g = np.random.default_rng(9)
    X = g.random((B, f.n)).astype(np.float32)
    X[:, ::11] = 0.5
    Y = g.uniform(-1.0, 2.0, (B, f.n)).astype(np.float32)
    p = W.gda_params("maxsat", B=B, T=1, scale=s, g="quad")
    ctx = P.maxsat_gda_init(f, p, X.astype(np.float64))
    ctx.set_state(X, Y, 0)
    ctx.step(1)
    Xg, Yg, _ = ctx.get_state()
    G64 = om.grad_f(f, X.astype(np.float64), s)
    gabs = 1e-5 * float(np.max(np.abs(G64))) + 1e-6
    dx, dy, namb, _, _ = lockstep_compare(X.astype(np.float64), Y.astype(np.float64), G64, Xg, Yg, p, gabs)
    say(f"   max|dX|={dx:.3e} max|dY|={dy:.3e} excluded={namb}/{X.size}")
    assert dx <= p["alpha"] * gabs + 2e-6
    assert dy <= 1e-5
    assert namb <= 0.2 * X.size
    assert np.array_equal(ctx.objectives(), om.objective(f, Xg > 0.5))


def test_autograd_function_against_oracle():
    P = require_gpu()
    import torch
    f = CASES["3sat_n500"][0]()
    s = W.maxsat_scale(f)
    B = 6
    ctx = P.maxsat_gda_init(f, W.gda_params("maxsat", B=B, T=1, scale=s), W.x0_uniform(5, 3, B, f.n))
    g = np.random.default_rng(9)
    X = g.random((B, f.n))
    Y = g.uniform(-1, 2, (B, f.n))
    x = torch.tensor(X, dtype=torch.float32, device="cuda", requires_grad=True)
    y = torch.tensor(Y, dtype=torch.float32, device="cuda", requires_grad=True)
    L = P.MaxSATLagrangian.apply(x, y, ctx)
    w = torch.arange(1, B + 1, dtype=torch.float32, device="cuda")
    (L * w).sum().backward()
    Xf, Yf = X.astype(np.float32).astype(np.float64), Y.astype(np.float32).astype(np.float64)
    ent = Entropy()
    L64 = om.f_multilinear(f, Xf) / s + np.sum(Yf * ent.value(Xf), axis=1)
    assert np.max(np.abs(L.detach().cpu().numpy() - L64) / (1 + np.abs(L64))) <= 1e-5
    dx64 = (om.grad_f(f, Xf, s) + Yf * ent.deriv(Xf)) * np.arange(1, B + 1)[:, None]
    dy64 = ent.value(Xf) * np.arange(1, B + 1)[:, None]
    assert normwise(x.grad.cpu().numpy(), dx64) <= 1e-5
    assert normwise(y.grad.cpu().numpy(), dy64) <= 1e-5
    # central finite differences of the float64 Lagrangian along a random direction
    v = g.standard_normal((B, f.n))
    h = 1e-6

    def Lf(Xe):
        return om.f_multilinear(f, Xe) / s + np.sum(Yf * ent.value(Xe), axis=1)
    fd = (Lf(Xf + h * v) - Lf(Xf - h * v)) / (2 * h)
    dd = np.sum(x.grad.cpu().numpy() / np.arange(1, B + 1)[:, None] * v, axis=1)
    assert np.max(np.abs(fd - dd) / (1 + np.abs(fd))) <= 1e-4


def test_persistent_run_invariants_and_quality():
    P = require_gpu()
    f = W.random_maxsat(2000, 8400, 3, 1, 10, W.rng_for(5, 0, 0, 2000, 8400))
    s = W.maxsat_scale(f)
    B, T = 64, 400
    x0 = W.x0_uniform(5, 0, B, f.n)
    p = W.gda_params("maxsat", B=B, T=T, scale=s)
    say("[sat run] n=2000 m=8400 B=64 T=400")
    ctx = P.maxsat_gda_init(f, p, x0)
    ctx.step(150)
    ctx.step(250)
    X, Y, t = ctx.get_state()
    r = ctx.result()
    assert t == T and np.all((X >= 0) & (X <= 1)) and np.all(Y <= p["y0"])
    assert r["best_obj"] == om.objective(f, r["best_x"][None])[0]
    ref = gda.run(om.MaxSatProblem(f, s), x0[:8], p, T=T)
    say(f"   GPU best unsat weight {r['best_obj']}; oracle (8 restarts) {ref.inc.F}")
    assert r["best_obj"] <= ref.inc.F * 1.02 + 5
