"""The dual certificate (App. D, Dual Certificate) through the C ABI: projected
descent on L(., ybar 1) in the context's own kernels, then the float64 bound
with rounding control, against the oracle's bound at the same point, the
oracle's descent, brute force, and the incumbent of a run."""
import numpy as np
import pytest

import workloads as W
from gpu_util import require_gpu, say
from oracle import dual
from oracle import enumerate as en
from oracle import qubo as oq

pytestmark = pytest.mark.gpu


def _check_at_point(q, s, ybar, r):
    prob = oq.QuboProblem(q, s)
    lb_o, val_o, gap_o = dual.certificate(prob, r["x"].astype(np.float64), ybar)
    say(f"   bound {r['lower_bound']:.6f} (oracle at the same x {lb_o:.6f}), s L(x) {r['value']:.6f}, "
        f"gap {r['gap']:.3e}, rounding bound {r['rounding']:.3e}")
    assert r["lower_bound"] <= lb_o + 1e-12 * max(1.0, abs(lb_o))
    assert lb_o - r["lower_bound"] <= 2 * r["rounding"] + 1e-9 * max(1.0, abs(lb_o))
    assert abs(r["value"] - val_o) <= 1e-9 * max(1.0, abs(val_o)) + r["rounding"]
    return prob, lb_o


@pytest.mark.parametrize("prec", ["fp32", "bf16", "i8"])
def test_dense_small_brute_force(prec):
    P = require_gpu()
    n = 14
    q = W.random_dense_qubo(n, -20, 20, np.random.default_rng(40 + n))
    s = 3.0
    A, _ = oq.canonicalize(q)
    ev = np.linalg.eigvalsh(A / s)
    ybar = 1.5 * (-ev.min() / 2) + 0.1
    L = ev.max() + 2 * ybar
    p = W.gda_params("qubo", B=8, T=1, scale=s, precision=prec, alpha=1.0 / L, y0=ybar)
    ctx = P.qubo_gda_init(q, p, W.x0_uniform(3, 50, 8, n))
    say(f"[dual dense n={n}] prec={prec} ybar={ybar:.3f}")
    r = P.qubo_dual_bound(ctx, iters=3000)
    prob, _ = _check_at_point(q, s, ybar, r)
    Fstar, _ = en.brute_force(lambda Xb: oq.objective(q, Xb), n)
    assert r["lower_bound"] <= Fstar
    xo = dual.projected_descent(prob, ybar, p["alpha"], 3000)
    tol = 1e-5 if prec == "fp32" else 2e-2
    say(f"   max|x - x_oracle| {np.max(np.abs(r['x'] - xo)):.3e}, brute-force min F {Fstar}")
    assert np.max(np.abs(r["x"] - xo)) <= tol
    if prec == "fp32":
        assert r["gap"] <= 1e-6 * max(1.0, abs(r["value"]))
    ctx.destroy()


def test_dense_n2000_against_run():
    P = require_gpu()
    n, B = 2000, 64
    q = W.random_dense_qubo(n, -100, 100, W.rng_for(3, 51, 0, n))
    s = W.qubo_scale(q)
    p = W.gda_params("qubo", B=B, T=1, scale=s, precision="bf16")
    ctx = P.qubo_gda_init(q, p, W.x0_uniform(3, 51, B, n))
    ctx.step(300)
    best = ctx.result()["best_obj"]
    say(f"[dual dense n={n}] s={s:.2f} ybar={p['y0']}")
    r = P.qubo_dual_bound(ctx, iters=400)
    _check_at_point(q, s, p["y0"], r)
    assert r["lower_bound"] <= best
    X, _, t = ctx.get_state()
    assert t == 300  # the run is untouched
    ctx.step(10)
    assert ctx.result()["best_obj"] <= best
    say(f"   incumbent {best}, lower bound {r['lower_bound']:.1f}")
    ctx.destroy()


@pytest.mark.parametrize("tile", [1, 2])
def test_csr_maxcut_and_mis(tile):
    P = require_gpu()
    for q, B, s in ((W.maxcut_c2(0), 256, 1.0), (W.mis_qubo(10000, 3, 0), 10, None)):
        s = W.qubo_scale(q) if s is None else s
        p = W.gda_params("maxcut", B=B, T=1, scale=s, tile=tile)
        ctx = P.qubo_gda_init(q, p, W.x0_uniform(2, 52, B, q.n))
        ctx.step(200)
        best = ctx.result()["best_obj"]
        say(f"[dual csr tile={tile}] {q.name} n={q.n} s={s:.3f}")
        r = P.qubo_dual_bound(ctx, iters=400)
        _check_at_point(q, s, p["y0"], r)
        assert r["lower_bound"] <= best
        say(f"   incumbent {best}, lower bound {r['lower_bound']:.2f}")
        ctx.destroy()
