"""Dense QUBOs whose canonical couplings leave the int8 range (Eq. 1 allows
any integer Q): the exact evaluation multiplies Ahat = sum_l 256^l Ahat_l one
int8 limb at a time and combines the limbs in int64, in the evaluation GEMM,
the incremental kernel and the by-rows evaluation.  Objectives bit-exact with
the oracle's int64 evaluation of the original (Q, c); gradient within the
form's tolerance."""
import numpy as np
import pytest

import workloads as W
from gpu_util import normwise, require_gpu, say
from oracle import qubo as oq

pytestmark = pytest.mark.gpu

# asymmetric Q makes A = offdiag(Q + Q^T) odd somewhere (kappa = 1)
CASES = {
    "asym_u100_n517": (lambda: W.random_asym_qubo(517, -100, 100, W.rng_for(3, 20, 0, 517)), 2),
    "sym_u2000_n600": (lambda: W.random_dense_qubo(600, -2000, 2000, W.rng_for(3, 21, 0, 600)), 2),
    "asym_u2000_n300": (lambda: W.random_asym_qubo(300, -2000, 2000, W.rng_for(3, 22, 0, 300)), 2),
    "asym_u40000_n257": (lambda: W.random_asym_qubo(257, -40000, 40000, W.rng_for(3, 23, 0, 257)), 3),
}
GTOL = {"fp32": 1e-5, "bf16": 1e-2, "fp8": 1e-1}


def _limbs(q):
    A, _ = oq.canonicalize(q)
    kappa = 2 if np.all(A.astype(np.int64) % 2 == 0) else 1
    amax = int(np.max(np.abs(A))) // kappa
    L = 1
    while amax > 127 * ((256 ** L - 1) // 255):
        L += 1
    return L


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("name", list(CASES))
def test_wide_eval_and_gradient(name, prec):
    P = require_gpu()
    make, L = CASES[name]
    q = make()
    assert _limbs(q) == L  # the case reaches the intended number of limbs
    B = 70
    s = W.qubo_scale(q)
    p = W.gda_params("qubo", B=B, T=1, scale=s, precision=prec)
    say(f"[wide eval] {name} prec={prec} limbs={L}")
    ctx = P.qubo_gda_init(q, p, W.x0_uniform(3, 20, B, q.n))
    xr = np.random.default_rng(5).integers(0, 2, size=(B, q.n), dtype=np.uint8)
    xr[0] = 1
    xr[1] = 0
    assert np.array_equal(ctx.eval(xr), oq.objective(q, xr.astype(bool)))
    A, cp = oq.canonicalize(q)
    X = np.random.default_rng(6).random((B, q.n)).astype(np.float32)
    G64 = oq.grad_f(A, cp, X.astype(np.float64), s)
    err = normwise(ctx.grad(X), G64)
    say(f"   gradient normwise error {err:.3e}")
    assert err <= GTOL[prec]
    ctx.destroy()


@pytest.mark.parametrize("full_iters", ["64", "0"])
@pytest.mark.parametrize("name", list(CASES))
def test_wide_objectives_every_step(name, full_iters, monkeypatch):
    """Every step's objectives (evaluation GEMM in the transient then the
    incremental differences; with the transient at 0, the by-rows evaluation
    for restarts with many changes) equal the oracle's."""
    P = require_gpu()
    monkeypatch.setenv("PDBO_FULL_EVAL_ITERS", full_iters)
    q = CASES[name][0]()
    B = 96
    p = W.gda_params("qubo", B=B, T=1, scale=W.qubo_scale(q), precision="bf16")
    say(f"[wide steps] {name} transient={full_iters}")
    ctx = P.qubo_gda_init(q, p, W.x0_uniform(3, 21, B, q.n))
    prev = None
    few = many = 0
    for t in range(40):
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
    ctx.destroy()


def test_wide_int8_form_rejected():
    P = require_gpu()
    q = CASES["asym_u100_n517"][0]()
    p = W.gda_params("qubo", B=8, T=1, scale=10.0, precision="i8")
    with pytest.raises(P.PdboError) as ei:
        P.qubo_gda_init(q, p, W.x0_uniform(3, 20, 8, q.n))
    assert ei.value.status == 6
