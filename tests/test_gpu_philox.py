"""Starting points drawn by the library (x0 = NULL): Philox4x32-10 keyed by the
seed, mapped as pdbo.h states (App. C: x^0 uniform on [0,1]^n).  The iterate
after init equals the oracle's draw bit for bit, and a run from it equals the
run from the same points passed explicitly."""
import numpy as np
import pytest

import workloads as W
from gpu_util import require_gpu, say
from oracle.philox import x0_philox

pytestmark = pytest.mark.gpu

SEED = 0x5EED_0123_4567_89AB


def _check(P, make_ctx, n, B, y0):
    ref = x0_philox(SEED, B, n)
    ctx = make_ctx(None)
    X, Y, t = ctx.get_state()
    assert t == 0
    assert np.array_equal(X.astype(np.float64), ref)
    assert np.all(Y == np.float32(y0))
    ctx.step(25)
    r1 = ctx.result()
    ctx.restart(None)  # the same draw again
    X2, _, t2 = ctx.get_state()
    assert t2 == 0 and np.array_equal(X2, X)
    ctx.destroy()
    ctx = make_ctx(ref)
    ctx.step(25)
    r2 = ctx.result()
    assert (r1["best_obj"], r1["best_iter"], r1["best_restart"]) == \
        (r2["best_obj"], r2["best_iter"], r2["best_restart"])
    assert np.array_equal(r1["best_x"], r2["best_x"])
    ctx.destroy()


@pytest.mark.parametrize("prec", ["i8", "fp32"])
def test_philox_dense(prec):
    P = require_gpu()
    n, B = 301, 70
    q = W.random_dense_qubo(n, -50, 50, W.rng_for(3, 30, 0, n))
    p = W.gda_params("qubo", B=B, T=1, scale=W.qubo_scale(q), precision=prec, seed=SEED)
    say(f"[philox dense] prec={prec} n={n} B={B}")
    _check(P, lambda x0: P.qubo_gda_init(q, p, x0), n, B, p["y0"])


def test_philox_csr_and_maxsat():
    P = require_gpu()
    q = W.maxcut_c2(0, n=500, M=1500)
    p = W.gda_params("maxcut", B=40, T=1, seed=SEED)
    say("[philox csr]")
    _check(P, lambda x0: P.qubo_gda_init(q, p, x0), q.n, 40, p["y0"])
    f = W.random_maxsat(400, 1700, 3, 1, 10, W.rng_for(5, 30, 0))
    p = W.gda_params("maxsat", B=24, T=1, scale=W.maxsat_scale(f), seed=SEED)
    say("[philox maxsat]")
    _check(P, lambda x0: P.maxsat_gda_init(f, p, x0), f.n, 24, p["y0"])
