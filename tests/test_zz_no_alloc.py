"""qubo_gda_eval_noalloc, the evaluation entry point that allocates nothing,
against qubo_gda_eval on the same contexts and vectors (bit-exact int64), on
two calls in a row with the second smaller, through the C ABI; and its size
limit.  Runs on its own and after the other GPU tests."""
import numpy as np
import pytest

import workloads as W
from gpu_util import require_gpu, say
from oracle import maxsat as om
from oracle import qubo as oq

pytestmark = pytest.mark.gpu


def _vectors(rng, nb, n):
    # arbitrary bytes: the no-alloc entry point counts any nonzero byte as 1
    raw = rng.integers(0, 4, size=(nb, n), dtype=np.uint8)
    raw[0] = 0
    if nb > 1:
        raw[1] = 3
    return raw, (raw != 0).astype(np.uint8)


def _both(P, ctx, raw, bits):
    import torch
    xr = torch.from_numpy(raw).cuda()
    F = torch.full((raw.shape[0],), -7, dtype=torch.int64, device="cuda")
    P.qubo_gda_eval_noalloc(ctx, xr, F)
    torch.cuda.synchronize()
    return F.cpu().numpy(), ctx.eval(bits)


@pytest.mark.parametrize("prec", ["i8", "bf16", "fp32"])
def test_noalloc_dense_matches_eval(prec):
    P = require_gpu()
    n, B = 517, 300
    q = W.random_dense_qubo(n, -100, 100, W.rng_for(3, 9, 0, n))
    p = W.gda_params("qubo", B=B, T=1, scale=W.qubo_scale(q), precision=prec)
    ctx = P.qubo_gda_init(q, p, W.x0_uniform(3, 9, B, n))
    ctx.step(3)  # the context's own buffers hold a run; the scratch is separate
    rng = np.random.default_rng(11)
    for nb in (B, 37):
        say(f"[noalloc dense] prec={prec} n={n} nb={nb}")
        raw, bits = _vectors(rng, nb, n)
        Fn, Fe = _both(P, ctx, raw, bits)
        assert np.array_equal(Fn, Fe), nb
        assert np.array_equal(Fn, oq.objective(q, bits.astype(bool))), nb
    ctx.destroy()


def test_noalloc_sparse_and_maxsat_match_eval():
    P = require_gpu()
    rng = np.random.default_rng(12)
    q = W.maxcut_c2(0, n=301, M=900)
    ctx = P.qubo_gda_init(q, W.gda_params("maxcut", B=64, T=1), W.x0_uniform(2, 3, 64, q.n))
    for nb in (64, 5):
        say(f"[noalloc csr] n={q.n} nb={nb}")
        raw, bits = _vectors(rng, nb, q.n)
        Fn, Fe = _both(P, ctx, raw, bits)
        assert np.array_equal(Fn, Fe) and np.array_equal(Fn, oq.objective(q, bits.astype(bool)))
    ctx.destroy()
    f = W.random_maxsat(700, 2900, 3, 1, 10, W.rng_for(5, 7, 0))
    ctx = P.maxsat_gda_init(f, W.gda_params("maxsat", B=32, T=1, scale=W.maxsat_scale(f)),
                            W.x0_uniform(5, 7, 32, f.n))
    for nb in (32, 3):
        say(f"[noalloc maxsat] n={f.n} nb={nb}")
        raw, bits = _vectors(rng, nb, f.n)
        Fn, Fe = _both(P, ctx, raw, bits)
        assert np.array_equal(Fn, Fe) and np.array_equal(Fn, om.objective(f, bits.astype(bool)))
    ctx.destroy()


def test_noalloc_size_limit():
    """nb * ld + 16 nb + 512 bytes beyond the 16 MiB scratch: PDBO_EUNSUPPORTED,
    raised on the host before any launch."""
    import torch
    P = require_gpu()
    n, B = 13000, 1300  # ld = 13056: 1300 rows need 16.99e6 bytes > 16 MiB
    q = W.random_dense_qubo(n, -3, 3, W.rng_for(3, 10, 0, n))
    # tile 7 (160x256, DMA) given, so that no autotuning runs at this size
    p = W.gda_params("qubo", B=B, T=1, scale=1000.0, precision="i8", tile=7)
    say(f"[noalloc limit] n={n} B={B}")
    ctx = P.qubo_gda_init(q, p, W.x0_uniform(3, 10, B, n))
    xr = torch.zeros((B, n), dtype=torch.uint8, device="cuda")
    F = torch.zeros(B, dtype=torch.int64, device="cuda")
    with pytest.raises(P.PdboError) as ei:
        P.qubo_gda_eval_noalloc(ctx, xr, F)
    assert ei.value.status == 6
    # 1000 rows fit: the same call with fewer rows runs
    bits = np.random.default_rng(13).integers(0, 2, size=(1000, n), dtype=np.uint8)
    Fn, Fe = _both(P, ctx, bits, bits)
    assert np.array_equal(Fn, Fe)
    ctx.destroy()
