"""Per-instance choice between the dense and the CSR path for a large single
instance (n^2 B >= 2^30, tile 0, fp32 operands): the context that comes back
runs the path the timing picked, from the caller's starting point, and its run
is bit for bit that of a context built directly on that path."""
import json

import numpy as np
import pytest

import workloads as W
from gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu

N, B, T = 2048, 256, 300   # n^2 B = 2^30, the smallest size that is timed


def _csr_of(Q, c):
    """CSR of the nonzeros of a dense matrix, columns ascending in each row."""
    r, k = np.nonzero(Q)
    rp = np.zeros(Q.shape[0] + 1, np.int64)
    np.add.at(rp, r + 1, 1)
    return W.Qubo(n=Q.shape[0], row_ptr=np.cumsum(rp).astype(np.int32),
                  col_idx=k.astype(np.int32), vals=Q[r, k].astype(np.int32), c=c)


def _run(P, q, p, x0):
    ctx = P.qubo_gda_init(q, p, x0)
    P.qubo_gda_step(ctx, T)
    r = P.qubo_gda_result(ctx)
    x, y, t = P.qubo_gda_get_state(ctx)
    name = ctx.tile_name
    ctx.destroy()
    return name, r, x, y, t


def _same(a, b):
    assert a[1]["best_obj"] == b[1]["best_obj"]
    assert (a[1]["best_restart"], a[1]["best_iter"]) == (b[1]["best_restart"], b[1]["best_iter"])
    assert np.array_equal(a[1]["best_x"], b[1]["best_x"])
    assert a[4] == b[4] == T
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])


def _route_keys(path):
    with open(path) as f:
        return {k: v for k, v in json.load(f).items() if k.startswith("route/")}


@pytest.fixture
def cache(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("PDBO_AUTOTUNE_CACHE", str(path))
    monkeypatch.delenv("PDBO_ROUTE", raising=False)
    return path


def test_sparse_dense_matrix_runs_on_csr(cache, monkeypatch):
    """Max-Cut on G(n, 3n) handed over as a dense matrix: the CSR path is
    several times faster and takes the instance."""
    P = require_gpu()
    g = W.maxcut_c2(rep=3, n=N, M=3 * N)
    dense = W.Qubo(n=N, Q=g.dense(), c=g.c)
    p = W.gda_params("maxcut", B=B, T=T, precision="fp32")
    x0 = W.x0_uniform(2, 3, B, N)
    say("route dense->csr", N, B)
    routed = _run(P, dense, p, x0)
    assert routed[0].startswith("csr"), routed[0]
    keys = _route_keys(cache)
    assert list(keys.values()) == [1], keys
    monkeypatch.setenv("PDBO_ROUTE", "0")
    direct = _run(P, _csr_of(dense.Q, g.c), p, x0)
    _same(routed, direct)
    kept = _run(P, dense, p, x0)
    assert not kept[0].startswith("csr"), kept[0]
    monkeypatch.delenv("PDBO_ROUTE")
    again = _run(P, dense, p, x0)   # the cached choice, no timing
    _same(again, direct)


@pytest.mark.parametrize("gc", [0, 8])
def test_dense_csr_matrix_runs_dense(cache, monkeypatch, gc):
    """A QUBO with two thirds of its entries nonzero handed over as CSR: the
    dense path takes it.  x0 NULL: the generator's points of the seed.  With
    hipGraph chunks the timing iterations record a graph before the restart,
    and the replays after it must still match a fresh context."""
    P = require_gpu()
    q = W.random_dense_qubo(N, -1, 1, np.random.default_rng(11))
    csr = _csr_of(q.Q, q.c)
    p = W.gda_params("maxcut", B=B, T=T, precision="fp32", seed=77, graph_chunk=gc)
    say("route csr->dense", N, B, csr.col_idx.size, "graph_chunk", gc)
    routed = _run(P, csr, p, None)
    assert not routed[0].startswith("csr") and routed[0], routed[0]
    assert list(_route_keys(cache).values()) == [1]
    monkeypatch.setenv("PDBO_ROUTE", "0")
    direct = _run(P, q, p, None)
    _same(routed, direct)


def test_small_or_quantised_instances_are_not_routed(cache):
    """Below n^2 B = 2^30, or with int8 operands, the representation given is kept
    and nothing is timed."""
    P = require_gpu()
    g = W.maxcut_c2(rep=4, n=N, M=3 * N)
    dense = W.Qubo(n=N, Q=g.dense(), c=g.c)
    x0 = W.x0_uniform(2, 4, 128, N)
    ctx = P.qubo_gda_init(dense, W.gda_params("maxcut", B=128, T=T, precision="fp32"), x0)
    assert not ctx.tile_name.startswith("csr")
    ctx.destroy()
    ctx = P.qubo_gda_init(dense, W.gda_params("maxcut", B=B, T=T, precision="i8"),
                          W.x0_uniform(2, 4, B, N))
    assert not ctx.tile_name.startswith("csr")
    ctx.destroy()
    assert not cache.exists() or not _route_keys(cache)
