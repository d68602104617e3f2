"""CSR persistent path on the GPU against the oracle."""
import numpy as np
import pytest

import workloads as W
from gpu_util import lockstep_compare, normwise, require_gpu, say
from oracle import gda
from oracle import qubo as oq

pytestmark = pytest.mark.gpu


def _wide_weights(n=900, M=4000, seed=0):
    """A CSR QUBO with weights beyond int8 and an asymmetric part plus diagonal,
    which takes the int32 (non-compact) storage."""
    g = np.random.default_rng(seed)
    base = W.maxcut_c2(rep=seed, n=n, M=M)
    vals = g.integers(-900, 901, size=base.vals.shape[0]).astype(np.int32)
    rows = np.repeat(np.arange(n), np.diff(base.row_ptr))
    # add diagonal entries to some rows
    Qd = np.zeros((n, n), np.int64)
    Qd[rows, base.col_idx] = vals
    di = g.choice(n, n // 5, replace=False)
    Qd[di, di] = g.integers(-50, 51, size=di.size)
    import scipy.sparse as sp
    S = sp.csr_matrix(Qd)
    S.sort_indices()
    return W.Qubo(n=n, row_ptr=S.indptr.astype(np.int32), col_idx=S.indices.astype(np.int32),
                  vals=S.data.astype(np.int32), c=g.integers(-100, 101, n).astype(np.int64))


def _big_weights(n=700, M=2100, seed=5, mag=1 << 20):
    """Weights and linear terms up to 2^20 in magnitude: a wave's partial sums of
    the exact objective no longer fit in 32 bits, so the kernel keeps them in
    int64 (the per-row sums still fit in int32)."""
    base = W.maxcut_c2(rep=seed, n=n, M=M)
    g = np.random.default_rng(seed)
    vals = (g.integers(1, mag, size=base.vals.shape[0]) * np.sign(base.vals)).astype(np.int32)
    return W.Qubo(n=n, row_ptr=base.row_ptr, col_idx=base.col_idx, vals=vals,
                  c=g.integers(-mag, mag, n).astype(np.int64))


def _l2_weights(n=2000, M=6000, seed=6, mag=1 << 17):
    """Weights up to 2^17: beyond the 16-bit packed entries and too large for
    the wide-entry kernel's int32 totals, but with int32 wave sums."""
    base = W.maxcut_c2(rep=seed, n=n, M=M)
    g = np.random.default_rng(seed)
    vals = (g.integers(1, mag, size=base.vals.shape[0]) * np.sign(base.vals)).astype(np.int32)
    return W.Qubo(n=n, row_ptr=base.row_ptr, col_idx=base.col_idx, vals=vals,
                  c=g.integers(-mag, mag, n).astype(np.int64))


def _hub_weights(n=2000, M=6000, seed=7, hub=70, w=32001):
    """The C2-style graph plus one row with `hub` entries of weight w: packed
    16-bit entries still apply and a wave's partial sums fit in 32 bits, but n
    times the heaviest row does not, so the sum over waves runs in int64."""
    import scipy.sparse as sp
    base = W.maxcut_c2(rep=seed, n=n, M=M)
    rows = np.repeat(np.arange(n), np.diff(base.row_ptr))
    g = np.random.default_rng(seed)
    nb = g.choice(np.arange(1, n), hub, replace=False)
    r = np.concatenate([rows, np.zeros(hub, np.int64)])
    c = np.concatenate([base.col_idx, nb])
    v = np.concatenate([base.vals, np.full(hub, w)]).astype(np.int64)
    S = sp.csr_matrix((v, (r, c)), shape=(n, n))
    S.sum_duplicates()
    S.sort_indices()
    return W.Qubo(n=n, row_ptr=S.indptr.astype(np.int32), col_idx=S.indices.astype(np.int32),
                  vals=S.data.astype(np.int32), c=g.integers(-100, 101, n).astype(np.int64))


# Each case reaches a different variant of the persistent kernel (VARIANT):
#   n2000        packed 16-bit entries in LDS, interleaved by slices of 64 rows
#                (a wave's reads of entry r hit consecutive words), x
#                double-buffered, int32 wave sums and int32 totals over the waves
#   n301         the same in CSR order (the slices' padding would take more LDS
#                than row_ptr), one row per thread, ragged last wave
#   wide_n900    interleaved, with weights up to ~1800, an asymmetric part and a diagonal
#   n4000        interleaved, four rows per thread
#   hub_n2000    packed entries in CSR order (one heavy row), int32 wave sums, int64 totals
#   l2_n2000     int32 column/value arrays read through L2 (weights beyond 16 bits)
#   big_n700     the same with int64 wave sums
#   l2t_n2000    +-1 weights with too many entries for LDS: CSR through L2, int32
#                wave sums and int32 totals
#   n8000        interleaved packed entries in LDS, no room for a second x buffer
#                (by the CSR-order size): x updated in place
#   n12000       more than 8192 rows: 512 threads with 32 rows each, CSR through L2
CASES = {
    "maxcut_n2000": (lambda: W.maxcut_c2(0), 256, 1.0),
    "maxcut_n301_ragged": (lambda: W.maxcut_c2(1, n=301, M=900), 37, 1.0),
    "wide_n900": (lambda: _wide_weights(), 20, None),
    "maxcut_n4000_packed": (lambda: W.maxcut_c2(5, n=4000, M=8000), 24, 1.0),
    "hub_n2000": (lambda: _hub_weights(), 16, None),
    "l2_n2000": (lambda: _l2_weights(), 16, None),
    "big_n700": (lambda: _big_weights(), 24, None),
    "l2t_n2000": (lambda: W.maxcut_c2(6, n=2000, M=30000), 20, 1.0),
    "maxcut_n8000_inplace": (lambda: W.maxcut_c2(4, n=8000, M=8000), 24, 1.0),
    "maxcut_n12000_rows32": (lambda: W.maxcut_c2(3, n=12000, M=36000), 16, 1.0),
}
VARIANT = {
    "maxcut_n2000": "csr_sliced_dbuf_t32",
    "maxcut_n301_ragged": "csr_packed_dbuf_t32",
    "wide_n900": "csr_sliced_dbuf_t32",
    "maxcut_n4000_packed": "csr_sliced_dbuf_t32",
    "hub_n2000": "csr_packed_dbuf_i32",
    "l2_n2000": "csr_l2_dbuf_i32",
    "big_n700": "csr_l2_dbuf_i64",
    "l2t_n2000": "csr_l2_dbuf_t32",
    "maxcut_n8000_inplace": "csr_sliced_inplace_i32",
    "maxcut_n12000_rows32": "csr_l2_rows32",
}


@pytest.mark.parametrize("name", list(CASES))
def test_gradient_and_lockstep(name):
    P = require_gpu()
    mk, B, s = CASES[name]
    q = mk()
    s = W.qubo_scale(q) if s is None else s
    say(f"[csr lockstep] case={name} n={q.n} B={B}")
    g = np.random.default_rng(2)
    X = g.random((B, q.n)).astype(np.float32)
    X[:, ::9] = 0.5
    Y = g.uniform(-2.0, 6.0, (B, q.n)).astype(np.float32)
    # tile 1: the restart-resident kernel even for the few restarts of a test
    # (automatic routing sends B < 128 to the row-parallel path)
    p = W.gda_params("maxcut", B=B, T=1, scale=s, tile=1)
    ctx = P.qubo_gda_init(q, p, X.astype(np.float64))
    assert ctx.tile_name == VARIANT[name]
    G64 = oq.grad_f(*oq.canonicalize(q), X.astype(np.float64), s)
    G = ctx.grad(X)
    assert normwise(G, G64) <= 1e-5
    ctx.set_state(X, Y, 0)
    ctx.step(1)
    Xg, Yg, t = ctx.get_state()
    gabs = 1e-5 * float(np.max(np.abs(G64))) + 1e-6
    dx, dy, namb, _, _ = lockstep_compare(X.astype(np.float64), Y.astype(np.float64), G64, Xg, Yg, p, gabs)
    say(f"   max|dX|={dx:.3e} max|dY|={dy:.3e} excluded={namb}/{X.size}")
    assert dx <= p["alpha"] * gabs + 2e-6 and dy <= 2e-6 * 7
    assert namb <= 0.2 * X.size
    # the objective of round(x^1) is fused into the persistent kernel: bit-exact
    assert np.array_equal(ctx.objectives(), oq.objective(q, Xg > 0.5))


@pytest.mark.parametrize("name", ["maxcut_n2000", "maxcut_n301_ragged", "hub_n2000", "l2t_n2000",
                                  "maxcut_n8000_inplace", "maxcut_n12000_rows32"])
def test_lockstep_entropy_g(name):
    """The persistent kernel's variant for the entropy g (the Max-Cut workloads
    use the quadratic one): one iteration against the oracle, with x at 0, 1/2
    and 1."""
    P = require_gpu()
    mk, B, s = CASES[name]
    q = mk()
    s = W.qubo_scale(q) if s is None else s
    say(f"[csr lockstep entropy] case={name} n={q.n} B={B}")
    g = np.random.default_rng(8)
    X = g.random((B, q.n)).astype(np.float32)
    X[:, ::9] = 0.5
    X[:, 4::13] = 0.0
    X[:, 7::17] = 1.0
    Y = g.uniform(-2.0, 6.0, (B, q.n)).astype(np.float32)
    p = W.gda_params("maxcut", B=B, T=1, scale=s, g="entropy", tile=1)
    ctx = P.qubo_gda_init(q, p, X.astype(np.float64))
    assert ctx.tile_name == VARIANT[name]
    ctx.set_state(X, Y, 0)
    ctx.step(1)
    Xg, Yg, t = ctx.get_state()
    assert t == 1
    G64 = oq.grad_f(*oq.canonicalize(q), X.astype(np.float64), s)
    # float32 logarithms of g' near the clip: up to |y| * 2e-6 in dL
    gabs = 1e-5 * float(np.max(np.abs(G64))) + 2e-6 * float(np.max(np.abs(Y))) + 1e-6
    dx, dy, namb, _, _ = lockstep_compare(X.astype(np.float64), Y.astype(np.float64), G64, Xg, Yg, p, gabs)
    say(f"   max|dX|={dx:.3e} max|dY|={dy:.3e} excluded={namb}/{X.size}")
    assert dx <= p["alpha"] * gabs + 2e-6 and dy <= 2e-6 * 7
    assert namb <= 0.2 * X.size
    assert np.array_equal(ctx.objectives(), oq.objective(q, Xg > 0.5))


@pytest.mark.parametrize("name", list(CASES))
def test_eval_exact(name):
    P = require_gpu()
    mk, B, s = CASES[name]
    q = mk()
    ctx = P.qubo_gda_init(q, W.gda_params("maxcut", B=B, T=1, scale=1.0, tile=1),
                          W.x0_uniform(2, 3, B, q.n))
    assert ctx.tile_name == VARIANT[name]
    g = np.random.default_rng(4)
    xr = (g.random((B, q.n)) < 0.5).astype(np.uint8)
    assert np.array_equal(ctx.eval(xr), oq.objective(q, xr))


def test_full_c2_run_invariants_and_split_launches():
    P = require_gpu()
    q = W.maxcut_c2(0)
    B, T = 256, 5000
    x0 = W.x0_uniform(2, 0, B, q.n)
    p = W.gda_params("maxcut", B=B, T=T)
    say("[csr run] C2 n=2000 B=256 T=5000")
    ctx = P.qubo_gda_init(q, p, x0)
    ctx.step(T)
    X, Y, t = ctx.get_state()
    r = ctx.result()
    assert t == T and np.all((X >= 0) & (X <= 1)) and np.all(Y <= p["y0"])
    assert r["best_obj"] == oq.objective(q, r["best_x"][None])[0]
    # the same run split into uneven launches is bit-identical
    ctx2 = P.qubo_gda_init(q, p, x0)
    for k in (1, 999, 2000, 2000):
        ctx2.step(k)
    X2, Y2, _ = ctx2.get_state()
    r2 = ctx2.result()
    assert np.array_equal(X, X2) and np.array_equal(Y, Y2)
    assert (r2["best_obj"], r2["best_iter"], r2["best_restart"]) == (r["best_obj"], r["best_iter"], r["best_restart"])
    # quality against the oracle on a bounded sample of restarts and iterations
    ref = gda.run(oq.QuboProblem(q, 1.0), x0[:32], p, T=1000)
    say(f"   GPU best cut {-r['best_obj']} (t={r['best_iter']}); oracle 32 restarts x 1000 it: {-ref.inc.F}")
    assert r["best_obj"] <= ref.inc.F


def test_oracle_trajectory_short_horizon():
    """Over a few iterations the float32 trajectory tracks the float64 one."""
    P = require_gpu()
    q = W.maxcut_c2(1, n=301, M=900)
    B = 8
    x0 = W.x0_uniform(2, 1, B, q.n)
    p = W.gda_params("maxcut", B=B, T=5)
    ctx = P.qubo_gda_init(q, p, x0)
    ctx.step(5)
    X, Y, _ = ctx.get_state()
    ref = gda.run(oq.QuboProblem(q, 1.0), x0, p, T=5)
    assert np.max(np.abs(X - ref.X)) < 1e-4 and np.max(np.abs(Y - ref.Y)) < 1e-5


@pytest.mark.parametrize("name", ["maxcut_n2000", "wide_n900", "maxcut_n8000_inplace"])
def test_interleaved_layout_same_bits_as_csr_order(name, monkeypatch):
    """The interleaved entries (csr_sliced_*) run the same sums in the same order
    as the entries in CSR order: a run of 300 iterations ends in the same state
    and incumbent, bit for bit."""
    P = require_gpu()
    mk, B, s = CASES[name]
    q = mk()
    s = W.qubo_scale(q) if s is None else s
    p = W.gda_params("maxcut", B=B, T=300, scale=s, tile=1)
    x0 = W.x0_uniform(2, 9, B, q.n)
    say(f"[csr layouts] case={name} n={q.n} B={B}")
    out = []
    for sliced in ("1", "0"):
        monkeypatch.setenv("PDBO_CSR_SLICED", sliced)
        ctx = P.qubo_gda_init(q, p, x0)
        out.append(ctx.tile_name)
        ctx.step(300)
        out.append((ctx.get_state(), ctx.result()))
    assert out[0] == VARIANT[name] and out[2] == VARIANT[name].replace("sliced", "packed")
    (xa, ya, ta), ra = out[1]
    (xb, yb, tb), rb = out[3]
    assert ta == tb == 300 and np.array_equal(xa, xb) and np.array_equal(ya, yb)
    assert (ra["best_obj"], ra["best_restart"], ra["best_iter"]) == (rb["best_obj"], rb["best_restart"], rb["best_iter"])
    assert np.array_equal(ra["best_x"], rb["best_x"])
