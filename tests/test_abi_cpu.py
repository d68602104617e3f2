"""The C ABI on the CPU: the library loads, exports exactly what include/pdbo.h
declares, the ctypes structs match the C layout, and contract violations are
rejected before any HIP call (no GPU needed)."""
import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

import workloads as W
from paper_2509_21064_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdbo.h")


def _declared():
    txt = open(HEADER).read()
    return set(re.findall(r"^PDBO_API\s+[\w\s\*]+?\b(\w+)\s*\(", txt, flags=re.M))


@pytest.fixture(scope="module")
def lib():
    return _abi.load()


def test_exports_match_header(lib):
    names = _declared()
    assert len(names) >= 20
    assert names == set(_abi.SIGNATURES), names ^ set(_abi.SIGNATURES)
    out = subprocess.run(["nm", "-D", "--defined-only", _abi.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert names <= exported
    # internal C++ symbols are hidden
    assert not [s for s in exported if s.startswith("_ZN4pdbo")]


def test_struct_layout_matches_c():
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "pdbo.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("pdbo_qubo %zu\npdbo_maxsat %zu\npdbo_params %zu\npdbo_result %zu\n",
         sizeof(pdbo_qubo), sizeof(pdbo_maxsat), sizeof(pdbo_params), sizeof(pdbo_result));
  P(pdbo_qubo, nnz) P(pdbo_qubo, c) P(pdbo_qubo, wtype) P(pdbo_qubo, qd) P(pdbo_qubo, cd)
  P(pdbo_result, best_obj_f64) P(pdbo_params, alpha) P(pdbo_params, scale)
  P(pdbo_params, tile) P(pdbo_params, x0) P(pdbo_params, g_degree) P(pdbo_params, dual_kind)
  P(pdbo_params, seed) P(pdbo_result, best_iter) P(pdbo_result, best_x)
  P(pdbo_maxsat, lits) P(pdbo_maxsat, w)
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    vals = dict(l.rsplit(" ", 1) for l in out.strip().splitlines())
    assert int(vals["pdbo_qubo"]) == ctypes.sizeof(_abi.pdbo_qubo)
    assert int(vals["pdbo_maxsat"]) == ctypes.sizeof(_abi.pdbo_maxsat)
    assert int(vals["pdbo_params"]) == ctypes.sizeof(_abi.pdbo_params)
    assert int(vals["pdbo_result"]) == ctypes.sizeof(_abi.pdbo_result)
    for key, v in vals.items():
        if "." in key:
            T, f = key.split(".")
            assert int(v) == getattr(getattr(_abi, T), f).offset, key


def test_status_strings(lib):
    for s in range(7):
        assert lib.pdbo_status_str(s)
    assert lib.pdbo_status_str(99) == b"unknown status"


def _init(lib, q, p, x0):
    import paper_2509_21064_amd as P
    keep = P._Keep()
    prob = P._qubo_struct(q, keep)
    par = P._params_struct(p, x0, keep)
    h = ctypes.c_void_p()
    st = lib.qubo_gda_init(ctypes.byref(prob), ctypes.byref(par), None, ctypes.byref(h))
    if st == 0:
        lib.pdbo_destroy(h)
    return st


def _base():
    q = W.qubo_c1(0, n=20)
    p = W.gda_params("maxcut", B=4, T=10)
    x0 = W.x0_uniform(1, 0, 4, 20, 20)
    return q, p, x0


@pytest.mark.parametrize("field,value", [
    ("B", 0), ("alpha", 0.0), ("beta", -1.0), ("y0", 0.0), ("delta", 0.5), ("delta", 0.0),
    ("scale", 0.0), ("alpha", float("nan")), ("eval_every", 0), ("graph_chunk", 3), ("tile", 99),
    ("g_degree", 0), ("g_degree", 17),
])
def test_invalid_params(lib, field, value):
    q, p, x0 = _base()
    p = dict(p)
    p[field] = value
    if field == "g_degree":
        p["g"] = "poly"
    if field == "B":
        x0 = x0[:0]
    assert _init(lib, q, p, x0) == _abi.PDBO_EINVAL


def test_invalid_x0(lib):
    q, p, x0 = _base()
    bad = x0.copy()
    bad[1, 3] = 1.5
    assert _init(lib, q, p, bad) == _abi.PDBO_EINVAL
    bad[1, 3] = float("nan")
    assert _init(lib, q, p, bad) == _abi.PDBO_EINVAL
    # no x0: the library draws the starting points (on the CPU the first
    # device allocation then fails)
    import torch
    if not torch.cuda.is_available():
        assert _init(lib, q, p, None) in (_abi.PDBO_EDEVICE, _abi.PDBO_ENOMEM)


def test_real_weights_rejected_before_the_device(lib):
    """Float64 weights: non-finite entries (EINVAL), an exponent span beyond
    the 192 bits of the exact evaluation (ERANGE), the restart-resident tile and
    batches (EUNSUPPORTED) are refused on the host."""
    import paper_2509_21064_amd as P
    _, p, _ = _base()
    n = 12
    g = np.random.default_rng(3)
    Q = g.standard_normal((n, n))
    x0 = W.x0_uniform(1, 0, 4, n, n)
    bad = Q.copy()
    bad[2, 3] = float("inf")
    assert _init(lib, W.Qubo(n=n, Q=bad), p, x0) == _abi.PDBO_EINVAL
    c = np.zeros(n)
    c[4] = float("nan")
    assert _init(lib, W.Qubo(n=n, Q=Q, c=c), p, x0) == _abi.PDBO_EINVAL
    wide = Q.copy()
    wide[0, 1] = 2.0 ** 100
    wide[5, 6] = 2.0 ** -100          # bits 100 .. -152: 253 bits
    assert _init(lib, W.Qubo(n=n, Q=wide), p, x0) == _abi.PDBO_ERANGE
    assert _init(lib, W.Qubo(n=n, Q=Q), dict(p, tile=1), x0) == _abi.PDBO_EUNSUPPORTED
    keep = P._Keep()
    probs = (_abi.pdbo_qubo * 1)(P._qubo_struct(W.Qubo(n=n, Q=Q), keep))
    pars = (_abi.pdbo_params * 1)(P._params_struct(p, x0, keep))
    h = ctypes.c_void_p()
    assert lib.qubo_gda_batch_init(1, probs, pars, 1, None, ctypes.byref(h)) == _abi.PDBO_EUNSUPPORTED


def test_invalid_csr(lib):
    _, p, _ = _base()
    q = W.maxcut_c2(0, n=30, M=60)
    x0 = W.x0_uniform(2, 0, 4, 30)
    for mutate in ("col_range", "dup", "rowptr"):
        qq = W.Qubo(n=q.n, row_ptr=q.row_ptr.copy(), col_idx=q.col_idx.copy(), vals=q.vals.copy(), c=q.c)
        if mutate == "col_range":
            qq.col_idx[5] = 30
        elif mutate == "dup":
            r = int(np.argmax(np.diff(qq.row_ptr) >= 2))
            qq.col_idx[qq.row_ptr[r] + 1] = qq.col_idx[qq.row_ptr[r]]
        else:
            qq.row_ptr[3], qq.row_ptr[4] = qq.row_ptr[4], qq.row_ptr[3] - 1
        assert _init(lib, qq, p, x0) == _abi.PDBO_EINVAL, mutate
    assert b"" != lib.pdbo_last_global_error()


def test_exactness_guard(lib):
    q, p, x0 = _base()
    Q = q.Q.copy()
    Q[2, 3] = 1 << 30
    assert _init(lib, W.Qubo(n=q.n, Q=Q, c=None), p, x0) == _abi.PDBO_ERANGE


def test_limb_range_guards(lib):
    """Dense: |Ahat_ij| beyond the four int8 limbs (2,139,062,143) is ERANGE,
    and a row of |Ahat| summing to 2^31 or more is ERANGE; the INT8 operand
    form with |Ahat_ij| > 127 is EUNSUPPORTED.  All decided on the host, before
    any HIP call, so on any machine."""
    q, p, x0 = _base()
    Q = q.Q.copy()
    Q[:] = 0
    # A_01 = Q_01 + Q_10 = 2^31 - 3, odd (kappa = 1): above the limb range,
    # while its row sum stays below 2^31
    Q[0, 1], Q[1, 0] = (1 << 30) - 1, (1 << 30) - 2
    assert _init(lib, W.Qubo(n=q.n, Q=Q, c=None), p, x0) == _abi.PDBO_ERANGE
    Q[:] = 0
    Q[0, 1:] = (1 << 30) - 1  # a row of |A| far above 2^31
    assert _init(lib, W.Qubo(n=q.n, Q=Q, c=None), p, x0) == _abi.PDBO_ERANGE
    Q[:] = 0
    Q[0, 1] = 201  # A_01 = 201: two limbs, fine for FP32, not for the INT8 form
    assert _init(lib, W.Qubo(n=q.n, Q=Q, c=None), dict(p, precision="i8"), x0) == \
        _abi.PDBO_EUNSUPPORTED


def test_invalid_maxsat(lib):
    import paper_2509_21064_amd as P
    f = W.random_maxsat(10, 20, 3, 1, 5, np.random.default_rng(0))
    p = W.gda_params("maxsat", B=2, T=5)
    x0 = W.x0_uniform(5, 0, 2, 10)
    for bad in ("zero", "range", "repeat", "weight"):
        lits = f.lits.copy()
        w = f.w.copy()
        if bad == "zero":
            lits[3, 1] = 0
        elif bad == "range":
            lits[3, 1] = 11
        elif bad == "repeat":
            lits[3, 1] = -lits[3, 0]
        else:
            w[2] = 1 << 24
        keep = P._Keep()
        prob = P._maxsat_struct(W.MaxSat(n=10, lits=lits, w=w), keep)
        par = P._params_struct(p, x0, keep)
        h = ctypes.c_void_p()
        st = lib.maxsat_gda_init(ctypes.byref(prob), ctypes.byref(par), None, ctypes.byref(h))
        assert st == _abi.PDBO_EINVAL, bad


def test_null_context(lib):
    assert lib.qubo_gda_step(None, 1) == _abi.PDBO_ESTATE
    assert lib.maxsat_gda_step(None, 1) == _abi.PDBO_ESTATE
    lib.pdbo_destroy(None)


def test_valid_input_without_gpu_reports_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    q, p, x0 = _base()
    assert _init(lib, q, p, x0) in (_abi.PDBO_EDEVICE, _abi.PDBO_ENOMEM)


def test_autotune_cache_fresh_nested_directory(lib, tmp_path, monkeypatch):
    """The autotuner's cache is written into directories that do not exist yet
    (created with mkdir(2), no shell), and read back."""
    path = tmp_path / "a" / "b c" / "d'e" / "tune.json"
    monkeypatch.setenv("PDBO_AUTOTUNE_CACHE", str(path))
    cfg = ctypes.c_int32(7)
    assert lib.pdbo_autotune_lookup(b"gfx950/p3/B8/k1/nmax64/nsum1024", ctypes.byref(cfg)) == 0
    assert cfg.value == -1
    assert lib.pdbo_autotune_store(b"gfx950/p3/B8/k1/nmax64/nsum1024", 5) == 0
    assert lib.pdbo_autotune_store(b"gfx950/p1/B8/k1/nmax64/nsum1024", 2) == 0
    assert lib.pdbo_autotune_store(b"gfx950/p3/B8/k1/nmax64/nsum1024", 6) == 0
    assert path.is_file()
    import json
    assert json.loads(path.read_text()) == {"gfx950/p1/B8/k1/nmax64/nsum1024": 2,
                                            "gfx950/p3/B8/k1/nmax64/nsum1024": 6}
    assert lib.pdbo_autotune_lookup(b"gfx950/p3/B8/k1/nmax64/nsum1024", ctypes.byref(cfg)) == 0
    assert cfg.value == 6
    # keys that would break the file format, and unknown configurations
    assert lib.pdbo_autotune_store(b'bad"key', 1) == _abi.PDBO_EINVAL
    assert lib.pdbo_autotune_store(b"ok", 99) == _abi.PDBO_EINVAL
    # a path through a regular file cannot be created
    monkeypatch.setenv("PDBO_AUTOTUNE_CACHE", str(tmp_path / "a" / "b c" / "d'e" / "tune.json" / "x.json"))
    assert lib.pdbo_autotune_store(b"k", 1) == _abi.PDBO_EINVAL


def test_library_starts_no_processes():
    """The library builds no shell command lines and spawns nothing."""
    csrc = os.path.join(ROOT, "paper_2509_21064_amd", "csrc")
    for f in os.listdir(csrc):
        txt = open(os.path.join(csrc, f)).read()
        for pat in (r"\bsystem\s*\(", r"\bpopen\s*\(", r"\bfork\s*\(", r"\bexec[lv]p?e?\s*\(",
                    r"posix_spawn"):
            assert not re.search(pat, txt), (f, pat)
