// Host side of libpdbo: the extern "C" entry points declared in pdbo.h.
//
// Validation happens before any HIP call, so contract violations return
// PDBO_EINVAL on any machine.  Canonicalisation follows Prop. 2.4: on binary
// points x_i^2 = x_i, so the multilinear extension of x^T Q x + c^T x is
// 1/2 x^T A x + c'^T x with A = offdiag(Q + Q^T) and c' = c + diag(Q).  A is
// stored as Ahat = A / kappa with kappa = 2 when every entry of A is even (always
// the case for a symmetric integer Q) and 1 otherwise, so the exact objective
// is F = (kappa/2) x^T Ahat x + c'^T x and the gradient of f/s is
// (kappa/s) Ahat x + c'/s.
#include <algorithm>
#include <sys/stat.h>

#include <cerrno>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

using namespace pdbo;

namespace {

thread_local std::string g_last_error;

constexpr int kTraceCap = 4096;
constexpr int kMaxLimbs = 4;  // int8 limbs of the dense exact evaluation
// the automatic CSR choice gives each restart a workgroup of its own only when
// there are enough restarts to occupy the chip
constexpr int kResidentMinB = 128;
constexpr int64_t kI64Max = LLONG_MAX;

int roundup(int v, int a) { return (v + a - 1) / a * a; }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Fault injection for tests: PDBO_FAIL_ALLOC_AT=k makes the k-th device
// allocation after the variable last changed value fail with PDBO_ENOMEM
// (0 or unset: none fails).
std::mutex g_alloc_mu;
long g_alloc_count = 0;
std::string g_alloc_env;

bool inject_alloc_failure() {
  const char* e = std::getenv("PDBO_FAIL_ALLOC_AT");
  const std::string v = e ? e : "";
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  if (v != g_alloc_env) {
    g_alloc_env = v;
    g_alloc_count = 0;
  }
  const long fail_at = v.empty() ? 0L : std::atol(v.c_str());
  ++g_alloc_count;
  return fail_at > 0 && g_alloc_count == fail_at;
}

}  // namespace

struct TimedLaunch {
  hipEvent_t a, b;
  int cls;
};

struct pdbo_ctx {
  int kind = 0;  // 0 dense (one or many instances), 1 CSR resident, 2 MaxSAT, 3 CSR row-parallel,
                 // 4 Max-k-Cut
  hipStream_t stream = nullptr;
  std::string err;
  pdbo_params par{};
  int B = 0, prec = 0, cfg = 0, eval_every = 1;
  int64_t t_host = 0;
  int parity = 0;
  bool stamped = false;
  std::vector<void*> allocs;
  std::vector<int> n_of;  // n per instance
  // dense
  std::vector<InstDev> insts_h;
  InstDev* insts_d = nullptr;
  std::vector<TileDev> tiles_h;
  TileDev* tiles_d = nullptr;
  std::vector<int> tile_off, tile_cnt;
  // incremental evaluation: one workgroup per (instance, restart), in instance order
  int2* incr_work_d = nullptr;
  std::vector<int> incr_off;  // first work item of each instance, plus the total
  int grouped = 1;
  InstDev* scratch_inst_d = nullptr;
  float* gx_scratch = nullptr;     // fp32 x for grad()
  uint8_t* gs_scratch = nullptr;   // shadow for grad()
  float* g_scratch = nullptr;      // gradient out
  int8_t* xr_scratch = nullptr;
  int64_t *sp_scratch = nullptr, *cp_scratch = nullptr, *f_scratch = nullptr;
  // dual certificate: one descent point (two for ping-pong), its dual, shadow,
  // rounding, per-row terms and the result; per-restart records of the
  // resident CSR kernel and the partial sums of the row-parallel one
  float *cert_x = nullptr, *cert_y = nullptr;
  uint8_t* cert_xs = nullptr;
  int8_t* cert_xr = nullptr;
  double *cert_rows = nullptr, *cert_res = nullptr;
  int64_t *cert_i64 = nullptr;
  uint64_t* cert_u64 = nullptr;
  uint8_t* cert_bx = nullptr;
  // graph
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream used only to record the graph
  int graph_parity0 = -1;
  // the best of B of the last iteration has not run yet (incremental evaluation)
  bool argmin_pending = false;
  // with incremental evaluation, the evaluation GEMM runs in iterations before
  // this one (the transient after init or set_state, when many rounded
  // coordinates change); later iterations evaluate such restarts by rows
  int64_t full_until = 0;
  // CSR / MaxSAT persistent (kind 1, 2); row-parallel CSR (kind 3) keeps its
  // iterates in spmm and the canonical matrix also in csr (for qubo_gda_eval)
  SpmmDev spmm{};
  KcutDev kcut{};  // Max-k-Cut (kind 4)
  float *kz_scratch = nullptr, *kg_scratch = nullptr;  // node-major (B, n, k) for grad()
  CsrDev csr{};
  bool compact = false;
  SatDev sat{};
  Incumbent* inc_d = nullptr;
  uint8_t* best_x_d = nullptr;
  uint64_t* ts0_d = nullptr;
  // timing
  bool timing = false;
  uint32_t tmask = 0;  // kernel classes being timed (bit k = PDBO_K_k)
  int tstride = 1;     // time every tstride-th launch of a timed class
  int64_t tseen[PDBO_K_COUNT] = {};  // launches of each class since timing was set
  std::vector<TimedLaunch> pending;
  std::vector<hipEvent_t> ev_pool;  // events already read, reused by later launches
  double ms[PDBO_K_COUNT] = {};
  int64_t cnt[PDBO_K_COUNT] = {};
};

namespace {

pdbo_status fail(pdbo_ctx* c, pdbo_status s, const std::string& msg) {
  if (c)
    c->err = msg;
  g_last_error = msg;
  return s;
}

pdbo_status hipfail(pdbo_ctx* c, const char* what, hipError_t e) {
  std::string m = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  return fail(c, e == hipErrorOutOfMemory ? PDBO_ENOMEM : PDBO_EDEVICE, m);
}

#define HIPCHK(ctx, call)                              \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hipfail(ctx, #call, e_); \
  } while (0)

#define STCHK(call)                     \
  do {                                  \
    pdbo_status s_ = (call);            \
    if (s_ != PDBO_OK) return s_;       \
  } while (0)

template <typename T>
pdbo_status dalloc(pdbo_ctx* c, T** p, size_t count) {
  *p = nullptr;
  if (inject_alloc_failure()) return fail(c, PDBO_ENOMEM, "injected allocation failure");
  const size_t bytes = std::max<size_t>(count * sizeof(T), 16);
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) return hipfail(c, "hipMalloc", e);
  c->allocs.push_back(q);
  e = hipMemsetAsync(q, 0, bytes, c->stream);
  if (e != hipSuccess) return hipfail(c, "hipMemsetAsync", e);
  *p = (T*)q;
  return PDBO_OK;
}

void free_all(pdbo_ctx* c) {
  if (!c) return;
  // the context's stream may be the null (legacy default) stream: synchronise it either way
  (void)hipStreamSynchronize(c->stream);
  for (auto& t : c->pending) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  c->pending.clear();
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  c->ev_pool.clear();
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (void* p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
}

// Temporary device buffer freed at scope exit (init-time uploads).
struct TempDev {
  void* p = nullptr;
  ~TempDev() {
    if (p) (void)hipFree(p);
  }
};

pdbo_status temp_upload(pdbo_ctx* c, TempDev& t, const void* host, size_t bytes) {
  if (inject_alloc_failure()) return fail(c, PDBO_ENOMEM, "injected allocation failure");
  hipError_t e = hipMalloc(&t.p, std::max<size_t>(bytes, 16));
  if (e != hipSuccess) return hipfail(c, "hipMalloc", e);
  if (bytes) {
    e = hipMemcpyAsync(t.p, host, bytes, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return hipfail(c, "hipMemcpyAsync", e);
  }
  return PDBO_OK;
}

// ---------------------------------------------------------------- validation

// Uploads the caller's starting points, or leaves t empty when there are none
// (the init kernel then draws them from the generator keyed by the seed).
pdbo_status upload_x0(pdbo_ctx* c, TempDev& t, const double* x0, size_t count) {
  if (!x0) return PDBO_OK;
  return temp_upload(c, t, x0, count * sizeof(double));
}

pdbo_status check_params(const pdbo_params* p, int n, bool x0_required = true) {
  if (!p) return fail(nullptr, PDBO_EINVAL, "params is NULL");
  if (p->B < 1 || p->B > (1 << 20)) return fail(nullptr, PDBO_EINVAL, "B must be in [1, 2^20]");
  if (!finite_pos(p->alpha) || !finite_pos(p->beta))
    return fail(nullptr, PDBO_EINVAL, "alpha and beta must be finite and > 0");
  if (!finite_pos(p->y0)) return fail(nullptr, PDBO_EINVAL, "y0 must be finite and > 0");
  if (!finite_pos(p->scale)) return fail(nullptr, PDBO_EINVAL, "scale must be finite and > 0");
  if (!(std::isfinite(p->delta) && p->delta > 0.0 && p->delta < 0.5))
    return fail(nullptr, PDBO_EINVAL, "delta must be in (0, 1/2)");
  if (p->g_kind != PDBO_G_QUAD && p->g_kind != PDBO_G_ENTROPY && p->g_kind != PDBO_G_POLY)
    return fail(nullptr, PDBO_EINVAL, "unknown g_kind");
  if (p->precision < PDBO_FP32 || p->precision > PDBO_I8)
    return fail(nullptr, PDBO_EINVAL, "unknown precision");
  if (p->eval_every < 1) return fail(nullptr, PDBO_EINVAL, "eval_every must be >= 1");
  if (p->graph_chunk < 0 || (p->graph_chunk & 1))
    return fail(nullptr, PDBO_EINVAL, "graph_chunk must be 0 or a positive even number");
  if (p->tile < 0 || p->tile > dense_num_cfgs())
    return fail(nullptr, PDBO_EINVAL, "unknown tile configuration");
  if (p->g_kind == PDBO_G_POLY && (p->g_degree < 1 || p->g_degree > 16))
    return fail(nullptr, PDBO_EINVAL, "g_degree must be in [1, 16]");
  if (p->dual_kind != PDBO_DUAL_VECTOR && p->dual_kind != PDBO_DUAL_SCALAR)
    return fail(nullptr, PDBO_EINVAL, "unknown dual_kind");
  if (x0_required && p->x0) {  // NULL: drawn by the library's generator
    const size_t tot = (size_t)p->B * (size_t)n;
    for (size_t i = 0; i < tot; ++i) {
      const double v = p->x0[i];
      if (!(v >= 0.0 && v <= 1.0)) return fail(nullptr, PDBO_EINVAL, "x0 must lie in [0,1]");
    }
  }
  return PDBO_OK;
}

pdbo_status check_qubo(const pdbo_qubo* q) {
  if (!q) return fail(nullptr, PDBO_EINVAL, "problem is NULL");
  if (q->n < 1 || q->n > 65536) return fail(nullptr, PDBO_EINVAL, "n must be in [1, 65536]");
  if (q->wtype != PDBO_W_INT32 && q->wtype != PDBO_W_F64)
    return fail(nullptr, PDBO_EINVAL, "unknown wtype");
  const bool real = q->wtype == PDBO_W_F64;
  const int n = q->n;
  // weight checks: int32 entries below 2^30, float64 entries finite
  auto bad_q = [&](size_t k) -> pdbo_status {
    if (real) {
      if (!std::isfinite(q->qd[k])) return fail(nullptr, PDBO_EINVAL, "Q_ij must be finite");
    } else if (q->q[k] >= (1 << 30) || q->q[k] <= -(1 << 30)) {
      return fail(nullptr, PDBO_ERANGE, "|Q_ij| must be below 2^30");
    }
    return PDBO_OK;
  };
  const bool have_q = real ? q->qd != nullptr : q->q != nullptr;
  if (q->format == PDBO_DENSE) {
    if (!have_q) return fail(nullptr, PDBO_EINVAL, "dense Q is NULL");
    const size_t tot = (size_t)n * n;
    for (size_t i = 0; i < tot; ++i) STCHK(bad_q(i));
  } else if (q->format == PDBO_CSR) {
    if (!q->row_ptr || (q->nnz > 0 && (!q->col_idx || !have_q)))
      return fail(nullptr, PDBO_EINVAL, "CSR arrays are NULL");
    if (q->nnz < 0 || q->nnz > (int64_t)INT_MAX) return fail(nullptr, PDBO_EINVAL, "bad nnz");
    if (q->row_ptr[0] != 0 || (int64_t)q->row_ptr[n] != q->nnz)
      return fail(nullptr, PDBO_EINVAL, "row_ptr must start at 0 and end at nnz");
    for (int i = 0; i < n; ++i) {
      if (q->row_ptr[i + 1] < q->row_ptr[i])
        return fail(nullptr, PDBO_EINVAL, "row_ptr must be non-decreasing");
      for (int p = q->row_ptr[i]; p < q->row_ptr[i + 1]; ++p) {
        const int j = q->col_idx[p];
        if (j < 0 || j >= n) return fail(nullptr, PDBO_EINVAL, "column index out of range");
        if (p > q->row_ptr[i] && j <= q->col_idx[p - 1])
          return fail(nullptr, PDBO_EINVAL, "columns of a row must be strictly increasing");
        STCHK(bad_q((size_t)p));
      }
    }
  } else {
    return fail(nullptr, PDBO_EINVAL, "unknown format");
  }
  if (real) {
    if (q->cd)
      for (int i = 0; i < n; ++i)
        if (!std::isfinite(q->cd[i])) return fail(nullptr, PDBO_EINVAL, "c_i must be finite");
  } else if (q->c) {
    for (int i = 0; i < n; ++i)
      if (q->c[i] >= (int64_t(1) << 40) || q->c[i] <= -(int64_t(1) << 40))
        return fail(nullptr, PDBO_ERANGE, "|c_i| must be below 2^40");
  }
  return PDBO_OK;
}

// ---------------------------------------------------------------- canonical form

struct DenseCanon {
  int n = 0, kappa = 1;
  std::vector<int32_t> Ahat;   // n*n
  std::vector<int64_t> cp;     // n
  int32_t amax = 0;
  int nlimb = 1;               // int8 limbs of the exact evaluation copy
  std::vector<float> rowmax;   // max_j |Ahat_ij|
};

pdbo_status canon_dense(const pdbo_qubo* q, DenseCanon& C) {
  const int n = q->n;
  C.n = n;
  C.cp.assign(n, 0);
  if (q->c)
    for (int i = 0; i < n; ++i) C.cp[i] = q->c[i];
  std::vector<int64_t> A;
  try {
    A.assign((size_t)n * n, 0);
  } catch (...) {
    return fail(nullptr, PDBO_ENOMEM, "host allocation failed");
  }
  if (q->format == PDBO_DENSE) {
    constexpr int T = 64;
    for (int i0 = 0; i0 < n; i0 += T)
      for (int j0 = 0; j0 < n; j0 += T)
        for (int i = i0; i < std::min(n, i0 + T); ++i)
          for (int j = j0; j < std::min(n, j0 + T); ++j) {
            const int64_t v = q->q[(size_t)i * n + j];
            if (i == j)
              C.cp[i] += v;
            else {
              A[(size_t)i * n + j] += v;
              A[(size_t)j * n + i] += v;
            }
          }
  } else {
    for (int i = 0; i < n; ++i)
      for (int p = q->row_ptr[i]; p < q->row_ptr[i + 1]; ++p) {
        const int j = q->col_idx[p];
        const int64_t v = q->q[p];
        if (i == j)
          C.cp[i] += v;
        else {
          A[(size_t)i * n + j] += v;
          A[(size_t)j * n + i] += v;
        }
      }
  }
  bool even = true;
  for (size_t k = 0; k < A.size() && even; ++k) even = (A[k] & 1) == 0;
  C.kappa = even ? 2 : 1;
  try {
    C.Ahat.resize((size_t)n * n);
  } catch (...) {
    return fail(nullptr, PDBO_ENOMEM, "host allocation failed");
  }
  C.rowmax.assign(n, 0.f);
  for (int i = 0; i < n; ++i) {
    int64_t rs = 0;
    int32_t rm = 0;
    for (int j = 0; j < n; ++j) {
      const int64_t v = A[(size_t)i * n + j] / C.kappa;
      C.Ahat[(size_t)i * n + j] = (int32_t)v;
      const int32_t av = (int32_t)(v < 0 ? -v : v);
      rs += av;
      rm = std::max(rm, av);
    }
    if (rs >= (int64_t(1) << 31)) return fail(nullptr, PDBO_ERANGE, "a row of |Ahat| sums to 2^31 or more");
    C.rowmax[i] = (float)rm;
    C.amax = std::max(C.amax, rm);
  }
  // The exact evaluation copy holds Ahat as nlimb signed base-256 int8 digits,
  // which cover |Ahat_ij| <= 127 (256^nlimb - 1) / 255.
  auto limb_max = [](int L) { return 127 * (((int64_t(1) << (8 * L)) - 1) / 255); };
  C.nlimb = 1;
  while (C.nlimb < kMaxLimbs && (int64_t)C.amax > limb_max(C.nlimb)) ++C.nlimb;
  if ((int64_t)C.amax > limb_max(C.nlimb))
    return fail(nullptr, PDBO_ERANGE, "|Ahat_ij| beyond the four int8 limbs of the exact evaluation");
  return PDBO_OK;
}

struct CsrCanon {
  int n = 0, kappa = 1;
  std::vector<int32_t> rp, col, val;
  std::vector<int64_t> cp;
  int32_t amax = 0;
  int64_t rowabs = 0;  // max_i sum_j |Ahat_ij|
};

pdbo_status canon_csr(const pdbo_qubo* q, CsrCanon& C) {
  const int n = q->n;
  C.n = n;
  C.cp.assign(n, 0);
  if (q->c)
    for (int i = 0; i < n; ++i) C.cp[i] = q->c[i];
  struct E {
    int32_t i, j;
    int64_t v;
  };
  std::vector<E> e;
  e.reserve((size_t)q->nnz * 2);
  for (int i = 0; i < n; ++i)
    for (int p = q->row_ptr[i]; p < q->row_ptr[i + 1]; ++p) {
      const int j = q->col_idx[p];
      const int64_t v = q->q[p];
      if (i == j) {
        C.cp[i] += v;
      } else {
        e.push_back({i, j, v});
        e.push_back({j, i, v});
      }
    }
  std::sort(e.begin(), e.end(), [](const E& a, const E& b) { return a.i != b.i ? a.i < b.i : a.j < b.j; });
  std::vector<E> m;
  for (const E& x : e) {
    if (!m.empty() && m.back().i == x.i && m.back().j == x.j)
      m.back().v += x.v;
    else
      m.push_back(x);
  }
  bool even = true;
  for (const E& x : m) even = even && ((x.v & 1) == 0);
  C.kappa = even ? 2 : 1;
  C.rp.assign(n + 1, 0);
  std::vector<int64_t> rs(n, 0);
  for (const E& x : m) {
    const int64_t v = x.v / C.kappa;
    if (v == 0) continue;
    C.rp[x.i + 1]++;
    C.col.push_back(x.j);
    C.val.push_back((int32_t)v);
    const int64_t av = v < 0 ? -v : v;
    rs[x.i] += av;
    C.amax = std::max<int32_t>(C.amax, (int32_t)av);
  }
  for (int i = 0; i < n; ++i) {
    C.rp[i + 1] += C.rp[i];
    if (rs[i] >= (int64_t(1) << 31)) return fail(nullptr, PDBO_ERANGE, "a row of |Ahat| sums to 2^31 or more");
    C.rowabs = std::max(C.rowabs, rs[i]);
  }
  return PDBO_OK;
}

// Float64 weights: the canonical A = offdiag(Q + Q^T) and c' = c + diag(Q)
// (Prop. 2.4) in exact fixed point.  Every finite nonzero weight is m 2^e with
// m odd; with elo the least such e over all weights, a weight is the integer
// m 2^(e - elo) in units of 2^elo, written as ndig signed base-2^24 digits
// (the digits of |m| 2^(e - elo), each carrying the weight's sign).  The two
// weights that make up a canonical entry are added digit by digit, without
// carries, so every digit stays below 2^25 in magnitude.  The gradient uses
// A/s and c'/s rounded to float32.
struct RealCanon {
  int n = 0, ndig = 0, elo = 0;
  std::vector<int32_t> rp, col;
  std::vector<float> valf;     // A/s
  std::vector<int32_t> Adig;   // [ndig][nnz]
  std::vector<int32_t> Cdig;   // [ndig][n]
  std::vector<float> cps;      // c'/s
};

struct OddPow {  // v = m 2^e, m odd (v != 0)
  int64_t m;
  int e;
};

OddPow odd_pow(double v) {
  int E = 0;
  const double f = std::frexp(v, &E);  // v = f 2^E, 1/2 <= |f| < 1
  OddPow r{(int64_t)std::ldexp(f, 53), E - 53};
  while ((r.m & 1) == 0) {
    r.m /= 2;
    ++r.e;
  }
  return r;
}

int bit_length(uint64_t a) { return a ? 64 - __builtin_clzll(a) : 0; }

// dst[d * stride] += digit d of m 2^sh (digits of |m| 2^sh, sign of m)
void add_digits(int32_t* dst, size_t stride, int ndig, int64_t m, int sh) {
  const uint64_t a = (uint64_t)(m < 0 ? -m : m);
  const int32_t sg = m < 0 ? -1 : 1;
  for (int d = 0; d < ndig; ++d) {
    const int lo = 24 * d - sh;  // bit of |m| that lands on bit 0 of digit d
    uint64_t chunk;
    if (lo >= 0)
      chunk = lo >= 64 ? 0 : (a >> lo) & 0xFFFFFFu;
    else
      chunk = -lo >= 24 ? 0 : (a << -lo) & 0xFFFFFFu;
    dst[(size_t)d * stride] += sg * (int32_t)chunk;
  }
}

pdbo_status canon_real(const pdbo_qubo* q, double scale, RealCanon& R) {
  const int n = q->n;
  R.n = n;
  const bool dense = q->format == PDBO_DENSE;
  const size_t nq = dense ? (size_t)n * n : (size_t)q->nnz;
  // the exponent range over all weights
  int elo = INT_MAX, hi = INT_MIN;
  auto scan = [&](double v) {
    if (v == 0.0) return;
    const OddPow o = odd_pow(v);
    elo = std::min(elo, o.e);
    hi = std::max(hi, o.e + bit_length((uint64_t)(o.m < 0 ? -o.m : o.m)) - 1);
  };
  for (size_t k = 0; k < nq; ++k) scan(q->qd[k]);
  if (q->cd)
    for (int i = 0; i < n; ++i) scan(q->cd[i]);
  if (elo == INT_MAX) elo = hi = 0;  // all weights zero
  R.elo = elo;
  R.ndig = (hi - elo) / 24 + 1;
  if (R.ndig > kMaxDigits)
    return fail(nullptr, PDBO_ERANGE, "the weights' binary exponents span more than 192 bits");
  const int nd = R.ndig;
  // (i, j, weight index) contributions to canonical entries, i != j
  struct E {
    int32_t i, j;
    int64_t k;
  };
  std::vector<E> e;
  std::vector<double> cpd(n, 0.0);
  std::vector<int32_t> Cd;
  try {
    R.Cdig.assign((size_t)nd * n, 0);
    if (dense) {
      e.reserve(nq);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          if (i == j) continue;
          if (q->qd[(size_t)i * n + j] != 0.0) e.push_back({i, j, (int64_t)i * n + j});
          if (q->qd[(size_t)j * n + i] != 0.0) e.push_back({i, j, (int64_t)j * n + i});
        }
    } else {
      e.reserve(2 * nq);
      for (int i = 0; i < n; ++i)
        for (int p = q->row_ptr[i]; p < q->row_ptr[i + 1]; ++p) {
          const int j = q->col_idx[p];
          if (i == j || q->qd[p] == 0.0) continue;
          e.push_back({i, j, p});
          e.push_back({j, i, p});
        }
      std::stable_sort(e.begin(), e.end(),
                       [](const E& a, const E& b) { return a.i != b.i ? a.i < b.i : a.j < b.j; });
    }
  } catch (...) {
    return fail(nullptr, PDBO_ENOMEM, "host allocation failed");
  }
  // linear part: c' = c + diag(Q)
  auto add_lin = [&](int i, double v) {
    if (v == 0.0) return;
    const OddPow o = odd_pow(v);
    add_digits(R.Cdig.data() + i, (size_t)n, nd, o.m, o.e - elo);
    cpd[i] += v;
  };
  for (int i = 0; i < n; ++i) {
    if (q->cd) add_lin(i, q->cd[i]);
    if (dense)
      add_lin(i, q->qd[(size_t)i * n + i]);
    else
      for (int p = q->row_ptr[i]; p < q->row_ptr[i + 1]; ++p)
        if (q->col_idx[p] == i) add_lin(i, q->qd[p]);
  }
  // canonical entries: runs of equal (i, j); an exact cancellation (all digits
  // zero) leaves no entry
  std::vector<int32_t> dig;  // [nnz][nd] while building
  R.rp.assign(n + 1, 0);
  std::vector<int32_t> cur(nd);
  try {
    for (size_t a = 0; a < e.size();) {
      size_t b = a;
      double v = 0.0;
      std::fill(cur.begin(), cur.end(), 0);
      while (b < e.size() && e[b].i == e[a].i && e[b].j == e[a].j) {
        const double w = q->qd[e[b].k];
        const OddPow o = odd_pow(w);
        add_digits(cur.data(), 1, nd, o.m, o.e - elo);
        v += w;
        ++b;
      }
      bool any = false;
      for (int d = 0; d < nd; ++d) any = any || cur[d] != 0;
      if (any) {
        R.rp[e[a].i + 1]++;
        R.col.push_back(e[a].j);
        R.valf.push_back((float)(v / scale));
        dig.insert(dig.end(), cur.begin(), cur.end());
      }
      a = b;
    }
    const size_t nnz = R.col.size();
    R.Adig.resize((size_t)nd * nnz);
    for (size_t k = 0; k < nnz; ++k)
      for (int d = 0; d < nd; ++d) R.Adig[(size_t)d * nnz + k] = dig[k * nd + d];
  } catch (...) {
    return fail(nullptr, PDBO_ENOMEM, "host allocation failed");
  }
  for (int i = 0; i < n; ++i) R.rp[i + 1] += R.rp[i];
  R.cps.resize(n);
  // the float32 gradient needs every row of |A/s| and |c'/s| within range
  for (int i = 0; i < n; ++i) {
    R.cps[i] = (float)(cpd[i] / scale);
    double rs = std::fabs((double)R.cps[i]);
    for (int p = R.rp[i]; p < R.rp[i + 1]; ++p) rs += std::fabs((double)R.valf[p]);
    if (!(rs <= 3.0e38))
      return fail(nullptr, PDBO_ERANGE, "a row of |A/s| exceeds the float32 range of the gradient");
  }
  return PDBO_OK;
}

GdaP make_gp(const pdbo_params* p) {
  GdaP g;
  g.alpha = (float)p->alpha;
  g.beta = (float)p->beta;
  g.delta = (float)p->delta;
  g.gkind = p->g_kind;
  g.deg = p->g_kind == PDBO_G_POLY ? p->g_degree : 1;
  return g;
}

int32_t f32_bits(float v) {
  int32_t b;
  std::memcpy(&b, &v, sizeof(b));
  return b;
}

int element_bytes(int prec) { return prec == PDBO_FP32 ? 4 : prec == PDBO_BF16 ? 2 : 1; }
static_assert((int)PDBO_I8 == (int)P_I8, "ABI and kernel precision codes agree");

// Estimated cost of a tile configuration for a set of instances: the launch
// runs in ceil(tiles / (256 CUs x workgroups per CU)) rounds, each costing the
// per-CU output area, inflated when the wave tile needs more LDS bytes per MFMA
// than the LDS can deliver at the MFMA rate (wave tiles below 64x64).
double cfg_cost(int cfg, const std::vector<int>& ns, int B) {
  const TileCfgInfo& cf = dense_cfg(cfg);
  const int lds = cf.dma ? 3 * (cf.BM + cf.BN) * 128 : 2 * (cf.BM + cf.BN) * 144;
  const int occ = std::max(1, std::min(4, (160 * 1024) / lds));
  double tiles = 0;
  for (int n : ns) tiles += (double)((n + cf.BM - 1) / cf.BM) * ((B + cf.BN - 1) / cf.BN);
  const double rounds = std::ceil(tiles / (256.0 * occ));
  const double fm = cf.BM / cf.WM / 16.0, fn = cf.BN / cf.WN / 16.0;
  const double lds_per_mfma = (fm + fn) / (fm * fn);
  const double ineff = std::max(1.0, lds_per_mfma / 0.5);
  return rounds * occ * cf.BM * cf.BN * ineff;
}

int default_cfg(const std::vector<int>& ns, int B) {
  // small tiles first so that they win ties on small problems
  static const int order[] = {1, 9, 0, 7, 2, 8, 3, 4, 6, 5};
  int best = 1;
  double bc = 1e300;
  for (int id : order) {
    if (id >= dense_num_cfgs()) continue;
    const double cst = cfg_cost(id, ns, B);
    if (cst < bc) {
      bc = cst;
      best = id;
    }
  }
  return best;
}

// ---------------------------------------------------------------- timing

hipEvent_t ev_get(pdbo_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

// Brackets one launch with a pair of events on the context's stream.
void t_begin(pdbo_ctx* c, TimedLaunch& tl, int cls) {
  tl.cls = -1;
  if (!c->timing || !((c->tmask >> cls) & 1u)) return;
  if (c->tseen[cls]++ % c->tstride != 0) return;
  tl.a = ev_get(c);
  if (!tl.a) return;
  tl.b = ev_get(c);
  if (!tl.b) {
    c->ev_pool.push_back(tl.a);
    return;
  }
  tl.cls = cls;
  (void)hipEventRecord(tl.a, c->stream);
}
void t_end(pdbo_ctx* c, TimedLaunch& tl) {
  if (tl.cls < 0) return;
  (void)hipEventRecord(tl.b, c->stream);
  c->pending.push_back(tl);
}

void t_collect(pdbo_ctx* c) {
  for (auto& t : c->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(t.b) == hipSuccess && hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      c->ms[t.cls] += ms;
      c->cnt[t.cls] += 1;
    }
    c->ev_pool.push_back(t.a);
    c->ev_pool.push_back(t.b);
  }
  c->pending.clear();
}

// ---------------------------------------------------------------- dense setup

pdbo_status setup_dense_instance(pdbo_ctx* c, const DenseCanon& C, const pdbo_params* p,
                                 InstDev& I) {
  const int n = C.n, B = p->B, prec = c->prec;
  const int ld = roundup(n, kLdAlign);
  const int EB = element_bytes(prec);
  const TileCfgInfo& cf = dense_cfg(c->cfg);
  std::memset(&I, 0, sizeof(I));
  I.n = n;
  I.ld = ld;
  I.B = B;
  I.mblocks = (n + cf.BM - 1) / cf.BM;
  I.kappa = C.kappa;
  I.kos = (float)((double)C.kappa / p->scale);
  I.gp = make_gp(p);
  I.trace_cap = kTraceCap;
  const int nlimb = C.nlimb;
  I.nlimb = nlimb;
  I.limb_stride = (int64_t)n * ld;

  uint8_t* A = nullptr;
  int8_t* A8 = nullptr;
  float* rs = nullptr;
  STCHK(dalloc(c, &A8, (size_t)nlimb * n * ld));
  if (prec == PDBO_I8) {
    // the exact int8 matrix is the gradient operand as well
    int64_t worst = 0;
    std::vector<int32_t> hsum(ld, 0);
    for (int i = 0; i < n; ++i) {
      int64_t sa = 0, sg = 0;
      for (int j = 0; j < n; ++j) {
        const int32_t v = C.Ahat[(size_t)i * n + j];
        sg += v;
        sa += v < 0 ? -v : v;
      }
      hsum[i] = (int32_t)sg;
      worst = std::max(worst, sa);
    }
    if (127 * worst >= (int64_t(1) << 31))
      return fail(c, PDBO_EUNSUPPORTED, "INT8 form needs 127 * sum_j |Ahat_ij| < 2^31");
    int32_t* dsum = nullptr;
    STCHK(dalloc(c, &dsum, ld));
    HIPCHK(c, hipMemcpyAsync(dsum, hsum.data(), ld * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    I.rsum = dsum;
  } else {
    STCHK(dalloc(c, &A, (size_t)n * ld * EB));
  }
  std::vector<float> hs(ld, 1.f);  // alive until the stream is synchronised below
  if (prec == PDBO_FP8) {
    for (int i = 0; i < n; ++i) hs[i] = C.rowmax[i] > 0.f ? C.rowmax[i] / 448.f : 1.f;
    STCHK(dalloc(c, &rs, ld));
    HIPCHK(c, hipMemcpyAsync(rs, hs.data(), ld * sizeof(float), hipMemcpyHostToDevice, c->stream));
  }
  {
    TempDev t;
    STCHK(temp_upload(c, t, C.Ahat.data(), (size_t)n * n * sizeof(int32_t)));
    HIPCHK(c, launch_quantize_A((const int32_t*)t.p, n, ld, prec, A, A8, nlimb, rs, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  if (prec == PDBO_I8) A = (uint8_t*)A8;
  I.A = A;
  I.A8 = A8;
  I.rscale = rs;

  std::vector<float> hcps(ld, 0.f);
  std::vector<int64_t> hcp(ld, 0);
  for (int i = 0; i < n; ++i) {
    hcp[i] = C.cp[i];
    hcps[i] = (float)((double)C.cp[i] / p->scale);
  }
  float* cps = nullptr;
  int64_t* cpd = nullptr;
  STCHK(dalloc(c, &cps, ld));
  STCHK(dalloc(c, &cpd, ld));
  HIPCHK(c, hipMemcpyAsync(cps, hcps.data(), ld * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(cpd, hcp.data(), ld * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
  I.cps = cps;
  I.cp = cpd;

  const size_t sz = (size_t)B * ld;
  STCHK(dalloc(c, &I.X[0], sz));
  STCHK(dalloc(c, &I.Y, sz));
  if (prec == PDBO_FP32) {
    // x is the GEMM operand itself: tiles of one step read x^t while others
    // write x^{t+1}, so the two must be distinct
    STCHK(dalloc(c, &I.X[1], sz));
    I.Xs[0] = (uint8_t*)I.X[0];
    I.Xs[1] = (uint8_t*)I.X[1];
  } else {
    // the GEMM reads the operand shadow; each x value is read and rewritten
    // by the same thread of the step epilogue, so x is updated in place (one
    // buffer less to keep in the last-level cache)
    I.X[1] = I.X[0];
    STCHK(dalloc(c, &I.Xs[0], sz * EB));
    STCHK(dalloc(c, &I.Xs[1], sz * EB));
  }
  STCHK(dalloc(c, &I.Xr, sz));
  STCHK(dalloc(c, &I.Sacc, (size_t)B));
  STCHK(dalloc(c, &I.Cacc, (size_t)B));
  STCHK(dalloc(c, &I.Fall, (size_t)B));
  I.nflip = nullptr;
  I.fbits = nullptr;
  I.cand = nullptr;
  if (p->eval_every == 1) {
    // the first evaluation is a full product (nflip above kFlipMax); the
    // bitmap starts clear (dalloc zeroes)
    STCHK(dalloc(c, &I.nflip, (size_t)B));
    STCHK(dalloc(c, &I.fbits, (size_t)B * (ld / 32)));
    STCHK(dalloc(c, &I.cand, (size_t)B * ld));
    HIPCHK(c, launch_fill_i32(I.nflip, kFlipMax + 1, B, c->stream));
  }
  I.ys = nullptr;
  if (p->dual_kind == PDBO_DUAL_SCALAR) {
    STCHK(dalloc(c, &I.ys, (size_t)B));
    HIPCHK(c, launch_fill_i32((int32_t*)I.ys, f32_bits((float)p->y0), B, c->stream));
  }
  STCHK(dalloc(c, &I.inc, 1));
  STCHK(dalloc(c, &I.best_x, (size_t)ld));
  STCHK(dalloc(c, &I.trace, kTraceCap));
  STCHK(dalloc(c, &I.trace_len, 1));
  STCHK(dalloc(c, &I.t_dev, 1));
  I.ts0 = c->ts0_d;
  Incumbent init{kI64Max, -1, -1, 0};
  HIPCHK(c, hipMemcpyAsync(I.inc, &init, sizeof(init), hipMemcpyHostToDevice, c->stream));
  {
    TempDev t;
    STCHK(upload_x0(c, t, p->x0, (size_t)B * n));
    HIPCHK(c, launch_init_state((const double*)t.p, B, n, ld, (float)p->y0, I.X[0], I.Y,
                                prec == PDBO_FP32 ? nullptr : I.Xs[0], prec, I.Xr, p->seed, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return PDBO_OK;
}

// Tile table: row groups (instance, m-block) are assigned round-robin to the
// 8 XCDs (workgroup w of a launch runs on XCD w % 8) so that the column tiles
// sharing one block of Ahat rows run on the same XCD, back to back, and reuse
// that block from the XCD's L2.  PDBO_TILE_ORDER=1 selects plain row-group
// order instead (for measurement).
void build_tiles(pdbo_ctx* c) {
  const TileCfgInfo& cf = dense_cfg(c->cfg);
  c->tiles_h.clear();
  c->tile_off.clear();
  c->tile_cnt.clear();
  static const int order = [] {
    const char* e = std::getenv("PDBO_TILE_ORDER");
    return e ? std::atoi(e) : 0;
  }();
  // Instances in decreasing order of n (longest-processing-time first): a
  // tile's work is proportional to its instance's n (its K loop), and the
  // grouped launch hands tiles to the CUs in list order, so the long tiles
  // start first and the short ones fill in behind them.
  const int ninst = (int)c->insts_h.size();
  std::vector<int> by_cost(ninst);
  for (int k = 0; k < ninst; ++k) by_cost[k] = k;
  std::stable_sort(by_cost.begin(), by_cost.end(),
                   [&](int a, int b) { return c->insts_h[a].n > c->insts_h[b].n; });
  c->tile_off.assign(ninst, 0);
  c->tile_cnt.assign(ninst, 0);
  for (int k : by_cost) {
    InstDev& I = c->insts_h[k];
    I.mblocks = (I.n + cf.BM - 1) / cf.BM;
    const int nb = (I.B + cf.BN - 1) / cf.BN;
    if (order == 1) {
      c->tile_off[k] = (int)c->tiles_h.size();
      for (int m = 0; m < I.mblocks; ++m)
        for (int j = 0; j < nb; ++j) c->tiles_h.push_back(TileDev{(int)k, m * cf.BM, j * cf.BN, m});
      c->tile_cnt[k] = (int)c->tiles_h.size() - c->tile_off[k];
      continue;
    }
    std::vector<std::vector<TileDev>> q(8);
    for (int m = 0; m < I.mblocks; ++m)
      for (int j = 0; j < nb; ++j) q[m % 8].push_back(TileDev{(int)k, m * cf.BM, j * cf.BN, m});
    c->tile_off[k] = (int)c->tiles_h.size();
    size_t longest = 0;
    for (auto& v : q) longest = std::max(longest, v.size());
    std::vector<TileDev> rest;
    for (size_t r = 0; r < longest; ++r) {
      bool full = true;
      for (auto& v : q) full = full && r < v.size();
      for (auto& v : q) {
        if (r >= v.size()) continue;
        if (full)
          c->tiles_h.push_back(v[r]);
        else
          rest.push_back(v[r]);
      }
    }
    c->tiles_h.insert(c->tiles_h.end(), rest.begin(), rest.end());
    c->tile_cnt[k] = (int)c->tiles_h.size() - c->tile_off[k];
  }
}

pdbo_status upload_dense_tables(pdbo_ctx* c) {
  build_tiles(c);
  std::vector<int2> work;  // alive until the stream is synchronised below
  c->incr_off.clear();
  for (size_t k = 0; k < c->insts_h.size(); ++k) {
    c->incr_off.push_back((int)work.size());
    if (!c->insts_h[k].nflip) continue;
    for (int b = 0; b < c->insts_h[k].B; ++b) work.push_back(make_int2((int)k, b));
  }
  c->incr_off.push_back((int)work.size());
  if (!work.empty()) {
    STCHK(dalloc(c, &c->incr_work_d, work.size()));
    HIPCHK(c, hipMemcpyAsync(c->incr_work_d, work.data(), work.size() * sizeof(int2),
                             hipMemcpyHostToDevice, c->stream));
  }
  STCHK(dalloc(c, &c->insts_d, c->insts_h.size()));
  STCHK(dalloc(c, &c->tiles_d, c->tiles_h.size()));
  HIPCHK(c, hipMemcpyAsync(c->insts_d, c->insts_h.data(), c->insts_h.size() * sizeof(InstDev),
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->tiles_d, c->tiles_h.data(), c->tiles_h.size() * sizeof(TileDev),
                           hipMemcpyHostToDevice, c->stream));
  // set the dynamic LDS limit of every kernel this context launches, outside
  // of any stream capture
  HIPCHK(c, launch_dense_gemm(c->cfg, c->prec, EPI_STEP, c->par.g_kind, nullptr, 0, nullptr, 0, 0,
                              c->stream));
  HIPCHK(c, launch_dense_gemm(c->cfg, c->prec, EPI_GRAD, 0, nullptr, 0, nullptr, 0, 0, c->stream));
  HIPCHK(c, launch_dense_gemm(c->cfg, c->prec, EPI_EVAL, 0, nullptr, 0, nullptr, 0, 0, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PDBO_OK;
}

// ---------------------------------------------------------------- autotuner
//
// Times the STEP variant of the dense GEMM (main loop and the Alg. 1
// epilogue, as the iterations launch it) for every tile configuration on
// scratch copies of the context's iterate, so the timing launches leave the
// state untouched, and keeps the fastest.  Every output element is accumulated
// along K in the same order whatever the tile shape, so the choice never
// changes results.  Choices are cached as a flat JSON object {"key": cfg, ...}
// in $PDBO_AUTOTUNE_CACHE (default $HOME/.cache/pdbo_autotune.json), keyed by
// architecture, operand type, B, instance count and the instance sizes.  The
// cache directory is created with mkdir(2), one path component at a time; the
// library starts no child process.

std::string autotune_key(const pdbo_ctx* c) {
  int dev = 0;
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  long long nsum = 0;
  int nmax = 0;
  for (const InstDev& I : c->insts_h) {
    nsum += I.n;
    nmax = std::max(nmax, I.n);
  }
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s/p%d/g%d/B%d/k%zu/nmax%d/nsum%lld", arch.c_str(), c->prec,
                c->par.g_kind, c->B, c->insts_h.size(), (nmax + 63) / 64 * 64,
                (nsum + 1023) / 1024 * 1024);
  return buf;
}

std::string autotune_path() {
  const char* e = std::getenv("PDBO_AUTOTUNE_CACHE");
  if (e && *e) return e;
  const char* h = std::getenv("HOME");
  return std::string(h ? h : "/tmp") + "/.cache/pdbo_autotune.json";
}

// Keys are written between double quotes, one entry per line.
bool autotune_key_ok(const std::string& k) {
  if (k.empty() || k.size() >= 400) return false;
  for (char ch : k)
    if (ch == '"' || ch == '\\' || (unsigned char)ch < 0x20) return false;
  return true;
}

// mkdir -p without a shell: every prefix of `dir` ending before a '/'.
bool make_dirs(const std::string& dir) {
  for (size_t pos = 1; pos <= dir.size(); ++pos) {
    if (pos < dir.size() && dir[pos] != '/') continue;
    const std::string part = dir.substr(0, pos);
    struct stat sb;
    if (::stat(part.c_str(), &sb) == 0) {
      if (!S_ISDIR(sb.st_mode)) return false;
      continue;
    }
    if (::mkdir(part.c_str(), 0755) != 0 && errno != EEXIST) return false;
  }
  return true;
}

std::mutex g_tune_mu;

std::vector<std::pair<std::string, int>> autotune_read(const std::string& path) {
  std::vector<std::pair<std::string, int>> ent;
  if (FILE* f = std::fopen(path.c_str(), "r")) {
    char line[512];
    while (std::fgets(line, sizeof(line), f)) {
      char k[400];
      int v;
      if (std::sscanf(line, " \"%399[^\"]\" : %d", k, &v) == 2) ent.emplace_back(k, v);
    }
    std::fclose(f);
  }
  return ent;
}

int autotune_lookup(const std::string& key) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  int found = -1;
  for (const auto& e : autotune_read(autotune_path()))
    if (e.first == key) found = e.second;
  return found;
}

// Rewrites the cache with `key` set to `cfg` (through a temporary file renamed
// over the old one).  Returns false when the file cannot be written.
bool autotune_store(const std::string& key, int cfg) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const std::string path = autotune_path();
  std::vector<std::pair<std::string, int>> ent;
  for (const auto& e : autotune_read(path))
    if (e.first != key) ent.push_back(e);
  ent.emplace_back(key, cfg);
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos && slash > 0 && !make_dirs(path.substr(0, slash))) return false;
  const std::string tmp = path + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  std::fprintf(f, "{\n");
  for (size_t i = 0; i < ent.size(); ++i)
    std::fprintf(f, "  \"%s\": %d%s\n", ent[i].first.c_str(), ent[i].second,
                 i + 1 < ent.size() ? "," : "");
  std::fprintf(f, "}\n");
  const bool ok = std::fclose(f) == 0;
  return ok && std::rename(tmp.c_str(), path.c_str()) == 0;
}

// Device buffers and events of the timing runs, released on every exit path.
struct TuneScratch {
  std::vector<void*> bufs;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~TuneScratch() {
    for (void* p : bufs) (void)hipFree(p);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
  template <typename T>
  hipError_t alloc(T** p, size_t count) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count * sizeof(T), 16));
    if (e == hipSuccess) bufs.push_back(q);
    *p = (T*)q;
    return e;
  }
};

pdbo_status upload_dense_tables(pdbo_ctx* c);

pdbo_status autotune_dense(pdbo_ctx* c) {
  const std::string key = autotune_key(c);
  const int cached = autotune_lookup(key);
  if (cached >= 0 && cached < dense_num_cfgs()) {
    c->cfg = cached;
    return PDBO_OK;
  }
  // Scratch copies of everything the step writes: x (both buffers for FP32,
  // whose operand is x itself), y, the operand shadows and x_r.  The rounding
  // changes are not recorded (nflip = nullptr) and no best of B runs.
  TuneScratch ts;
  std::vector<InstDev> tune = c->insts_h;
  const int EB = element_bytes(c->prec);
  for (InstDev& I : tune) {
    const size_t sz = (size_t)I.B * I.ld;
    float *x0 = nullptr, *x1 = nullptr, *y = nullptr;
    uint8_t *s0 = nullptr, *s1 = nullptr;
    int8_t* xr = nullptr;
    HIPCHK(c, ts.alloc(&x0, sz));
    HIPCHK(c, ts.alloc(&y, sz));
    HIPCHK(c, ts.alloc(&xr, sz));
    HIPCHK(c, hipMemcpyAsync(x0, I.X[c->parity], sz * 4, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(y, I.Y, sz * 4, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(xr, I.Xr, sz, hipMemcpyDeviceToDevice, c->stream));
    if (c->prec == PDBO_FP32) {
      HIPCHK(c, ts.alloc(&x1, sz));
      HIPCHK(c, hipMemcpyAsync(x1, x0, sz * 4, hipMemcpyDeviceToDevice, c->stream));
      I.X[c->parity] = x0;
      I.X[c->parity ^ 1] = x1;
      I.Xs[c->parity] = (uint8_t*)x0;
      I.Xs[c->parity ^ 1] = (uint8_t*)x1;
    } else {
      HIPCHK(c, ts.alloc(&s0, sz * EB));
      HIPCHK(c, ts.alloc(&s1, sz * EB));
      HIPCHK(c, hipMemcpyAsync(s0, I.Xs[c->parity], sz * EB, hipMemcpyDeviceToDevice, c->stream));
      I.X[0] = I.X[1] = x0;
      I.Xs[c->parity] = s0;
      I.Xs[c->parity ^ 1] = s1;
    }
    I.Y = y;
    I.Xr = xr;
    I.nflip = nullptr;
    I.fbits = nullptr;
  }
  InstDev* idv = nullptr;
  HIPCHK(c, ts.alloc(&idv, tune.size()));
  HIPCHK(c, hipEventCreate(&ts.e0));
  HIPCHK(c, hipEventCreate(&ts.e1));
  const int cfg0 = c->cfg;
  int best = cfg0;
  float best_ms = 1e30f;
  for (int id = 0; id < dense_num_cfgs(); ++id) {
    c->cfg = id;
    build_tiles(c);
    for (size_t k = 0; k < tune.size(); ++k) tune[k].mblocks = c->insts_h[k].mblocks;
    TileDev* td = nullptr;
    HIPCHK(c, ts.alloc(&td, c->tiles_h.size()));
    HIPCHK(c, hipMemcpyAsync(td, c->tiles_h.data(), c->tiles_h.size() * sizeof(TileDev),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(idv, tune.data(), tune.size() * sizeof(InstDev), hipMemcpyHostToDevice,
                             c->stream));
    const int nt = (int)c->tiles_h.size();
    // one untimed launch (first use of the kernel), then three timed ones; the
    // scratch iterate advances from launch to launch as in a run
    int par = c->parity;
    HIPCHK(c, launch_dense_gemm(id, c->prec, EPI_STEP, c->par.g_kind, td, nt, idv, par, 0, c->stream));
    par ^= 1;
    HIPCHK(c, hipEventRecord(ts.e0, c->stream));
    constexpr int reps = 3;
    for (int r = 0; r < reps; ++r, par ^= 1)
      HIPCHK(c, launch_dense_gemm(id, c->prec, EPI_STEP, c->par.g_kind, td, nt, idv, par, 0,
                                  c->stream));
    HIPCHK(c, hipEventRecord(ts.e1, c->stream));
    HIPCHK(c, hipEventSynchronize(ts.e1));
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, ts.e0, ts.e1));
    if (ms < best_ms) {
      best_ms = ms;
      best = id;
    }
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));  // before the scratch buffers are freed
  c->cfg = best;
  (void)autotune_store(key, best);  // an unwritable cache only costs a re-tune next time
  return PDBO_OK;
}

// Iterations after init or set_state in which the evaluation GEMM runs:
// PDBO_FULL_EVAL_ITERS, default 64.  Afterwards a restart whose rounded
// iterate changed in more than kFlipMax coordinates is evaluated by rows in
// the incremental kernel, which is exact but slow; on the workloads here no
// restart does after about 20 iterations.
int64_t full_eval_iters() {
  const char* e = std::getenv("PDBO_FULL_EVAL_ITERS");
  if (e && *e) {
    const long v = std::strtol(e, nullptr, 10);
    if (v >= 0) return v;
  }
  return 64;
}

// Workgroups of a row-parallel launch (MIS, Max-k-Cut): each writes one partial
// objective per restart of its slice, which the best-of-B launch then sums, so
// more workgroups hide more gather latency in the step and cost more in the
// best of B.  Measured per iteration (2048 / 1024 / 512 workgroups): Max-3-Cut
// n = 10^4, B = 100: 43.7 / 41.9 / 54.7 us; MIS n = 5*10^4, B = 10, d = 3:
// 19.5 / 17.9 / 19.4 us, d = 100: 63.1 / 61.9 / 66.2 us.  PDBO_ROWPAR_GRID
// overrides the default of 1024.
int rowpar_grid_cap() {
  const char* e = std::getenv("PDBO_ROWPAR_GRID");
  if (e && *e) {
    const long v = std::strtol(e, nullptr, 10);
    if (v >= 1 && v <= (1 << 20)) return (int)v;
  }
  return 1024;
}

// With incremental evaluation an iteration's best of B is left pending: it
// runs in extra workgroups of the next step launch (on CUs the tiles leave
// free), or in a launch of its own when the steps stop (flush_argmin).
// The evaluation GEMM, one pass per int8 limb of Ahat (instances with fewer
// limbs skip the later passes).
hipError_t launch_eval_gemm(const pdbo_ctx* c, const TileDev* tiles, int ntiles,
                            const InstDev* insts, hipStream_t s) {
  int L = 1;
  for (const InstDev& I : c->insts_h) L = std::max(L, I.nlimb);
  for (int l = 0; l < L; ++l) {
    hipError_t e = launch_dense_gemm(c->cfg, c->prec, EPI_EVAL, 0, tiles, ntiles, insts, l, 0, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

pdbo_status dense_one_step(pdbo_ctx* c) {
  const bool do_eval = ((c->t_host + 1) % c->eval_every) == 0;
  const int ninst = (int)c->insts_h.size();
  const bool incr = c->incr_off.back() > 0;  // every instance, eval_every = 1
  const bool full = do_eval && (!incr || c->t_host < c->full_until);
  TimedLaunch tl;
  if (c->par.dual_kind == PDBO_DUAL_SCALAR)
    HIPCHK(c, launch_dual_scalar(c->insts_d, ninst, c->B, c->par.g_kind, c->parity, c->stream));
  if (c->grouped) {
    t_begin(c, tl, PDBO_K_STEP);
    HIPCHK(c, launch_dense_gemm(c->cfg, c->prec, EPI_STEP, c->par.g_kind, c->tiles_d,
                                (int)c->tiles_h.size(), c->insts_d, c->parity, 0, c->stream, 0,
                                c->argmin_pending ? ninst : 0));
    t_end(c, tl);
    if (do_eval) {
      // full products only for the column blocks that need them; then the
      // exact differences of every restart with few rounding changes
      if (full) {
        t_begin(c, tl, PDBO_K_EVAL);
        HIPCHK(c, launch_eval_gemm(c, c->tiles_d, (int)c->tiles_h.size(), c->insts_d, c->stream));
        t_end(c, tl);
      }
      if (incr) {
        t_begin(c, tl, PDBO_K_INCR);
        HIPCHK(c, launch_eval_incr(c->insts_d, c->incr_work_d, c->incr_off.back(), full ? 1 : 0,
                                   c->stream));
        t_end(c, tl);
      }
    }
    if (!incr) {
      t_begin(c, tl, PDBO_K_ARGMIN);
      HIPCHK(c, launch_argmin(c->insts_d, 0, ninst, do_eval ? 1 : 0, c->stream));
      t_end(c, tl);
    }
  } else {
    for (int k = 0; k < ninst; ++k) {
      t_begin(c, tl, PDBO_K_STEP);
      HIPCHK(c, launch_dense_gemm(c->cfg, c->prec, EPI_STEP, c->par.g_kind,
                                  c->tiles_d + c->tile_off[k], c->tile_cnt[k], c->insts_d,
                                  c->parity, 0, c->stream, k, c->argmin_pending ? 1 : 0));
      t_end(c, tl);
    }
    if (do_eval)
      for (int k = 0; k < ninst; ++k) {
        if (full) {
          t_begin(c, tl, PDBO_K_EVAL);
          HIPCHK(c, launch_eval_gemm(c, c->tiles_d + c->tile_off[k], c->tile_cnt[k], c->insts_d,
                                     c->stream));
          t_end(c, tl);
        }
        const int w0 = c->incr_off[k], nw = c->incr_off[k + 1] - w0;
        if (nw > 0) {
          t_begin(c, tl, PDBO_K_INCR);
          HIPCHK(c, launch_eval_incr(c->insts_d, c->incr_work_d + w0, nw, full ? 1 : 0, c->stream));
          t_end(c, tl);
        }
      }
    if (!incr)
      for (int k = 0; k < ninst; ++k) {
        t_begin(c, tl, PDBO_K_ARGMIN);
        HIPCHK(c, launch_argmin(c->insts_d, k, 1, do_eval ? 1 : 0, c->stream));
        t_end(c, tl);
      }
  }
  c->argmin_pending = incr;
  c->parity ^= 1;
  c->t_host += 1;
  return PDBO_OK;
}

pdbo_status flush_argmin(pdbo_ctx* c) {
  if (!c->argmin_pending) return PDBO_OK;
  TimedLaunch tl;
  t_begin(c, tl, PDBO_K_ARGMIN);
  HIPCHK(c, launch_argmin(c->insts_d, 0, (int)c->insts_h.size(), 1, c->stream));
  t_end(c, tl);
  c->argmin_pending = false;
  return PDBO_OK;
}

pdbo_status dense_steps(pdbo_ctx* c, int nsteps) {
  const int K = c->par.graph_chunk;
  const bool use_graph = K > 0 && c->eval_every == 1 && !c->timing;
  int left = nsteps;
  while (left > 0) {
    // graphs hold iterations past the transient (no evaluation GEMM)
    if (use_graph && left >= K && c->t_host >= c->full_until) {
      if (!c->gexec) {
        // The caller's stream may be the legacy default stream, which cannot
        // be captured: record the K iterations on a private stream (nothing
        // executes there) and launch the graph on the caller's stream.
        if (!c->cap_stream)
          HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        STCHK(flush_argmin(c));  // a graph starts and ends with nothing pending
        HIPCHK(c, hipStreamSynchronize(c->stream));
        const int64_t t_save = c->t_host;
        const int par_save = c->parity;
        hipStream_t user = c->stream;
        c->stream = c->cap_stream;
        hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
          c->stream = user;
          return hipfail(c, "hipStreamBeginCapture", e);
        }
        pdbo_status st = PDBO_OK;
        for (int s = 0; s < K && st == PDBO_OK; ++s) st = dense_one_step(c);
        if (st == PDBO_OK) st = flush_argmin(c);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(c->stream, &g);
        c->stream = user;
        c->t_host = t_save;
        c->parity = par_save;
        c->argmin_pending = false;
        if (st != PDBO_OK) {
          if (g) (void)hipGraphDestroy(g);
          return st;
        }
        if (e != hipSuccess) return hipfail(c, "hipStreamEndCapture", e);
        c->graph = g;
        HIPCHK(c, hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0));
        c->graph_parity0 = par_save;
      }
      if (c->parity != c->graph_parity0) {
        STCHK(dense_one_step(c));
        --left;
        continue;
      }
      STCHK(flush_argmin(c));
      HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
      c->t_host += K;
      left -= K;
    } else {
      STCHK(dense_one_step(c));
      --left;
    }
  }
  return flush_argmin(c);
}

double clock_rate_hz() {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1e8;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    return 1e8;
  return (double)khz * 1e3;
}

bool is_real(const pdbo_ctx* c) { return c->kind == 3 && c->spmm.ndig > 0; }

pdbo_status fill_result(pdbo_ctx* c, const Incumbent* inc_d, const uint8_t* best_x_d, int n,
                        pdbo_result* r) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  Incumbent inc;
  uint64_t ts0 = 0;
  HIPCHK(c, hipMemcpy(&inc, inc_d, sizeof(inc), hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(&ts0, c->ts0_d, sizeof(ts0), hipMemcpyDeviceToHost));
  r->steps_done = c->t_host;
  if (inc.F == kI64Max) {
    r->best_obj = 0;
    r->best_obj_f64 = HUGE_VAL;
    r->best_restart = -1;
    r->best_iter = -1;
    r->time_to_best_s = 0.0;
    return PDBO_OK;
  }
  if (is_real(c)) {  // the incumbent holds the bits of the rounded value
    std::memcpy(&r->best_obj_f64, &inc.F, sizeof(double));
    r->best_obj = 0;
  } else {
    r->best_obj = inc.F;
    r->best_obj_f64 = (double)inc.F;
  }
  r->best_restart = (int32_t)inc.b;
  r->best_iter = inc.t;
  r->time_to_best_s = (inc.ts >= ts0 && ts0) ? (double)(inc.ts - ts0) / clock_rate_hz() : 0.0;
  if (r->best_x) HIPCHK(c, hipMemcpy(r->best_x, best_x_d, (size_t)n, hipMemcpyDeviceToHost));
  return PDBO_OK;
}

pdbo_status begin_ctx(pdbo_ctx* c, void* stream, const pdbo_params* p) {
  c->stream = (hipStream_t)stream;
  c->par = *p;
  c->par.x0 = nullptr;
  c->B = p->B;
  c->prec = p->precision;
  c->eval_every = p->eval_every;
  STCHK(dalloc(c, &c->ts0_d, 1));
  return PDBO_OK;
}


// ------------------------------------------------ evaluation without allocation
//
// qubo_gda_eval_noalloc stages the caller's rounded vectors and keeps the
// integer partial sums of the dense evaluation in this file-scope array, so
// that it calls no allocator.  Each GPU the library runs on holds its own copy
// until the process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (the array's name is a
// host-side stand-in, not a device address).
constexpr size_t kNoallocScratchBytes = size_t(16) << 20;
constexpr size_t kNoallocDescBytes = 512;  // room for one InstDev, 256-byte aligned
static_assert(sizeof(InstDev) <= kNoallocDescBytes, "descriptor slot");
static __device__ __align__(256) uint8_t scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch_ptr[kMaxDevices] = {};

pdbo_status scratch_for_current_device(pdbo_ctx* c, uint8_t** out) {
  int dev = -1;
  HIPCHK(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(c, PDBO_EUNSUPPORTED, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(c, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = (uint8_t*)p;
  }
  *out = g_scratch_ptr[dev];
  return PDBO_OK;
}

// xs[b][j] = [xr[b][j] != 0] for j < n, 0 for n <= j < ld (the padding the
// 128-byte K chunks of the evaluation GEMM read).
__global__ void stage_rounded_kernel(const uint8_t* __restrict__ xr, int nb, int n, int ld,
                                     int8_t* __restrict__ xs) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nb * ld) return;
  const int b = (int)(idx / ld), j = (int)(idx % ld);
  xs[idx] = j < n ? (int8_t)(xr[(size_t)b * n + j] != 0) : (int8_t)0;
}

// Writes the instance descriptor of the evaluation into the scratch array and
// clears the integer partial sums S, C that the evaluation GEMM accumulates
// into (the last call on this GPU may have left anything there).
__global__ void put_eval_desc_kernel(InstDev* dst, InstDev v, int64_t* S, int64_t* C, int nb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *dst = v;
  if (i < nb) {
    S[i] = 0;
    C[i] = 0;
  }
}

}  // namespace

// =================================================================== ABI

extern "C" {

const char* pdbo_status_str(pdbo_status s) {
  switch (s) {
    case PDBO_OK: return "ok";
    case PDBO_EINVAL: return "invalid argument";
    case PDBO_ENOMEM: return "out of memory";
    case PDBO_EDEVICE: return "device error";
    case PDBO_ERANGE: return "exactness guard failed";
    case PDBO_ESTATE: return "invalid state";
    case PDBO_EUNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* pdbo_last_error(const pdbo_ctx* ctx) { return ctx ? ctx->err.c_str() : g_last_error.c_str(); }
const char* pdbo_last_global_error(void) { return g_last_error.c_str(); }

const char* pdbo_tile_name(const pdbo_ctx* ctx) {
  if (!ctx) return "";
  if (ctx->kind == 0) return dense_cfg(ctx->cfg).name;
  if (ctx->kind == 1) return csr_variant_name(ctx->csr, ctx->compact);
  if (ctx->kind == 3) return "csr_rows";
  return "";
}

void pdbo_destroy(pdbo_ctx* ctx) {
  if (!ctx) return;
  free_all(ctx);
  delete ctx;
}

static pdbo_status dense_init(int k, const pdbo_qubo* probs, const pdbo_params* pars, int grouped,
                              void* stream, pdbo_ctx** out) {
  if (!out) return fail(nullptr, PDBO_EINVAL, "out is NULL");
  *out = nullptr;
  if (k < 1) return fail(nullptr, PDBO_EINVAL, "k must be >= 1");
  if (!probs || !pars) return fail(nullptr, PDBO_EINVAL, "problem or params is NULL");
  for (int i = 0; i < k; ++i) {
    STCHK(check_qubo(&probs[i]));
    STCHK(check_params(&pars[i], probs[i].n));
    if (probs[i].wtype != PDBO_W_INT32)
      return fail(nullptr, PDBO_EUNSUPPORTED, "batches and dense contexts take int32 weights");
    if (pars[i].B != pars[0].B || pars[i].precision != pars[0].precision ||
        pars[i].g_kind != pars[0].g_kind || pars[i].eval_every != pars[0].eval_every ||
        pars[i].dual_kind != pars[0].dual_kind)
      return fail(nullptr, PDBO_EINVAL, "B, precision, g_kind, dual_kind and eval_every must agree");
  }
  pdbo_ctx* c = new pdbo_ctx();
  c->kind = 0;
  c->grouped = grouped ? 1 : 0;
  c->full_until = full_eval_iters();
  if (pars[0].tile > 0) {
    c->cfg = pars[0].tile - 1;
  } else {
    std::vector<int> ns;
    for (int i = 0; i < k; ++i) ns.push_back(probs[i].n);
    c->cfg = default_cfg(ns, pars[0].B);
  }
  c->insts_h.resize(k);
  // The first instance is canonicalised (host only) before any HIP call, so
  // that its range errors come back on any machine.
  pdbo_status st = PDBO_OK;
  for (int i = 0; i < k && st == PDBO_OK; ++i) {
    DenseCanon C;
    st = canon_dense(&probs[i], C);
    if (st == PDBO_OK && pars[i].precision == PDBO_I8 && C.amax > 127)
      st = fail(nullptr, PDBO_EUNSUPPORTED, "the INT8 operand form needs |Ahat_ij| <= 127");
    if (st == PDBO_OK && i == 0) st = begin_ctx(c, stream, &pars[0]);
    if (st == PDBO_OK) st = setup_dense_instance(c, C, &pars[i], c->insts_h[i]);
    c->n_of.push_back(probs[i].n);
  }
  if (st == PDBO_OK && pars[0].tile == 0) {
    // autotune large problems (or when asked); PDBO_AUTOTUNE=0 keeps the heuristic
    const char* e = std::getenv("PDBO_AUTOTUNE");
    double work = 0;
    for (const InstDev& I : c->insts_h) work += (double)I.n * I.n * I.B;
    const bool want = e ? std::atoi(e) != 0 : work >= (double)(1 << 30);
    if (want) st = autotune_dense(c);
  }
  if (st == PDBO_OK) st = upload_dense_tables(c);
  if (st != PDBO_OK) {
    const std::string msg = c->err.empty() ? g_last_error : c->err;
    pdbo_destroy(c);
    g_last_error = msg;
    return st;
  }
  *out = c;
  return PDBO_OK;
}

// The persistent CSR and MaxSAT kernels are built for the quadratic and the
// entropy g with one dual variable per coordinate.
static bool persistent_ok(const pdbo_params* p) {
  return p->g_kind != PDBO_G_POLY && p->dual_kind == PDBO_DUAL_VECTOR;
}

static pdbo_status persistent_supported(const pdbo_params* p) {
  if (p->g_kind == PDBO_G_POLY)
    return fail(nullptr, PDBO_EUNSUPPORTED, "the persistent kernels take the quadratic or entropy g");
  if (p->dual_kind != PDBO_DUAL_VECTOR)
    return fail(nullptr, PDBO_EUNSUPPORTED, "the scalar dual is built for the dense path only");
  return PDBO_OK;
}

static pdbo_status spmm_init(const CsrCanon* C, const RealCanon* R, const pdbo_params* p,
                             void* stream, pdbo_ctx** out);

static pdbo_status csr_init(const pdbo_qubo* q, const pdbo_params* p, void* stream, pdbo_ctx** out) {
  if (p->eval_every != 1) return fail(nullptr, PDBO_EUNSUPPORTED, "the CSR path evaluates every iteration");
  if (p->tile > PDBO_CSR_ROWS)
    return fail(nullptr, PDBO_EINVAL, "CSR instances take tile 0 (automatic), 1 (restart-resident) "
                                      "or 2 (row-parallel)");
  CsrCanon C;
  STCHK(canon_csr(q, C));
  const int n = q->n;
  const bool compact = n <= 65536 && C.amax <= 32767;  // packed 16-bit column / 16-bit value
  const bool fits = csr_fits(n, (int64_t)C.col.size(), compact, nullptr);
  int path = p->tile;
  if (path == PDBO_CSR_AUTO)
    path = (fits && p->B >= kResidentMinB && persistent_ok(p)) ? PDBO_CSR_RESIDENT : PDBO_CSR_ROWS;
  if (path == PDBO_CSR_ROWS) return spmm_init(&C, nullptr, p, stream, out);
  STCHK(persistent_supported(p));
  if (!fits)
    return fail(nullptr, PDBO_EUNSUPPORTED, "instance too large for the restart-resident CSR kernel");
  pdbo_ctx* c = new pdbo_ctx();
  c->kind = 1;
  c->compact = compact;
  c->n_of.push_back(n);
  pdbo_status st = begin_ctx(c, stream, p);
  auto run = [&]() -> pdbo_status {
    const int B = p->B, ld = roundup(n, kLdAlign);
    const int64_t nnz = (int64_t)C.col.size();
    CsrDev& d = c->csr;
    std::memset(&d, 0, sizeof(d));
    d.n = n;
    d.ld = ld;
    d.B = B;
    d.kappa = C.kappa;
    d.nnz = nnz;
    d.kos = (float)((double)C.kappa / p->scale);
    d.gp = make_gp(p);
    int64_t cmax = 0;
    for (int i = 0; i < n; ++i) cmax = std::max<int64_t>(cmax, C.cp[i] < 0 ? -C.cp[i] : C.cp[i]);
    {
      // a wave of the 1024-thread kernel sums at most 64 x 8 rows
      const int64_t lim = int64_t(1) << 31;
      d.small32 = (512 * C.rowabs < lim && 512 * cmax < lim) ? 1 : 0;
      d.tot32 = (d.small32 && (int64_t)n * C.rowabs < lim && (int64_t)n * cmax < lim) ? 1 : 0;
    }
    int32_t* rp = nullptr;
    STCHK(dalloc(c, &rp, n + 1));
    HIPCHK(c, hipMemcpyAsync(rp, C.rp.data(), (n + 1) * 4, hipMemcpyHostToDevice, c->stream));
    d.row_ptr = rp;
    // rows by decreasing degree (ties by index): a wave's rows then have
    // nearly the same number of entries
    std::vector<int32_t> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
      return C.rp[a + 1] - C.rp[a] > C.rp[b + 1] - C.rp[b];
    });
    int32_t* ord = nullptr;
    STCHK(dalloc(c, &ord, n));
    HIPCHK(c, hipMemcpyAsync(ord, order.data(), (size_t)n * 4, hipMemcpyHostToDevice, c->stream));
    d.order = ord;
    // host staging lives until the stream is synchronised at the end of init
    std::vector<uint32_t> pk, psl;
    std::vector<int32_t> slo;
    int32_t* col = nullptr;
    int32_t* val = nullptr;
    STCHK(dalloc(c, &col, nnz));
    STCHK(dalloc(c, &val, nnz));
    HIPCHK(c, hipMemcpyAsync(col, C.col.data(), nnz * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(val, C.val.data(), nnz * 4, hipMemcpyHostToDevice, c->stream));
    d.col = col;
    d.val = val;
    if (compact) {
      pk.resize(nnz);
      for (int64_t q = 0; q < nnz; ++q)
        pk[q] = (uint32_t)C.col[q] | ((uint32_t)(uint16_t)(int16_t)C.val[q] << 16);
      uint32_t* dp = nullptr;
      STCHK(dalloc(c, &dp, nnz));
      HIPCHK(c, hipMemcpyAsync(dp, pk.data(), nnz * 4, hipMemcpyHostToDevice, c->stream));
      d.packed = dp;
    }
    const char* sl_env = std::getenv("PDBO_CSR_SLICED");
    if (compact && n <= 8192 && !(sl_env && std::atoi(sl_env) == 0)) {
      // the interleaved layout of the 1024-thread kernels (slices of 64
      // positions, each as long as its longest row), used when it takes no
      // more LDS than row_ptr and the entries in CSR order
      const int ns = (n + 63) / 64;
      slo.assign(ns, 0);
      int64_t tot = 0;
      for (int s = 0; s < ns; ++s) {
        slo[s] = (int32_t)tot;
        int lmax = 0;
        for (int q = s * 64; q < std::min(n, s * 64 + 64); ++q)
          lmax = std::max(lmax, (int)(C.rp[order[q] + 1] - C.rp[order[q]]));
        tot += (int64_t)64 * lmax;
      }
      auto a16 = [](int64_t v) { return (v + 15) / 16 * 16; };
      if (a16(4 * tot) <= a16(4 * (int64_t)(n + 1)) + a16(4 * nnz)) {
        psl.assign((size_t)tot, 0u);
        for (int q = 0; q < n; ++q) {
          const int i = order[q];
          size_t f = (size_t)slo[q / 64] + (q % 64);
          for (int64_t e = C.rp[i]; e < C.rp[i + 1]; ++e, f += 64) psl[f] = pk[e];
        }
        uint32_t* dsl = nullptr;
        int32_t* dso = nullptr;
        STCHK(dalloc(c, &dsl, std::max<int64_t>(tot, 1)));
        STCHK(dalloc(c, &dso, ns));
        HIPCHK(c, hipMemcpyAsync(dsl, psl.data(), (size_t)tot * 4, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(dso, slo.data(), (size_t)ns * 4, hipMemcpyHostToDevice, c->stream));
        d.psl = dsl;
        d.slice = dso;
        d.nsl = tot;
      }
    }
    std::vector<float> hcps(ld, 0.f);
    std::vector<int64_t> hcp(ld, 0);
    for (int i = 0; i < n; ++i) {
      hcp[i] = C.cp[i];
      hcps[i] = (float)((double)C.cp[i] / p->scale);
    }
    float* cps = nullptr;
    int64_t* cp = nullptr;
    STCHK(dalloc(c, &cps, ld));
    STCHK(dalloc(c, &cp, ld));
    HIPCHK(c, hipMemcpyAsync(cps, hcps.data(), ld * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(cp, hcp.data(), ld * 8, hipMemcpyHostToDevice, c->stream));
    d.cps = cps;
    d.cp = cp;
    STCHK(dalloc(c, &d.X, (size_t)B * ld));
    STCHK(dalloc(c, &d.Y, (size_t)B * ld));
    STCHK(dalloc(c, &d.rbestF, B));
    STCHK(dalloc(c, &d.rbestT, B));
    STCHK(dalloc(c, &d.rbestTs, B));
    STCHK(dalloc(c, &d.best_xr, (size_t)B * n));
    STCHK(dalloc(c, &d.Flast, B));
    STCHK(dalloc(c, &c->inc_d, 1));
    STCHK(dalloc(c, &c->best_x_d, n));
    HIPCHK(c, launch_fill_i64(d.rbestF, kI64Max, B, c->stream));
    HIPCHK(c, launch_fill_i64(d.rbestT, kI64Max, B, c->stream));
    Incumbent init{kI64Max, -1, -1, 0};
    HIPCHK(c, hipMemcpyAsync(c->inc_d, &init, sizeof(init), hipMemcpyHostToDevice, c->stream));
    TempDev t;
    STCHK(upload_x0(c, t, p->x0, (size_t)B * n));
    HIPCHK(c, launch_init_state((const double*)t.p, B, n, ld, (float)p->y0, d.X, d.Y, nullptr,
                                P_F32, nullptr, p->seed, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PDBO_OK;
  };
  if (st == PDBO_OK) st = run();
  if (st != PDBO_OK) {
    const std::string msg = c->err.empty() ? g_last_error : c->err;
    pdbo_destroy(c);
    g_last_error = msg;
    return st;
  }
  *out = c;
  return PDBO_OK;
}

// Row-parallel CSR path (spmm.hip): node-major iterates, one launch per
// iteration over all rows plus the best of B.  C: integer weights; R: float64
// weights (realw.hip).
static pdbo_status spmm_init(const CsrCanon* C, const RealCanon* R, const pdbo_params* p,
                             void* stream, pdbo_ctx** out) {
  if (p->dual_kind != PDBO_DUAL_VECTOR)
    return fail(nullptr, PDBO_EUNSUPPORTED, "the scalar dual is built for the dense path only");
  const int n = C ? C->n : R->n, B = p->B;
  pdbo_ctx* c = new pdbo_ctx();
  c->kind = 3;
  c->n_of.push_back(n);
  pdbo_status st = begin_ctx(c, stream, p);
  auto run = [&]() -> pdbo_status {
    const std::vector<int32_t>& hrp = C ? C->rp : R->rp;
    const std::vector<int32_t>& hcol = C ? C->col : R->col;
    const int64_t nnz = (int64_t)hcol.size();
    std::vector<uint32_t> hpk;  // host staging, alive until init syncs
    SpmmDev& d = c->spmm;
    std::memset(&d, 0, sizeof(d));
    d.n = n;
    d.B = B;
    d.nnz = nnz;
    d.kappa = C ? C->kappa : 1;
    d.trace_cap = kTraceCap;
    d.kos = C ? (float)((double)C->kappa / p->scale) : 1.f;
    d.gp = make_gp(p);
    d.W = std::min(B, 64);
    d.G = 64 / d.W;
    d.nslices = (B + d.W - 1) / d.W;
    const int rows_per_wg = 4 * d.G;
    const int nrb = (n + rows_per_wg - 1) / rows_per_wg;
    const int gpw = std::max(1, std::min(nrb, std::max(1, rowpar_grid_cap() / d.nslices)));
    d.grid = gpw * d.nslices;
    int32_t *rp = nullptr, *col = nullptr;
    float* cps = nullptr;
    STCHK(dalloc(c, &rp, n + 1));
    STCHK(dalloc(c, &col, nnz));
    STCHK(dalloc(c, &cps, n));
    HIPCHK(c, hipMemcpyAsync(rp, hrp.data(), (n + 1) * 4, hipMemcpyHostToDevice, c->stream));
    if (nnz > 0)
      HIPCHK(c, hipMemcpyAsync(col, hcol.data(), nnz * 4, hipMemcpyHostToDevice, c->stream));
    d.row_ptr = rp;
    d.col = col;
    d.cps = cps;
    std::vector<float> hcps(n);
    if (C) {
      int32_t* val = nullptr;
      int64_t* cp = nullptr;
      STCHK(dalloc(c, &val, nnz));
      STCHK(dalloc(c, &cp, n));
      for (int i = 0; i < n; ++i) hcps[i] = (float)((double)C->cp[i] / p->scale);
      if (nnz > 0)
        HIPCHK(c, hipMemcpyAsync(val, C->val.data(), nnz * 4, hipMemcpyHostToDevice, c->stream));
      HIPCHK(c, hipMemcpyAsync(cp, C->cp.data(), n * 8, hipMemcpyHostToDevice, c->stream));
      d.val = val;
      d.cp = cp;
      if (n <= 65536 && C->amax <= 32767 && nnz > 0) {
        // one 4-byte word per entry (16-bit column, 16-bit value)
        hpk.resize((size_t)nnz);
        for (int64_t q = 0; q < nnz; ++q)
          hpk[q] = (uint32_t)hcol[q] | ((uint32_t)(uint16_t)(int16_t)C->val[q] << 16);
        uint32_t* dpk = nullptr;
        STCHK(dalloc(c, &dpk, nnz));
        HIPCHK(c, hipMemcpyAsync(dpk, hpk.data(), (size_t)nnz * 4, hipMemcpyHostToDevice, c->stream));
        d.packed = dpk;
      }
    } else {
      float* valf = nullptr;
      int32_t *Adig = nullptr, *Cdig = nullptr;
      d.ndig = R->ndig;
      d.elo = R->elo;
      STCHK(dalloc(c, &valf, nnz));
      STCHK(dalloc(c, &Adig, (size_t)R->ndig * nnz));
      STCHK(dalloc(c, &Cdig, (size_t)R->ndig * n));
      hcps = R->cps;
      if (nnz > 0) {
        HIPCHK(c, hipMemcpyAsync(valf, R->valf.data(), nnz * 4, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(Adig, R->Adig.data(), (size_t)R->ndig * nnz * 4,
                                 hipMemcpyHostToDevice, c->stream));
      }
      HIPCHK(c, hipMemcpyAsync(Cdig, R->Cdig.data(), (size_t)R->ndig * n * 4, hipMemcpyHostToDevice,
                               c->stream));
      d.valf = valf;
      d.Adig = Adig;
      d.Cdig = Cdig;
      STCHK(dalloc(c, &d.incw, 4));
      STCHK(dalloc(c, &d.Fd, B));
      const uint64_t top[4] = {~0ull, ~0ull, ~0ull, ~0ull >> 1};
      HIPCHK(c, hipMemcpyAsync(d.incw, top, sizeof(top), hipMemcpyHostToDevice, c->stream));
    }
    HIPCHK(c, hipMemcpyAsync(cps, hcps.data(), n * 4, hipMemcpyHostToDevice, c->stream));
    const size_t sz = (size_t)n * B;
    STCHK(dalloc(c, &d.X[0], sz));
    STCHK(dalloc(c, &d.X[1], sz));
    STCHK(dalloc(c, &d.Y, sz));
    STCHK(dalloc(c, &d.part, (size_t)d.grid * 2 * d.W * std::max(1, d.ndig)));
    STCHK(dalloc(c, &d.Flast, B));
    STCHK(dalloc(c, &d.inc, 1));
    STCHK(dalloc(c, &d.best_x, n));
    STCHK(dalloc(c, &d.trace, kTraceCap));
    STCHK(dalloc(c, &d.trace_len, 1));
    STCHK(dalloc(c, &d.t_dev, 1));
    d.ts0 = c->ts0_d;
    Incumbent init{kI64Max, -1, -1, 0};
    HIPCHK(c, hipMemcpyAsync(d.inc, &init, sizeof(init), hipMemcpyHostToDevice, c->stream));
    d.win = nullptr;
    if (C) {  // integer weights: the winner copy rides on the next step launch
      STCHK(dalloc(c, &d.win, 1));
      HIPCHK(c, launch_fill_i32(d.win, -1, 1, c->stream));
    }
    if (C) {
      // qubo_gda_eval of given vectors goes through the restart-major CSR kernel
      CsrDev& e = c->csr;
      std::memset(&e, 0, sizeof(e));
      e.row_ptr = rp;
      e.col = col;
      e.val = d.val;
      e.cps = cps;
      e.cp = d.cp;
      e.nnz = nnz;
      e.n = n;
      e.ld = roundup(n, kLdAlign);
      e.B = B;
      e.kappa = C->kappa;
      e.kos = d.kos;
      e.gp = d.gp;
    }
    TempDev t;
    STCHK(upload_x0(c, t, p->x0, (size_t)B * n));
    HIPCHK(c, launch_spmm_init((const double*)t.p, d, (float)p->y0, p->seed, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PDBO_OK;
  };
  if (st == PDBO_OK) st = run();
  if (st != PDBO_OK) {
    const std::string msg = c->err.empty() ? g_last_error : c->err;
    pdbo_destroy(c);
    g_last_error = msg;
    return st;
  }
  *out = c;
  return PDBO_OK;
}

// Float64 weights: exact fixed-point canonical form, row-parallel CSR path.
static pdbo_status real_init(const pdbo_qubo* q, const pdbo_params* p, void* stream,
                             pdbo_ctx** out) {
  if (p->eval_every != 1) return fail(nullptr, PDBO_EUNSUPPORTED, "the CSR path evaluates every iteration");
  if (p->tile != PDBO_CSR_AUTO && p->tile != PDBO_CSR_ROWS)
    return fail(nullptr, PDBO_EUNSUPPORTED, "float64 weights run on the row-parallel CSR path "
                                            "(tile 0 or 2)");
  RealCanon R;
  STCHK(canon_real(q, p->scale, R));
  return spmm_init(nullptr, &R, p, stream, out);
}

pdbo_status spmm_one_step(pdbo_ctx* c) {
  TimedLaunch tl;
  t_begin(c, tl, PDBO_K_STEP);
  HIPCHK(c, launch_spmm(c->spmm, 0, c->parity, nullptr, c->stream));
  t_end(c, tl);
  t_begin(c, tl, PDBO_K_ARGMIN);
  HIPCHK(c, launch_spmm_best(c->spmm, c->parity, 1, c->stream));
  t_end(c, tl);
  c->parity ^= 1;
  c->t_host += 1;
  return PDBO_OK;
}

pdbo_status kcut_one_step(pdbo_ctx* c) {
  TimedLaunch tl;
  t_begin(c, tl, PDBO_K_STEP);
  HIPCHK(c, launch_kcut(c->kcut, 0, c->parity, nullptr, c->stream));
  t_end(c, tl);
  t_begin(c, tl, PDBO_K_ARGMIN);
  HIPCHK(c, launch_kcut_best(c->kcut, c->parity, 1, c->stream));
  t_end(c, tl);
  c->parity ^= 1;
  c->t_host += 1;
  return PDBO_OK;
}

// The row-parallel paths (kinds 3 and 4): each iteration evaluates round(x^t)
// in the gathers of its own gradient, so after the last one the rounded x^T
// is evaluated by a pass of its own.  With graph_chunk = K, K iterations are
// recorded once (on a private stream: the caller's may be the legacy default)
// and replayed.
pdbo_status rowpar_steps(pdbo_ctx* c, int nsteps, pdbo_status (*one)(pdbo_ctx*)) {
  const int K = c->par.graph_chunk;
  const bool use_graph = K > 0 && !c->timing;
  int left = nsteps;
  while (left > 0) {
    if (use_graph && left >= K) {
      if (!c->gexec) {
        if (!c->cap_stream)
          HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        const int64_t t_save = c->t_host;
        const int par_save = c->parity;
        hipStream_t user = c->stream;
        c->stream = c->cap_stream;
        hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
          c->stream = user;
          return hipfail(c, "hipStreamBeginCapture", e);
        }
        pdbo_status st = PDBO_OK;
        for (int k = 0; k < K && st == PDBO_OK; ++k) st = one(c);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(c->stream, &g);
        c->stream = user;
        c->t_host = t_save;
        c->parity = par_save;
        if (st != PDBO_OK) {
          if (g) (void)hipGraphDestroy(g);
          return st;
        }
        if (e != hipSuccess) return hipfail(c, "hipStreamEndCapture", e);
        c->graph = g;
        HIPCHK(c, hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0));
        c->graph_parity0 = par_save;
      }
      if (c->parity != c->graph_parity0) {
        STCHK(one(c));
        --left;
        continue;
      }
      HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
      c->t_host += K;
      c->parity ^= (K & 1);
      left -= K;
    } else {
      STCHK(one(c));
      --left;
    }
  }
  TimedLaunch tl;
  t_begin(c, tl, PDBO_K_EVAL);
  if (c->kind == 3)
    HIPCHK(c, launch_spmm(c->spmm, 1, c->parity, nullptr, c->stream));
  else
    HIPCHK(c, launch_kcut(c->kcut, 1, c->parity, nullptr, c->stream));
  t_end(c, tl);
  t_begin(c, tl, PDBO_K_ARGMIN);
  if (c->kind == 3)
    HIPCHK(c, launch_spmm_best(c->spmm, c->parity, 0, c->stream));
  else
    HIPCHK(c, launch_kcut_best(c->kcut, c->parity, 0, c->stream));
  t_end(c, tl);
  return PDBO_OK;
}

// ---------------------------------------------------------------- dense or CSR per instance
//
// A large single instance (n^2 B >= 2^30) given with tile 0 and FP32 operands
// may run on the path of the other representation when that is faster: a dense
// matrix with at most 10% nonzeros on the CSR paths, a CSR matrix with
// n <= 16384 on the dense one.  Both compute with exact integer weights and
// FP32 iterates; only the order of the FP32 sums differs.
// Both contexts are built and timed over 8 iterations past the dense path's
// evaluation transient; the faster (the other only when at least 10% faster)
// is restarted from x0 and kept.  The choice is cached beside the tile
// configurations, under "route/<arch>/f<format>/n<n>/B<B>/nz<nnz bucket>/p<precision>/g<g kind>"
// with 0 for the given representation and 1 for the other.  PDBO_ROUTE=0 keeps
// the given representation.

struct HostQubo {
  pdbo_qubo q{};
  std::vector<int32_t> vals, rp, ci;
};

// dense row-major -> CSR of the nonzero entries, rows sorted by column
static void host_to_csr(const pdbo_qubo* in, HostQubo& h) {
  const int n = in->n;
  h.rp.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) {
      const int32_t v = in->q[(size_t)i * n + j];
      if (v) {
        h.ci.push_back(j);
        h.vals.push_back(v);
      }
    }
    h.rp[i + 1] = (int32_t)h.ci.size();
  }
  h.q = *in;
  h.q.format = PDBO_CSR;
  h.q.q = h.vals.data();
  h.q.row_ptr = h.rp.data();
  h.q.col_idx = h.ci.data();
  h.q.nnz = (int64_t)h.ci.size();
}

// CSR -> dense row-major
static void host_to_dense(const pdbo_qubo* in, HostQubo& h) {
  const int n = in->n;
  h.vals.assign((size_t)n * n, 0);
  for (int i = 0; i < n; ++i)
    for (int p = in->row_ptr[i]; p < in->row_ptr[i + 1]; ++p)
      h.vals[(size_t)i * n + in->col_idx[p]] = in->q[p];
  h.q = *in;
  h.q.format = PDBO_DENSE;
  h.q.q = h.vals.data();
  h.q.row_ptr = nullptr;
  h.q.col_idx = nullptr;
  h.q.nnz = 0;
}

static pdbo_status init_as_given(const pdbo_qubo* prob, const pdbo_params* par, void* stream,
                                 pdbo_ctx** out) {
  if (prob->format == PDBO_CSR) return csr_init(prob, par, stream, out);
  return dense_init(1, prob, par, 1, stream, out);
}

// Milliseconds of k iterations after `warm` untimed ones.
static pdbo_status time_iterations(pdbo_ctx* c, int warm, int k, float* ms) {
  STCHK(qubo_gda_step(c, warm));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(c, hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
  pdbo_status st = e == hipSuccess ? qubo_gda_step(c, k) : PDBO_OK;
  if (e == hipSuccess && st == PDBO_OK) e = hipEventRecord(e1, c->stream);
  if (e == hipSuccess && st == PDBO_OK) e = hipEventSynchronize(e1);
  if (e == hipSuccess && st == PDBO_OK) e = hipEventElapsedTime(ms, e0, e1);
  (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st != PDBO_OK) return st;
  HIPCHK(c, e);
  return PDBO_OK;
}

pdbo_status qubo_gda_init(const pdbo_qubo* prob, const pdbo_params* par, void* stream,
                          pdbo_ctx** out) {
  if (!out) return fail(nullptr, PDBO_EINVAL, "out is NULL");
  *out = nullptr;
  STCHK(check_qubo(prob));
  STCHK(check_params(par, prob->n));
  if (prob->wtype == PDBO_W_F64) return real_init(prob, par, stream, out);
  const int n = prob->n;
  const char* env = std::getenv("PDBO_ROUTE");
  const bool may = par->tile == 0 && !(env && std::atoi(env) == 0) &&
                   (double)n * n * par->B >= (double)(1 << 30) && par->precision == PDBO_FP32 &&
                   par->eval_every == 1 && par->dual_kind == PDBO_DUAL_VECTOR;
  if (!may) return init_as_given(prob, par, stream, out);
  int64_t nnz = 0;
  if (prob->format == PDBO_DENSE) {
    const size_t tot = (size_t)n * n;
    for (size_t e = 0; e < tot; ++e) nnz += prob->q[e] != 0;
    if (nnz > (int64_t)(tot / 10)) return init_as_given(prob, par, stream, out);
  } else {
    nnz = prob->nnz;
    if (n > 16384) return init_as_given(prob, par, stream, out);
  }
  std::string arch = "unknown";
  {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
  }
  char key[256];
  std::snprintf(key, sizeof(key), "route/%s/f%d/n%d/B%d/nz%lld/p%d/g%d", arch.c_str(), prob->format, n,
                par->B, (long long)((nnz + 1023) / 1024 * 1024), par->precision, par->g_kind);
  const int cached = autotune_lookup(key);
  if (cached == 0) return init_as_given(prob, par, stream, out);
  HostQubo h;
  if (prob->format == PDBO_DENSE)
    host_to_csr(prob, h);
  else
    host_to_dense(prob, h);
  const std::string err0 = g_last_error;  // a refusal of the other path is no error of the call
  if (cached == 1) {
    if (init_as_given(&h.q, par, stream, out) == PDBO_OK) return PDBO_OK;
    g_last_error = err0;
    return init_as_given(prob, par, stream, out);
  }
  pdbo_ctx* a = nullptr;
  STCHK(init_as_given(prob, par, stream, &a));
  pdbo_ctx* b = nullptr;
  if (init_as_given(&h.q, par, stream, &b) != PDBO_OK) {
    g_last_error = err0;
    *out = a;
    return PDBO_OK;
  }
  float ma = 0.f, mb = 0.f;
  pdbo_status st = time_iterations(a, 70, 8, &ma);
  if (st == PDBO_OK) st = time_iterations(b, 70, 8, &mb);
  if (st != PDBO_OK) {
    pdbo_destroy(a);
    pdbo_destroy(b);
    return st;
  }
  const bool other = mb < 0.9f * ma;
  (void)autotune_store(key, other ? 1 : 0);  // an unwritable cache only costs a re-measurement
  pdbo_ctx* keep = other ? b : a;
  pdbo_destroy(other ? a : b);
  st = qubo_gda_restart(keep, par->x0);
  if (st != PDBO_OK) {
    pdbo_destroy(keep);
    return st;
  }
  *out = keep;
  return PDBO_OK;
}

pdbo_status qubo_gda_batch_init(int32_t k, const pdbo_qubo* probs, const pdbo_params* par,
                                int32_t grouped, void* stream, pdbo_ctx** out) {
  return dense_init(k, probs, par, grouped, stream, out);
}

pdbo_status qubo_gda_step(pdbo_ctx* c, int32_t nsteps) {
  if (!c) return fail(nullptr, PDBO_ESTATE, "context is NULL");
  if (nsteps < 0) return fail(c, PDBO_EINVAL, "nsteps must be >= 0");
  if (nsteps == 0) return PDBO_OK;
  if (!c->stamped) {
    HIPCHK(c, launch_stamp(c->ts0_d, c->stream));
    c->stamped = true;
  }
  if (c->kind == 0) return dense_steps(c, nsteps);
  if (c->kind == 3) return rowpar_steps(c, nsteps, spmm_one_step);
  if (c->kind == 4) return rowpar_steps(c, nsteps, kcut_one_step);
  TimedLaunch tl;
  t_begin(c, tl, PDBO_K_PERSISTENT);
  if (c->kind == 1)
    HIPCHK(c, launch_csr_persistent(c->csr, c->compact, c->t_host, nsteps, c->stream));
  else
    HIPCHK(c, launch_sat_persistent(c->sat, c->t_host, nsteps, c->stream));
  t_end(c, tl);
  c->t_host += nsteps;
  return PDBO_OK;
}

pdbo_status qubo_gda_result(pdbo_ctx* c, pdbo_result* r) {
  if (!c || !r) return fail(c, PDBO_EINVAL, "NULL argument");
  if (c->kind == 0) {
    if (c->insts_h.size() != 1) return fail(c, PDBO_ESTATE, "use qubo_gda_batch_result");
    return fill_result(c, c->insts_h[0].inc, c->insts_h[0].best_x, c->insts_h[0].n, r);
  }
  const int B = c->B;
  const int n = c->n_of[0];
  if (c->kind == 3) return fill_result(c, c->spmm.inc, c->spmm.best_x, n, r);
  if (c->kind == 4) return fill_result(c, c->kcut.inc, c->kcut.best_x, n, r);
  if (c->kind == 1)
    HIPCHK(c, launch_restart_best(c->csr.rbestF, c->csr.rbestT, c->csr.rbestTs, c->csr.best_xr, B,
                                  n, c->inc_d, c->best_x_d, c->stream));
  else
    HIPCHK(c, launch_restart_best(c->sat.rbestF, c->sat.rbestT, c->sat.rbestTs, c->sat.best_xr, B,
                                  n, c->inc_d, c->best_x_d, c->stream));
  return fill_result(c, c->inc_d, c->best_x_d, n, r);
}

pdbo_status qubo_gda_batch_result(pdbo_ctx* c, int32_t inst, pdbo_result* r) {
  if (!c || !r) return fail(c, PDBO_EINVAL, "NULL argument");
  if (c->kind != 0 || inst < 0 || inst >= (int)c->insts_h.size())
    return fail(c, PDBO_EINVAL, "instance index out of range");
  return fill_result(c, c->insts_h[inst].inc, c->insts_h[inst].best_x, c->insts_h[inst].n, r);
}

static void state_ptrs(pdbo_ctx* c, float** X, float** Y, int* ld, int* n) {
  if (c->kind == 0) {
    InstDev& I = c->insts_h[0];
    *X = I.X[c->parity];
    *Y = I.Y;
    *ld = I.ld;
    *n = I.n;
  } else if (c->kind == 1) {
    *X = c->csr.X;
    *Y = c->csr.Y;
    *ld = c->csr.ld;
    *n = c->csr.n;
  } else if (c->kind == 3) {  // node-major: callers transpose
    *X = c->spmm.X[c->parity];
    *Y = c->spmm.Y;
    *ld = c->spmm.n;
    *n = c->spmm.n;
  } else {
    *X = c->sat.X;
    *Y = c->sat.Y;
    *ld = c->sat.ld;
    *n = c->sat.n;
  }
}

// Row-parallel CSR: node-major device arrays <-> restart-major host arrays.
static pdbo_status spmm_download(pdbo_ctx* c, const float* src, float* dst) {
  const int n = c->spmm.n, B = c->B;
  std::vector<float> h((size_t)n * B);
  HIPCHK(c, hipMemcpy(h.data(), src, h.size() * sizeof(float), hipMemcpyDeviceToHost));
  for (int i = 0; i < n; ++i)
    for (int b = 0; b < B; ++b) dst[(size_t)b * n + i] = h[(size_t)i * B + b];
  return PDBO_OK;
}

static pdbo_status spmm_upload(pdbo_ctx* c, const float* src, float* dst) {
  const int n = c->spmm.n, B = c->B;
  std::vector<float> h((size_t)n * B);
  for (int i = 0; i < n; ++i)
    for (int b = 0; b < B; ++b) h[(size_t)i * B + b] = src[(size_t)b * n + i];
  HIPCHK(c, hipMemcpy(dst, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
  return PDBO_OK;
}

// Max-k-Cut: node-major [n][B][m] <-> restart-major [B][n][m] (m = k or 1).
static pdbo_status kcut_download(pdbo_ctx* c, const float* src, float* dst, int m) {
  const int n = c->kcut.n, B = c->B;
  std::vector<float> h((size_t)n * B * m);
  HIPCHK(c, hipMemcpy(h.data(), src, h.size() * sizeof(float), hipMemcpyDeviceToHost));
  for (int i = 0; i < n; ++i)
    for (int b = 0; b < B; ++b)
      for (int u = 0; u < m; ++u) dst[((size_t)b * n + i) * m + u] = h[((size_t)i * B + b) * m + u];
  return PDBO_OK;
}

static pdbo_status kcut_upload(pdbo_ctx* c, const float* src, float* dst, int m) {
  const int n = c->kcut.n, B = c->B;
  std::vector<float> h((size_t)n * B * m);
  for (int i = 0; i < n; ++i)
    for (int b = 0; b < B; ++b)
      for (int u = 0; u < m; ++u) h[((size_t)i * B + b) * m + u] = src[((size_t)b * n + i) * m + u];
  HIPCHK(c, hipMemcpy(dst, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
  return PDBO_OK;
}

pdbo_status qubo_gda_get_state(pdbo_ctx* c, float* x, float* y, int64_t* t) {
  if (!c) return fail(nullptr, PDBO_ESTATE, "context is NULL");
  if (c->kind == 0 && c->insts_h.size() != 1) return fail(c, PDBO_ESTATE, "batched context");
  if (c->kind == 4) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (x) STCHK(kcut_download(c, c->kcut.Z, x, c->kcut.k));
    if (y) STCHK(kcut_download(c, c->kcut.Y, y, 1));
    if (t) *t = c->t_host;
    return PDBO_OK;
  }
  if (c->kind == 3) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (x) STCHK(spmm_download(c, c->spmm.X[c->parity], x));
    if (y) STCHK(spmm_download(c, c->spmm.Y, y));
    if (t) *t = c->t_host;
    return PDBO_OK;
  }
  float *X, *Y;
  int ld, n;
  state_ptrs(c, &X, &Y, &ld, &n);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (x)
    HIPCHK(c, hipMemcpy2D(x, n * sizeof(float), X, ld * sizeof(float), n * sizeof(float), c->B,
                          hipMemcpyDeviceToHost));
  if (y && c->kind == 0 && c->insts_h[0].ys) {
    // scalar dual: every coordinate of restart b carries the restart's y
    std::vector<float> ys(c->B);
    HIPCHK(c, hipMemcpy(ys.data(), c->insts_h[0].ys, c->B * sizeof(float), hipMemcpyDeviceToHost));
    for (int b = 0; b < c->B; ++b) std::fill(y + (size_t)b * n, y + (size_t)(b + 1) * n, ys[b]);
  } else if (y) {
    HIPCHK(c, hipMemcpy2D(y, n * sizeof(float), Y, ld * sizeof(float), n * sizeof(float), c->B,
                          hipMemcpyDeviceToHost));
  }
  if (t) *t = c->t_host;
  return PDBO_OK;
}

pdbo_status qubo_gda_set_state(pdbo_ctx* c, const float* x, const float* y, int64_t t) {
  if (!c) return fail(nullptr, PDBO_ESTATE, "context is NULL");
  if (c->kind == 0 && c->insts_h.size() != 1) return fail(c, PDBO_ESTATE, "batched context");
  if (t < 0) return fail(c, PDBO_EINVAL, "t must be >= 0");
  if (c->kind == 4) {  // x: the logits Z (B, n, k); X = softmax(Z) follows
    KcutDev& d = c->kcut;
    const size_t tz = (size_t)c->B * d.n * d.k, ty = (size_t)c->B * d.n;
    if (x)
      for (size_t i = 0; i < tz; ++i)
        if (!std::isfinite(x[i])) return fail(c, PDBO_EINVAL, "Z must be finite");
    if (y)
      for (size_t i = 0; i < ty; ++i)
        if (!std::isfinite(y[i])) return fail(c, PDBO_EINVAL, "y must be finite");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (x) {
      TempDev tx, tyd;
      STCHK(temp_upload(c, tx, x, tz * sizeof(float)));
      if (y) STCHK(temp_upload(c, tyd, y, ty * sizeof(float)));
      HIPCHK(c, launch_kcut_set((const float*)tx.p, (const float*)tyd.p, d, c->parity, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
    } else if (y) {
      STCHK(kcut_upload(c, y, d.Y, 1));
    }
    c->t_host = t;
    HIPCHK(c, hipMemcpy(d.t_dev, &t, sizeof(t), hipMemcpyHostToDevice));
    return PDBO_OK;
  }
  float *X, *Y;
  int ld, n;
  state_ptrs(c, &X, &Y, &ld, &n);
  const size_t tot = (size_t)c->B * n;
  if (x)
    for (size_t i = 0; i < tot; ++i)
      if (!(x[i] >= 0.f && x[i] <= 1.f)) return fail(c, PDBO_EINVAL, "x must lie in [0,1]");
  if (y)
    for (size_t i = 0; i < tot; ++i)
      if (!std::isfinite(y[i])) return fail(c, PDBO_EINVAL, "y must be finite");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->kind == 3) {
    if (x) STCHK(spmm_upload(c, x, c->spmm.X[c->parity]));
    if (y) STCHK(spmm_upload(c, y, c->spmm.Y));
    c->t_host = t;
    HIPCHK(c, hipMemcpy(c->spmm.t_dev, &t, sizeof(t), hipMemcpyHostToDevice));
    return PDBO_OK;
  }
  TempDev tx, ty;
  if (x) STCHK(temp_upload(c, tx, x, tot * sizeof(float)));
  if (y) STCHK(temp_upload(c, ty, y, tot * sizeof(float)));
  uint8_t* Xs = nullptr;
  if (c->kind == 0 && c->prec != PDBO_FP32) Xs = c->insts_h[0].Xs[c->parity];
  HIPCHK(c, launch_set_state((const float*)tx.p, (const float*)ty.p, c->B, n, ld, X, Y, Xs, c->prec,
                             c->stream));
  c->t_host = t;
  c->full_until = t + full_eval_iters();
  if (c->kind == 0 && y && c->insts_h[0].ys) {
    // scalar dual: restart b's y is y[b][0]
    std::vector<float> ys(c->B);
    for (int b = 0; b < c->B; ++b) ys[b] = y[(size_t)b * n];
    HIPCHK(c, hipMemcpyAsync(c->insts_h[0].ys, ys.data(), c->B * sizeof(float), hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  if (c->kind == 0) {
    HIPCHK(c, hipMemcpyAsync(c->insts_h[0].t_dev, &t, sizeof(t), hipMemcpyHostToDevice, c->stream));
    // the rounded iterate no longer follows the recorded changes
    if (c->insts_h[0].nflip)
      HIPCHK(c, launch_fill_i32(c->insts_h[0].nflip, kFlipMax + 1, c->B, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PDBO_OK;
}

pdbo_status qubo_gda_restart(pdbo_ctx* c, const double* x0) {
  if (!c) return fail(nullptr, PDBO_ESTATE, "context is NULL");
  if (c->kind == 0 && c->insts_h.size() != 1) return fail(c, PDBO_ESTATE, "batched context");
  const int n = c->n_of[0], B = c->B;
  if (c->kind == 4) {  // x0: the logits Z^0 (B, n, k)
    KcutDev& d = c->kcut;
    const size_t tz = (size_t)B * n * d.k;
    if (x0)
      for (size_t i = 0; i < tz; ++i)
        if (!std::isfinite(x0[i])) return fail(c, PDBO_EINVAL, "Z^0 must be finite");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    TempDev t;
    STCHK(upload_x0(c, t, x0, tz));
    c->parity = 0;
    HIPCHK(c, launch_kcut_init((const double*)t.p, d, (float)c->par.y0, c->par.seed, c->stream));
    const int64_t zero = 0;
    Incumbent init{kI64Max, -1, -1, 0};
    HIPCHK(c, hipMemcpyAsync(d.t_dev, &zero, sizeof(zero), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(d.inc, &init, sizeof(init), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_fill_i32(d.trace_len, 0, 1, c->stream));
    HIPCHK(c, launch_fill_i32(d.win, -1, 1, c->stream));
    HIPCHK(c, launch_fill_i64((int64_t*)c->ts0_d, 0, 1, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->t_host = 0;
    c->stamped = false;
    return PDBO_OK;
  }
  const size_t tot = (size_t)B * n;
  if (x0)
    for (size_t i = 0; i < tot; ++i)
      if (!(x0[i] >= 0.0 && x0[i] <= 1.0)) return fail(c, PDBO_EINVAL, "x0 must lie in [0,1]");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  TempDev t;
  STCHK(upload_x0(c, t, x0, tot));
  const float y0 = (float)c->par.y0;
  Incumbent init{kI64Max, -1, -1, 0};
  if (c->kind == 0) {
    InstDev& I = c->insts_h[0];
    c->parity = 0;
    HIPCHK(c, launch_init_state((const double*)t.p, B, n, I.ld, y0, I.X[0], I.Y,
                                c->prec == PDBO_FP32 ? nullptr : I.Xs[0], c->prec, I.Xr, c->par.seed,
                                c->stream));
    const int64_t zero = 0;
    HIPCHK(c, hipMemcpyAsync(I.t_dev, &zero, sizeof(zero), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(I.inc, &init, sizeof(init), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_fill_i32(I.trace_len, 0, 1, c->stream));
    HIPCHK(c, launch_fill_i64(I.Sacc, 0, (size_t)B, c->stream));
    HIPCHK(c, launch_fill_i64(I.Cacc, 0, (size_t)B, c->stream));
    if (I.nflip) {
      // the first evaluation is a full product; the change bitmap starts clear
      HIPCHK(c, launch_fill_i32(I.nflip, kFlipMax + 1, B, c->stream));
      HIPCHK(c, launch_fill_i32((int32_t*)I.fbits, 0, (int64_t)B * (I.ld / 32), c->stream));
    }
    if (I.ys) HIPCHK(c, launch_fill_i32((int32_t*)I.ys, f32_bits(y0), B, c->stream));
    c->argmin_pending = false;
  } else if (c->kind == 3) {
    SpmmDev& d = c->spmm;
    c->parity = 0;
    HIPCHK(c, launch_spmm_init((const double*)t.p, d, y0, c->par.seed, c->stream));
    const int64_t zero = 0;
    HIPCHK(c, hipMemcpyAsync(d.t_dev, &zero, sizeof(zero), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(d.inc, &init, sizeof(init), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_fill_i32(d.trace_len, 0, 1, c->stream));
    if (d.incw) {
      const uint64_t top[4] = {~0ull, ~0ull, ~0ull, ~0ull >> 1};
      HIPCHK(c, hipMemcpyAsync(d.incw, top, sizeof(top), hipMemcpyHostToDevice, c->stream));
    }
    if (d.win) HIPCHK(c, launch_fill_i32(d.win, -1, 1, c->stream));
  } else {
    float* X = c->kind == 1 ? c->csr.X : c->sat.X;
    float* Y = c->kind == 1 ? c->csr.Y : c->sat.Y;
    const int ld = c->kind == 1 ? c->csr.ld : c->sat.ld;
    int64_t* rbF = c->kind == 1 ? c->csr.rbestF : c->sat.rbestF;
    int64_t* rbT = c->kind == 1 ? c->csr.rbestT : c->sat.rbestT;
    HIPCHK(c, launch_init_state((const double*)t.p, B, n, ld, y0, X, Y, nullptr, P_F32, nullptr,
                                c->par.seed, c->stream));
    HIPCHK(c, launch_fill_i64(rbF, kI64Max, B, c->stream));
    HIPCHK(c, launch_fill_i64(rbT, kI64Max, B, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->inc_d, &init, sizeof(init), hipMemcpyHostToDevice, c->stream));
  }
  // the time origin is the first step after the restart
  HIPCHK(c, launch_fill_i64((int64_t*)c->ts0_d, 0, 1, c->stream));
  c->stamped = false;
  c->t_host = 0;
  c->full_until = full_eval_iters();
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PDBO_OK;
}

pdbo_status qubo_gda_objectives_f64(pdbo_ctx* c, double* F) {
  if (!c || !F) return fail(c, PDBO_EINVAL, "NULL argument");
  if (c->kind == 2 || c->kind == 4) return fail(c, PDBO_ESTATE, "not a QUBO context");
  if (!is_real(c)) {
    std::vector<int64_t> Fi(c->B);
    STCHK(qubo_gda_objectives(c, Fi.data()));
    for (int b = 0; b < c->B; ++b) F[b] = (double)Fi[b];
    return PDBO_OK;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(F, c->spmm.Fd, c->B * sizeof(double), hipMemcpyDeviceToHost));
  return PDBO_OK;
}

pdbo_status qubo_gda_objectives(pdbo_ctx* c, int64_t* F) {
  if (!c || !F) return fail(c, PDBO_EINVAL, "NULL argument");
  if (c->kind == 0 && c->insts_h.size() != 1) return fail(c, PDBO_ESTATE, "batched context");
  if (is_real(c)) return fail(c, PDBO_EUNSUPPORTED, "float64 weights: use qubo_gda_objectives_f64");
  const int64_t* src = c->kind == 0   ? c->insts_h[0].Fall
                       : c->kind == 1 ? c->csr.Flast
                       : c->kind == 3 ? c->spmm.Flast
                       : c->kind == 4 ? c->kcut.Flast
                                      : c->sat.Flast;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(F, src, c->B * sizeof(int64_t), hipMemcpyDeviceToHost));
  return PDBO_OK;
}

static pdbo_status ensure_scratch(pdbo_ctx* c) {
  if (c->g_scratch) return PDBO_OK;
  int ld = 0;
  if (c->kind == 0)
    ld = c->insts_h[0].ld;
  else if (c->kind == 1)
    ld = c->csr.ld;
  else if (c->kind == 3)
    ld = roundup(c->spmm.n, kLdAlign);
  else if (c->kind == 4)
    ld = roundup(c->kcut.n, kLdAlign);
  else
    ld = c->sat.ld;
  const size_t sz = (size_t)c->B * ld;
  STCHK(dalloc(c, &c->g_scratch, sz));
  STCHK(dalloc(c, &c->gx_scratch, sz));
  STCHK(dalloc(c, &c->xr_scratch, sz));
  STCHK(dalloc(c, &c->f_scratch, c->B));
  if (c->kind == 0) {
    STCHK(dalloc(c, &c->gs_scratch, sz * element_bytes(c->prec)));
    STCHK(dalloc(c, &c->sp_scratch, (size_t)c->B));
    STCHK(dalloc(c, &c->cp_scratch, (size_t)c->B));
    STCHK(dalloc(c, &c->scratch_inst_d, 1));
  }
  return PDBO_OK;
}

pdbo_status qubo_gda_grad(pdbo_ctx* c, const float* x, float* G) {
  if (!c || !x || !G) return fail(c, PDBO_EINVAL, "NULL argument");
  if (c->kind == 0 && c->insts_h.size() != 1) return fail(c, PDBO_ESTATE, "batched context");
  STCHK(ensure_scratch(c));
  if (c->kind == 4) {  // x: the logits Z (B, n, k); G: d(f/s)/dZ, same layout
    KcutDev d = c->kcut;
    const size_t tz = (size_t)c->B * d.n * d.k;
    for (size_t i = 0; i < tz; ++i)
      if (!std::isfinite(x[i])) return fail(c, PDBO_EINVAL, "Z must be finite");
    if (!c->kz_scratch) {
      STCHK(dalloc(c, &c->kz_scratch, 3 * tz));
      STCHK(dalloc(c, &c->kg_scratch, tz));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    TempDev tx;
    STCHK(temp_upload(c, tx, x, tz * sizeof(float)));
    d.Z = c->kz_scratch;
    d.X[0] = c->kz_scratch + tz;
    d.X[1] = c->kz_scratch + 2 * tz;
    HIPCHK(c, launch_kcut_set((const float*)tx.p, nullptr, d, 0, c->stream));
    HIPCHK(c, launch_kcut(d, 2, 0, c->kg_scratch, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return kcut_download(c, c->kg_scratch, G, d.k);
  }
  int n = c->n_of[0];
  const size_t tot = (size_t)c->B * n;
  for (size_t i = 0; i < tot; ++i)
    if (!(x[i] >= 0.f && x[i] <= 1.f)) return fail(c, PDBO_EINVAL, "x must lie in [0,1]");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->kind == 3) {  // node-major operand and result
    STCHK(spmm_upload(c, x, c->gx_scratch));
    SpmmDev d = c->spmm;
    d.X[0] = c->gx_scratch;
    HIPCHK(c, launch_spmm(d, 2, 0, c->g_scratch, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return spmm_download(c, c->g_scratch, G);
  }
  TempDev tx;
  STCHK(temp_upload(c, tx, x, tot * sizeof(float)));
  int ld;
  if (c->kind == 0) {
    InstDev I = c->insts_h[0];
    ld = I.ld;
    uint8_t* Xs = c->prec == PDBO_FP32 ? (uint8_t*)c->gx_scratch : c->gs_scratch;
    HIPCHK(c, launch_set_state((const float*)tx.p, nullptr, c->B, n, ld, c->gx_scratch, nullptr,
                               c->prec == PDBO_FP32 ? nullptr : Xs, c->prec, c->stream));
    I.Xs[0] = I.Xs[1] = Xs;
    I.G = c->g_scratch;
    HIPCHK(c, hipMemcpyAsync(c->scratch_inst_d, &I, sizeof(I), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_dense_gemm(c->cfg, c->prec, EPI_GRAD, 0, c->tiles_d, (int)c->tiles_h.size(),
                                c->scratch_inst_d, 0, 0, c->stream));
  } else if (c->kind == 1) {
    ld = c->csr.ld;
    HIPCHK(c, launch_set_state((const float*)tx.p, nullptr, c->B, n, ld, c->gx_scratch, nullptr,
                               nullptr, P_F32, c->stream));
    HIPCHK(c, launch_csr_grad(c->csr, c->gx_scratch, c->g_scratch, c->B, c->stream));
  } else {
    ld = c->sat.ld;
    HIPCHK(c, launch_set_state((const float*)tx.p, nullptr, c->B, n, ld, c->gx_scratch, nullptr,
                               nullptr, P_F32, c->stream));
    HIPCHK(c, launch_sat_grad(c->sat, c->gx_scratch, ld, c->g_scratch, c->B, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy2D(G, n * sizeof(float), c->g_scratch, ld * sizeof(float), n * sizeof(float),
                        c->B, hipMemcpyDeviceToHost));
  return PDBO_OK;
}

pdbo_status qubo_gda_eval_f64(pdbo_ctx* c, const uint8_t* xr, int32_t nb, double* F) {
  if (!c || !xr || !F) return fail(c, PDBO_EINVAL, "NULL argument");
  if (c->kind == 2 || c->kind == 4) return fail(c, PDBO_ESTATE, "not a QUBO context");
  if (!is_real(c)) {
    if (nb < 1 || nb > c->B) return fail(c, PDBO_EINVAL, "nb must be in [1, B]");
    std::vector<int64_t> Fi(nb);
    STCHK(qubo_gda_eval(c, xr, nb, Fi.data()));
    for (int b = 0; b < nb; ++b) F[b] = (double)Fi[b];
    return PDBO_OK;
  }
  if (nb < 1 || nb > c->B) return fail(c, PDBO_EINVAL, "nb must be in [1, B]");
  const int n = c->n_of[0];
  for (size_t i = 0; i < (size_t)nb * n; ++i)
    if (xr[i] > 1) return fail(c, PDBO_EINVAL, "xr must be 0/1 bytes");
  STCHK(ensure_scratch(c));
  // X[parity ^ 1] holds the previous iterate, which the next step overwrites
  // before reading: the vectors are evaluated there
  SpmmDev& d = c->spmm;
  const int q = c->parity ^ 1;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(c->xr_scratch, xr, (size_t)nb * n, hipMemcpyHostToDevice));
  HIPCHK(c, launch_real_load_x((const uint8_t*)c->xr_scratch, nb, d, q, c->stream));
  HIPCHK(c, launch_spmm_real(d, 1, q, nullptr, c->stream));
  HIPCHK(c, launch_spmm_real_best(d, q, 0, (double*)c->f_scratch, nb, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(F, c->f_scratch, nb * sizeof(double), hipMemcpyDeviceToHost));
  return PDBO_OK;
}

pdbo_status qubo_gda_eval(pdbo_ctx* c, const uint8_t* xr, int32_t nb, int64_t* F) {
  if (!c || !xr || !F) return fail(c, PDBO_EINVAL, "NULL argument");
  if (c->kind == 0 && c->insts_h.size() != 1) return fail(c, PDBO_ESTATE, "batched context");
  if (is_real(c)) return fail(c, PDBO_EUNSUPPORTED, "float64 weights: use qubo_gda_eval_f64");
  if (nb < 1 || nb > c->B) return fail(c, PDBO_EINVAL, "nb must be in [1, B]");
  const int n = c->n_of[0];
  const int vmax = c->kind == 4 ? c->kcut.k - 1 : 1;  // Max-k-Cut: categories 0..k-1
  for (size_t i = 0; i < (size_t)nb * n; ++i)
    if (xr[i] > vmax) return fail(c, PDBO_EINVAL, "xr must be 0/1 bytes (categories 0..k-1 for Max-k-Cut)");
  STCHK(ensure_scratch(c));
  if (c->kind == 4) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->xr_scratch, xr, (size_t)nb * n, hipMemcpyHostToDevice));
    HIPCHK(c, launch_kcut_eval(c->kcut, (const uint8_t*)c->xr_scratch, nb, c->f_scratch, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(F, c->f_scratch, nb * sizeof(int64_t), hipMemcpyDeviceToHost));
    return PDBO_OK;
  }
  const int ld = c->kind == 0 ? c->insts_h[0].ld : (c->kind == 1 || c->kind == 3) ? c->csr.ld : c->sat.ld;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemsetAsync(c->xr_scratch, 0, (size_t)c->B * ld, c->stream));
  HIPCHK(c, hipMemcpy2DAsync(c->xr_scratch, ld, xr, n, n, nb, hipMemcpyHostToDevice, c->stream));
  if (c->kind == 0) {
    InstDev I = c->insts_h[0];
    I.Xr = c->xr_scratch;
    I.Sacc = c->sp_scratch;
    I.Cacc = c->cp_scratch;
    I.Fall = c->f_scratch;
    I.nflip = nullptr;  // full product for every restart
    I.B = nb;
    HIPCHK(c, hipMemcpyAsync(c->scratch_inst_d, &I, sizeof(I), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, launch_eval_gemm(c, c->tiles_d, (int)c->tiles_h.size(), c->scratch_inst_d, c->stream));
    HIPCHK(c, launch_argmin(c->scratch_inst_d, 0, 1, 2, c->stream));
  } else if (c->kind == 1 || c->kind == 3) {
    HIPCHK(c, launch_csr_eval(c->csr, c->xr_scratch, nb, c->f_scratch, c->stream));
  } else {
    HIPCHK(c, launch_sat_eval(c->sat, c->xr_scratch, nb, c->f_scratch, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(F, c->f_scratch, nb * sizeof(int64_t), hipMemcpyDeviceToHost));
  return PDBO_OK;
}

pdbo_status qubo_gda_eval_noalloc(pdbo_ctx* c, const uint8_t* xr, int32_t nb, int64_t* F,
                                  void* stream) {
  if (!c || !xr || !F) return fail(c, PDBO_EINVAL, "NULL argument");
  if (c->kind == 0 && c->insts_h.size() != 1) return fail(c, PDBO_ESTATE, "batched context");
  if (is_real(c)) return fail(c, PDBO_EUNSUPPORTED, "float64 weights: no int64 objectives");
  if (nb < 1 || nb > c->B) return fail(c, PDBO_EINVAL, "nb must be in [1, B]");
  const hipStream_t s = (hipStream_t)stream;
  const int n = c->n_of[0];
  if (c->kind != 0) {
    // the CSR, MaxSAT and Max-k-Cut evaluation kernels read the caller's rows
    // directly (row stride n; nonzero bytes are 1, or categories for
    // Max-k-Cut) and need no scratch
    if (c->kind == 4) {
      HIPCHK(c, launch_kcut_eval(c->kcut, xr, nb, F, s));
    } else if (c->kind == 1 || c->kind == 3) {
      CsrDev d = c->csr;
      d.ld = n;
      HIPCHK(c, launch_csr_eval(d, (const int8_t*)xr, nb, F, s));
    } else {
      SatDev d = c->sat;
      d.ld = n;
      HIPCHK(c, launch_sat_eval(d, (const int8_t*)xr, nb, F, s));
    }
    return PDBO_OK;
  }
  const InstDev& I0 = c->insts_h[0];
  const size_t need = kNoallocDescBytes + 2 * sizeof(int64_t) * (size_t)nb + (size_t)nb * I0.ld;
  if (need > kNoallocScratchBytes)
    return fail(c, PDBO_EUNSUPPORTED,
                "nb * ld + 16 nb + 512 = " + std::to_string(need) + " bytes exceeds the " +
                    std::to_string(kNoallocScratchBytes) + "-byte scratch of qubo_gda_eval_noalloc");
  uint8_t* base = nullptr;
  STCHK(scratch_for_current_device(c, &base));
  InstDev* desc = (InstDev*)base;
  int64_t* S = (int64_t*)(base + kNoallocDescBytes);
  int64_t* C = S + nb;
  int8_t* xs = (int8_t*)(C + nb);  // 256 + 16 nb bytes in: 16-byte aligned
  InstDev I = I0;
  I.Xr = xs;
  I.Sacc = S;
  I.Cacc = C;
  I.Fall = F;
  I.nflip = nullptr;  // full product for every vector
  I.B = nb;
  const size_t tot = (size_t)nb * I0.ld;
  hipLaunchKernelGGL(stage_rounded_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, xr,
                     nb, n, I0.ld, xs);
  HIPCHK(c, hipGetLastError());
  hipLaunchKernelGGL(put_eval_desc_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, desc,
                     I, S, C, nb);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, launch_eval_gemm(c, c->tiles_d, (int)c->tiles_h.size(), desc, s));
  HIPCHK(c, launch_argmin(desc, 0, 1, 2, s));
  return PDBO_OK;
}

pdbo_status qubo_dual_bound(pdbo_ctx* c, double ybar, int32_t iters, double* lower_bound,
                            double* value, float* x_out) {
  if (!c || !lower_bound) return fail(c, PDBO_EINVAL, "NULL argument");
  if (c->kind == 0 && c->insts_h.size() != 1) return fail(c, PDBO_ESTATE, "batched context");
  if (c->kind == 2 || c->kind == 4)
    return fail(c, PDBO_EUNSUPPORTED, "the dual certificate is built for QUBO contexts");
  if (c->par.g_kind != PDBO_G_QUAD)
    return fail(c, PDBO_EUNSUPPORTED, "the dual certificate is built for the quadratic g");
  if (is_real(c)) return fail(c, PDBO_EUNSUPPORTED, "the dual certificate takes integer weights");
  if (ybar == 0.0) ybar = c->par.y0;
  if (!finite_pos(ybar)) return fail(c, PDBO_EINVAL, "ybar must be finite and > 0 (or 0 for y0)");
  if (iters < 0) return fail(c, PDBO_EINVAL, "iters must be >= 0");
  const int n = c->n_of[0];
  const int ld = roundup(n, kLdAlign);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (!c->cert_x) {
    STCHK(dalloc(c, &c->cert_x, 2 * (size_t)ld));
    STCHK(dalloc(c, &c->cert_y, (size_t)ld));
    STCHK(dalloc(c, &c->cert_xs, 2 * (size_t)ld * 4));
    STCHK(dalloc(c, &c->cert_xr, (size_t)ld));
    STCHK(dalloc(c, &c->cert_rows, 4 * (size_t)n));
    STCHK(dalloc(c, &c->cert_res, 4));
    STCHK(dalloc(c, &c->cert_i64, 4 + 2 * (size_t)std::max(1, 2048)));
    STCHK(dalloc(c, &c->cert_u64, 1));
    STCHK(dalloc(c, &c->cert_bx, (size_t)n));
  }
  if (c->kind == 0 && !c->scratch_inst_d) STCHK(dalloc(c, &c->scratch_inst_d, 1));
  float* x0 = c->cert_x;
  float* x1 = c->cert_x + ld;
  // projected gradient descent on L(., ybar 1) (Alg. 1 with beta = 0: y stays
  // positive, so the perturbation never applies) from x = 1/2
  HIPCHK(c, launch_fill_f32(x0, 0.5f, n, c->stream));
  HIPCHK(c, launch_fill_f32(x1, 0.f, ld, c->stream));
  HIPCHK(c, launch_fill_f32(c->cert_y, (float)ybar, ld, c->stream));
  const float* xhat = x0;
  if (c->kind == 0) {
    InstDev I = c->insts_h[0];
    I.B = 1;
    I.X[0] = x0;
    I.X[1] = c->prec == PDBO_FP32 ? x1 : x0;
    I.Y = c->cert_y;
    I.Xs[0] = c->prec == PDBO_FP32 ? (uint8_t*)x0 : c->cert_xs;
    I.Xs[1] = c->prec == PDBO_FP32 ? (uint8_t*)x1 : c->cert_xs + (size_t)ld * 4;
    I.Xr = c->cert_xr;
    I.nflip = nullptr;
    I.fbits = nullptr;
    I.cand = nullptr;
    I.ys = nullptr;
    I.gp.beta = 0.f;
    I.gp.gkind = PDBO_G_QUAD;
    if (c->prec != PDBO_FP32)
      HIPCHK(c, launch_set_state(x0, nullptr, 1, n, ld, x0, nullptr, I.Xs[0], c->prec, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->scratch_inst_d, &I, sizeof(I), hipMemcpyHostToDevice, c->stream));
    int parity = 0;
    for (int t = 0; t < iters; ++t) {
      HIPCHK(c, launch_dense_gemm(c->cfg, c->prec, EPI_STEP, PDBO_G_QUAD, c->tiles_d,
                                  (int)c->tiles_h.size(), c->scratch_inst_d, parity, 0, c->stream));
      parity ^= 1;
    }
    xhat = I.X[parity];
    HIPCHK(c, launch_cert_dense(c->insts_h[0], xhat, c->par.scale, ybar, c->cert_rows, c->cert_res,
                                c->stream));
  } else if (c->kind == 1) {
    CsrDev d = c->csr;
    d.B = 1;
    d.X = x0;
    d.Y = c->cert_y;
    d.rbestF = c->cert_i64;
    d.rbestT = c->cert_i64 + 1;
    d.Flast = c->cert_i64 + 2;
    d.rbestTs = c->cert_u64;
    d.best_xr = c->cert_bx;
    d.gp.beta = 0.f;
    d.gp.gkind = PDBO_G_QUAD;
    if (iters > 0) HIPCHK(c, launch_csr_persistent(d, c->compact, 0, iters, c->stream));
    HIPCHK(c, launch_cert_csr(c->csr, x0, c->par.scale, ybar, c->cert_rows, c->cert_res, c->stream));
  } else {
    SpmmDev d = c->spmm;
    d.win = nullptr;  // no incumbent here: the step launches copy nothing
    d.B = 1;
    d.W = 1;
    d.G = 64;
    d.nslices = 1;
    d.grid = std::max(1, std::min((n + 255) / 256, 2048));
    d.X[0] = x0;
    d.X[1] = x1;
    d.Y = c->cert_y;
    d.part = c->cert_i64 + 4;
    d.gp.beta = 0.f;
    d.gp.gkind = PDBO_G_QUAD;
    int parity = 0;
    for (int t = 0; t < iters; ++t) {
      HIPCHK(c, launch_spmm(d, 0, parity, nullptr, c->stream));
      parity ^= 1;
    }
    xhat = d.X[parity];
    HIPCHK(c, launch_cert_csr(c->csr, xhat, c->par.scale, ybar, c->cert_rows, c->cert_res, c->stream));
  }
  double res[4];
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(res, c->cert_res, sizeof(res), hipMemcpyDeviceToHost));
  *lower_bound = res[0];
  if (value) {
    value[0] = res[1];
    value[1] = res[2];
    value[2] = res[3];
  }
  if (x_out) HIPCHK(c, hipMemcpy(x_out, xhat, (size_t)n * sizeof(float), hipMemcpyDeviceToHost));
  return PDBO_OK;
}

pdbo_status qubo_gda_solve(const pdbo_qubo* prob, const pdbo_params* par, int32_t T, void* stream,
                           pdbo_result* result) {
  if (T < 0 || !result) return fail(nullptr, PDBO_EINVAL, "T must be >= 0 and result non-NULL");
  pdbo_ctx* c = nullptr;
  STCHK(qubo_gda_init(prob, par, stream, &c));
  pdbo_status st = qubo_gda_step(c, T);
  if (st == PDBO_OK) st = qubo_gda_result(c, result);
  if (st != PDBO_OK) g_last_error = c->err;
  pdbo_destroy(c);
  return st;
}

pdbo_status qubo_gda_batch_solve(int32_t k, const pdbo_qubo* probs, const pdbo_params* par,
                                 int32_t T, int32_t grouped, void* stream, pdbo_result* results) {
  if (T < 0 || !results) return fail(nullptr, PDBO_EINVAL, "T must be >= 0 and results non-NULL");
  pdbo_ctx* c = nullptr;
  STCHK(qubo_gda_batch_init(k, probs, par, grouped, stream, &c));
  pdbo_status st = qubo_gda_step(c, T);
  for (int i = 0; i < k && st == PDBO_OK; ++i) st = qubo_gda_batch_result(c, i, &results[i]);
  if (st != PDBO_OK) g_last_error = c->err;
  pdbo_destroy(c);
  return st;
}

// ---------------------------------------------------------------- MaxSAT

static pdbo_status check_maxsat(const pdbo_maxsat* s) {
  if (!s) return fail(nullptr, PDBO_EINVAL, "problem is NULL");
  if (s->n < 1 || s->n > (1 << 24)) return fail(nullptr, PDBO_EINVAL, "n must be in [1, 2^24]");
  if (s->m < 1) return fail(nullptr, PDBO_EINVAL, "m must be >= 1");
  if (s->k < 1 || s->k > 16) return fail(nullptr, PDBO_EINVAL, "k must be in [1, 16]");
  if (!s->lits) return fail(nullptr, PDBO_EINVAL, "lits is NULL");
  for (int j = 0; j < s->m; ++j) {
    for (int l = 0; l < s->k; ++l) {
      const int32_t v = s->lits[(size_t)j * s->k + l];
      if (v == 0 || v > s->n || v < -s->n)
        return fail(nullptr, PDBO_EINVAL, "literal out of range (DIMACS 1..n with sign)");
      for (int l2 = 0; l2 < l; ++l2) {
        const int32_t u = s->lits[(size_t)j * s->k + l2];
        if ((u < 0 ? -u : u) == (v < 0 ? -v : v))
          return fail(nullptr, PDBO_EINVAL, "a clause repeats a variable");
      }
    }
    if (s->w && (s->w[j] < 0 || s->w[j] >= (1 << 24)))
      return fail(nullptr, PDBO_EINVAL, "clause weights must be in [0, 2^24)");
  }
  return PDBO_OK;
}

static pdbo_status check_kcut(const pdbo_kcut* g, const pdbo_params* p) {
  if (!g) return fail(nullptr, PDBO_EINVAL, "problem is NULL");
  if (g->n < 1 || g->n > 65536) return fail(nullptr, PDBO_EINVAL, "n must be in [1, 65536]");
  if (g->k < 2 || g->k > 8) return fail(nullptr, PDBO_EINVAL, "k must be in [2, 8]");
  if (!g->row_ptr || (g->nnz > 0 && (!g->col_idx || !g->w)))
    return fail(nullptr, PDBO_EINVAL, "CSR arrays are NULL");
  if (g->nnz < 0 || g->nnz > (int64_t)INT_MAX) return fail(nullptr, PDBO_EINVAL, "bad nnz");
  const int n = g->n;
  if (g->row_ptr[0] != 0 || (int64_t)g->row_ptr[n] != g->nnz)
    return fail(nullptr, PDBO_EINVAL, "row_ptr must start at 0 and end at nnz");
  for (int i = 0; i < n; ++i) {
    if (g->row_ptr[i + 1] < g->row_ptr[i]) return fail(nullptr, PDBO_EINVAL, "row_ptr must be non-decreasing");
    int64_t rs = 0;
    for (int q = g->row_ptr[i]; q < g->row_ptr[i + 1]; ++q) {
      const int j = g->col_idx[q];
      if (j < 0 || j >= n || j == i) return fail(nullptr, PDBO_EINVAL, "column out of range or on the diagonal");
      if (q > g->row_ptr[i] && j <= g->col_idx[q - 1])
        return fail(nullptr, PDBO_EINVAL, "columns of a row must be strictly increasing");
      // the mirror entry (j, i) with the same weight
      const int32_t* b = g->col_idx + g->row_ptr[j];
      const int32_t* e = g->col_idx + g->row_ptr[j + 1];
      const int32_t* f = std::lower_bound(b, e, i);
      if (f == e || *f != i || g->w[g->row_ptr[j] + (f - b)] != g->w[q])
        return fail(nullptr, PDBO_EINVAL, "W must be symmetric with both directions stored");
      rs += g->w[q] < 0 ? -(int64_t)g->w[q] : g->w[q];
    }
    if (rs >= (int64_t(1) << 31)) return fail(nullptr, PDBO_ERANGE, "a row of |W| sums to 2^31 or more");
  }
  STCHK(check_params(p, n, false));
  if (p->x0) {
    const size_t tot = (size_t)p->B * n * g->k;
    for (size_t i = 0; i < tot; ++i)
      if (!std::isfinite(p->x0[i])) return fail(nullptr, PDBO_EINVAL, "x0 (the logits Z^0) must be finite");
  }
  if (p->g_kind == PDBO_G_POLY || p->dual_kind != PDBO_DUAL_VECTOR)
    return fail(nullptr, PDBO_EUNSUPPORTED, "Max-k-Cut takes the quadratic or entropy g with a dual per node");
  if (p->eval_every != 1) return fail(nullptr, PDBO_EUNSUPPORTED, "Max-k-Cut evaluates every iteration");
  return PDBO_OK;
}

pdbo_status kcut_gda_init(const pdbo_kcut* g, const pdbo_params* p, void* stream, pdbo_ctx** out) {
  if (!out) return fail(nullptr, PDBO_EINVAL, "out is NULL");
  *out = nullptr;
  STCHK(check_kcut(g, p));
  const int n = g->n, B = p->B, k = g->k;
  pdbo_ctx* c = new pdbo_ctx();
  c->kind = 4;
  c->n_of.push_back(n);
  pdbo_status st = begin_ctx(c, stream, p);
  auto run = [&]() -> pdbo_status {
    KcutDev& d = c->kcut;
    std::memset(&d, 0, sizeof(d));
    d.n = n;
    d.B = B;
    d.k = k;
    d.trace_cap = kTraceCap;
    d.tos = (float)(2.0 / p->scale);
    d.gp = make_gp(p);
    d.W = std::min(B, 64);
    d.G = 64 / d.W;
    d.nslices = (B + d.W - 1) / d.W;
    const int nrb = (n + 4 * d.G - 1) / (4 * d.G);
    d.grid = std::max(1, std::min(nrb, std::max(1, rowpar_grid_cap() / d.nslices))) * d.nslices;
    const int64_t nnz = g->nnz;
    int32_t *rp = nullptr, *col = nullptr, *w = nullptr;
    STCHK(dalloc(c, &rp, n + 1));
    STCHK(dalloc(c, &col, nnz));
    STCHK(dalloc(c, &w, nnz));
    HIPCHK(c, hipMemcpyAsync(rp, g->row_ptr, (n + 1) * 4, hipMemcpyHostToDevice, c->stream));
    if (nnz > 0) {
      HIPCHK(c, hipMemcpyAsync(col, g->col_idx, nnz * 4, hipMemcpyHostToDevice, c->stream));
      HIPCHK(c, hipMemcpyAsync(w, g->w, nnz * 4, hipMemcpyHostToDevice, c->stream));
    }
    d.row_ptr = rp;
    d.col = col;
    d.w = w;
    const size_t sz = (size_t)n * B * k;
    STCHK(dalloc(c, &d.Z, sz));
    STCHK(dalloc(c, &d.X[0], sz));
    STCHK(dalloc(c, &d.X[1], sz));
    STCHK(dalloc(c, &d.Y, (size_t)n * B));
    STCHK(dalloc(c, &d.part, (size_t)d.grid * d.W));
    STCHK(dalloc(c, &d.Flast, B));
    STCHK(dalloc(c, &d.inc, 1));
    STCHK(dalloc(c, &d.best_x, n));
    STCHK(dalloc(c, &d.win, 1));
    STCHK(dalloc(c, &d.trace, kTraceCap));
    STCHK(dalloc(c, &d.trace_len, 1));
    STCHK(dalloc(c, &d.t_dev, 1));
    d.ts0 = c->ts0_d;
    Incumbent init{kI64Max, -1, -1, 0};
    HIPCHK(c, hipMemcpyAsync(d.inc, &init, sizeof(init), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_fill_i32(d.win, -1, 1, c->stream));
    TempDev t;
    STCHK(upload_x0(c, t, p->x0, (size_t)B * n * k));
    HIPCHK(c, launch_kcut_init((const double*)t.p, d, (float)p->y0, p->seed, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PDBO_OK;
  };
  if (st == PDBO_OK) st = run();
  if (st != PDBO_OK) {
    const std::string msg = c->err.empty() ? g_last_error : c->err;
    pdbo_destroy(c);
    g_last_error = msg;
    return st;
  }
  *out = c;
  return PDBO_OK;
}

pdbo_status maxsat_gda_init(const pdbo_maxsat* prob, const pdbo_params* p, void* stream,
                            pdbo_ctx** out) {
  if (!out) return fail(nullptr, PDBO_EINVAL, "out is NULL");
  *out = nullptr;
  STCHK(check_maxsat(prob));
  STCHK(check_params(p, prob->n));
  STCHK(persistent_supported(p));
  if (p->eval_every != 1) return fail(nullptr, PDBO_EUNSUPPORTED, "the MaxSAT path evaluates every iteration");
  const int n = prob->n, m = prob->m, k = prob->k;
  if (!sat_fits(n, nullptr))
    return fail(nullptr, PDBO_EUNSUPPORTED, "n too large for the restart-resident MaxSAT kernel");
  // literal codes and the variable-major occurrence lists
  std::vector<int32_t> codes((size_t)m * k), wv(m);
  std::vector<int32_t> ptr(n + 1, 0);
  for (int j = 0; j < m; ++j) {
    wv[j] = prob->w ? prob->w[j] : 1;
    for (int l = 0; l < k; ++l) {
      const int32_t v = prob->lits[(size_t)j * k + l];
      const int32_t var = (v < 0 ? -v : v) - 1;
      codes[(size_t)j * k + l] = (int32_t)((uint32_t)var | (v < 0 ? 0x80000000u : 0u));
      ptr[var + 1]++;
    }
  }
  for (int i = 0; i < n; ++i) ptr[i + 1] += ptr[i];
  // Every clause is counted in the exact evaluation by one of its variables,
  // its owner: the variable with the fewest clauses owned so far when the
  // clause comes up, so that each variable owns about m/n of them (the
  // evaluation work of the threads stays even).
  std::vector<int32_t> owner(m);
  {
    std::vector<int32_t> owned(n, 0);
    for (int j = 0; j < m; ++j) {
      int best = 0;
      for (int l = 1; l < k; ++l)
        if (owned[codes[(size_t)j * k + l] & 0x7fffffff] < owned[codes[(size_t)j * k + best] & 0x7fffffff])
          best = l;
      owner[j] = best;
      owned[codes[(size_t)j * k + best] & 0x7fffffff]++;
    }
  }
  std::vector<int32_t> inc((size_t)ptr[n] * k);
  std::vector<int32_t> fillp(ptr.begin(), ptr.end() - 1);
  for (int j = 0; j < m; ++j)
    for (int l = 0; l < k; ++l) {
      const int32_t code = codes[(size_t)j * k + l];
      const int var = code & 0x7fffffff;
      const int e = fillp[var]++;
      int o = 0;
      for (int l2 = 0; l2 < k; ++l2)
        if (l2 != l) inc[(size_t)e * k + o++] = codes[(size_t)j * k + l2];
      const int32_t meta = wv[j] | ((code < 0 ? 1 : 0) << 30) | ((l == owner[j] ? 1 : 0) << 29);
      inc[(size_t)e * k + (k - 1)] = meta;
    }

  std::vector<uint64_t> pinc3;  // host staging, alive until init syncs
  std::vector<int32_t> slice;
  std::vector<int32_t> ord, pptr, pinc;
  pdbo_ctx* c = new pdbo_ctx();
  c->kind = 2;
  c->n_of.push_back(n);
  pdbo_status st = begin_ctx(c, stream, p);
  auto run = [&]() -> pdbo_status {
    const int B = p->B, ld = roundup(n, kLdAlign);
    SatDev& d = c->sat;
    std::memset(&d, 0, sizeof(d));
    d.n = n;
    d.m = m;
    d.k = k;
    d.ld = ld;
    d.B = B;
    d.ios = (float)(1.0 / p->scale);
    d.gp = make_gp(p);
    int32_t *dp = nullptr, *di = nullptr, *dl = nullptr, *dw = nullptr;
    STCHK(dalloc(c, &dp, n + 1));
    STCHK(dalloc(c, &di, inc.size()));
    STCHK(dalloc(c, &dl, codes.size()));
    STCHK(dalloc(c, &dw, m));
    HIPCHK(c, hipMemcpyAsync(dp, ptr.data(), (n + 1) * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(di, inc.data(), inc.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(dl, codes.data(), codes.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(dw, wv.data(), m * 4, hipMemcpyHostToDevice, c->stream));
    d.inc_ptr = dp;
    d.inc = di;
    d.lits = dl;
    d.w = dw;
    // position space of the persistent kernel: variables by decreasing
    // occurrence count, their lists with the other literals' codes renamed
    // to positions
    ord.resize(n);
    for (int v = 0; v < n; ++v) ord[v] = v;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b2) {
      return ptr[a + 1] - ptr[a] > ptr[b2 + 1] - ptr[b2];
    });
    std::vector<int32_t> posv(n);
    for (int q = 0; q < n; ++q) posv[ord[q]] = q;
    pptr.assign(n + 1, 0);
    for (int q = 0; q < n; ++q) pptr[q + 1] = pptr[q] + (ptr[ord[q] + 1] - ptr[ord[q]]);
    pinc.resize(inc.size());
    auto rename = [&](int32_t code) {
      return (int32_t)(((uint32_t)code & 0x80000000u) | (uint32_t)posv[code & 0x7fffffff]);
    };
    for (int q = 0; q < n; ++q) {
      const int v = ord[q];
      for (int e = ptr[v], f = pptr[q]; e < ptr[v + 1]; ++e, ++f) {
        for (int o = 0; o < k - 1; ++o) pinc[(size_t)f * k + o] = rename(inc[(size_t)e * k + o]);
        pinc[(size_t)f * k + (k - 1)] = inc[(size_t)e * k + (k - 1)];
      }
    }
    int32_t *dord = nullptr, *dpp = nullptr, *dpi = nullptr;
    STCHK(dalloc(c, &dord, n));
    STCHK(dalloc(c, &dpp, n + 1));
    STCHK(dalloc(c, &dpi, pinc.size()));
    HIPCHK(c, hipMemcpyAsync(dord, ord.data(), (size_t)n * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(dpp, pptr.data(), (size_t)(n + 1) * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(dpi, pinc.data(), pinc.size() * 4, hipMemcpyHostToDevice, c->stream));
    d.order = dord;
    d.pinc_ptr = dpp;
    d.pinc = dpi;
    if (k == 3) {
      // compact 8-byte entries (16-bit codes: position | negated << 15,
      // n <= 32768), each position's owned clauses first, interleaved by
      // slices of 64 positions; a slice is as long as its longest list (its
      // first: positions are in decreasing count order), shorter lists leave
      // zero slots that are never read
      const int ns = (n + 63) / 64;
      slice.assign(ns, 0);
      int64_t tot = 0;
      for (int s = 0; s < ns; ++s) {
        slice[s] = (int32_t)tot;
        int lmax = 0;
        for (int q = s * 64; q < std::min(n, s * 64 + 64); ++q) lmax = std::max(lmax, pptr[q + 1] - pptr[q]);
        tot += (int64_t)64 * lmax;
        if (tot > INT32_MAX) return fail(c, PDBO_ERANGE, "3-SAT occurrence slices exceed 2^31 entries");
      }
      pinc3.assign((size_t)tot, 0);
      auto c16 = [](int32_t code) {
        return (uint32_t)(code & 0x7fffffff) | ((code < 0 ? 1u : 0u) << 15);
      };
      for (int q = 0; q < n; ++q) {
        size_t f = (size_t)slice[q / 64] + (q % 64);
        for (int pass = 0; pass < 2; ++pass)
          for (int e = pptr[q]; e < pptr[q + 1]; ++e) {
            const int32_t meta = pinc[(size_t)e * 3 + 2];
            if ((((meta >> 29) & 1) != 0) != (pass == 0)) continue;
            const uint32_t lo = c16(pinc[(size_t)e * 3]) | (c16(pinc[(size_t)e * 3 + 1]) << 16);
            pinc3[f] = (uint64_t)lo | ((uint64_t)(uint32_t)meta << 32);
            f += 64;
          }
      }
      uint64_t* d3 = nullptr;
      int32_t* dsl = nullptr;
      STCHK(dalloc(c, &d3, std::max<size_t>(pinc3.size(), 1)));
      STCHK(dalloc(c, &dsl, ns));
      HIPCHK(c, hipMemcpyAsync(d3, pinc3.data(), pinc3.size() * sizeof(uint64_t),
                               hipMemcpyHostToDevice, c->stream));
      HIPCHK(c, hipMemcpyAsync(dsl, slice.data(), (size_t)ns * 4, hipMemcpyHostToDevice, c->stream));
      d.pinc3 = d3;
      d.pinc3_slice = dsl;
    }
    STCHK(dalloc(c, &d.X, (size_t)B * ld));
    STCHK(dalloc(c, &d.Y, (size_t)B * ld));
    STCHK(dalloc(c, &d.rbestF, B));
    STCHK(dalloc(c, &d.rbestT, B));
    STCHK(dalloc(c, &d.rbestTs, B));
    STCHK(dalloc(c, &d.best_xr, (size_t)B * n));
    STCHK(dalloc(c, &d.Flast, B));
    STCHK(dalloc(c, &c->inc_d, 1));
    STCHK(dalloc(c, &c->best_x_d, n));
    HIPCHK(c, launch_fill_i64(d.rbestF, kI64Max, B, c->stream));
    HIPCHK(c, launch_fill_i64(d.rbestT, kI64Max, B, c->stream));
    Incumbent init{kI64Max, -1, -1, 0};
    HIPCHK(c, hipMemcpyAsync(c->inc_d, &init, sizeof(init), hipMemcpyHostToDevice, c->stream));
    TempDev t;
    STCHK(upload_x0(c, t, p->x0, (size_t)B * n));
    HIPCHK(c, launch_init_state((const double*)t.p, B, n, ld, (float)p->y0, d.X, d.Y, nullptr,
                                P_F32, nullptr, p->seed, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PDBO_OK;
  };
  if (st == PDBO_OK) st = run();
  if (st != PDBO_OK) {
    const std::string msg = c->err.empty() ? g_last_error : c->err;
    pdbo_destroy(c);
    g_last_error = msg;
    return st;
  }
  *out = c;
  return PDBO_OK;
}

pdbo_status maxsat_gda_step(pdbo_ctx* c, int32_t nsteps) {
  if (!c || c->kind != 2) return fail(c, PDBO_ESTATE, "not a MaxSAT context");
  return qubo_gda_step(c, nsteps);
}

pdbo_status maxsat_gda_result(pdbo_ctx* c, pdbo_result* r) {
  if (!c || c->kind != 2) return fail(c, PDBO_ESTATE, "not a MaxSAT context");
  return qubo_gda_result(c, r);
}

pdbo_status maxsat_gda_solve(const pdbo_maxsat* prob, const pdbo_params* par, int32_t T,
                             void* stream, pdbo_result* result) {
  if (T < 0 || !result) return fail(nullptr, PDBO_EINVAL, "T must be >= 0 and result non-NULL");
  pdbo_ctx* c = nullptr;
  STCHK(maxsat_gda_init(prob, par, stream, &c));
  pdbo_status st = qubo_gda_step(c, T);
  if (st == PDBO_OK) st = qubo_gda_result(c, result);
  if (st != PDBO_OK) g_last_error = c->err;
  pdbo_destroy(c);
  return st;
}

pdbo_status maxsat_lagrangian_fwd(pdbo_ctx* c, const float* x, const float* y, int32_t nb,
                                  float* L, void* stream) {
  if (!c || c->kind != 2) return fail(c, PDBO_ESTATE, "not a MaxSAT context");
  if (!x || !y || !L || nb < 1) return fail(c, PDBO_EINVAL, "bad arguments");
  HIPCHK(c, launch_sat_fwd(c->sat, x, y, nb, L, (hipStream_t)stream));
  return PDBO_OK;
}

pdbo_status maxsat_lagrangian_bwd(pdbo_ctx* c, const float* x, const float* y, const float* dL,
                                  int32_t nb, float* dx, float* dy, void* stream) {
  if (!c || c->kind != 2) return fail(c, PDBO_ESTATE, "not a MaxSAT context");
  if (!x || !y || !dL || !dx || !dy || nb < 1) return fail(c, PDBO_EINVAL, "bad arguments");
  HIPCHK(c, launch_sat_bwd(c->sat, x, y, dL, nb, dx, dy, (hipStream_t)stream));
  return PDBO_OK;
}

static pdbo_status trace_records(pdbo_ctx* c, int32_t cap, int64_t* t, int64_t* F, double* Fd,
                                 int32_t* b, double* sec, int32_t* len);

pdbo_status qubo_gda_trace(pdbo_ctx* c, int32_t cap, int64_t* t, int64_t* F, int32_t* b,
                           double* sec, int32_t* len) {
  if (c && is_real(c)) return fail(c, PDBO_EUNSUPPORTED, "float64 weights: use qubo_gda_trace_f64");
  return trace_records(c, cap, t, F, nullptr, b, sec, len);
}

pdbo_status qubo_gda_trace_f64(pdbo_ctx* c, int32_t cap, int64_t* t, double* F, int32_t* b,
                               double* sec, int32_t* len) {
  return trace_records(c, cap, t, nullptr, F, b, sec, len);
}

static pdbo_status trace_records(pdbo_ctx* c, int32_t cap, int64_t* t, int64_t* F, double* Fd,
                                 int32_t* b, double* sec, int32_t* len) {
  if (!c || !len) return fail(c, PDBO_EINVAL, "NULL argument");
  if (cap < 0) return fail(c, PDBO_EINVAL, "cap must be >= 0");
  *len = 0;
  const TraceRec* trace_d = nullptr;
  const int32_t* len_d = nullptr;
  if (c->kind == 0 && c->insts_h.size() == 1) {
    trace_d = c->insts_h[0].trace;
    len_d = c->insts_h[0].trace_len;
  } else if (c->kind == 3) {
    trace_d = c->spmm.trace;
    len_d = c->spmm.trace_len;
  } else if (c->kind == 4) {
    trace_d = c->kcut.trace;
    len_d = c->kcut.trace_len;
  } else {
    return PDBO_OK;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  int32_t k = 0;
  uint64_t ts0 = 0;
  HIPCHK(c, hipMemcpy(&k, len_d, sizeof(k), hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(&ts0, c->ts0_d, sizeof(ts0), hipMemcpyDeviceToHost));
  k = std::min(k, cap);
  std::vector<TraceRec> tr(k);
  if (k > 0) HIPCHK(c, hipMemcpy(tr.data(), trace_d, k * sizeof(TraceRec), hipMemcpyDeviceToHost));
  const double hz = clock_rate_hz();
  for (int i = 0; i < k; ++i) {
    if (t) t[i] = tr[i].t;
    if (F) F[i] = tr[i].F;
    if (Fd) {  // float64 weights keep the bits of the rounded value
      if (is_real(c))
        std::memcpy(&Fd[i], &tr[i].F, sizeof(double));
      else
        Fd[i] = (double)tr[i].F;
    }
    if (b) b[i] = (int32_t)tr[i].b;
    if (sec) sec[i] = (tr[i].ts >= ts0 && ts0) ? (double)(tr[i].ts - ts0) / hz : 0.0;
  }
  *len = k;
  return PDBO_OK;
}

// ---------------------------------------------------------------- timing

pdbo_status pdbo_timing_classes(pdbo_ctx* c, uint32_t mask) {
  if (!c) return fail(nullptr, PDBO_ESTATE, "context is NULL");
  if (mask >> PDBO_K_COUNT) return fail(c, PDBO_EINVAL, "mask names an unknown kernel class");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  t_collect(c);
  for (int k = 0; k < PDBO_K_COUNT; ++k) {
    c->ms[k] = 0.0;
    c->cnt[k] = 0;
    c->tseen[k] = 0;
  }
  c->tmask = mask;
  c->timing = mask != 0;
  return PDBO_OK;
}

pdbo_status pdbo_timing_stride(pdbo_ctx* c, int32_t stride) {
  if (!c) return fail(nullptr, PDBO_ESTATE, "context is NULL");
  if (stride < 1) return fail(c, PDBO_EINVAL, "stride must be >= 1");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  t_collect(c);
  for (int k = 0; k < PDBO_K_COUNT; ++k) {
    c->ms[k] = 0.0;
    c->cnt[k] = 0;
    c->tseen[k] = 0;
  }
  c->tstride = stride;
  return PDBO_OK;
}

pdbo_status pdbo_autotune_store(const char* key, int32_t cfg) {
  if (!key || !autotune_key_ok(key)) return fail(nullptr, PDBO_EINVAL, "bad autotune key");
  if (cfg < 0 || cfg >= dense_num_cfgs()) return fail(nullptr, PDBO_EINVAL, "unknown tile configuration");
  if (!autotune_store(key, cfg))
    return fail(nullptr, PDBO_EINVAL, "cannot write the autotune cache " + autotune_path());
  return PDBO_OK;
}

pdbo_status pdbo_autotune_lookup(const char* key, int32_t* cfg) {
  if (!key || !cfg || !autotune_key_ok(key)) return fail(nullptr, PDBO_EINVAL, "bad autotune key");
  *cfg = autotune_lookup(key);
  return PDBO_OK;
}

pdbo_status pdbo_timing(pdbo_ctx* c, int32_t enable) {
  return pdbo_timing_classes(c, enable ? (1u << PDBO_K_COUNT) - 1u : 0u);
}

pdbo_status pdbo_kernel_time(pdbo_ctx* c, int32_t which, double* total_ms, int64_t* launches) {
  if (!c) return fail(nullptr, PDBO_ESTATE, "context is NULL");
  if (which < 0 || which >= PDBO_K_COUNT || !total_ms || !launches)
    return fail(c, PDBO_EINVAL, "bad arguments");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  t_collect(c);
  *total_ms = c->ms[which];
  *launches = c->cnt[which];
  return PDBO_OK;
}

}  // extern "C"
