/*
 * pdbo.h - C ABI of the PDBO hot path on MI355X (gfx950).
 *
 * PDBO (primal-dual binary optimisation) minimises F(x) over x in {0,1}^n
 * (Eq. 1) by running Algorithm 1 - simultaneous projected gradient
 * descent-ascent on the Lagrangian L(x,y) = f(x) + sum_i y_i g(x_i), with a
 * perturbation away from 1/2 - from B independent starting points at once, and
 * keeping the best rounded solution over all restarts (Sec. 4.2, Model
 * Settings).  f is the multilinear extension of F (Def. 2.2; closed form by
 * Prop. 2.4) and g a binarity constraint function (Sec. 3.1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns a pdbo_status; nothing aborts, exits or throws
 *   across the ABI.  On failure a message is available from pdbo_last_error()
 *   (per context) or pdbo_last_global_error() (when no context exists yet).
 * - Arrays of iterates are restart-major: an (B, n) array holds restart b in
 *   elements [b*n, (b+1)*n).  Unless stated otherwise these are HOST pointers;
 *   they are read (or written) during the call only and remain caller-owned.
 * - A context owns all device memory it allocates; pdbo_destroy() frees it.
 *   The HIP stream passed at init is borrowed, never created or destroyed; all
 *   device work of the context is enqueued on it.  One context per stream;
 *   calls on one context must not overlap.
 * - Objectives are always those of the ORIGINAL instance (Q, c) or clause
 *   weights, evaluated exactly in int64, never of the scaled or quantised data.
 * - Alg. 1 requires y^0 > 0, alpha, beta > 0 and delta > 0 (its Require line);
 *   this library additionally requires delta < 1/2 and scale > 0.
 */
#ifndef PDBO_H
#define PDBO_H

#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define PDBO_API __attribute__((visibility("default")))
#else
#define PDBO_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PDBO_OK = 0,
  PDBO_EINVAL = 1,       /* an argument violates the documented contract   */
  PDBO_ENOMEM = 2,       /* host or device allocation failed               */
  PDBO_EDEVICE = 3,      /* a HIP runtime call failed (text in last_error) */
  PDBO_ERANGE = 4,       /* an exactness guard of the integer paths failed */
  PDBO_ESTATE = 5,       /* call not valid for this context or its state   */
  PDBO_EUNSUPPORTED = 6  /* valid request outside what this build supports */
} pdbo_status;

typedef struct pdbo_ctx pdbo_ctx;

enum { PDBO_DENSE = 0, PDBO_CSR = 1 };
enum { PDBO_G_QUAD = 0, PDBO_G_ENTROPY = 1, PDBO_G_POLY = 2 };
enum { PDBO_DUAL_VECTOR = 0, PDBO_DUAL_SCALAR = 1 };
/* values of pdbo_params.tile for CSR instances */
enum { PDBO_CSR_AUTO = 0, PDBO_CSR_RESIDENT = 1, PDBO_CSR_ROWS = 2 };
enum { PDBO_FP32 = 0, PDBO_BF16 = 1, PDBO_FP8 = 2, PDBO_I8 = 3 };
/* values of pdbo_qubo.wtype */
enum { PDBO_W_INT32 = 0, PDBO_W_F64 = 1 };

/*
 * QUBO instance (Eq. 1 with quadratic F): minimise F(x) = x^T Q x + c^T x over
 * x in {0,1}^n.  Q may be asymmetric and may have a diagonal; the library works
 * on the multilinear extension f(x) = 1/2 x^T A x + c'^T x with
 * A = offdiag(Q + Q^T), c' = c + diag(Q) (Prop. 2.4), which equals F on {0,1}^n.
 *   format == PDBO_DENSE: Q is n*n, row-major (Q_ij at element i*n+j).
 *   format == PDBO_CSR:   row_ptr[n+1], col_idx[nnz], values[nnz], rows sorted
 *                         by column, no duplicate (i,j) in a row.
 *   wtype == PDBO_W_INT32: q holds Q (int32) and c holds n int64 linear
 *                         coefficients or is NULL for c = 0.
 *   wtype == PDBO_W_F64:  real weights: qd holds Q (float64, finite) and cd
 *                         holds c (float64) or is NULL; q and c are ignored.
 *                         The canonical A and c' are formed exactly (in fixed
 *                         point, not in float64), objectives are the exact
 *                         real sums compared exactly and reported correctly
 *                         rounded to float64 (pdbo_result.best_obj_f64, the
 *                         _f64 entry points).  Such instances run on the
 *                         row-parallel CSR path whatever their format (a dense
 *                         Q is stored as the CSR of its nonzeros); tile must be
 *                         0 or PDBO_CSR_ROWS.  ERANGE when the weights' binary
 *                         exponents span more than the 192 bits the exact
 *                         evaluation carries (from the highest bit of the
 *                         largest |weight| to the lowest set bit of any
 *                         weight, the one of the canonical sums included).
 * A zero-initialised struct is an int32 instance (wtype 0).  All pointers are
 * host pointers.
 */
typedef struct {
  int32_t n;
  int32_t format;
  const int32_t* q;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  int64_t nnz;
  const int64_t* c;
  int32_t wtype;
  int32_t _pad;
  const double* qd;
  const double* cd;
} pdbo_qubo;

/*
 * Weighted Max-k-SAT (Sec. 4.1, Max-k-SAT): minimise the total weight of the
 * unsatisfied clauses.  lits holds m*k int32 literals, clause j in
 * lits[j*k .. j*k+k), DIMACS convention: +v is x_v, -v is not x_v, v in 1..n;
 * the k variables of a clause must be distinct.  w: m clause weights in
 * [0, 2^24), or NULL for all ones.  Host pointers.
 */
typedef struct {
  int32_t n;
  int32_t m;
  int32_t k;
  const int32_t* lits;
  const int32_t* w;
} pdbo_maxsat;

/*
 * Weighted graph for Max-k-Cut (App. B): partition the n nodes into k
 * categories so as to maximise the weight of the edges between categories.
 * W is symmetric CSR with both directions of every edge stored (row_ptr[n+1],
 * col_idx[nnz] strictly increasing per row, w[nnz] int32), no diagonal;
 * 2 <= k <= 8.  Host pointers.
 */
typedef struct {
  int32_t n;
  int32_t k;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const int32_t* w;
  int64_t nnz;
} pdbo_kcut;

/*
 * Parameters of Alg. 1 and of the execution.
 *   B          number of restarts, >= 1.
 *   alpha,beta primal / dual step sizes (> 0).
 *   y0         initial dual value y^0 = y0 * 1 (> 0).
 *   delta      perturbation tolerance, in (0, 1/2).
 *   scale      s > 0: the method runs on f/s (gradient (A x + c')/s); the
 *              objective is still reported unscaled.
 *   g_kind     the binarity constraint function g of Sec. 3.1: PDBO_G_QUAD
 *              (x^2 - x), PDBO_G_ENTROPY (x log x + (1-x) log(1-x), derivative
 *              taken at x clipped to [2^-20, 1 - 2^-20]) or PDBO_G_POLY
 *              ((2x - 1)^(2d) - 1 with d = g_degree).
 *   precision  operand type of the dense gradient product A.X: PDBO_FP32,
 *              PDBO_BF16 (A and a bf16 copy of X), PDBO_FP8 (A as OCP e4m3 with
 *              one fp32 scale per row, X as e4m3), all with FP32 accumulation;
 *              or PDBO_I8 (A exactly as int8, X quantised to q = round(254 x) -
 *              127 so that x ~ (q + 127)/254 within 1/508, int32 accumulation;
 *              needs |Ahat_ij| <= 127 and 127 sum_j |Ahat_ij| < 2^31, else
 *              EUNSUPPORTED; the other forms take any |Ahat_ij| the exact
 *              evaluation covers).
 *              Ignored by the CSR and MaxSAT paths, whose integer weights are
 *              stored exactly.
 *   eval_every evaluate round(x^t) every eval_every iterations (>= 1); the
 *              persistent CSR and MaxSAT paths require 1.
 *   tile       dense: tile configuration id (0 = default for the shape).
 *              CSR: PDBO_CSR_RESIDENT (one workgroup per restart for all T
 *              iterations, x in LDS; n <= 32768, quadratic or entropy g),
 *              PDBO_CSR_ROWS (one launch per iteration over all rows, the
 *              restarts of a row in adjacent lanes; any n, any g), or
 *              PDBO_CSR_AUTO (resident when it fits and B >= 128).  With
 *              n <= 8192 the resident kernel stages its packed entries
 *              interleaved by slices of 64 rows when that takes no more LDS
 *              than CSR order (same sums in the same order, so the same
 *              results); PDBO_CSR_SLICED=0 keeps CSR order.
 *   graph_chunk  dense and row-parallel CSR paths: 0 = eager launches;
 *              K > 0 (even) = capture K iterations in one hipGraph and replay it.
 *   g_degree   d of PDBO_G_POLY, in [1, 16]; ignored for the other kinds.
 *   dual_kind  PDBO_DUAL_VECTOR: one dual variable per coordinate (Alg. 1);
 *              PDBO_DUAL_SCALAR: one per restart for the single constraint
 *              sum_i g(x_i) = 0 (the PDBO-s variant of Sec. 4.5), updated as
 *              y += beta * sum_i g(x_i^t); dense path only (else EUNSUPPORTED).
 *   x0         HOST (B, n) float64 starting points in [0,1], or NULL: then the
 *              library draws X^0 uniformly on [0,1)^n (App. C) with the
 *              counter-based generator Philox4x32-10 (Salmon et al., SC 2011)
 *              keyed by (seed mod 2^32, seed div 2^32): coordinate i of restart
 *              b is word (i mod 4) of the output for the counter
 *              (i div 4, b, 0, 0), and x = (word >> 8) * 2^-24.
 *   seed       key of that generator; ignored when x0 is given.
 */
typedef struct {
  int32_t B;
  int32_t g_kind;
  int32_t precision;
  int32_t eval_every;
  double alpha;
  double beta;
  double y0;
  double delta;
  double scale;
  int32_t tile;
  int32_t graph_chunk;
  int32_t g_degree;
  int32_t dual_kind;
  const double* x0;
  uint64_t seed;
} pdbo_params;

/* Incumbent of a run: the lexicographic minimum of (F, t, b) over all
 * evaluated rounded iterates x_r = [x^t > 1/2], t >= 1. */
typedef struct {
  int64_t best_obj;       /* exact F of best_x (weighted unsat count for MaxSAT);
                             0 for float64 weights                                */
  int32_t best_restart;   /* b, or -1 when nothing has been evaluated yet        */
  int32_t _pad;
  int64_t best_iter;      /* iteration t (1-based) at which it was first reached */
  double time_to_best_s;  /* device clock, from the start of the first step      */
  int64_t steps_done;     /* iterations run so far                               */
  uint8_t* best_x;        /* caller-owned host buffer of n bytes, or NULL        */
  double best_obj_f64;    /* F of best_x correctly rounded to float64 (integer
                             weights: best_obj converted); +inf before the first
                             evaluation                                           */
} pdbo_result;

/* ---- QUBO (dense MFMA path or CSR persistent path) ------------------------ */

/* Validates, canonicalises (Prop. 2.4) and uploads the instance, sets
 * X^0 = x0 and Y^0 = y0 (Alg. 1 input), and returns a context.  EINVAL for any
 * contract violation (checked before any HIP call); ERANGE when the exact
 * int64 evaluation cannot be guaranteed (|Q_ij| >= 2^30, or a row of |A| or
 * |c'| summing to 2^31 or more; dense: |Ahat_ij| above 2,139,062,143, the range
 * of the four int8 limbs Ahat = sum_l 256^l Ahat_l that the exact evaluation
 * multiplies one by one); EUNSUPPORTED for a CSR instance too large for the
 * restart-resident kernel when that kernel is asked for, or the INT8 form with
 * |Ahat_ij| > 127.  The dense
 * instance is canonicalised before any HIP call, so its range errors come back
 * on any machine.  `stream` is a hipStream_t (NULL = default).
 * Dense or CSR per instance: an int32 instance with n^2 B >= 2^30, tile 0,
 * PDBO_FP32, eval_every 1 and the vector dual, given dense with at most 10%
 * nonzeros or as CSR with n <= 16384, is built on both paths, each timed over
 * 8 iterations after 70, and kept on the other representation's path when that
 * is at least 10% faster; the context is then restarted from x0 (or the
 * generator's points), so its run is that of a context built on the chosen
 * path.  The choice is cached with the tile configurations under a key
 * "route/<arch>/f<format>/n<n>/B<B>/nz<nnz rounded up to 1024>/p<precision>/g<g_kind>"
 * (0 keeps the given representation, 1 takes the other); PDBO_ROUTE=0 turns
 * the choice off.  pdbo_tile_name tells which path runs. */
PDBO_API pdbo_status qubo_gda_init(const pdbo_qubo* prob, const pdbo_params* par, void* stream,
                          pdbo_ctx** out);

/* Enqueues nsteps >= 0 iterations of Alg. 1 on the context's stream,
 * asynchronously.  After each iteration t the rounded iterate of every
 * restart is evaluated exactly and the incumbent updated. */
PDBO_API pdbo_status qubo_gda_step(pdbo_ctx* ctx, int32_t nsteps);

/* Synchronises the stream and reports the incumbent (result->best_x, if not
 * NULL, receives n bytes). */
PDBO_API pdbo_status qubo_gda_result(pdbo_ctx* ctx, pdbo_result* result);

/* Copies the current iterate (x, y: host (B, n) float32, either may be NULL)
 * and iteration count.  Synchronises. */
PDBO_API pdbo_status qubo_gda_get_state(pdbo_ctx* ctx, float* x, float* y, int64_t* t);

/* Replaces the iterate (host (B, n) float32, x in [0,1]) and the iteration
 * count t >= 0; the incumbent is kept.  Synchronises. */
PDBO_API pdbo_status qubo_gda_set_state(pdbo_ctx* ctx, const float* x, const float* y, int64_t t);

/* Starts the run over on the same instance and parameters: X^0 = x0 (HOST
 * (B, n) float64 in [0,1], or NULL for the generator's points of the
 * parameters' seed), Y^0 = y0, t = 0, incumbent, trace and time origin
 * cleared (Alg. 1 input), without uploading the instance again.  Not for
 * batched contexts (ESTATE).  EINVAL when x0 lies outside [0,1].
 * Synchronises. */
PDBO_API pdbo_status qubo_gda_restart(pdbo_ctx* ctx, const double* x0);

/* Exact objectives (host int64[B]) of the rounded iterate evaluated last.
 * EUNSUPPORTED for float64 weights (use qubo_gda_objectives_f64). */
PDBO_API pdbo_status qubo_gda_objectives(pdbo_ctx* ctx, int64_t* F);

/* The same objectives (Eq. 1) correctly rounded to float64 (host double[B]);
 * for float64 weights the exact real sums, for integer weights the int64
 * values converted.  QUBO contexts (dense, CSR, row-parallel). */
PDBO_API pdbo_status qubo_gda_objectives_f64(pdbo_ctx* ctx, double* F);

/* Gradient of f/s, (A x + c')/s, at the host (B, n) float32 points x, written
 * to the host (B, n) float32 array G, computed by the same GEMM (dense: same
 * precision and tiles) that the step uses.  Does not change the iterate. */
PDBO_API pdbo_status qubo_gda_grad(pdbo_ctx* ctx, const float* x, float* G);

/* Exact objectives F (host int64[nb]) of nb host binary vectors xr (nb, n)
 * bytes in {0,1}, nb <= B, through the step's evaluation kernels.
 * EUNSUPPORTED for float64 weights (use qubo_gda_eval_f64). */
PDBO_API pdbo_status qubo_gda_eval(pdbo_ctx* ctx, const uint8_t* xr, int32_t nb, int64_t* F);

/* Objectives (Eq. 1) of nb host binary vectors xr (nb, n) bytes in {0,1},
 * 1 <= nb <= B, correctly rounded to float64 (host double[nb]): for float64
 * weights the exact real sum of the selected terms, rounded once. */
PDBO_API pdbo_status qubo_gda_eval_f64(pdbo_ctx* ctx, const uint8_t* xr, int32_t nb, double* F);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the exact
 * objectives of qubo_gda_eval with DEVICE arguments, enqueued on `stream`
 * (hipStream_t, NULL = the null stream), asynchronous, with no allocation,
 * free, memset or synchronisation.
 *   xr: device (nb, n) bytes, a nonzero byte counts as 1; F: device int64[nb];
 *   1 <= nb <= B.
 * The dense path stages xr and keeps the evaluation's integer partial sums in
 * a 16 MiB device array that the library holds on each GPU it runs on until
 * the process ends; PDBO_EUNSUPPORTED when nb * ld + 16 nb + 512 bytes exceed
 * it (ld = n rounded up to 128; nb <= 1656 at n = 10^4).  All calls on one GPU
 * share that array: calls that overlap on one GPU (other streams, threads or
 * contexts) race, calls ordered on one stream do not.  The CSR and MaxSAT
 * paths read xr in place and use no scratch.  ESTATE for batched contexts. */
PDBO_API pdbo_status qubo_gda_eval_noalloc(pdbo_ctx* ctx, const uint8_t* xr, int32_t nb, int64_t* F,
                                           void* stream);

/* Dual certificate (App. D, Dual Certificate): a lower bound on min F over
 * {0,1}^n.  For any y, the minimum of L(., y) over [0,1]^n is at most its
 * minimum over {0,1}^n, where L = F/s (weak duality, proof of Thm. 3.2).  With
 * the quadratic g and y = ybar * 1 the function L(., y) is convex when
 * A/s + 2 ybar I is positive semidefinite (ybar >= -lambda_min(A) / (2 s));
 * the caller vouches for that, the library does not check it.  The call runs
 * `iters` iterations of projected gradient descent on L(., ybar 1) (Alg. 1
 * with beta = 0, from x = 1/2, through the context's own step kernels and
 * precision) and then, at the point x reached, evaluates in float64 the bound
 *   s * (L(x) + sum_i min(-d_i x_i, d_i (1 - x_i))),  d = grad L(x),
 * less a bound on its rounding errors, into *lower_bound (valid at any x when
 * L is convex; tight at the minimiser).  value (or NULL) receives s L(x), the
 * Frank-Wolfe gap s * max_z d.(x - z) >= 0 and the rounding bound subtracted;
 * x_out (host float[n] or NULL) the point.  ybar = 0 takes the parameters'
 * y0.  Dense (single instance) and CSR contexts with the quadratic g and
 * integer weights, else EUNSUPPORTED.  The run's own iterate and incumbent are left untouched.
 * Synchronises. */
PDBO_API pdbo_status qubo_dual_bound(pdbo_ctx* ctx, double ybar, int32_t iters, double* lower_bound,
                                     double* value, float* x_out);

/* init + step(T) + result + destroy. */
PDBO_API pdbo_status qubo_gda_solve(const pdbo_qubo* prob, const pdbo_params* par, int32_t T,
                           void* stream, pdbo_result* result);

/* Many dense instances of uneven n stepped together: each iteration of all k
 * instances is ONE grouped launch per kernel (grouped != 0) or k launches per
 * kernel (grouped == 0), optionally captured in a hipGraph (par[0].graph_chunk).
 * par[i] gives instance i's parameters; B, precision, g_kind and eval_every
 * must agree across instances (and dual_kind).  results[i] (with its own best_x) receives
 * instance i's incumbent. */
PDBO_API pdbo_status qubo_gda_batch_init(int32_t k, const pdbo_qubo* probs, const pdbo_params* par,
                                int32_t grouped, void* stream, pdbo_ctx** out);
PDBO_API pdbo_status qubo_gda_batch_result(pdbo_ctx* ctx, int32_t inst, pdbo_result* result);
PDBO_API pdbo_status qubo_gda_batch_solve(int32_t k, const pdbo_qubo* probs, const pdbo_params* par,
                                 int32_t T, int32_t grouped, void* stream, pdbo_result* results);

/* ---- Max-k-Cut (softmax reparametrisation, row-parallel kernel) ----------- */

/* Max-k-Cut through the softmax reparametrisation of App. B: node i of a
 * restart has logits Z_{:,i} (k reals) and probabilities X_{:,i} =
 * softmax(Z_{:,i}); simultaneous gradient descent-ascent on
 * L(Z, y) = Tr(X W X^T)/s + sum_i y_i g(X_{:,i}) over (Z, y), with g quadratic
 * (sum_c X_ci^2 - 1, g_kind PDBO_G_QUAD) or entropy (sum_c X_ci log X_ci with
 * log taken at X clipped below at 2^-20, PDBO_G_ENTROPY):
 *   Z_ci -= alpha X_ci (G_ci - sum_c' X_c'i G_c'i),
 *   G_ci = (2/s) (X W)_ci + y_i dg/dX_ci,   y_i += beta g(X_{:,i}) (old X);
 * Z is unconstrained, so Alg. 1's projection and perturbation do not apply.
 * Every iteration the assignment c_i = argmax_c X_ci (lowest c on ties) is
 * evaluated exactly: F = the weight of the edges whose ends share a category
 * (each edge once; minimised, the cut is the total weight minus F).
 * x0: HOST (B, n, k) float64 logits Z^0 (finite), or NULL for the library's
 * generator (coordinate index i k + c, values in [0, 1)).  Step, result
 * (best_x: the n categories), objectives, trace, restart, timing and
 * destroy use the qubo_gda_* / pdbo_* entry points; get_state / set_state take
 * x as the logits Z, host (B, n, k) float32, and y as (B, n); eval takes
 * categories (nb, n) bytes in [0, k); grad returns d(Tr(X W X^T)/s)/dZ at
 * logits x, (B, n, k).  EINVAL for an asymmetric W, a diagonal entry, k out of
 * range; ERANGE for a row of |W| summing to 2^31 or more; EUNSUPPORTED for the
 * polynomial g or the scalar dual. */
PDBO_API pdbo_status kcut_gda_init(const pdbo_kcut* prob, const pdbo_params* par, void* stream,
                                   pdbo_ctx** out);

/* ---- weighted MaxSAT (persistent, restart-resident kernel) ---------------- */

/* Like qubo_gda_init for a MaxSAT formula; g_kind is usually PDBO_G_ENTROPY
 * (the paper's choice for Max-k-SAT).  Step, result, get/set_state,
 * objectives and grad use the qubo_gda_* entry points or the aliases below. */
PDBO_API pdbo_status maxsat_gda_init(const pdbo_maxsat* prob, const pdbo_params* par, void* stream,
                            pdbo_ctx** out);
PDBO_API pdbo_status maxsat_gda_step(pdbo_ctx* ctx, int32_t nsteps);
PDBO_API pdbo_status maxsat_gda_result(pdbo_ctx* ctx, pdbo_result* result);
PDBO_API pdbo_status maxsat_gda_solve(const pdbo_maxsat* prob, const pdbo_params* par, int32_t T,
                             void* stream, pdbo_result* result);

/* Lagrangian of a MaxSAT context for nb restarts given as DEVICE arrays:
 * L[b] = f(x_b)/s + sum_i y_bi g(x_bi)  (Sec. 3.1; f as in Sec. 4.1).
 * x, y: device (nb, n) float32 (x in [0,1]); L: device float32[nb].
 * Enqueued on `stream` (hipStream_t); asynchronous. */
PDBO_API pdbo_status maxsat_lagrangian_fwd(pdbo_ctx* ctx, const float* x, const float* y, int32_t nb,
                                  float* L, void* stream);

/* Adjoint of maxsat_lagrangian_fwd: given dL (device float32[nb]) writes
 * dx = dL_b * (grad f(x_b)/s + y_b * g'(x_b)) and dy = dL_b * g(x_b) as device
 * (nb, n) float32 arrays.  Deterministic (no atomics). */
PDBO_API pdbo_status maxsat_lagrangian_bwd(pdbo_ctx* ctx, const float* x, const float* y,
                                  const float* dL, int32_t nb, float* dx, float* dy,
                                  void* stream);

/* ---- instrumentation ------------------------------------------------------ */

/* Incumbent improvements of a dense context, in order: iteration t, objective
 * F, restart b and device-clock seconds since the start of the first step, for
 * at most `cap` records (host arrays, any may be NULL); *len receives the
 * number of records kept (the device keeps the first 4096).  Persistent
 * (CSR, MaxSAT) contexts keep per-restart bests instead and report len = 0.
 * Synchronises. */
PDBO_API pdbo_status qubo_gda_trace(pdbo_ctx* ctx, int32_t cap, int64_t* t, int64_t* F, int32_t* b,
                                    double* sec, int32_t* len);

/* qubo_gda_trace with the objectives correctly rounded to float64 (the only
 * form for float64 weights, where qubo_gda_trace returns EUNSUPPORTED). */
PDBO_API pdbo_status qubo_gda_trace_f64(pdbo_ctx* ctx, int32_t cap, int64_t* t, double* F,
                                        int32_t* b, double* sec, int32_t* len);

/* Kernel classes of pdbo_kernel_time:
 *   PDBO_K_STEP        dense GEMM with the Alg. 1 update fused (one per iteration)
 *   PDBO_K_EVAL        dense int8 GEMM of the exact objectives (Eq. 1); a column
 *                      block of restarts is skipped when none of them needs a
 *                      full product
 *   PDBO_K_ARGMIN      best of B and incumbent update, when it has a launch of its
 *                      own: with incremental evaluation (eval_every = 1) an
 *                      iteration's best of B runs in extra workgroups of the
 *                      next step launch, and only the last iteration of each
 *                      qubo_gda_step call (or graph of iterations) launches it
 *   PDBO_K_PERSISTENT  the CSR and MaxSAT persistent kernels (one per step call)
 *   PDBO_K_INCR        exact objective differences from the recorded rounding
 *                      changes: when at most 32 coordinates of a restart's
 *                      rounded iterate changed since the previous evaluation,
 *                      F(x') - F(x) = sum_i d_i (c'_i + kappa (Ahat x')_i)
 *                                     - kappa sum_{i<j} d_i d_j Ahat_ij
 *                      (d = x' - x, all in integers) replaces the full product;
 *                      the first evaluation after init or set_state, and any
 *                      restart with more changes, take the full product.  This
 *                      kernel also finalises every restart's objective. */
enum { PDBO_K_STEP = 0, PDBO_K_EVAL = 1, PDBO_K_ARGMIN = 2, PDBO_K_PERSISTENT = 3,
       PDBO_K_INCR = 4, PDBO_K_COUNT = 5 };

/* Enables (1) or disables (0) HIP-event timing of every kernel launch of the
 * context, on the context's stream.  Clears the accumulated times. */
PDBO_API pdbo_status pdbo_timing(pdbo_ctx* ctx, int32_t enable);

/* Times only the launches of the kernel classes in mask (bit k = PDBO_K_k;
 * 0 disables timing): every timed launch costs two event records on the
 * stream, so a caller that needs one class measures the others separately.
 * Clears the accumulated times.  PDBO_EINVAL for bits beyond PDBO_K_COUNT. */
PDBO_API pdbo_status pdbo_timing_classes(pdbo_ctx* ctx, uint32_t mask);

/* Times only every stride-th launch of each timed class, counting from the
 * first launch after this call or pdbo_timing / pdbo_timing_classes (1, the
 * default, times every launch), so that a long timed run carries fewer event
 * records.  Clears the accumulated times.  PDBO_EINVAL for stride < 1. */
PDBO_API pdbo_status pdbo_timing_stride(pdbo_ctx* ctx, int32_t stride);

/* Accumulated device time (ms) and launch count of kernel class `which`
 * (PDBO_K_*) since timing was enabled.  Synchronises. */
PDBO_API pdbo_status pdbo_kernel_time(pdbo_ctx* ctx, int32_t which, double* total_ms, int64_t* launches);

/* The dense tile autotuner's cache, a JSON object of "key": cfg lines in
 * $PDBO_AUTOTUNE_CACHE (default $HOME/.cache/pdbo_autotune.json).  A context
 * whose tile is chosen automatically looks its key up there and, when absent,
 * times every configuration and stores the fastest.  pdbo_autotune_store sets
 * `key` to tile configuration `cfg` (0-based; the params' `tile` is cfg + 1),
 * creating missing directories of the path; pdbo_autotune_lookup writes the
 * cached configuration to *cfg, or -1 when there is none.  Keys are at most
 * 399 printable bytes without '"' or '\'.  EINVAL for a bad key or
 * configuration, or when the cache cannot be written.  No device work. */
PDBO_API pdbo_status pdbo_autotune_store(const char* key, int32_t cfg);
PDBO_API pdbo_status pdbo_autotune_lookup(const char* key, int32_t* cfg);

/* Name of the tile configuration the dense path uses, of the kernel variant
 * the restart-resident CSR path uses, or "csr_rows" for the row-parallel CSR
 * path (static string; empty for the other paths). */
PDBO_API const char* pdbo_tile_name(const pdbo_ctx* ctx);

PDBO_API void pdbo_destroy(pdbo_ctx* ctx);
PDBO_API const char* pdbo_status_str(pdbo_status s);
PDBO_API const char* pdbo_last_error(const pdbo_ctx* ctx);
PDBO_API const char* pdbo_last_global_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PDBO_H */
