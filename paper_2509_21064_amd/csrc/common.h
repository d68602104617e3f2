// Internal declarations shared by the HIP translation units of libpdbo.
//
// Layout in HBM (all per-restart arrays are restart-major):
//   X[2], Y      float32 [B][ld]   ping-pong primal iterate, dual iterate
//   Xs[2]        GEMM shadow of X in the operand type (bf16 / e4m3) [B][ld]
//   Xr           int8 {0,1} [B][ld] rounded iterate [x > 1/2]
//   A            canonical Ahat = offdiag(Q + Q^T)/kappa in the operand type,
//                n rows x ld columns (columns n..ld-1 are zero)
//   A8           the same matrix exactly, as nlimb int8 limbs of n x ld each
//                (evaluation operand; one limb when every |Ahat_ij| <= 127)
// ld is n rounded up to a multiple of 128 elements, so every row of every
// operand is a whole number of 128-byte K chunks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pdbo.h"

namespace pdbo {

enum Prec { P_F32 = 0, P_BF16 = 1, P_FP8 = 2, P_I8 = 3 };
enum Epi { EPI_STEP = 0, EPI_GRAD = 1, EPI_EVAL = 2 };

constexpr int kLdAlign = 128;        // elements
constexpr float kEntropyEps = 9.5367431640625e-07f;  // 2^-20

struct Incumbent {
  int64_t F;        // INT64_MAX when empty
  int64_t t;        // iteration (1-based)
  int64_t b;        // restart
  uint64_t ts;      // device wall clock at the improvement
};

struct TraceRec {
  int64_t t;
  int64_t F;
  int64_t b;
  uint64_t ts;
};

// Alg. 1 step-size parameters, kernel-argument sized.
struct GdaP {
  float alpha, beta, delta;
  int gkind;        // 0 quadratic, 1 entropy, 2 polynomial
  int deg;          // d of the polynomial g
};

// One dense instance as seen by the kernels.
struct InstDev {
  const uint8_t* A;       // Ahat in the GEMM operand type
  const int8_t* A8;       // Ahat as nlimb int8 limbs (evaluation): limb l at A8 + l * limb_stride,
                          // Ahat = sum_l 256^l Ahat_l with signed digits Ahat_l in [-128, 127]
  const float* rscale;    // e4m3 row scale (FP8 form), else nullptr
  const int32_t* rsum;    // sum_j Ahat_ij (INT8 form: offset of the quantised x)
  const float* cps;       // c'/s, padded to ld with zeros
  const int64_t* cp;      // c', padded to ld with zeros
  float* X[2];
  float* Y;
  uint8_t* Xs[2];         // shadows; for FP32 these alias X
  int8_t* Xr;
  float* G;               // gradient output of the GRAD epilogue
  int64_t* Sacc;          // [B] x_r^T Ahat x_r, accumulated by integer atomics
  int64_t* Cacc;          // [B] c'^T x_r, accumulated by integer atomics
  int64_t* Fall;          // [B] objectives of the last evaluation
  Incumbent* inc;
  uint8_t* best_x;        // [ld]; the first n bytes are the best rounded vector
  TraceRec* trace;
  int32_t* trace_len;
  int64_t* t_dev;         // completed iterations
  // Incremental evaluation (nullptr: every evaluation is a full product).
  // The step epilogue records the coordinates whose rounding changed; an
  // evaluation then updates F_b exactly from them unless more than kFlipMax
  // changed (or nflip[b] was set above kFlipMax to ask for a full product).
  // The incremental kernel finalises every F_b (Fall) and keeps the rounded
  // row of each restart that beats the incumbent (cand), so that the best of
  // B can run while the next step already rewrites x_r.
  int32_t* nflip;         // [B] rounding changes since the last evaluation
  uint32_t* fbits;        // [B][ld / 32] bitmap of the changed coordinates
  uint8_t* cand;          // [B][ld] rounded rows that beat the incumbent when evaluated
  uint64_t* ts0;          // clock at the first step
  // Scalar dual (PDBO-s, single constraint sum_i g(x_i) = 0): one y per
  // restart, or nullptr for the vector dual of Alg. 1.  Before each step the
  // scalar of restart b is copied into its row of Y (which the step reads as
  // y_i) and raised by beta * sum_i g(x_i^t).
  float* ys;              // [B]
  int n, ld, B, mblocks;
  int kappa, trace_cap;
  int nlimb;              // int8 limbs of Ahat (1 when every |Ahat_ij| <= 127)
  int64_t limb_stride;    // bytes between limbs (n * ld)
  float kos;              // kappa / s
  GdaP gp;
};

struct TileDev {
  int inst, m0, n0, mblk;
};

// ---- device helpers -------------------------------------------------------

// The binarity constraint functions of Sec. 3.1: quadratic x^2 - x, entropy
// x log x + (1-x) log(1-x) (continuous at 0 and 1), and the even polynomial
// (2x - 1)^(2d) - 1, whose derivative is 4d (2x - 1)^(2d-1).
__device__ __forceinline__ float poly_pow(float u2, int deg) {  // u2^(deg-1)
  float t = 1.f;
  for (int k = 1; k < deg; ++k) t *= u2;
  return t;
}

__device__ __forceinline__ float g_value(float x, int gkind, int deg = 1) {
  if (gkind == 0) return x * x - x;
  if (gkind == 2) {
    const float u = 2.f * x - 1.f, u2 = u * u;
    return u2 * poly_pow(u2, deg) - 1.f;
  }
  float a = x > 0.f ? x * logf(x) : 0.f;
  float b = x < 1.f ? (1.f - x) * logf(1.f - x) : 0.f;
  return a + b;
}

__device__ __forceinline__ float g_deriv(float x, int gkind, int deg = 1) {
  if (gkind == 0) return 2.f * x - 1.f;
  if (gkind == 2) {
    const float u = 2.f * x - 1.f;
    return 4.f * (float)deg * u * poly_pow(u * u, deg);
  }
  float xc = fminf(fmaxf(x, kEntropyEps), 1.f - kEntropyEps);
  return logf(xc) - logf(1.f - xc);
}

// One coordinate of Alg. 1: perturbation test, projected primal step and dual
// ascent with g evaluated at the old x (simultaneous update, Eq. 6).
__device__ __forceinline__ void gda_update(float x, float y, float G, const GdaP& p,
                                           float& xn, float& yn) {
  float dL = fmaf(y, g_deriv(x, p.gkind, p.deg), G);
  bool pert = (fabsf(x - 0.5f) <= p.delta) && (fabsf(dL) <= 2.f * p.delta) && (y <= 0.f);
  float xs = fminf(fmaxf(fmaf(-p.alpha, dL, x), 0.f), 1.f);
  float xp = x <= 0.5f ? 0.5f - p.delta : 0.5f + p.delta;
  xn = pert ? xp : xs;
  yn = fmaf(p.beta, g_value(x, p.gkind, p.deg), y);
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ uint64_t wall_clock() { return __builtin_amdgcn_s_memrealtime(); }

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011): ten rounds of
// (c0, c1, c2, c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1,
// lo(M0 c0)) with the key raised by the Weyl constants between rounds.  The
// starting point of coordinate i of restart b is word i mod 4 of the output for
// the counter (i / 4, b, 0, 0) under the key (seed lo, seed hi), scaled to a
// multiple of 2^-24 in [0, 1) (App. C: x^0 uniform on [0,1]^n).
__device__ __forceinline__ float philox_start(uint64_t seed, uint32_t b, uint32_t i) {
  uint32_t c0 = i >> 2, c1 = b, c2 = 0u, c3 = 0u;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
  }
  const uint32_t w = (i & 3u) == 0u ? c0 : (i & 3u) == 1u ? c1 : (i & 3u) == 2u ? c2 : c3;
  return (float)(w >> 8) * 5.9604644775390625e-08f;  // 2^-24
}


// Sum of an int32 over the 64 lanes of a wave through DPP moves (no LDS):
// shifts by 1, 2, 4 and 8 within each row of 16 lanes leave the row's total in
// its lane 15; row_bcast:15 adds row 0's total into row 1 and row 2's into
// row 3, row_bcast:31 adds lane 31 into rows 2 and 3, so lane 63 ends with
// the wave's total.  Lanes a move does not reach add 0.
__device__ __forceinline__ int wave_sum_i32(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15, rows 1 and 3
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31, rows 2 and 3
  return __builtin_amdgcn_readlane(v, 63);
}

// One step of a row reduction: v plus the value of the lane SHR lanes lower
// in the same row of 16 lanes (0 for the first SHR lanes of a row), on the two
// 32-bit halves of an int64 with the carry.
template <int CTL>
__device__ __forceinline__ int64_t row_shr_add_i64(int64_t v) {
  const uint32_t lo = (uint32_t)v, hi = (uint32_t)((uint64_t)v >> 32);
  const uint32_t slo = __builtin_amdgcn_update_dpp(0u, lo, CTL, 0xf, 0xf, true);
  const uint32_t shi = __builtin_amdgcn_update_dpp(0u, hi, CTL, 0xf, 0xf, true);
  return v + (int64_t)(((uint64_t)shi << 32) | slo);
}

// Sum of v over lanes 0..15 (row 0 of the wave), returned in every lane: row
// shifts by 1, 2, 4 and 8 leave each row's total in its lane 15.  Exact in int64.
__device__ __forceinline__ int64_t row16_sum_i64(int64_t v) {
  v = row_shr_add_i64<0x111>(v);  // row_shr:1
  v = row_shr_add_i64<0x112>(v);  // row_shr:2
  v = row_shr_add_i64<0x114>(v);  // row_shr:4
  v = row_shr_add_i64<0x118>(v);  // row_shr:8
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, 15);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)((uint64_t)v >> 32), 15);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// ---- launchers (dense.hip) --------------------------------------------------

constexpr int kFlipMax = 32;

struct TileCfgInfo {
  const char* name;
  int BM, BN, WM, WN, threads;  // block tile, waves along M and N
  int dma;                       // 1: three-stage direct-to-LDS main loop
};
int dense_num_cfgs();
const TileCfgInfo& dense_cfg(int id);

// gkind: the kind of g (GdaP::gkind) of every instance of the launch; only the
// step epilogue uses it.  parity: the operand shadow the step and gradient
// epilogues read (STEP, GRAD); the limb of Ahat an evaluation launch adds
// (EVAL: pass l adds 256^l Ahat_l x_r, and c'^T x_r in pass 0; instances with
// fewer limbs skip the pass)
// A step launch may also run the best of B of the previous iteration for
// instances am0 .. am0 + amn - 1 (incremental evaluation only), in amn extra
// workgroups after the tiles.
hipError_t launch_dense_gemm(int cfg, int prec, int epi, int gkind, const TileDev* tiles,
                             int ntiles, const InstDev* insts, int parity, int grid, hipStream_t s,
                             int am0 = 0, int amn = 0);
hipError_t launch_argmin(const InstDev* insts, int inst0, int ninst, int mode, hipStream_t s);
// work[w] = (instance, first restart) of the workgroups of the incremental evaluation
// full_done: the evaluation GEMM ran in this iteration (its partials hold the
// full products); otherwise restarts that need one are evaluated by rows
hipError_t launch_eval_incr(const InstDev* insts, const int2* work, int nwork, int full_done,
                            hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t s);
// Scalar dual of every restart of ninst instances (grid B x ninst): writes y^t
// into the restart's row of Y and sets y^{t+1} = y^t + beta sum_i g(x_i^t),
// with x^t in X[parity].
hipError_t launch_dual_scalar(const InstDev* insts, int ninst, int B, int gkind, int parity,
                              hipStream_t s);
hipError_t launch_stamp(uint64_t* ts0, hipStream_t s);
// x0 == nullptr: X^0 is drawn by Philox4x32-10 keyed by seed (pdbo_params)
hipError_t launch_init_state(const double* x0, int B, int n, int ld, float y0, float* X,
                             float* Y, uint8_t* Xs, int xs_prec, int8_t* Xr, uint64_t seed,
                             hipStream_t s);
hipError_t launch_set_state(const float* x, const float* y, int B, int n, int ld, float* X,
                            float* Y, uint8_t* Xs, int xs_prec, hipStream_t s);
hipError_t launch_quantize_A(const int32_t* Ahat, int n, int ld, int prec, uint8_t* A,
                             int8_t* A8, int nlimb, const float* rscale, hipStream_t s);
hipError_t launch_fill_i64(int64_t* p, int64_t v, size_t cnt, hipStream_t s);

// ---- launchers (sparse.hip) -------------------------------------------------

struct CsrDev {
  const int32_t* row_ptr;
  const void* col;        // int32 column indices
  const void* val;        // int32 values of Ahat
  const uint32_t* packed; // column | value << 16 when n <= 65536 and |Ahat_ij| < 2^15
  const float* cps;
  const int64_t* cp;
  float* X;               // [B][ld]
  float* Y;
  int64_t* rbestF;        // [B]
  int64_t* rbestT;
  uint64_t* rbestTs;
  uint8_t* best_xr;       // [B][n]
  int64_t* Flast;         // [B]
  const int32_t* order;   // [n] rows by decreasing degree: thread t of the
                          // persistent kernel owns rows order[t + j * threads]
  // the packed entries interleaved by slices of 64 positions (the rows
  // order[q] of one wave round): entry r of row order[q] is
  // psl[slice[q / 64] + 64 r + q % 64], so a wave's LDS reads of entry r hit
  // consecutive words; null when the layout is not used (1024-thread packed
  // kernels only, and only when it takes no more LDS than row_ptr + entries)
  const uint32_t* psl;
  const int32_t* slice;   // [ceil(n / 64)]
  int64_t nsl;            // words of psl
  int64_t nnz;
  int n, ld, B, kappa;
  int small32;            // 512 * max_i sum_j |Ahat_ij| and 512 * max_i |c'_i| are below 2^31
  int tot32;              // n times each of those is below 2^31 too: a restart's totals fit int32
  float kos;
  GdaP gp;
};
bool csr_fits(int n, int64_t nnz, bool packed, size_t* lds_bytes);
const char* csr_variant_name(const CsrDev& d, bool packed);
hipError_t launch_csr_persistent(const CsrDev& d, bool packed, int64_t t0, int nsteps,
                                 hipStream_t s);
hipError_t launch_csr_grad(const CsrDev& d, const float* X, float* G, int nb, hipStream_t s);
hipError_t launch_csr_eval(const CsrDev& d, const int8_t* xr, int nb, int64_t* F, hipStream_t s);

// ---- launchers (spmm.hip) ---------------------------------------------------
//
// Sparse path that is not restart-resident: one launch per iteration over all
// rows, the restarts of a row in adjacent lanes.  Iterates are node-major
// ([n][B]: the B restarts of coordinate i are contiguous), so gathering x_j
// for all restarts of a group reads B contiguous floats.  Used when x of one
// restart does not fit in LDS, or when there are too few restarts to fill the
// chip with one workgroup each.
struct SpmmDev {
  const int32_t* row_ptr;
  const int32_t* col;
  const int32_t* val;     // canonical Ahat
  const uint32_t* packed; // column | value << 16 when n <= 65536 and |Ahat_ij| < 2^15 (integer
                          // weights), read instead of col and val; else null
  const float* cps;       // c'/s
  const int64_t* cp;      // c'
  float* X[2];            // node-major ping-pong iterate
  float* Y;               // node-major dual iterate
  int64_t* part;          // [nslices][2][W][grid / nslices]: partial sums S, C of each
                          // restart from every workgroup of its slice
  int64_t* Flast;         // [B] objectives of the last evaluation
  Incumbent* inc;
  uint8_t* best_x;        // [n]
  int32_t* win;           // [1] integer weights: restart whose rounded iterate became the
                          // incumbent and still has to be copied into best_x, or -1 (the
                          // next step launch copies it while it overwrites that iterate,
                          // the last best-of-B launch of a call at once); null: no deferral
  TraceRec* trace;
  int32_t* trace_len;
  int64_t* t_dev;         // completed iterations
  uint64_t* ts0;
  int n, B, kappa, trace_cap;
  int W;                  // restarts per lane group (slice width, <= 64)
  int G;                  // lane groups per wave (64 / W)
  int nslices;            // ceil(B / W)
  int grid;               // workgroups of a launch (a multiple of nslices)
  float kos;              // kappa / s
  GdaP gp;
  // float64 weights (ndig > 0): the gradient reads valf = A/s in float32, the
  // exact objective ndig signed base-2^24 digits of the canonical integers in
  // units of 2^elo (A = sum_d 2^(24 d) Adig[d], c' likewise), with
  // F = N 2^(elo - 1), N = S + 2 C (S over ordered pairs, C the linear part).
  // part then holds [nslices][2 ndig][W][grid / nslices].
  const float* valf;
  const int32_t* Adig;    // [ndig][nnz]
  const int32_t* Cdig;    // [ndig][n]
  int64_t nnz;
  int ndig, elo;
  uint64_t* incw;         // [4] the incumbent's N, 256-bit two's complement
  double* Fd;             // [B] objectives of the last evaluation, rounded to float64
};
constexpr int kMaxDigits = 8;  // 192 bits of fixed point
// mode 0: gradient, Alg. 1 update into X[parity ^ 1] and Y, and the exact
// objective of round(X[parity]) into the partials; mode 1: the objective only;
// mode 2: the gradient only, into G (node-major)
hipError_t launch_spmm(const SpmmDev& d, int mode, int parity, float* G, hipStream_t s);
// Objectives from the partials, first argmin over b, incumbent update for
// evaluations of x^t with t >= 1 (label: the completed iterations), and, for
// advance != 0, the iteration counter moves on.  The winning rounded vector
// is read from X[parity], at once or (integer weights, advance != 0) by the
// next step launch.
hipError_t launch_spmm_best(const SpmmDev& d, int parity, int advance, hipStream_t s);
// float64-weight forms (realw.hip).  launch_spmm and launch_spmm_best call
// these when d.ndig > 0.  With Fout != NULL, launch_spmm_real_best writes the
// objectives of X[parity]'s first nb restarts, correctly rounded, into Fout,
// without touching the incumbent (after a mode-1 pass over X[parity]).
hipError_t launch_spmm_real(const SpmmDev& d, int mode, int parity, float* G, hipStream_t s);
hipError_t launch_spmm_real_best(const SpmmDev& d, int parity, int advance, double* Fout, int nb,
                                 hipStream_t s);
// restart-major host bytes (nb, n) -> node-major 0/1 floats of X[parity], other restarts 0
hipError_t launch_real_load_x(const uint8_t* xr, int nb, const SpmmDev& d, int parity,
                              hipStream_t s);
// node-major state <-> restart-major host layout helpers on the device
hipError_t launch_spmm_init(const double* x0, const SpmmDev& d, float y0, uint64_t seed,
                            hipStream_t s);
// ---- launchers (kcut.hip) ---------------------------------------------------
//
// Max-k-Cut through the softmax reparametrisation: logits Z, probabilities X,
// node-major [n][B][k]; duals Y [n][B]; the same lane groups as SpmmDev.
struct KcutDev {
  const int32_t* row_ptr;
  const int32_t* col;
  const int32_t* w;       // symmetric edge weights, both directions stored
  float* Z;
  float* X[2];            // softmax(Z), ping-pong
  float* Y;
  int64_t* part;          // [nslices][W][grid / nslices]: same-category weight (edges
                          // twice) of each restart from every workgroup of its slice
  int64_t* Flast;
  Incumbent* inc;
  uint8_t* best_x;        // [n] categories of the incumbent
  int32_t* win;           // [1] restart whose rounded iterate became the incumbent
                          // and still has to be copied into best_x, or -1: the
                          // next step launch copies it while it overwrites that
                          // iterate, the last best-of-B launch of a call at once
  TraceRec* trace;
  int32_t* trace_len;
  int64_t* t_dev;
  uint64_t* ts0;
  int n, B, k, trace_cap;
  int W, G, nslices, grid;
  float tos;              // 2 / s
  GdaP gp;
};
hipError_t launch_kcut(const KcutDev& d, int mode, int parity, float* G, hipStream_t s);
hipError_t launch_kcut_best(const KcutDev& d, int parity, int advance, hipStream_t s);
hipError_t launch_kcut_init(const double* z0, const KcutDev& d, float y0, uint64_t seed,
                            hipStream_t s);
hipError_t launch_kcut_set(const float* z, const float* y, const KcutDev& d, int parity,
                           hipStream_t s);
hipError_t launch_kcut_eval(const KcutDev& d, const uint8_t* cat, int nb, int64_t* F,
                            hipStream_t s);

// ---- launchers (cert.hip) ---------------------------------------------------
//
// Certified lower bound on min F from the Lagrangian at y = ybar * 1 with the
// quadratic g, evaluated at one box point x (device float[ld] / float[n]) in
// float64 with rounding bounds: rows = device double[4 n] scratch; res = device
// double[4]: bound, s L(x), Frank-Wolfe gap, rounding bound subtracted.
hipError_t launch_cert_dense(const InstDev& I, const float* x, double s, double ybar, double* rows,
                             double* res, hipStream_t st);
hipError_t launch_cert_csr(const CsrDev& d, const float* x, double s, double ybar, double* rows,
                           double* res, hipStream_t st);
hipError_t launch_fill_f32(float* p, float v, int64_t cnt, hipStream_t st);

// Reduction of per-restart bests to the incumbent (persistent paths).
hipError_t launch_restart_best(const int64_t* rbestF, const int64_t* rbestT,
                               const uint64_t* rbestTs, const uint8_t* best_xr, int B, int n,
                               Incumbent* inc, uint8_t* best_x, hipStream_t s);

// ---- launchers (maxsat.hip) -------------------------------------------------

struct SatDev {
  const int32_t* inc_ptr;   // [n+1] per-variable incidence ranges
  const int32_t* inc;       // entries of k int32: (k-1) other literal codes, then meta
  const int32_t* lits;      // [m][k] literal codes (var | neg<<31)
  const int32_t* w;         // [m]
  float* X;                 // [B][ld]
  float* Y;
  int64_t* rbestF;
  int64_t* rbestT;
  uint64_t* rbestTs;
  uint8_t* best_xr;
  int64_t* Flast;
  // the persistent kernel works on positions p = 0..n-1 holding the variables
  // order[p] in order of decreasing occurrence count (the variables of a wave
  // round then have lists of nearly the same length): its occurrence lists are
  // indexed by position and their literal codes name positions
  const int32_t* order;     // [n] variable at position p
  const int32_t* pinc_ptr;  // [n+1]
  const int32_t* pinc;      // as inc, codes in positions
  // 3-SAT: the entries in 8 bytes, the two other literals as 16-bit codes
  // (position | negated << 15) in the low word, the meta word in the high
  // word; each position's list starts with the clauses it owns.  Interleaved
  // by slices of 64 positions (the positions of one wave): entry r of
  // position p is pinc3[pinc3_slice[p / 64] + 64 r + p % 64], so a wave's
  // load of entry r reads 512 contiguous bytes; a position's count is
  // pinc_ptr[p + 1] - pinc_ptr[p]
  const uint64_t* pinc3;
  const int32_t* pinc3_slice;  // [ceil(n / 64)]
  int n, m, k, ld, B;
  float ios;                // 1/s
  GdaP gp;
};
bool sat_fits(int n, size_t* lds_bytes);
hipError_t launch_sat_persistent(const SatDev& d, int64_t t0, int nsteps, hipStream_t s);
hipError_t launch_sat_grad(const SatDev& d, const float* X, int ldx, float* G, int nb,
                           hipStream_t s);
hipError_t launch_sat_eval(const SatDev& d, const int8_t* xr, int nb, int64_t* F,
                           hipStream_t s);
hipError_t launch_sat_fwd(const SatDev& d, const float* x, const float* y, int nb, float* L,
                          hipStream_t s);
hipError_t launch_sat_bwd(const SatDev& d, const float* x, const float* y, const float* dL,
                          int nb, float* dx, float* dy, hipStream_t s);

}  // namespace pdbo
