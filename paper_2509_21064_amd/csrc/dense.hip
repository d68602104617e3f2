// Dense QUBO path: one MFMA GEMM kernel family for gfx950.
//
//   EPI_STEP : G = (kappa/s) * Ahat . X + c'/s, then Alg. 1 for every (i, b) in
//              the tile, in registers (perturbation, projection, dual ascent),
//              writing X^{t+1}, Y^{t+1}, the operand shadow of X^{t+1} and the
//              rounded iterate [x^{t+1} > 1/2].
//   EPI_GRAD : G only (tests and autotuning).
//   EPI_EVAL : E = Ahat . Xr in int8 x int8 -> int32, reduced on the fly to
//              x_r^T Ahat x_r and c'^T x_r per restart with int64 atomics
//              (integer addition is exact in any order, so the totals are
//              bit-reproducible); a tile whose restarts all changed few
//              rounded coordinates exits at once, their objectives come from
//              eval_incr_kernel (the incremental evaluation below).
//
// Operands are both K-contiguous: row i of Ahat (Ahat is symmetric) and row b
// of the restart-major shadow.  Every K step consumes one 128-byte chunk of
// each row, whatever the element type, so a lane always reads 32 bytes per
// 16-row fragment: row (lane % 16), two 16-byte pieces of the chunk (bytes
// [32*(lane/16), +32) in the register-staged kernel, pieces lane/16 and
// lane/16 + 4 in the DMA kernel).  The same lane->k mapping is used for both
// operands, which is all the MFMA dot product needs.  Output layout of the 16x16 MFMA: lane holds rows
// 4*(lane/16)+r, r = 0..3, of column lane % 16.
#include <climits>

#include "common.h"

// This file is compiled four times (see build.py): part 0 holds everything but
// the step kernels, part 1 + k the step kernels of the k-th kind of g, so that
// the parts compile in parallel.
#ifndef PDBO_DENSE_PART
#define PDBO_DENSE_PART 0
#endif

namespace pdbo {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int P> struct PT;
template <> struct PT<P_F32> { static constexpr int EB = 4; using Acc = f32x4; };
template <> struct PT<P_BF16> { static constexpr int EB = 2; using Acc = f32x4; };
template <> struct PT<P_FP8> { static constexpr int EB = 1; using Acc = f32x4; };
template <> struct PT<P_I8> { static constexpr int EB = 1; using Acc = i32x4; };

// One 128-byte K chunk of a 16x16 output fragment.
template <int P>
__device__ __forceinline__ void mfma_chunk(typename PT<P>::Acc& c, const u32x4 (&a)[2],
                                           const u32x4 (&b)[2]);

template <>
__device__ __forceinline__ void mfma_chunk<P_F32>(f32x4& c, const u32x4 (&a)[2],
                                                  const u32x4 (&b)[2]) {
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int s = 0; s < 4; ++s)
      c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a[h][s]),
                                               __uint_as_float(b[h][s]), c, 0, 0, 0);
}

template <>
__device__ __forceinline__ void mfma_chunk<P_BF16>(f32x4& c, const u32x4 (&a)[2],
                                                   const u32x4 (&b)[2]) {
#pragma unroll
  for (int h = 0; h < 2; ++h)
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[h]),
                                                __builtin_bit_cast(bf16x8, b[h]), c, 0, 0, 0);
}

template <>
__device__ __forceinline__ void mfma_chunk<P_FP8>(f32x4& c, const u32x4 (&a)[2],
                                                  const u32x4 (&b)[2]) {
  i32x8 av = {(int)a[0][0], (int)a[0][1], (int)a[0][2], (int)a[0][3],
              (int)a[1][0], (int)a[1][1], (int)a[1][2], (int)a[1][3]};
  i32x8 bv = {(int)b[0][0], (int)b[0][1], (int)b[0][2], (int)b[0][3],
              (int)b[1][0], (int)b[1][1], (int)b[1][2], (int)b[1][3]};
  // format 0 = e4m3 for both operands; E8M0 scales of 2^0
  c = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv, c, 0, 0, 0, 0x7f7f7f7f, 0,
                                                       0x7f7f7f7f);
}

template <>
__device__ __forceinline__ void mfma_chunk<P_I8>(i32x4& c, const u32x4 (&a)[2],
                                                 const u32x4 (&b)[2]) {
#pragma unroll
  for (int h = 0; h < 2; ++h)
    c = __builtin_amdgcn_mfma_i32_16x16x64_i8(__builtin_bit_cast(i32x4, a[h]),
                                              __builtin_bit_cast(i32x4, b[h]), c, 0, 0, 0);
}

// Half of a 128-byte K chunk (the 16 bytes a lane holds of one fragment row):
// the software-pipelined main loop issues the MFMAs of one half while it reads
// the other half's fragments.  Per accumulator the sequence of MFMAs is the
// same as mfma_chunk's (half 0, then half 1 of every chunk).  FP8 has no half
// form: its single MFMA per chunk consumes all 32 bytes of a lane.
template <int P> struct HasHalf { static constexpr bool value = P != P_FP8; };
template <int P> struct HalfMfmas { static constexpr int value = P == P_F32 ? 4 : 1; };

template <int P>
__device__ __forceinline__ void mfma_half(typename PT<P>::Acc& c, const u32x4& a, const u32x4& b);

template <>
__device__ __forceinline__ void mfma_half<P_F32>(f32x4& c, const u32x4& a, const u32x4& b) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a[s]), __uint_as_float(b[s]), c, 0, 0,
                                             0);
}

template <>
__device__ __forceinline__ void mfma_half<P_BF16>(f32x4& c, const u32x4& a, const u32x4& b) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                              __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

template <>
__device__ __forceinline__ void mfma_half<P_I8>(i32x4& c, const u32x4& a, const u32x4& b) {
  c = __builtin_amdgcn_mfma_i32_16x16x64_i8(__builtin_bit_cast(i32x4, a),
                                            __builtin_bit_cast(i32x4, b), c, 0, 0, 0);
}

// x in [0,1] -> q = round(254 x) - 127 in [-127, 127] (x ~ (q + 127) / 254)
__device__ __forceinline__ uint32_t quant8(float x) {
  return (uint32_t)(uint8_t)(int8_t)((int)rintf(x * 254.f) - 127);
}

__device__ __forceinline__ uint32_t pack_q8x4(float a, float b, float c, float d) {
  return quant8(a) | (quant8(b) << 8) | (quant8(c) << 16) | (quant8(d) << 24);
}

__device__ __forceinline__ uint32_t pack_fp8x4(float a, float b, float c, float d) {
  int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
  return (uint32_t)w;
}

// Pointers read from the instance table are generic; casting them to the
// global address space makes the compiler emit global_load/global_store rather
// than flat accesses, which would also count against the LDS wait counter and
// serialise the operand prefetch with the fragment reads.
#define PDBO_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ PDBO_GLOBAL T* gptr(T* p) {
  return (PDBO_GLOBAL T*)p;
}

constexpr int kRow = 144;  // LDS bytes per operand row: one 128-byte chunk + 16 pad

template <int BM, int BN>
constexpr int gemm_lds_bytes() {
  return 2 * (BM + BN) * kRow;
}

// Best of B for one instance, by one workgroup of NT threads: the objectives
// F_b, first argmin over b, strict-improvement update of the incumbent, copy
// of the winning rounded vector.
// mode 0: no evaluation this iteration (only the iteration counter advances);
// mode 1: evaluation and incumbent update; mode 2: objectives only.
// Without incremental evaluation (nflip absent), F_b = (kappa * S_b) / 2 + C_b
// from the evaluation's integer partials, which are reset to zero for the next
// evaluation, and the winner is copied from x_r.  With it, the incremental
// kernel has already finalised F_b in Fall, reset the partials and kept the
// rows that beat the incumbent in cand: only Fall is read and the winner is
// copied from cand, so this can run while the next step rewrites x_r.
//
// The kernel is a short chain of dependent steps, so its length is set by how
// many memory round trips it waits for: every load it needs (including the
// incumbent and the trace length) goes out in one batch, the reduction runs in
// registers and through LDS, and the stores are issued last, after the
// barriers, so that no barrier waits for them.
__device__ __forceinline__ void argmin_pair(int64_t& F, int& b, int64_t F2, int b2) {
  if (F2 < F || (F2 == F && b2 < b)) {
    F = F2;
    b = b2;
  }
}

template <int NT>
__device__ void best_of_B(const InstDev& I, int mode, int tid, int64_t* sF, int* sb,
                          int* improved) {
  static_assert(NT % 64 == 0 && NT / 64 <= 64, "whole waves, one per lane of the last step");
  constexpr int NW = NT / 64, U = 4;
  const int64_t t = *gptr(I.t_dev) + 1;
  if (mode == 0) {
    if (tid == 0) *I.t_dev = t;
    return;
  }
  const int lane = tid & 63, wid = tid >> 6;
  int64_t incF = 0;
  int tlen = 0;
  if (tid == 0 && mode == 1) {
    incF = *gptr(&I.inc->F);
    tlen = *gptr(I.trace_len);
  }
  const bool fin = I.nflip != nullptr;  // objectives finalised by the incremental kernel
  int64_t bestF = LLONG_MAX;
  int bestb = INT_MAX;
  // Each thread visits its restarts in increasing order, so the strict
  // comparison keeps the first minimum.
  int64_t F1[U];  // the objectives of the first batch, stored after the barriers
  for (int b0 = 0; b0 < I.B; b0 += U * NT) {
    int64_t S[U], C[U], Fp[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = b0 + u * NT + tid;
      const bool ok = b < I.B;
      S[u] = (ok && !fin) ? *gptr(I.Sacc + b) : 0;
      C[u] = (ok && !fin) ? *gptr(I.Cacc + b) : 0;
      Fp[u] = (ok && fin) ? *gptr(I.Fall + b) : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = b0 + u * NT + tid;
      const int64_t F = fin ? Fp[u] : (I.kappa == 2 ? S[u] : S[u] / 2) + C[u];
      if (b < I.B && F < bestF) {
        bestF = F;
        bestb = b;
      }
      if (b0 == 0) {
        F1[u] = F;
      } else if (b < I.B && !fin) {  // more than U * NT restarts: store as we go
        I.Sacc[b] = 0;
        I.Cacc[b] = 0;
        I.Fall[b] = F;
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
    argmin_pair(bestF, bestb, __shfl_xor(bestF, o), __shfl_xor(bestb, o));
  if (lane == 0) {
    sF[wid] = bestF;
    sb[wid] = bestb;
  }
  __syncthreads();
  if (wid == 0) {
    bestF = lane < NW ? sF[lane] : LLONG_MAX;
    bestb = lane < NW ? sb[lane] : INT_MAX;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
      argmin_pair(bestF, bestb, __shfl_xor(bestF, o), __shfl_xor(bestb, o));
    if (lane == 0) {
      int imp = 0;
      if (mode == 1 && bestF < incF) {
        const uint64_t ts = wall_clock();
        I.inc->F = bestF;
        I.inc->t = t;
        I.inc->b = bestb;
        I.inc->ts = ts;
        if (tlen < I.trace_cap) {
          I.trace[tlen] = TraceRec{t, bestF, (int64_t)bestb, ts};
          *I.trace_len = tlen + 1;
        }
        imp = 1;
      }
      *improved = imp;
      sb[0] = bestb;
      if (mode != 2) *I.t_dev = t;
    }
  }
  __syncthreads();
  if (!fin) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = u * NT + tid;
      if (b >= I.B) continue;
      I.Sacc[b] = 0;  // ready for the next evaluation
      I.Cacc[b] = 0;
      I.Fall[b] = F1[u];
    }
  }
  if (*improved) {
    // whole 16-byte words of the winning row (best_x holds ld bytes)
    const u32x4* src = (const u32x4*)((fin ? I.cand : (const uint8_t*)I.Xr) + (size_t)sb[0] * I.ld);
    u32x4* dst = (u32x4*)I.best_x;
    const int nv = I.ld / 16;
    for (int v0 = 0; v0 < nv; v0 += U * NT) {
      u32x4 r[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int v = v0 + u * NT + tid;
        if (v < nv) r[u] = src[v];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int v = v0 + u * NT + tid;
        if (v < nv) dst[v] = r[u];
      }
    }
  }
}

// Rounding changes of coordinates i..i+3 of restart b (bytes of the old and
// new rounded words; coordinates at or past n are padding): counted in
// nflip[b] and marked in the restart's bitmap.  Neither atomic returns a
// value, so nothing waits on them (a returned value would make the step wait
// for every older memory operation, the epilogue's prefetches included).
__device__ __forceinline__ void record_flips(const InstDev& I, int b, int i, int n, uint32_t oldw,
                                             uint32_t neww) {
  uint32_t chg = (oldw ^ neww) & 0x01010101u;
  const int valid = n - i;
  if (valid < 4) chg &= (1u << (8 * valid)) - 1u;
  if (!chg) return;
  atomicAdd(I.nflip + b, __builtin_popcount(chg));
  const uint32_t bits = (chg | (chg >> 7) | (chg >> 14) | (chg >> 21)) & 0xfu;
  atomicOr(I.fbits + (size_t)b * (I.ld / 32) + (i >> 5), bits << (i & 31));
}

// An evaluation tile is needed only if some restart of its column block asks
// for a full product (more than kFlipMax changes, or a fresh state).
template <int BN, int NT>
__device__ __forceinline__ bool eval_block_needed(const InstDev& I, int n0, int tid) {
  bool need = false;
  for (int q = tid; q < BN; q += NT) {
    const int b = n0 + q;
    if (b < I.B && I.nflip[b] > kFlipMax) need = true;
  }
  return __syncthreads_or(need);
}

// Workgroups of a step launch past its tiles run the best of B of the
// previous iteration, one instance each (incremental evaluation only: it reads
// the finalised objectives and the kept rows, nothing the step writes).
template <int NT>
__device__ __forceinline__ void best_of_B_extra(const InstDev& I) {
  __shared__ int64_t sF[NT / 64];
  __shared__ int sb[NT / 64];
  __shared__ int improved;
  best_of_B<NT>(I, 1, threadIdx.x, sF, sb, &improved);
}

// Epilogue of one tile, shared by both main loops.  STEP/GRAD: lane holds
// rows ibase+16*fm+r (r = 0..3) of restart column bbase+16*fn.  GK is the kind
// of g (0 quadratic, 1 entropy) as a constant: with the kind read at run time
// the compiler evaluates both forms of g and g' for every element, and the
// entropy's logarithms alone cost more than the rest of the update.
template <int BM, int BN, int WM, int WN, int P, int EPI, int GK = 0>
__device__ __forceinline__ void gemm_epilogue(
    typename PT<P>::Acc (&acc)[BM / WM / 16][BN / WN / 16], const TileDev& td, const InstDev& I,
    int parity, int lane, int wm, int wn) {
  constexpr int WTM = BM / WM, WTN = BN / WN;
  constexpr int FM = WTM / 16, FN = WTN / 16;
  const int n = I.n, ld = I.ld, B = I.B;
  const int ibase = td.m0 + wm * WTM + 4 * (lane >> 4);
  const int bbase = td.n0 + wn * WTN + (lane & 15);
  if constexpr (EPI == EPI_STEP || EPI == EPI_GRAD) {
    const float kos = I.kos;
    GdaP gp = I.gp;
    gp.gkind = GK;
    float* Xc = I.X[parity];
    float* Xn = I.X[parity ^ 1];
    float* Yp = I.Y;
    uint8_t* Xsn = I.Xs[parity ^ 1];
    // Row group fm (16 rows of the wave tile) needs c'/s, the row scales and,
    // for STEP, x and y at every (row, restart) of the group.  The loads of
    // group fm+1 are issued before the stores of group fm: Y is updated in
    // place, so the compiler may not move a load above an earlier store, and
    // in plain program order every fragment would wait a full memory round
    // trip.  Loads use clamped (always valid) offsets; only stores are guarded.
    struct Rows {
      f32x4 cs, sc;
      i32x4 off8;
      f32x4 x[FN], y[FN];
      uint32_t xro[FN];  // rounded word before this step
    };
    auto fetch = [&](int fm, Rows& r) {
      const int ic = min(ibase + fm * 16, ld - 4);
      r.cs = *gptr((const f32x4*)(I.cps + ic));
      r.sc = f32x4{kos, kos, kos, kos};
      if constexpr (P == P_FP8) r.sc = r.sc * *gptr((const f32x4*)(I.rscale + ic));
      r.off8 = i32x4{0, 0, 0, 0};
      if constexpr (P == P_I8) {
        // A x ~ (A q + 127 A 1) / 254 for the quantised iterate q
        r.sc = r.sc * (1.f / 254.f);
        r.off8 = *gptr((const i32x4*)(I.rsum + ic)) * 127;
      }
      if constexpr (EPI == EPI_STEP) {
#pragma unroll
        for (int fn = 0; fn < FN; ++fn) {
          const size_t off = (size_t)min(bbase + fn * 16, B - 1) * ld + ic;
          r.x[fn] = *gptr((const f32x4*)(Xc + off));
          r.y[fn] = *gptr((const f32x4*)(Yp + off));
          r.xro[fn] = *gptr((const uint32_t*)(I.Xr + off));
        }
      }
    };
    Rows rb[2];
    fetch(0, rb[0]);
#pragma unroll
    for (int fm = 0; fm < FM; ++fm) {
      if (fm + 1 < FM) fetch(fm + 1, rb[(fm + 1) & 1]);
      const Rows& r = rb[fm & 1];
      const int i = ibase + fm * 16;
      if (i >= n) continue;
#pragma unroll
      for (int fn = 0; fn < FN; ++fn) {
        const int b = bbase + fn * 16;
        if (b >= B) continue;
        const size_t off = (size_t)b * ld + i;
        f32x4 G;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if constexpr (P == P_I8)
            G[q] = fmaf((float)(acc[fm][fn][q] + r.off8[q]), r.sc[q], r.cs[q]);
          else
            G[q] = fmaf(acc[fm][fn][q], r.sc[q], r.cs[q]);
        }
        if constexpr (EPI == EPI_GRAD) {
          *gptr((f32x4*)(I.G + off)) = G;
        } else {
          const f32x4 xv = r.x[fn];
          const f32x4 yv = r.y[fn];
          f32x4 xo, yo;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            float a, c;
            gda_update(xv[q], yv[q], G[q], gp, a, c);
            xo[q] = a;
            yo[q] = c;
          }
          *gptr((f32x4*)(Xn + off)) = xo;
          *gptr((f32x4*)(Yp + off)) = yo;
          const uint32_t xr = (uint32_t)(xo[0] > 0.5f) | ((uint32_t)(xo[1] > 0.5f) << 8) |
                              ((uint32_t)(xo[2] > 0.5f) << 16) |
                              ((uint32_t)(xo[3] > 0.5f) << 24);
          *gptr((uint32_t*)(I.Xr + off)) = xr;
          if (I.nflip) record_flips(I, b, i, n, r.xro[fn], xr);
          if constexpr (P == P_BF16) {
            u32x2 v;
            v.x = (uint32_t)f32_to_bf16_rne(xo[0]) | ((uint32_t)f32_to_bf16_rne(xo[1]) << 16);
            v.y = (uint32_t)f32_to_bf16_rne(xo[2]) | ((uint32_t)f32_to_bf16_rne(xo[3]) << 16);
            *gptr((u32x2*)(Xsn + off * 2)) = v;
          } else if constexpr (P == P_FP8) {
            *gptr((uint32_t*)(Xsn + off)) = pack_fp8x4(xo[0], xo[1], xo[2], xo[3]);
          } else if constexpr (P == P_I8) {
            *gptr((uint32_t*)(Xsn + off)) = pack_q8x4(xo[0], xo[1], xo[2], xo[3]);
          }
        }
      }
    }
  } else {
    // parity is the limb: this pass adds 256^limb (Ahat_limb x_r)_i, and the
    // linear term only in pass 0
    const int64_t lmul = int64_t(1) << (8 * parity);
    int64_t sS[FN], sC[FN];
#pragma unroll
    for (int fn = 0; fn < FN; ++fn) sS[fn] = sC[fn] = 0;
    // x_r and c' of row group fm+1 are fetched before group fm is reduced
    // (clamped offsets; c' is zero-padded to ld), so the loads never wait
    // behind the data-dependent selection of the previous group.
    struct ERows {
      int64_t cp[4];
      uint32_t xr[FN];
    };
    auto fetch = [&](int fm, ERows& r) {
      const int ic = min(ibase + fm * 16, ld - 4);
#pragma unroll
      for (int q = 0; q < 4; ++q) r.cp[q] = *gptr(I.cp + ic + q);
#pragma unroll
      for (int fn = 0; fn < FN; ++fn)
        r.xr[fn] = *gptr((const uint32_t*)(I.Xr + (size_t)min(bbase + fn * 16, B - 1) * ld + ic));
    };
    ERows rb[2];
    fetch(0, rb[0]);
#pragma unroll
    for (int fm = 0; fm < FM; ++fm) {
      if (fm + 1 < FM) fetch(fm + 1, rb[(fm + 1) & 1]);
      const ERows& r = rb[fm & 1];
      const int i = ibase + fm * 16;
      if (i >= n) continue;
#pragma unroll
      for (int fn = 0; fn < FN; ++fn) {
        const int b = bbase + fn * 16;
        if (b >= B) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (((r.xr[fn] >> (8 * q)) & 1u) && (i + q < n)) {
            sS[fn] += (int64_t)acc[fm][fn][q] * lmul;
            sC[fn] += r.cp[q];
          }
        }
      }
    }
#pragma unroll
    for (int fn = 0; fn < FN; ++fn) {
      sS[fn] += __shfl_xor(sS[fn], 16);
      sS[fn] += __shfl_xor(sS[fn], 32);
      sC[fn] += __shfl_xor(sC[fn], 16);
      sC[fn] += __shfl_xor(sC[fn], 32);
      const int b = bbase + fn * 16;
      if (lane < 16 && b < B) {
        if (sS[fn]) atomicAdd((unsigned long long*)(I.Sacc + b), (unsigned long long)sS[fn]);
        if (sC[fn] && parity == 0)
          atomicAdd((unsigned long long*)(I.Cacc + b), (unsigned long long)sC[fn]);
      }
    }
  }
}

// STEP/GRAD epilogue through LDS, for the DMA kernel.  The fragment layout
// gives a store instruction 16 restarts x 64 contiguous bytes; moving G
// through LDS lets the whole workgroup walk each restart's BM contiguous
// floats instead, which takes the x/y traffic from about 3.7 to 6.8 TB/s.
// The tile is done in passes of PR restarts, whose G block fits in one stage
// buffer (the stages must stay distinct LDS objects: over one array the
// compiler cannot tell the DMA into one stage from the reads of another and
// makes every DMA wait for all outstanding LDS reads).  Passes alternate
// between two stage buffers, so one barrier per pass suffices.
//   phase 1 of pass p: the waves owning restarts [PR p, PR p + PR) write G
//            for those fragments, row = restart within the pass, 16-byte
//            column group c (BM/4 per row) stored at (c & ~7) | ((c ^ row) & 7)
//            so that the 16 restarts of one fragment store and the
//            consecutive columns of one row read both hit distinct banks;
//   phase 2 of pass p: element e = (row, c) goes to thread e mod NT.  x and y
//            are fetched one group of PF elements ahead, across passes (y is
//            updated in place, so the compiler keeps loads behind earlier
//            stores and would otherwise wait a memory round trip per group).
template <int BM, int BN, int STAGE>
constexpr int rows_per_pass() {
  return (64 * BM * 4 <= STAGE && BN % 64 == 0) ? 64 : (32 * BM * 4 <= STAGE && BN % 32 == 0) ? 32 : 16;
}

template <int BM, int BN, int WM, int WN, int P, int EPI, int STAGE, int GK = 0>
__device__ __forceinline__ void gemm_epilogue_rows(
    typename PT<P>::Acc (&acc)[BM / WM / 16][BN / WN / 16], const TileDev& td, const InstDev& I,
    int parity, int tid, int lane, int wm, int wn, uint8_t* buf0, uint8_t* buf1) {
  static_assert(EPI == EPI_STEP || EPI == EPI_GRAD, "row epilogue is for STEP and GRAD");
  constexpr int NT = 64 * WM * WN;
  constexpr int WTM = BM / WM, WTN = BN / WN;
  constexpr int FM = WTM / 16, FN = WTN / 16;
  constexpr int C4 = BM / 4;                       // 16-byte column groups per tile row
  constexpr int PR = rows_per_pass<BM, BN, STAGE>();
  constexpr int NP = BN / PR;                      // passes
  constexpr int EPP = PR * C4 / NT;                // elements per thread and pass
  // elements per prefetch group: as many as divide the thread's share of a pass
  // (up to 5), so that enough x/y loads are in flight to cover the latency
  constexpr int PF = EPP % 5 == 0 ? 5 : EPP % 4 == 0 ? 4 : EPP % 2 == 0 ? 2 : 1;
  constexpr int GPP = EPP / PF;                    // groups per pass
  static_assert(PR * BM * 4 <= STAGE && BN % PR == 0 && PR % 16 == 0, "pass shape");
  static_assert(C4 % 8 == 0 && (PR * C4) % NT == 0 && EPP % PF == 0, "row epilogue shape");
  const int n = I.n, ld = I.ld, B = I.B;
  // Opaque copies of the thread and lane ids: the index arithmetic below
  // depends on nothing else, and hoisted above the main loop (whose registers
  // are all in use) it would spill.
  asm volatile("" : "+v"(tid), "+v"(lane));
  auto slot = [](int row, int c) { return row * C4 + ((c & ~7) | ((c ^ row) & 7)); };

  // scale and offset of every row group of the wave tile
  const float kos = I.kos;
  const int ibase = td.m0 + wm * WTM + 4 * (lane >> 4);
  f32x4 cs[FM], sc[FM];
  i32x4 off8[FM];
#pragma unroll
  for (int fm = 0; fm < FM; ++fm) {
    const int ic = min(ibase + fm * 16, ld - 4);
    cs[fm] = *gptr((const f32x4*)(I.cps + ic));
    sc[fm] = f32x4{kos, kos, kos, kos};
    if constexpr (P == P_FP8) sc[fm] = sc[fm] * *gptr((const f32x4*)(I.rscale + ic));
    off8[fm] = i32x4{0, 0, 0, 0};
    if constexpr (P == P_I8) {
      // A x ~ (A q + 127 A 1) / 254 for the quantised iterate q
      sc[fm] = sc[fm] * (1.f / 254.f);
      off8[fm] = *gptr((const i32x4*)(I.rsum + ic)) * 127;
    }
  }
  auto write_pass = [&](int p, uint8_t* buf) {
    f32x4* G4 = (f32x4*)buf;
#pragma unroll
    for (int fn = 0; fn < FN; ++fn) {
      const int r0 = wn * WTN + 16 * fn;            // first restart of the fragment
      if (r0 / PR != p) continue;                   // uniform over the wave
      const int row = r0 - p * PR + (lane & 15);
#pragma unroll
      for (int fm = 0; fm < FM; ++fm) {
        const int c = (wm * WTM) / 4 + 4 * fm + (lane >> 4);
        f32x4 G;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if constexpr (P == P_I8)
            G[q] = fmaf((float)(acc[fm][fn][q] + off8[fm][q]), sc[fm][q], cs[fm][q]);
          else
            G[q] = fmaf(acc[fm][fn][q], sc[fm][q], cs[fm][q]);
        }
        G4[slot(row, c)] = G;
      }
    }
  };

  GdaP gp = I.gp;
  gp.gkind = GK;  // a constant: only this kind's g and g' are computed
  float* Xc = I.X[parity];
  float* Xn = I.X[parity ^ 1];
  float* Yp = I.Y;
  uint8_t* Xsn = I.Xs[parity ^ 1];
  struct Vals {
    f32x4 x[PF], y[PF];
    uint32_t xro[PF];  // rounded word before this step
  };
  // element u of group g: pass g / GPP, index e = (g mod GPP) * PF + u within the
  // thread's share of that pass
  auto coords = [&](int g, int u, int& row, int& c) {
    const int e = ((g % GPP) * PF + u) * NT + tid;
    row = e / C4;
    c = e % C4;
  };
  auto fetch = [&](int g, Vals& v) {
    if constexpr (EPI == EPI_STEP) {
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        int row, c;
        coords(g, u, row, c);
        const int b = min(td.n0 + (g / GPP) * PR + row, B - 1);
        const size_t off = (size_t)b * ld + min(td.m0 + 4 * c, ld - 4);
        v.x[u] = *gptr((const f32x4*)(Xc + off));
        v.y[u] = *gptr((const f32x4*)(Yp + off));
        v.xro[u] = *gptr((const uint32_t*)(I.Xr + off));
      }
    }
  };
  Vals vb[2];
  fetch(0, vb[0]);
#pragma unroll
  for (int g = 0; g < NP * GPP; ++g) {
    const int p = g / GPP;
    uint8_t* buf = (p & 1) ? buf1 : buf0;
    if (g % GPP == 0) {
      write_pass(p, buf);
      __syncthreads();
    }
    if (g + 1 < NP * GPP) fetch(g + 1, vb[(g + 1) & 1]);
    const Vals& v = vb[g & 1];
    const f32x4* G4 = (const f32x4*)buf;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      int row, c;
      coords(g, u, row, c);
      const int b = td.n0 + p * PR + row, i = td.m0 + 4 * c;
      if (b >= B || i >= n) continue;
      const size_t off = (size_t)b * ld + i;
      const f32x4 G = G4[slot(row, c)];
      if constexpr (EPI == EPI_GRAD) {
        *gptr((f32x4*)(I.G + off)) = G;
      } else {
        f32x4 xo, yo;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float a, cc;
          gda_update(v.x[u][q], v.y[u][q], G[q], gp, a, cc);
          xo[q] = a;
          yo[q] = cc;
        }
        *gptr((f32x4*)(Xn + off)) = xo;
        *gptr((f32x4*)(Yp + off)) = yo;
        const uint32_t xr = (uint32_t)(xo[0] > 0.5f) | ((uint32_t)(xo[1] > 0.5f) << 8) |
                            ((uint32_t)(xo[2] > 0.5f) << 16) | ((uint32_t)(xo[3] > 0.5f) << 24);
        *gptr((uint32_t*)(I.Xr + off)) = xr;
        if (I.nflip) record_flips(I, b, i, n, v.xro[u], xr);
        if constexpr (P == P_BF16) {
          u32x2 w;
          w.x = (uint32_t)f32_to_bf16_rne(xo[0]) | ((uint32_t)f32_to_bf16_rne(xo[1]) << 16);
          w.y = (uint32_t)f32_to_bf16_rne(xo[2]) | ((uint32_t)f32_to_bf16_rne(xo[3]) << 16);
          *gptr((u32x2*)(Xsn + off * 2)) = w;
        } else if constexpr (P == P_FP8) {
          *gptr((uint32_t*)(Xsn + off)) = pack_fp8x4(xo[0], xo[1], xo[2], xo[3]);
        } else if constexpr (P == P_I8) {
          *gptr((uint32_t*)(Xsn + off)) = pack_q8x4(xo[0], xo[1], xo[2], xo[3]);
        }
      }
    }
  }
}

template <int BM, int BN, int WM, int WN, int P, int EPI, int GK>
__global__ void __launch_bounds__(64 * WM * WN)
    dense_gemm(const TileDev* __restrict__ tiles, int ntiles, const InstDev* __restrict__ insts,
               int parity, int am0) {
  if (blockIdx.x >= ntiles) {
    if constexpr (EPI == EPI_STEP) best_of_B_extra<64 * WM * WN>(insts[am0 + blockIdx.x - ntiles]);
    return;
  }
  constexpr int NT = 64 * WM * WN;
  constexpr int WTM = BM / WM, WTN = BN / WN;
  constexpr int FM = WTM / 16, FN = WTN / 16;
  constexpr int STAGE = (BM + BN) * kRow;
  constexpr int APC = BM * 8 / NT, BPC = BN * 8 / NT;
  constexpr int EB = PT<P>::EB;
  static_assert((BM * 8) % NT == 0 && (BN * 8) % NT == 0, "tile / thread mismatch");
  static_assert(WTM % 16 == 0 && WTN % 16 == 0, "wave tile must be whole fragments");
  using Acc = typename PT<P>::Acc;

  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int wm = wid % WM, wn = wid / WM;

  for (int w = blockIdx.x; w < ntiles; w += gridDim.x) {
    const TileDev td = tiles[w];
    const InstDev& I = insts[td.inst];
    if constexpr (EPI == EPI_EVAL) {
      if (parity >= I.nlimb) continue;
      if (I.nflip && !eval_block_needed<BN, 64 * WM * WN>(I, td.n0, threadIdx.x)) continue;
    }
    const int n = I.n, ld = I.ld, B = I.B;
    const size_t rbytes = (size_t)ld * EB;
    const int nk = (int)(rbytes / 128);
    const uint8_t* Ag = (EPI == EPI_EVAL) ? (const uint8_t*)I.A8 + parity * I.limb_stride : I.A;
    const uint8_t* Bg = (EPI == EPI_EVAL) ? (const uint8_t*)I.Xr : I.Xs[parity];

    const uint8_t* pa[APC];
    const uint8_t* pb[BPC];
    int la[APC], lb[BPC];
#pragma unroll
    for (int j = 0; j < APC; ++j) {
      const int p = tid + j * NT, r = p >> 3, c = p & 7;
      const int row = min(td.m0 + r, n - 1);
      pa[j] = Ag + (size_t)row * rbytes + c * 16;
      la[j] = r * kRow + c * 16;
    }
#pragma unroll
    for (int j = 0; j < BPC; ++j) {
      const int p = tid + j * NT, r = p >> 3, c = p & 7;
      const int row = min(td.n0 + r, B - 1);
      pb[j] = Bg + (size_t)row * rbytes + c * 16;
      lb[j] = (BM + r) * kRow + c * 16;
    }

    Acc acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = Acc{0, 0, 0, 0};

    u32x4 ra[APC], rb[BPC];
#pragma unroll
    for (int j = 0; j < APC; ++j) ra[j] = *gptr((const u32x4*)(pa[j]));
#pragma unroll
    for (int j = 0; j < BPC; ++j) rb[j] = *gptr((const u32x4*)(pb[j]));
#pragma unroll
    for (int j = 0; j < APC; ++j) *(u32x4*)(smem + la[j]) = ra[j];
#pragma unroll
    for (int j = 0; j < BPC; ++j) *(u32x4*)(smem + lb[j]) = rb[j];
    __syncthreads();

    const int frow = (lane & 15) * kRow + (lane >> 4) * 32;
    for (int kc = 0; kc < nk; ++kc) {
      const int cur = kc & 1;
      const bool more = kc + 1 < nk;
      if (more) {
        const size_t off = (size_t)(kc + 1) * 128;
#pragma unroll
        for (int j = 0; j < APC; ++j) ra[j] = *gptr((const u32x4*)(pa[j] + off));
#pragma unroll
        for (int j = 0; j < BPC; ++j) rb[j] = *gptr((const u32x4*)(pb[j] + off));
      }
      const uint8_t* sA = smem + cur * STAGE + (wm * WTM) * kRow + frow;
      const uint8_t* sB = smem + cur * STAGE + (BM + wn * WTN) * kRow + frow;
      u32x4 fa[FM][2], fb[FN][2];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        fa[i][0] = *(const u32x4*)(sA + i * 16 * kRow);
        fa[i][1] = *(const u32x4*)(sA + i * 16 * kRow + 16);
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        fb[j][0] = *(const u32x4*)(sB + j * 16 * kRow);
        fb[j][1] = *(const u32x4*)(sB + j * 16 * kRow + 16);
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) mfma_chunk<P>(acc[i][j], fa[i], fb[j]);
      if (more) {
        uint8_t* nxt = smem + (cur ^ 1) * STAGE;
#pragma unroll
        for (int j = 0; j < APC; ++j) *(u32x4*)(nxt + la[j]) = ra[j];
#pragma unroll
        for (int j = 0; j < BPC; ++j) *(u32x4*)(nxt + lb[j]) = rb[j];
      }
      __syncthreads();
    }

    gemm_epilogue<BM, BN, WM, WN, P, EPI, GK>(acc, td, I, parity, lane, wm, wn);
  }
}

// ------------------------------------------------- three-stage LDS pipeline
//
// Same tile, same MFMA sequence and same epilogue as dense_gemm, but the
// operands go from global memory straight into LDS (global_load_lds_dwordx4:
// lane L of a wave writes 16 bytes at LDS base + 16 L), so no registers are
// spent on staging and two K chunks are in flight while a third is consumed.
// Rows are stored unpadded (128 bytes) with the 16-byte chunks XOR-swizzled by
// (row / 2) mod 8: one DMA instruction fills 8 whole rows, and a fragment read
// (16 rows, chunks q or q + 4 for the four quarter-waves q) is free of bank
// conflicts.  The three stages are
// distinct LDS objects and the K loop is unrolled by three, so every stage is
// addressed statically.

// Waits until at most N vector-memory operations (here: this wave's LDS DMAs)
// are outstanding AND every LDS read of this wave has returned, so that after
// the following s_barrier no wave can refill a stage another wave still reads.
template <int N>
__device__ __forceinline__ void wait_vmcnt_lds() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  // gfx9 encoding: vmcnt[3:0] and [15:14], expcnt[6:4], lgkmcnt[11:8] (= 0 here)
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (0 << 8) | ((N >> 4) << 14));
}

typedef __attribute__((address_space(3))) void* lds_ptr;

template <int BM, int BN, int WM, int WN, int P, int EPI, int GK>
__global__ void __launch_bounds__(64 * WM * WN)
    dense_gemm_dma(const TileDev* __restrict__ tiles, int ntiles, const InstDev* __restrict__ insts,
                   int parity, int am0) {
  if (blockIdx.x >= ntiles) {
    if constexpr (EPI == EPI_STEP) best_of_B_extra<64 * WM * WN>(insts[am0 + blockIdx.x - ntiles]);
    return;
  }
  constexpr int NW = WM * WN;
  constexpr int WTM = BM / WM, WTN = BN / WN;
  constexpr int FM = WTM / 16, FN = WTN / 16;
  constexpr int ROWS = BM + BN;
  constexpr int STAGE = ROWS * 128;
  constexpr int NI = ROWS / (8 * NW);
  constexpr int EB = PT<P>::EB;
  static_assert(ROWS % (8 * NW) == 0, "stage rows must split into 8-row DMA groups per wave");
  static_assert(BM % 16 == 0 && WTM % 16 == 0 && WTN % 16 == 0, "fragment alignment");
  using Acc = typename PT<P>::Acc;

  __shared__ __attribute__((aligned(1024))) uint8_t st0[STAGE];
  __shared__ __attribute__((aligned(1024))) uint8_t st1[STAGE];
  __shared__ __attribute__((aligned(1024))) uint8_t st2[STAGE];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int wm = wid % WM, wn = wid / WM;
  // fragment read offsets: row (lane % 16) of a 16-row group, logical chunk q
  // for the first half of the K step and q + 4 for the second (q = lane / 16),
  // stored at physical chunk c ^ ((row / 2) mod 8).  Both operands pair the
  // same k with the same lane slot, which is all the MFMA needs; with chunks
  // q (not 2q) in one read the 64 lanes hit the LDS banks without conflicts
  // (measured: 4 cycles per ds_read_b128 instead of 8 for chunks 2q, 2q + 1)
  const int sw = (lane & 15) >> 1, q = lane >> 4;
  const int fo0 = (lane & 15) * 128 + ((q ^ sw) << 4);
  const int fo1 = (lane & 15) * 128 + (((q + 4) ^ sw) << 4);

  for (int w = blockIdx.x; w < ntiles; w += gridDim.x) {
    const TileDev td = tiles[w];
    const InstDev& I = insts[td.inst];
    if constexpr (EPI == EPI_EVAL) {
      if (parity >= I.nlimb) continue;
      if (I.nflip && !eval_block_needed<BN, 64 * WM * WN>(I, td.n0, threadIdx.x)) continue;
    }
    const int n = I.n, B = I.B;
    const size_t rbytes = (size_t)I.ld * EB;
    const int nk = (int)(rbytes / 128);
    const uint8_t* Ag = (EPI == EPI_EVAL) ? (const uint8_t*)I.A8 + parity * I.limb_stride : I.A;
    const uint8_t* Bg = (EPI == EPI_EVAL) ? (const uint8_t*)I.Xr : I.Xs[parity];

    // DMA instruction j of this wave fills stage rows r0 .. r0+7, r0 = 8 (j NW + wid);
    // lane L writes physical chunk L % 8 of row r = r0 + L / 8, so it loads
    // logical chunk (L % 8) ^ ((r / 2) mod 8).
    const uint8_t* src[NI];
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int r = (j * NW + wid) * 8 + (lane >> 3);
      const int c = (lane & 7) ^ ((r >> 1) & 7);
      const uint8_t* row = r < BM ? Ag + (size_t)min(td.m0 + r, n - 1) * rbytes
                                  : Bg + (size_t)min(td.n0 + (r - BM), B - 1) * rbytes;
      src[j] = row + c * 16;
    }
    auto issue = [&](uint8_t* st, int kc) {
      const size_t off = (size_t)kc * 128;
#pragma unroll
      for (int j = 0; j < NI; ++j)
        __builtin_amdgcn_global_load_lds(gptr((const void*)(src[j] + off)),
                                         (lds_ptr)(st + (j * NW + wid) * 1024), 16, 0, 0);
    };

    Acc acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = Acc{0, 0, 0, 0};

    auto compute = [&](const uint8_t* st) {
      const uint8_t* sA = st + (wm * WTM) * 128;
      const uint8_t* sB = st + (BM + wn * WTN) * 128;
      u32x4 fa[FM][2], fb[FN][2];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        fa[i][0] = *(const u32x4*)(sA + i * 16 * 128 + fo0);
        fa[i][1] = *(const u32x4*)(sA + i * 16 * 128 + fo1);
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        fb[j][0] = *(const u32x4*)(sB + j * 16 * 128 + fo0);
        fb[j][1] = *(const u32x4*)(sB + j * 16 * 128 + fo1);
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) mfma_chunk<P>(acc[i][j], fa[i], fb[j]);
    };

    // one K step: wait for chunk k, publish it, refill the stage freed by
    // chunk k-1 with chunk k+2, then consume chunk k
    // A bare s_barrier, not __syncthreads(): the latter's workgroup fence would
    // wait for every outstanding DMA, including the two chunks being prefetched.
    // This wave's DMAs for chunk k are complete after the explicit vmcnt wait,
    // and its LDS reads of the stage being refilled were consumed by MFMAs
    // issued before the barrier.
    // Every step issues exactly one chunk of DMAs (past the end it reloads the
    // last chunk into a stage nobody reads again), so the number of DMAs in
    // flight is always the same and the steady-state loop has no branches that
    // would make the compiler give up tracking which stage each DMA writes.
    auto kstep = [&](const uint8_t* cur, uint8_t* nxt, int k) {
      wait_vmcnt_lds<NI>();
      __builtin_amdgcn_s_barrier();
      issue(nxt, min(k + 2, nk - 1));
      compute(cur);
    };

    wait_vmcnt_lds<63>();
    __builtin_amdgcn_s_barrier();  // the previous tile's last reads of the stages are done
    if constexpr (!HasHalf<P>::value) {
      issue(st0, 0);
      issue(st1, min(1, nk - 1));
      int kc = 0;
      for (; kc + 3 <= nk; kc += 3) {
        kstep(st0, st2, kc);
        kstep(st1, st0, kc + 1);
        kstep(st2, st1, kc + 2);
      }
      if (kc < nk) kstep(st0, st2, kc);
      if (kc + 1 < nk) kstep(st1, st0, kc + 1);
    } else {
      // Software pipeline over half chunks.  Entering step k, the registers
      // f0 hold half 0 of chunk k.  First half: read half 1 of chunk k into
      // f1 while the MFMAs on f0 run.  Then wait for this wave's DMAs of chunk
      // k+1 and for its reads of f1, and pass the barrier: now every wave is
      // done with the stage of chunk k and chunk k+1 is in LDS.  Second half:
      // refill chunk k's stage with chunk k+3, and read half 0 of chunk k+1
      // into f0 while the MFMAs on f1 run.  The sched_group_barrier chains
      // spread the LDS reads and DMA issues between the MFMAs; left to itself
      // the scheduler clusters the reads, and the MFMA pipe idles behind them.
      constexpr int MPH = FM * FN * HalfMfmas<P>::value;  // MFMAs per half step
      constexpr int NDS = FM + FN;                        // fragment reads per half step
      constexpr int MF = MPH / NDS >= 3 ? 3 : (MPH / NDS >= 1 ? MPH / NDS : 1);
      u32x4 f0a[FM], f0b[FN], f1a[FM], f1b[FN];
      auto load = [&](u32x4 (&fa)[FM], u32x4 (&fb)[FN], const uint8_t* st, int fo) {
        const uint8_t* sA = st + (wm * WTM) * 128;
        const uint8_t* sB = st + (BM + wn * WTN) * 128;
#pragma unroll
        for (int i = 0; i < FM; ++i) fa[i] = *(const u32x4*)(sA + i * 16 * 128 + fo);
#pragma unroll
        for (int j = 0; j < FN; ++j) fb[j] = *(const u32x4*)(sB + j * 16 * 128 + fo);
      };
      auto mm = [&](const u32x4 (&fa)[FM], const u32x4 (&fb)[FN]) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) mfma_half<P>(acc[i][j], fa[i], fb[j]);
      };
      auto interleave = [&](bool with_dma) {
#pragma unroll
        for (int u = 0; u < NDS; ++u) {
          if (with_dma && u < NI) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // VMEM
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);                          // DS read
          if (MF * (u + 1) <= MPH) __builtin_amdgcn_sched_group_barrier(0x008, MF, 0);  // MFMA
        }
        if (with_dma && NI > NDS) __builtin_amdgcn_sched_group_barrier(0x020, NI - NDS, 0);
        if (MPH > MF * NDS) __builtin_amdgcn_sched_group_barrier(0x008, MPH - MF * NDS, 0);
      };
      auto pstep = [&](const uint8_t* cur, const uint8_t* nx, int k) {
        load(f1a, f1b, cur, fo1);
        mm(f0a, f0b);
        interleave(false);
        wait_vmcnt_lds<NI>();  // chunk k+1 landed; chunk k+2 may be in flight
        __builtin_amdgcn_s_barrier();
        issue((uint8_t*)cur, min(k + 3, nk - 1));
        load(f0a, f0b, nx, fo0);  // past the last chunk: reads a stage nobody uses
        mm(f1a, f1b);
        interleave(true);
      };
      issue(st0, 0);
      issue(st1, min(1, nk - 1));
      issue(st2, min(2, nk - 1));
      wait_vmcnt_lds<2 * NI>();
      __builtin_amdgcn_s_barrier();
      load(f0a, f0b, st0, fo0);
      int kc = 0;
      for (; kc + 3 <= nk; kc += 3) {
        pstep(st0, st1, kc);
        pstep(st1, st2, kc + 1);
        pstep(st2, st0, kc + 2);
      }
      if (kc < nk) pstep(st0, st1, kc);
      if (kc + 1 < nk) pstep(st1, st2, kc + 1);
    }
    if constexpr (EPI == EPI_EVAL) {
      gemm_epilogue<BM, BN, WM, WN, P, EPI>(acc, td, I, parity, lane, wm, wn);
    } else {
      // every DMA of this wave (including the reloads past the last chunk) has
      // landed and every wave is done reading the stages before G goes in
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      gemm_epilogue_rows<BM, BN, WM, WN, P, EPI, STAGE, GK>(acc, td, I, parity, tid, lane, wm, wn,
                                                            st0, st1);
    }
  }
  __builtin_amdgcn_s_waitcnt(0);  // no DMA into LDS may outlive the workgroup
}

// ---------------------------------------------------------------- tile table

// id, block tile BM x BN, waves WM x WN, main loop (0: register-staged double
// buffer, 1: three-stage direct-to-LDS pipeline)
#define PDBO_TILE_CFGS(X)      \
  X(0, 128, 128, 2, 2, 0)      \
  X(1, 64, 64, 2, 2, 0)        \
  X(2, 256, 128, 4, 2, 0)      \
  X(3, 128, 256, 2, 4, 0)      \
  X(4, 160, 256, 2, 2, 0)      \
  X(5, 192, 256, 2, 2, 0)      \
  X(6, 160, 256, 2, 2, 1)      \
  X(7, 128, 128, 2, 2, 1)      \
  X(8, 256, 128, 4, 2, 1)      \
  X(9, 64, 64, 2, 2, 1)

template <int BM, int BN, int WM, int WN, int P, int EPI, int DMA, int GK>
static hipError_t launch_one(const TileDev* tiles, int ntiles, const InstDev* insts, int parity,
                             int grid, hipStream_t s, int am0, int amn) {
  if (grid <= 0 || grid > ntiles) grid = ntiles;
  if (EPI == EPI_STEP && amn > 0 && ntiles > 0) grid = ntiles + amn;  // one tile per workgroup
  if constexpr (DMA) {
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL((dense_gemm_dma<BM, BN, WM, WN, P, EPI, GK>), dim3(grid), dim3(64 * WM * WN),
                       0, s, tiles, ntiles, insts, parity, am0);
  } else {
    constexpr int lds = gemm_lds_bytes<BM, BN>();
    auto kern = dense_gemm<BM, BN, WM, WN, P, EPI, GK>;
    static bool attr_done = false;
    if (!attr_done) {
      hipError_t e =
          hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
      if (e != hipSuccess) return e;
      attr_done = true;
    }
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * WM * WN), lds, s, tiles, ntiles, insts, parity,
                       am0);
  }
  return hipGetLastError();
}

// Step launches of one kind of g (0 quadratic, 1 entropy, 2 polynomial), each
// defined in its own part.
hipError_t launch_step_g0(int cfg, int prec, const TileDev* tiles, int ntiles, const InstDev* insts,
                          int parity, int grid, hipStream_t s, int am0, int amn);
hipError_t launch_step_g1(int cfg, int prec, const TileDev* tiles, int ntiles, const InstDev* insts,
                          int parity, int grid, hipStream_t s, int am0, int amn);
hipError_t launch_step_g2(int cfg, int prec, const TileDev* tiles, int ntiles, const InstDev* insts,
                          int parity, int grid, hipStream_t s, int am0, int amn);

#if PDBO_DENSE_PART >= 1
#if PDBO_DENSE_PART == 1
#define PDBO_STEP_FN launch_step_g0
#elif PDBO_DENSE_PART == 2
#define PDBO_STEP_FN launch_step_g1
#else
#define PDBO_STEP_FN launch_step_g2
#endif
// The kind of g of this part's step kernels is a compile-time constant: read at
// run time it made the compiler evaluate every form of g and g' for each
// element.
template <int BM, int BN, int WM, int WN, int DMA>
static hipError_t launch_step_cfg(int prec, const TileDev* tiles, int ntiles, const InstDev* insts,
                                  int parity, int grid, hipStream_t s, int am0, int amn) {
  constexpr int GK = PDBO_DENSE_PART - 1;
#define PDBO_L(P) \
  launch_one<BM, BN, WM, WN, P, EPI_STEP, DMA, GK>(tiles, ntiles, insts, parity, grid, s, am0, amn)
  switch (prec) {
    case P_F32: return PDBO_L(P_F32);
    case P_BF16: return PDBO_L(P_BF16);
    case P_FP8: return PDBO_L(P_FP8);
    case P_I8: return PDBO_L(P_I8);
    default: return hipErrorInvalidValue;
  }
#undef PDBO_L
}

hipError_t PDBO_STEP_FN(int cfg, int prec, const TileDev* tiles, int ntiles, const InstDev* insts,
                        int parity, int grid, hipStream_t s, int am0, int amn) {
  switch (cfg) {
#define X(id, bm, bn, wm, wn, dma) \
  case id:                         \
    return launch_step_cfg<bm, bn, wm, wn, dma>(prec, tiles, ntiles, insts, parity, grid, s, am0, amn);
    PDBO_TILE_CFGS(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}
#endif  // PDBO_DENSE_PART >= 1

#if PDBO_DENSE_PART == 0
static const TileCfgInfo kCfgs[] = {
#define X(id, bm, bn, wm, wn, dma) \
  {#bm "x" #bn "_w" #wm "x" #wn "_" #dma, bm, bn, wm, wn, 64 * wm * wn, dma},
    PDBO_TILE_CFGS(X)
#undef X
};

int dense_num_cfgs() { return (int)(sizeof(kCfgs) / sizeof(kCfgs[0])); }
const TileCfgInfo& dense_cfg(int id) { return kCfgs[id]; }

// Gradient and evaluation launches (the kernels that do not use g).
template <int BM, int BN, int WM, int WN, int DMA>
static hipError_t launch_cfg(int prec, int epi, const TileDev* tiles, int ntiles,
                             const InstDev* insts, int parity, int grid, hipStream_t s) {
#define PDBO_L(P, E) launch_one<BM, BN, WM, WN, P, E, DMA, 0>(tiles, ntiles, insts, parity, grid, s, 0, 0)
  if (epi == EPI_EVAL) return PDBO_L(P_I8, EPI_EVAL);
  if (epi != EPI_GRAD) return hipErrorInvalidValue;
  switch (prec) {
    case P_F32: return PDBO_L(P_F32, EPI_GRAD);
    case P_BF16: return PDBO_L(P_BF16, EPI_GRAD);
    case P_FP8: return PDBO_L(P_FP8, EPI_GRAD);
    case P_I8: return PDBO_L(P_I8, EPI_GRAD);
    default: return hipErrorInvalidValue;
  }
#undef PDBO_L
}

hipError_t launch_dense_gemm(int cfg, int prec, int epi, int gkind, const TileDev* tiles,
                             int ntiles, const InstDev* insts, int parity, int grid, hipStream_t s,
                             int am0, int amn) {
  if (epi == EPI_STEP) {
    switch (gkind) {
      case 0: return launch_step_g0(cfg, prec, tiles, ntiles, insts, parity, grid, s, am0, amn);
      case 1: return launch_step_g1(cfg, prec, tiles, ntiles, insts, parity, grid, s, am0, amn);
      case 2: return launch_step_g2(cfg, prec, tiles, ntiles, insts, parity, grid, s, am0, amn);
      default: return hipErrorInvalidValue;
    }
  }
  switch (cfg) {
#define X(id, bm, bn, wm, wn, dma) \
  case id:                         \
    return launch_cfg<bm, bn, wm, wn, dma>(prec, epi, tiles, ntiles, insts, parity, grid, s);
    PDBO_TILE_CFGS(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------- best of B

constexpr int kArgThreads = 1024;

__global__ void __launch_bounds__(kArgThreads)
    argmin_kernel(const InstDev* __restrict__ insts, int inst0, int mode) {
  __shared__ int64_t sF[kArgThreads / 64];
  __shared__ int sb[kArgThreads / 64];
  __shared__ int improved;
  best_of_B<kArgThreads>(insts[inst0 + blockIdx.x], mode, threadIdx.x, sF, sb, &improved);
}

hipError_t launch_argmin(const InstDev* insts, int inst0, int ninst, int mode, hipStream_t s) {
  hipLaunchKernelGGL(argmin_kernel, dim3(ninst), dim3(kArgThreads), 0, s, insts, inst0, mode);
  return hipGetLastError();
}

__global__ void stamp_kernel(uint64_t* ts0) {
  if (*ts0 == 0) *ts0 = wall_clock();
}

hipError_t launch_stamp(uint64_t* ts0, hipStream_t s) {
  hipLaunchKernelGGL(stamp_kernel, dim3(1), dim3(1), 0, s, ts0);
  return hipGetLastError();
}

// ---------------------------------------------------------------- state

__device__ __forceinline__ void store_shadow(uint8_t* Xs, size_t off, float v, int prec) {
  if (!Xs) return;
  if (prec == P_BF16) {
    ((uint16_t*)Xs)[off] = f32_to_bf16_rne(v);
  } else if (prec == P_FP8) {
    Xs[off] = (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.f, 0, false) & 0xff);
  } else if (prec == P_I8) {
    Xs[off] = (uint8_t)quant8(v);
  }
}

__global__ void init_state_kernel(const double* __restrict__ x0, int B, int n, int ld, float y0,
                                  float* X, float* Y, uint8_t* Xs, int prec, int8_t* Xr,
                                  uint64_t seed) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)B * n) return;
  const int b = (int)(idx / n), i = (int)(idx % n);
  const size_t off = (size_t)b * ld + i;
  const float x = x0 ? (float)x0[idx] : philox_start(seed, (uint32_t)b, (uint32_t)i);
  X[off] = x;
  Y[off] = y0;
  store_shadow(Xs, off, x, prec);
  if (Xr) Xr[off] = (int8_t)(x > 0.5f);
}

hipError_t launch_init_state(const double* x0, int B, int n, int ld, float y0, float* X,
                             float* Y, uint8_t* Xs, int xs_prec, int8_t* Xr, uint64_t seed,
                             hipStream_t s) {
  const size_t tot = (size_t)B * n;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(init_state_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, x0,
                     B, n, ld, y0, X, Y, Xs, xs_prec, Xr, seed);
  return hipGetLastError();
}

__global__ void set_state_kernel(const float* __restrict__ x, const float* __restrict__ y, int B,
                                 int n, int ld, float* X, float* Y, uint8_t* Xs, int prec) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)B * n) return;
  const int b = (int)(idx / n), i = (int)(idx % n);
  const size_t off = (size_t)b * ld + i;
  if (x) {
    X[off] = x[idx];
    store_shadow(Xs, off, x[idx], prec);
  }
  if (y) Y[off] = y[idx];
}

hipError_t launch_set_state(const float* x, const float* y, int B, int n, int ld, float* X,
                            float* Y, uint8_t* Xs, int xs_prec, hipStream_t s) {
  const size_t tot = (size_t)B * n;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(set_state_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, x, y,
                     B, n, ld, X, Y, Xs, xs_prec);
  return hipGetLastError();
}

// Ahat (int32, n x n) -> operand copy (n x ld, zero padded) and the int8 copy.
// The int8 copy is written as nlimb signed base-256 digits: digit l is the
// sign-extended low byte of r_l, r_{l+1} = (r_l - digit_l) / 256, r_0 = v.
__global__ void quantize_A_kernel(const int32_t* __restrict__ Ah, int n, int ld, int prec,
                                  uint8_t* A, int8_t* A8, int nlimb,
                                  const float* __restrict__ rscale) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * ld) return;
  const int i = (int)(idx / ld), k = (int)(idx % ld);
  const int32_t v = k < n ? Ah[(size_t)i * n + k] : 0;
  if (A8) {
    int64_t r = v;
    for (int l = 0; l < nlimb; ++l) {
      const int8_t d = (int8_t)(r & 0xff);
      A8[(size_t)l * n * ld + idx] = d;
      r = (r - d) / 256;
    }
  }
  if (!A) return;
  if (prec == P_F32) {
    ((float*)A)[idx] = (float)v;
  } else if (prec == P_BF16) {
    ((uint16_t*)A)[idx] = f32_to_bf16_rne((float)v);
  } else if (prec == P_FP8) {
    const float q = (float)v / rscale[i];
    A[idx] = (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(q, 0.f, 0, false) & 0xff);
  }
}

hipError_t launch_quantize_A(const int32_t* Ahat, int n, int ld, int prec, uint8_t* A,
                             int8_t* A8, int nlimb, const float* rscale, hipStream_t s) {
  const size_t tot = (size_t)n * ld;
  hipLaunchKernelGGL(quantize_A_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, Ahat,
                     n, ld, prec, A, A8, nlimb, rscale);
  return hipGetLastError();
}

// ---------------------------------------------------------------- incremental evaluation
//
// x_r changes from x to x' = x + delta (delta_i = +-1 on the recorded
// coordinates D).  With F(x) = (kappa/2) x^T Ahat x + c'^T x and Ahat symmetric
// with zero diagonal,
//   F(x') - F(x) = sum_{i in D} delta_i (c'_i + kappa (Ahat x')_i)
//                  - kappa sum_{i < j in D} delta_i delta_j Ahat_ij,
// all in integers.  One workgroup per restart: D is read off (and cleared
// from) the restart's bitmap; then every thread takes 16-byte chunks of the
// new rounded row and accumulates the dot products of the rows i in D of Ahat
// with them (v_dot4_i32_i8, int32: |Ahat x'|_i <= 127 n); delta_i is +1 where
// x'_i = 1, and the pairs are spread over the threads.  Restarts evaluated in
// full (more than kFlipMax changes) take the product's partials.  Either way
// the kernel finalises the restart's objective and resets its counters, and
// keeps its rounded row when it beats the incumbent, for the best of B.
//
// At a few changes per restart the kernel is a chain of memory round trips,
// so the loads are issued in as few batches as possible: the count with the
// first bitmap words; then the row chunks of x', the chunks of up to
// kIncrE rows of D at once (each thread holds kIncrV chunks of every row, so
// one pass covers rows of up to kIncrThreads * kIncrV * 16 bytes), and the
// signs, linear terms and pair entries that the last stage needs.

constexpr int kIncrThreads = 256;
constexpr int kIncrV = 3;  // 16-byte chunks of a row per thread and pass
constexpr int kIncrE = 4;  // rows of D loaded together

// Objective of a rounded row from scratch, by rows of Ahat: with S the sum of
// (Ahat x')_i and C the sum of c'_i over the coordinates i where x'_i = 1,
// F = (kappa / 2) S + C.  The incremental kernel takes this path for a restart
// with more than kFlipMax changes (or a first evaluation after init or
// set_state) when the evaluation GEMM did not run in this iteration.  It reads
// n bytes of Ahat per set coordinate: slow, and meant to be rare.  The set
// coordinates are collected 4 * NT at a time into lst.
template <int NT, int V, int E>
__device__ int64_t objective_by_rows(const InstDev& I, const PDBO_GLOBAL int8_t* xrow, int ld,
                                     int nv, int tid, int* lst, int* cnt, int64_t* part) {
  const int lane = tid & 63, wid = tid >> 6;
  constexpr int NW = NT / 64;
  const PDBO_GLOBAL int8_t* A8 = gptr(I.A8);
  const int nw = ld / 4;  // 32-bit words of the row, four 0/1 bytes each
  int64_t accS = 0, accC = 0;
  for (int v0 = 0; v0 < nv; v0 += NT * V) {
    u32x4 x[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int idx = v0 + v * NT + tid;
      x[v] = *(const PDBO_GLOBAL u32x4*)(xrow + (size_t)min(idx, nv - 1) * 16);
      if (idx >= nv) x[v] = u32x4{0, 0, 0, 0};
    }
    for (int s0 = 0; s0 < nw; s0 += NT) {
      if (tid == 0) *cnt = 0;
      __syncthreads();
      const int w = s0 + tid;
      const uint32_t word = w < nw ? ((const PDBO_GLOBAL uint32_t*)xrow)[w] : 0u;
#pragma unroll
      for (int q = 0; q < 4; ++q)  // padding coordinates (>= n) are zero; never indexed
        if (((word >> (8 * q)) & 1u) && 4 * w + q < I.n) lst[atomicAdd(cnt, 1)] = 4 * w + q;
      __syncthreads();
      const int m = *cnt;  // at most 4 * NT
      if (v0 == 0)
        for (int e = tid; e < m; e += NT) accC += *gptr(I.cp + lst[e]);
      for (int l = 0; l < I.nlimb; ++l) {  // limb l adds 256^l (Ahat_l x')_i
        const PDBO_GLOBAL int8_t* Al = A8 + l * I.limb_stride;
        for (int g = 0; g < m; g += E) {
          u32x4 a[E][V];
#pragma unroll
          for (int j = 0; j < E; ++j) {
            const PDBO_GLOBAL int8_t* arow = Al + (size_t)lst[min(g + j, m - 1)] * ld;
#pragma unroll
            for (int v = 0; v < V; ++v)
              a[j][v] =
                  *(const PDBO_GLOBAL u32x4*)(arow + (size_t)min(v0 + v * NT + tid, nv - 1) * 16);
          }
#pragma unroll
          for (int j = 0; j < E; ++j) {
            if (g + j >= m) break;
            int d = 0;
#pragma unroll
            for (int v = 0; v < V; ++v) {
              d = __builtin_amdgcn_sdot4((int)a[j][v].x, (int)x[v].x, d, false);
              d = __builtin_amdgcn_sdot4((int)a[j][v].y, (int)x[v].y, d, false);
              d = __builtin_amdgcn_sdot4((int)a[j][v].z, (int)x[v].z, d, false);
              d = __builtin_amdgcn_sdot4((int)a[j][v].w, (int)x[v].w, d, false);
            }
            accS += (int64_t)d << (8 * l);
          }
        }
      }
      __syncthreads();  // every thread is done with lst
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    accS += __shfl_xor(accS, o);
    accC += __shfl_xor(accC, o);
  }
  if (lane == 0) part[wid] = accS;
  __syncthreads();
  int64_t S = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) S += part[w];
  __syncthreads();
  if (lane == 0) part[wid] = accC;
  __syncthreads();
  int64_t C = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) C += part[w];
  __syncthreads();
  return (I.kappa == 2 ? S : S / 2) + C;
}

__global__ void __launch_bounds__(kIncrThreads)
    eval_incr_kernel(const InstDev* __restrict__ insts, const int2* __restrict__ work,
                     int full_done) {
  constexpr int NT = kIncrThreads, NW = NT / 64, V = kIncrV, E = kIncrE;
  static_assert(kFlipMax % E == 0, "whole groups of rows");
  __shared__ int lst[4 * NT];
  __shared__ int lcnt;
  __shared__ int fl[kFlipMax];
  __shared__ int nfl;
  __shared__ int red[NW][kFlipMax];
  __shared__ int64_t part[NW];
  const int2 wk = work[blockIdx.x];
  const InstDev& I = insts[wk.x];
  const int b = wk.y;
  const int ld = I.ld, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int nw32 = ld / 32;
  PDBO_GLOBAL uint32_t* bits = gptr(I.fbits + (size_t)b * nw32);
  const int k = *gptr(I.nflip + b);
  const uint32_t m0 = tid < nw32 ? bits[tid] : 0u;  // with the count, before it is known
  const int64_t Fp = *gptr(I.Fall + b);
  const int64_t incF = *gptr(&I.inc->F);
  const PDBO_GLOBAL int8_t* xrow = gptr(I.Xr + (size_t)b * ld);
  const int nv = ld / 16;
  // Only thread 0 reads and resets the restart's partials, count and
  // objective.  The new objective F is the same in every thread; the rounded
  // row is kept when it beats the incumbent of the earlier iterations, whose
  // best of B has run by now.
  auto finish = [&](int64_t F) {
    if (tid == 0) {
      *gptr(I.Fall + b) = F;
      *gptr(I.nflip + b) = 0;
      *gptr(I.Sacc + b) = 0;  // ready for the next evaluation
      *gptr(I.Cacc + b) = 0;
    }
    if (F < incF) {
      PDBO_GLOBAL u32x4* dst = (PDBO_GLOBAL u32x4*)gptr(I.cand + (size_t)b * ld);
      for (int v = tid; v < nv; v += NT) dst[v] = ((const PDBO_GLOBAL u32x4*)xrow)[v];
    }
  };
  if (k == 0) {  // unchanged: F carries over, the bitmap is clear
    if (tid == 0) {  // partials of a column block that was evaluated in full
      *gptr(I.Sacc + b) = 0;
      *gptr(I.Cacc + b) = 0;
    }
    return;
  }
  if (tid == 0) nfl = 0;
  if (k > kFlipMax && tid == 0) {  // evaluated in full: the product's partials
    const int64_t S = *gptr(I.Sacc + b), C = *gptr(I.Cacc + b);
    part[0] = (I.kappa == 2 ? S : S / 2) + C;
  }
  __syncthreads();
  if (k > kFlipMax) {
    if (m0) bits[tid] = 0u;
    for (int w = tid + NT; w < nw32; w += NT) bits[w] = 0u;
    const int64_t F = part[0];  // the partials are zero when the GEMM did not run
    finish(full_done ? F : objective_by_rows<NT, V, E>(I, xrow, ld, nv, tid, lst, &lcnt, part));
    return;
  }
  auto take = [&](int w, uint32_t m) {
    if (!m) return;
    bits[w] = 0u;
    while (m) {
      const int r = __builtin_ctz(m);
      m &= m - 1u;
      const int slot = atomicAdd(&nfl, 1);  // LDS; the order only permutes a sum
      if (slot < kFlipMax) fl[slot] = 32 * w + r;
    }
  };
  take(tid, m0);
  for (int w = tid + NT; w < nw32; w += NT) take(w, bits[w]);
  __syncthreads();
  const int kk = min(nfl, kFlipMax);
  if (kk == 0) {  // a count without marks: nothing to add
    finish(Fp);
    return;
  }
  const PDBO_GLOBAL int8_t* A8 = gptr(I.A8);

  // operands of the last stage: sign and linear term of change tid, and the
  // first pass of pairs (e, f), e < f.  They are loaded without branches, at
  // clamped (valid) indices, and masked where they are used, so that the loads
  // stay in flight while the rows are read.
  const int ci = fl[min(tid, kk - 1)];
  const int64_t cpi = *gptr(I.cp + ci);
  const int xi = xrow[ci];
  const int pe = min(tid / kk, kk - 1), pf = tid - (tid / kk) * kk;
  const int pie = fl[pe], pjf = fl[pf];
  int64_t pa = A8[(size_t)pie * ld + pjf];
  for (int l = 1; l < I.nlimb; ++l)
    pa += (int64_t)A8[l * I.limb_stride + (size_t)pie * ld + pjf] << (8 * l);
  const int pxe = xrow[pie], pxf = xrow[pjf];
  const bool pair_ok = tid < kk * kk && tid / kk < pf;

  // red[w][e]: wave w's part of (Ahat_l x')_i for change e, summed over
  // passes; dsum (thread e < kk): (Ahat x')_i = sum over limbs l of 256^l times
  // the total over waves
  int64_t dsum = 0;
  for (int l = 0; l < I.nlimb; ++l) {
  const PDBO_GLOBAL int8_t* Al = A8 + l * I.limb_stride;
  if (lane < kFlipMax) red[wid][lane] = 0;
  for (int v0 = 0; v0 < nv; v0 += NT * V) {
    // chunks past the row end are loaded at the last chunk and x is zeroed there
    u32x4 x[V];
#pragma unroll
    for (int v = 0; v < V; ++v)
      x[v] = *(const PDBO_GLOBAL u32x4*)(xrow + (size_t)min(v0 + v * NT + tid, nv - 1) * 16);
    for (int g = 0; g < kk; g += E) {
      // rows past the last change repeat it; their sums are dropped
      u32x4 a[E][V];
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const PDBO_GLOBAL int8_t* arow = Al + (size_t)fl[min(g + j, kk - 1)] * ld;
#pragma unroll
        for (int v = 0; v < V; ++v)
          a[j][v] = *(const PDBO_GLOBAL u32x4*)(arow + (size_t)min(v0 + v * NT + tid, nv - 1) * 16);
      }
#pragma unroll
      for (int v = 0; v < V; ++v)
        if (v0 + v * NT + tid >= nv) x[v] = u32x4{0, 0, 0, 0};
#pragma unroll
      for (int j = 0; j < E; ++j) {
        int d = 0;
#pragma unroll
        for (int v = 0; v < V; ++v) {
          d = __builtin_amdgcn_sdot4((int)a[j][v].x, (int)x[v].x, d, false);
          d = __builtin_amdgcn_sdot4((int)a[j][v].y, (int)x[v].y, d, false);
          d = __builtin_amdgcn_sdot4((int)a[j][v].z, (int)x[v].z, d, false);
          d = __builtin_amdgcn_sdot4((int)a[j][v].w, (int)x[v].w, d, false);
        }
        d = wave_sum_i32(d);
        if (lane == 0 && g + j < kk) red[wid][g + j] += d;
      }
    }
  }
  __syncthreads();
  if (tid < kk) {
    int d = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) d += red[w][tid];
    dsum += (int64_t)d << (8 * l);
  }
  __syncthreads();  // red is cleared for the next limb
  }
  int64_t acc64 = 0;
  if (tid < kk) acc64 = (xi ? 1 : -1) * (cpi + (int64_t)I.kappa * dsum);
  if (pair_ok) acc64 -= (int64_t)I.kappa * ((pxe ? 1 : -1) * (pxf ? 1 : -1) * pa);
  for (int pq = tid + NT; pq < kk * kk; pq += NT) {
    const int e = pq / kk, f = pq % kk;
    if (e < f) {
      const int ie = fl[e], jf = fl[f];
      const int de = xrow[ie] ? 1 : -1, df = xrow[jf] ? 1 : -1;
      int64_t a = A8[(size_t)ie * ld + jf];
      for (int l = 1; l < I.nlimb; ++l)
        a += (int64_t)A8[l * I.limb_stride + (size_t)ie * ld + jf] << (8 * l);
      acc64 -= (int64_t)I.kappa * de * df * a;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc64 += __shfl_xor(acc64, o);
  if (lane == 0) part[wid] = acc64;
  __syncthreads();
  int64_t dF = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) dF += part[w];
  finish(Fp + dF);
}

hipError_t launch_eval_incr(const InstDev* insts, const int2* work, int nwork, int full_done,
                            hipStream_t s) {
  if (nwork == 0) return hipSuccess;
  hipLaunchKernelGGL(eval_incr_kernel, dim3(nwork), dim3(kIncrThreads), 0, s, insts, work,
                     full_done);
  return hipGetLastError();
}

// The dual step of the single-constraint variant (PDBO-s): y of restart b is
// one number, raised by beta times sum_i g(x_i^t) (the constraint's value at
// the old x, as in the simultaneous update of Alg. 1).  The sum is taken in
// float64 in a fixed order (strided per thread, then a tree), so runs are
// reproducible.  y^t is first copied into the restart's row of Y, where the
// step kernel reads it for the perturbation test and dL/dx_i = G_i + y g'(x_i).
template <int GK>
__global__ void __launch_bounds__(256) dual_scalar_kernel(const InstDev* __restrict__ insts,
                                                          int parity) {
  __shared__ double red[256];
  const InstDev& I = insts[blockIdx.y];
  const int b = blockIdx.x, tid = threadIdx.x;
  if (b >= I.B) return;
  const float* x = I.X[parity] + (size_t)b * I.ld;
  float* y = I.Y + (size_t)b * I.ld;
  const float yb = I.ys[b];
  double acc = 0.0;
  for (int i = tid; i < I.n; i += 256) {
    acc += (double)g_value(x[i], GK, I.gp.deg);
    y[i] = yb;
  }
  red[tid] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) I.ys[b] = (float)((double)yb + (double)I.gp.beta * red[0]);
}

hipError_t launch_dual_scalar(const InstDev* insts, int ninst, int B, int gkind, int parity,
                              hipStream_t s) {
  const dim3 grid(B, ninst);
  if (gkind == 0)
    hipLaunchKernelGGL(dual_scalar_kernel<0>, grid, dim3(256), 0, s, insts, parity);
  else if (gkind == 1)
    hipLaunchKernelGGL(dual_scalar_kernel<1>, grid, dim3(256), 0, s, insts, parity);
  else
    hipLaunchKernelGGL(dual_scalar_kernel<2>, grid, dim3(256), 0, s, insts, parity);
  return hipGetLastError();
}

__global__ void fill_i32_kernel(int32_t* p, int32_t v, int64_t cnt) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < cnt) p[idx] = v;
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, v,
                     count);
  return hipGetLastError();
}

__global__ void fill_i64_kernel(int64_t* p, int64_t v, size_t cnt) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < cnt) p[idx] = v;
}

hipError_t launch_fill_i64(int64_t* p, int64_t v, size_t cnt, hipStream_t s) {
  if (cnt == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i64_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, p, v,
                     cnt);
  return hipGetLastError();
}

#endif  // PDBO_DENSE_PART == 0

}  // namespace pdbo
