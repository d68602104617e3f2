// Sparse QUBO path: a persistent, restart-resident kernel for CSR couplings.
//
// Restarts are independent (Sec. 4.2, Model Settings), so one workgroup owns
// one restart for the whole launch: x of that restart lives in LDS (every row's
// neighbours are gathered from there), y and the thread's own x in registers,
// and when it fits the canonical CSR matrix Ahat = offdiag(Q + Q^T)/kappa is
// staged in LDS too.  Each iteration needs one barrier (two when x cannot be
// double-buffered in LDS) and no grid-wide synchronisation.  The exact objective of round(x^t) is fused into the same
// gathers: while row i accumulates sum_k Ahat_ik x_k for the gradient it also
// accumulates sum_k Ahat_ik [x_k > 1/2] in int32, so F(round(x^t)) =
// (kappa/2) x_r^T Ahat x_r + c'^T x_r costs no extra pass.  The best value of
// each restart over time (and the vector that attained it) is kept per restart
// and reduced to the incumbent by restart_best_kernel.
#include <climits>
#include <type_traits>

#include "common.h"

namespace pdbo {

__host__ __device__ static inline size_t align16(size_t v) { return (v + 15) & ~size_t(15); }

static size_t csr_lds_need(int n, int64_t nnz, bool packed) {
  size_t b = align16((size_t)n * 4);
  if (packed) b += align16((size_t)(n + 1) * 4) + align16((size_t)nnz * 4);
  return b;
}

constexpr size_t kLdsBudget = 150 * 1024;

// The persistent kernel needs x of one restart in LDS and at most 32768 rows
// (512 threads x 64 rows).  With packed entries (16-bit column,
// 16-bit value) the whole canonical matrix is staged in LDS too when it fits;
// otherwise the CSR arrays are read through the L2.
bool csr_fits(int n, int64_t nnz, bool packed, size_t* lds_bytes) {
  const bool in_lds = packed && csr_lds_need(n, nnz, true) <= kLdsBudget;
  const size_t need = csr_lds_need(n, nnz, in_lds);
  if (lds_bytes) *lds_bytes = need;
  return n <= 32768 && need <= kLdsBudget;
}

// sum_k Ahat_ik x_k (float) and sum_k Ahat_ik [x_k > 1/2] (int) over row i,
// four entries at a time so that their LDS reads are in flight together.
template <bool PACKED>
__device__ __forceinline__ void row_gather(int i, const int32_t* __restrict__ rp,
                                           const uint32_t* __restrict__ ent,
                                           const int32_t* __restrict__ col,
                                           const int32_t* __restrict__ val,
                                           const float* __restrict__ xs, float& acc, int& accr) {
  const int pe = rp[i + 1];
  int p = rp[i];
  float a0 = 0.f, a1 = 0.f;
  int r0 = 0, r1 = 0;
  for (; p + 4 <= pe; p += 4) {
    int c[4], v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if constexpr (PACKED) {
        const uint32_t e = ent[p + u];
        c[u] = (int)(e & 0xffffu);
        v[u] = (int)(int16_t)(e >> 16);
      } else {
        c[u] = col[p + u];
        v[u] = val[p + u];
      }
    }
    float xk[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) xk[u] = xs[c[u]];
    a0 = fmaf((float)v[0], xk[0], a0);
    a1 = fmaf((float)v[1], xk[1], a1);
    a0 = fmaf((float)v[2], xk[2], a0);
    a1 = fmaf((float)v[3], xk[3], a1);
    r0 += (xk[0] > 0.5f ? v[0] : 0) + (xk[2] > 0.5f ? v[2] : 0);
    r1 += (xk[1] > 0.5f ? v[1] : 0) + (xk[3] > 0.5f ? v[3] : 0);
  }
  for (; p < pe; ++p) {
    int c, v;
    if constexpr (PACKED) {
      const uint32_t e = ent[p];
      c = (int)(e & 0xffffu);
      v = (int)(int16_t)(e >> 16);
    } else {
      c = col[p];
      v = val[p];
    }
    const float xk = xs[c];
    a0 = fmaf((float)v, xk, a0);
    r0 += xk > 0.5f ? v : 0;
  }
  acc = a0 + a1;
  accr = r0 + r1;
}

// The same sums over a row of the interleaved layout: entry r at
// ent[base + 64 r], accumulated in the same order as row_gather.
__device__ __forceinline__ void row_gather_sl(int base, int len, const uint32_t* __restrict__ ent,
                                              const float* __restrict__ xs, float& acc, int& accr) {
  const uint32_t* e0 = ent + base;
  float a0 = 0.f, a1 = 0.f;
  int r0 = 0, r1 = 0;
  int p = 0;
  for (; p + 4 <= len; p += 4) {
    int c[4], v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t e = e0[(p + u) * 64];
      c[u] = (int)(e & 0xffffu);
      v[u] = (int)(int16_t)(e >> 16);
    }
    float xk[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) xk[u] = xs[c[u]];
    a0 = fmaf((float)v[0], xk[0], a0);
    a1 = fmaf((float)v[1], xk[1], a1);
    a0 = fmaf((float)v[2], xk[2], a0);
    a1 = fmaf((float)v[3], xk[3], a1);
    r0 += (xk[0] > 0.5f ? v[0] : 0) + (xk[2] > 0.5f ? v[2] : 0);
    r1 += (xk[1] > 0.5f ? v[1] : 0) + (xk[3] > 0.5f ? v[3] : 0);
  }
  for (; p < len; ++p) {
    const uint32_t e = e0[p * 64];
    const int c = (int)(e & 0xffffu), v = (int)(int16_t)(e >> 16);
    const float xk = xs[c];
    a0 = fmaf((float)v, xk, a0);
    r0 += xk > 0.5f ? v : 0;
  }
  acc = a0 + a1;
  accr = r0 + r1;
}

// Sum of an int32 over lanes 0..15 (row 0 of the wave), in every lane: row
// shifts by 1, 2, 4 and 8 leave the row's total in its lane 15.
__device__ __forceinline__ int32_t row16_sum_i32(int32_t v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);  // row_shr:8
  return __builtin_amdgcn_readlane(v, 15);
}

// DBUF: x is double-buffered in LDS (iteration t gathers from buffer t mod 2
// and writes x^{t+1} into the other), so one barrier per iteration suffices;
// otherwise x is updated in place between two barriers.
// SMALL: the host has bounded every wave's partial sums of x_r^T Ahat x_r and
// c'^T x_r below 2^31, so the wave reductions run in int32 (half the shuffles
// of int64).  TOT32 (with SMALL): the restart's totals are bounded below 2^31
// too, so the sum over waves is taken in int32 as well (a quarter of the
// instructions of the int64 row reduction); otherwise it is taken in int64.
// SL (with PACKED): the entries are staged in the interleaved layout (psl)
// instead of row_ptr + CSR order; each row's start and length stay in
// registers.
template <bool PACKED, int NT, int RMAX, bool DBUF, bool SMALL, int GK, bool TOT32 = false,
          bool SL = false>
__global__ void __launch_bounds__(NT)
    csr_persistent(CsrDev D, int64_t t0, int nsteps) {
  static_assert(!SL || PACKED, "the interleaved layout holds packed entries");
  constexpr int NW = NT / 64;
  static_assert(NW <= 16, "the partials of at most 16 waves are summed by one row of lanes");
  using Part = typename std::conditional<SMALL, int32_t, int64_t>::type;
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  __shared__ Part red[2][NW][2];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int b = blockIdx.x;
  const int n = D.n;
  float* xs = (float*)lds;
  const int32_t* rp = D.row_ptr;
  const uint32_t* ent = D.packed;
  const size_t xbytes = align16((size_t)n * 4) * (DBUF ? 2 : 1);
  if constexpr (SL) {
    uint32_t* entl = (uint32_t*)(lds + xbytes);
    const int nsl = (int)D.nsl;
    for (int q = tid; q < nsl; q += NT) entl[q] = D.psl[q];
    ent = entl;
  } else if constexpr (PACKED) {
    int32_t* rpl = (int32_t*)(lds + xbytes);
    uint32_t* entl = (uint32_t*)((uint8_t*)rpl + align16((size_t)(n + 1) * 4));
    const int nnz = (int)D.nnz;
    for (int q = tid; q <= n; q += NT) rpl[q] = D.row_ptr[q];
    for (int q = tid; q < nnz; q += NT) entl[q] = D.packed[q];
    rp = rpl;
    ent = entl;
  }
  const int32_t* col = (const int32_t*)D.col;
  const int32_t* val = (const int32_t*)D.val;
  const int xstride = (int)(align16((size_t)n * 4) / 4);  // floats between the two x buffers
  // c'/s and c' of the thread's rows stay in registers when there are few rows
  constexpr bool CREG = RMAX <= 8;
  float xr[RMAX], yr[RMAX], xn[RMAX], cps[CREG ? RMAX : 1];
  Part cpr[CREG ? RMAX : 1];
  // the thread's rows, taken in order of decreasing degree so that the 64 rows
  // of a wave round have nearly the same length (fewer idle lanes in the
  // gathers); -1 past the end
  int rows[RMAX];
#pragma unroll
  for (int j = 0; j < RMAX; ++j) rows[j] = tid + j * NT < n ? D.order[tid + j * NT] : -1;
  int rbase[SL ? RMAX : 1], rlen[SL ? RMAX : 1];
  if constexpr (SL) {
#pragma unroll
    for (int j = 0; j < RMAX; ++j) {
      const int q = tid + j * NT, i = rows[j];
      rbase[j] = i >= 0 ? D.slice[q >> 6] + (q & 63) : 0;
      rlen[j] = i >= 0 ? D.row_ptr[i + 1] - D.row_ptr[i] : 0;
    }
  }
#pragma unroll
  for (int j = 0; j < RMAX; ++j) {
    const int i = rows[j];
    xr[j] = 0.f;
    yr[j] = 0.f;
    if constexpr (CREG) {
      cps[j] = 0.f;
      cpr[j] = 0;
    }
    if (i >= 0) {
      xr[j] = D.X[(size_t)b * D.ld + i];
      yr[j] = D.Y[(size_t)b * D.ld + i];
      if constexpr (CREG) {
        cps[j] = D.cps[i];
        cpr[j] = (Part)D.cp[i];
      }
      xs[i] = xr[j];
    }
  }
  int64_t bF = D.rbestF[b], bT = D.rbestT[b];
  uint64_t bTs = D.rbestTs[b];
  int64_t Flast = D.Flast[b];
  const float kos = D.kos;
  GdaP gp = D.gp;
  gp.gkind = GK;  // a constant: only this kind's g and g' are computed
  __syncthreads();

  for (int s = 0; s <= nsteps; ++s) {
    const bool upd = s < nsteps;
    const bool ev = s > 0;
    const float* xcur = DBUF ? xs + (s & 1) * xstride : xs;
    Part S = 0, C = 0;
#pragma unroll
    for (int j = 0; j < RMAX; ++j) {
      const int i = rows[j];
      if (i >= 0) {
        float acc;
        int accr;
        if constexpr (SL)
          row_gather_sl(rbase[j], rlen[j], ent, xcur, acc, accr);
        else
          row_gather<PACKED>(i, rp, ent, col, val, xcur, acc, accr);
        if (ev && xr[j] > 0.5f) {
          S += (Part)accr;
          if constexpr (CREG)
            C += cpr[j];
          else
            C += (Part)D.cp[i];
        }
        if (upd) {
          float a, c;
          gda_update(xr[j], yr[j], fmaf(acc, kos, CREG ? cps[j] : D.cps[i]), gp, a, c);
          xn[j] = a;
          yr[j] = c;
        }
      }
    }
    if (ev) {
      if constexpr (SMALL) {
        S = wave_sum_i32(S);
        C = wave_sum_i32(C);
      } else {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          S += __shfl_xor(S, o);
          C += __shfl_xor(C, o);
        }
      }
      if (lane == 0) {
        red[s & 1][wid][0] = S;
        red[s & 1][wid][1] = C;
      }
    }
    // x^{t+1} goes into the other buffer before the single barrier; the
    // rounded x^t (xr) is still needed for the incumbent copy below
    if constexpr (DBUF) {
      if (upd) {
        float* xnext = xs + ((s + 1) & 1) * xstride;
#pragma unroll
        for (int j = 0; j < RMAX; ++j) {
          const int i = rows[j];
          if (i >= 0) xnext[i] = xn[j];
        }
      }
    }
    __syncthreads();
    if (ev) {
      // lane l of every wave takes wave (l mod 16)'s partials; a 16-lane row
      // reduction gives the totals to every lane (NW <= 16)
      const int w = lane & 15;
      int64_t St, Ct;
      if constexpr (TOT32) {
        static_assert(SMALL, "int32 totals need int32 wave sums");
        St = row16_sum_i32(w < NW ? (int32_t)red[s & 1][w][0] : 0);
        Ct = row16_sum_i32(w < NW ? (int32_t)red[s & 1][w][1] : 0);
      } else {
        St = row16_sum_i64(w < NW ? (int64_t)red[s & 1][w][0] : 0);
        Ct = row16_sum_i64(w < NW ? (int64_t)red[s & 1][w][1] : 0);
      }
      const int64_t F = (D.kappa == 2 ? St : St / 2) + Ct;
      Flast = F;
      if (F < bF) {
        bF = F;
        bT = t0 + s;
        if (tid == 0) bTs = wall_clock();
        uint8_t* dst = D.best_xr + (size_t)b * n;
#pragma unroll
        for (int j = 0; j < RMAX; ++j) {
          const int i = rows[j];
          if (i >= 0) dst[i] = (uint8_t)(xr[j] > 0.5f);
        }
      }
    }
    if (upd) {
#pragma unroll
      for (int j = 0; j < RMAX; ++j) {
        const int i = rows[j];
        if (i >= 0) {
          if constexpr (!DBUF) xs[i] = xn[j];
          xr[j] = xn[j];
        }
      }
    }
    if constexpr (!DBUF) __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < RMAX; ++j) {
    const int i = rows[j];
    if (i >= 0) {
      D.X[(size_t)b * D.ld + i] = xr[j];
      D.Y[(size_t)b * D.ld + i] = yr[j];
    }
  }
  if (tid == 0) {
    D.rbestF[b] = bF;
    D.rbestT[b] = bT;
    D.rbestTs[b] = bTs;
    D.Flast[b] = Flast;
  }
}

// LDS of the interleaved layout: x and the entries (the host builds it only
// when this is no more than csr_lds_need with packed entries).
static size_t csr_lds_need_sl(const CsrDev& d) {
  return align16((size_t)d.n * 4) + align16((size_t)d.nsl * 4);
}

template <bool PACKED, int NT, int RMAX, bool DBUF, bool SMALL, int GK, bool TOT32 = false,
          bool SL = false>
static hipError_t launch_csr_k(const CsrDev& d, int64_t t0, int nsteps, hipStream_t s) {
  auto kern = csr_persistent<PACKED, NT, RMAX, DBUF, SMALL, GK, TOT32, SL>;
  const size_t lds = (SL ? csr_lds_need_sl(d) : csr_lds_need(d.n, d.nnz, PACKED)) +
                     (DBUF ? align16((size_t)d.n * 4) : 0);
  hipError_t e =
      hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(d.B), dim3(NT), lds, s, d, t0, nsteps);
  return hipGetLastError();
}

template <bool PACKED, int NT, int RMAX, int GK, bool SL>
static hipError_t launch_csr_v2(const CsrDev& d, int64_t t0, int nsteps, hipStream_t s) {
  const bool dbuf = csr_lds_need(d.n, d.nnz, PACKED) + align16((size_t)d.n * 4) <= kLdsBudget;
  if (dbuf && d.tot32)
    return launch_csr_k<PACKED, NT, RMAX, true, true, GK, true, SL>(d, t0, nsteps, s);
  if (dbuf && d.small32)
    return launch_csr_k<PACKED, NT, RMAX, true, true, GK, false, SL>(d, t0, nsteps, s);
  if (dbuf) return launch_csr_k<PACKED, NT, RMAX, true, false, GK, false, SL>(d, t0, nsteps, s);
  if (d.small32) return launch_csr_k<PACKED, NT, RMAX, false, true, GK, false, SL>(d, t0, nsteps, s);
  return launch_csr_k<PACKED, NT, RMAX, false, false, GK, false, SL>(d, t0, nsteps, s);
}

template <bool PACKED, int NT, int RMAX, int GK>
static hipError_t launch_csr_v(const CsrDev& d, int64_t t0, int nsteps, hipStream_t s) {
  if constexpr (PACKED)
    if (d.psl) return launch_csr_v2<true, NT, RMAX, GK, true>(d, t0, nsteps, s);
  return launch_csr_v2<PACKED, NT, RMAX, GK, false>(d, t0, nsteps, s);
}

// 1024 threads per restart (sixteen waves keep enough LDS gathers in flight)
// up to 8 rows per thread; beyond that (n > 8192) 512 threads with 32 or 64
// rows per thread, whose per-row state does not fit the register budget and
// partly lives in scratch memory.
template <bool PACKED, int GK>
static hipError_t launch_csr_r(const CsrDev& d, int64_t t0, int nsteps, hipStream_t s) {
  const int r = (d.n + 1023) / 1024;
  if (r <= 1) return launch_csr_v<PACKED, 1024, 1, GK>(d, t0, nsteps, s);
  if (r <= 2) return launch_csr_v<PACKED, 1024, 2, GK>(d, t0, nsteps, s);
  if (r <= 4) return launch_csr_v<PACKED, 1024, 4, GK>(d, t0, nsteps, s);
  if (r <= 8) return launch_csr_v<PACKED, 1024, 8, GK>(d, t0, nsteps, s);
  const int r2 = (d.n + 511) / 512;
  if (r2 <= 32) return launch_csr_k<PACKED, 512, 32, false, false, GK>(d, t0, nsteps, s);
  if (r2 <= 64) return launch_csr_k<PACKED, 512, 64, false, false, GK>(d, t0, nsteps, s);
  return hipErrorInvalidValue;
}

// The variant launch_csr_persistent takes for an instance, by the same rules:
// packed (16-bit) entries in LDS or int32 arrays through L2, x double-buffered
// or updated in place, int32 or int64 wave sums (and, double-buffered, int32
// totals: "t32"), and beyond 8192 rows 512 threads with 32 or 64 rows each.
const char* csr_variant_name(const CsrDev& d, bool packed) {
  const bool pk = packed && csr_lds_need(d.n, d.nnz, true) <= kLdsBudget;
  if ((d.n + 1023) / 1024 > 8) {
    const bool r32 = (d.n + 511) / 512 <= 32;
    return pk ? (r32 ? "csr_packed_rows32" : "csr_packed_rows64")
              : (r32 ? "csr_l2_rows32" : "csr_l2_rows64");
  }
  const bool dbuf = csr_lds_need(d.n, d.nnz, pk) + align16((size_t)d.n * 4) <= kLdsBudget;
  const bool sl = pk && d.psl;
  if (dbuf && d.tot32) return sl ? "csr_sliced_dbuf_t32" : pk ? "csr_packed_dbuf_t32" : "csr_l2_dbuf_t32";
  static const char* names[3][2][2] = {
      {{"csr_l2_inplace_i64", "csr_l2_inplace_i32"}, {"csr_l2_dbuf_i64", "csr_l2_dbuf_i32"}},
      {{"csr_packed_inplace_i64", "csr_packed_inplace_i32"},
       {"csr_packed_dbuf_i64", "csr_packed_dbuf_i32"}},
      {{"csr_sliced_inplace_i64", "csr_sliced_inplace_i32"},
       {"csr_sliced_dbuf_i64", "csr_sliced_dbuf_i32"}}};
  return names[sl ? 2 : pk ? 1 : 0][dbuf][d.small32 ? 1 : 0];
}

// One kernel variant per kind of g (GK): read at run time, the kind would make
// the update evaluate both forms of g and g' for every coordinate.
hipError_t launch_csr_persistent(const CsrDev& d, bool packed, int64_t t0, int nsteps,
                                 hipStream_t s) {
  if (nsteps <= 0) return hipSuccess;
  const bool pk = packed && csr_lds_need(d.n, d.nnz, true) <= kLdsBudget;
  if (d.gp.gkind == 0)
    return pk ? launch_csr_r<true, 0>(d, t0, nsteps, s) : launch_csr_r<false, 0>(d, t0, nsteps, s);
  return pk ? launch_csr_r<true, 1>(d, t0, nsteps, s) : launch_csr_r<false, 1>(d, t0, nsteps, s);
}

// ---- gradient and exact evaluation at given points (tests, qubo_gda_grad/eval)

__global__ void csr_grad_kernel(CsrDev D, const float* __restrict__ X, float* __restrict__ G,
                                int nb) {
  using ColT = int32_t;
  using ValT = int32_t;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nb * D.n) return;
  const int b = (int)(idx / D.n), i = (int)(idx % D.n);
  const float* xb = X + (size_t)b * D.ld;
  const ColT* col = (const ColT*)D.col;
  const ValT* val = (const ValT*)D.val;
  float acc = 0.f;
  for (int p = D.row_ptr[i]; p < D.row_ptr[i + 1]; ++p) acc = fmaf((float)val[p], xb[col[p]], acc);
  G[(size_t)b * D.ld + i] = fmaf(acc, D.kos, D.cps[i]);
}

__global__ void __launch_bounds__(256)
    csr_eval_kernel(CsrDev D, const int8_t* __restrict__ xr, int64_t* __restrict__ F) {
  using ColT = int32_t;
  using ValT = int32_t;
  __shared__ int64_t red[4][2];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int8_t* x = xr + (size_t)b * D.ld;
  const ColT* col = (const ColT*)D.col;
  const ValT* val = (const ValT*)D.val;
  int64_t S = 0, C = 0;
  for (int i = tid; i < D.n; i += 256) {
    if (!x[i]) continue;
    int64_t a = 0;
    for (int p = D.row_ptr[i]; p < D.row_ptr[i + 1]; ++p) a += x[col[p]] ? (int64_t)val[p] : 0;
    S += a;
    C += D.cp[i];
  }
  for (int o = 32; o > 0; o >>= 1) {
    S += __shfl_xor(S, o);
    C += __shfl_xor(C, o);
  }
  if ((tid & 63) == 0) {
    red[tid >> 6][0] = S;
    red[tid >> 6][1] = C;
  }
  __syncthreads();
  if (tid == 0) {
    int64_t St = 0, Ct = 0;
    for (int w = 0; w < 4; ++w) {
      St += red[w][0];
      Ct += red[w][1];
    }
    F[b] = (D.kappa == 2 ? St : St / 2) + Ct;
  }
}

hipError_t launch_csr_grad(const CsrDev& d, const float* X, float* G, int nb, hipStream_t s) {
  const size_t tot = (size_t)nb * d.n;
  if (tot == 0) return hipSuccess;
  const dim3 grid((unsigned)((tot + 255) / 256));
  hipLaunchKernelGGL(csr_grad_kernel, grid, dim3(256), 0, s, d, X, G, nb);
  return hipGetLastError();
}

hipError_t launch_csr_eval(const CsrDev& d, const int8_t* xr, int nb, int64_t* F, hipStream_t s) {
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(csr_eval_kernel, dim3(nb), dim3(256), 0, s, d, xr, F);
  return hipGetLastError();
}

// ---- per-restart bests -> incumbent ----------------------------------------

__global__ void __launch_bounds__(256)
    restart_best_kernel(const int64_t* __restrict__ rbestF, const int64_t* __restrict__ rbestT,
                        const uint64_t* __restrict__ rbestTs, const uint8_t* __restrict__ best_xr,
                        int B, int n, Incumbent* inc, uint8_t* best_x) {
  __shared__ int64_t sF[256], sT[256];
  __shared__ int sb[256];
  const int tid = threadIdx.x;
  int64_t F = LLONG_MAX, T = LLONG_MAX;
  int bb = INT_MAX;
  for (int b = tid; b < B; b += 256) {
    const int64_t f = rbestF[b], t = rbestT[b];
    if (f < F || (f == F && t < T)) {
      F = f;
      T = t;
      bb = b;
    }
  }
  sF[tid] = F;
  sT[tid] = T;
  sb[tid] = bb;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      const int64_t f = sF[tid + h], t = sT[tid + h];
      const int b = sb[tid + h];
      if (f < sF[tid] || (f == sF[tid] && (t < sT[tid] || (t == sT[tid] && b < sb[tid])))) {
        sF[tid] = f;
        sT[tid] = t;
        sb[tid] = b;
      }
    }
    __syncthreads();
  }
  const int b = sb[0];
  if (sF[0] == LLONG_MAX || b == INT_MAX) return;
  if (tid == 0) {
    inc->F = sF[0];
    inc->t = sT[0];
    inc->b = b;
    inc->ts = rbestTs[b];
  }
  for (int i = tid; i < n; i += 256) best_x[i] = best_xr[(size_t)b * n + i];
}

hipError_t launch_restart_best(const int64_t* rbestF, const int64_t* rbestT,
                               const uint64_t* rbestTs, const uint8_t* best_xr, int B, int n,
                               Incumbent* inc, uint8_t* best_x, hipStream_t s) {
  hipLaunchKernelGGL(restart_best_kernel, dim3(1), dim3(256), 0, s, rbestF, rbestT, rbestTs,
                     best_xr, B, n, inc, best_x);
  return hipGetLastError();
}

}  // namespace pdbo
