// Weighted Max-k-SAT path (Sec. 4.1, Max-k-SAT; weighted clauses).
//
// f(x) = sum_j w_j prod_{l in C_j} p(x_l), p = x for a negated literal and
// 1 - x otherwise; its partial derivative in x_i sums, over the occurrences of
// variable i, w_j * (+1 if that literal is negated, else -1) times the product
// of p over the other literals of the clause.  The adjoint is computed
// variable-major: every variable owns the list of its occurrences, each entry
// carrying the codes of the clause's other literals and a meta word, so the
// gradient is a deterministic gather with no atomics.  The meta word holds the
// weight (bits 0-23), "this literal is negated" (bit 30) and "this variable
// owns the clause" (bit 29; the host spreads the clauses so that every variable
// owns about m/n of them); the exact weighted unsatisfied count of round(x) is
// fused into the same pass by counting each clause at its owner.  Literal codes
// are (variable index) | (negated << 31).  For 3-SAT the persistent kernel
// reads a compact 8-byte copy of each entry (two 16-bit codes and the meta
// word), a variable's owned clauses first, interleaved by slices of 64
// positions so that the 64 lanes of a wave read entry r of their lists from
// one contiguous 512-byte block.
#include <climits>

#include "common.h"

namespace pdbo {

__host__ __device__ static inline size_t align16s(size_t v) { return (v + 15) & ~size_t(15); }

constexpr size_t kSatLdsBudget = 150 * 1024;
// x and y of one restart, plus the kernel's small static arrays, in the 160 KB
constexpr size_t kSatYldsBudget = 160 * 1024 - 1024;

bool sat_fits(int n, size_t* lds_bytes) {
  const size_t need = align16s((size_t)n * 4);
  if (lds_bytes) *lds_bytes = need;
  return n <= 32768 && need <= kSatLdsBudget;
}

// Sum over the occurrences of variable i of the adjoint terms; also the
// weighted count of the clauses i owns whose literals are all false.
__device__ __forceinline__ float sat_adjoint(const SatDev& D, const float* __restrict__ xsrc,
                                             int i, float xi, bool want_eval, int64_t& unsat) {
  const int k = D.k;
  float g = 0.f;
  const bool own_true = xi > 0.5f;
  const int pe = D.inc_ptr[i + 1];
  for (int e = D.inc_ptr[i]; e < pe; ++e) {
    const int32_t* E = D.inc + (size_t)e * k;
    float prod = 1.f;
    bool others_false = true;
    for (int o = 0; o < k - 1; ++o) {
      const int32_t code = E[o];
      const float xv = xsrc[code & 0x7fffffff];
      const bool neg = code < 0;
      prod *= neg ? xv : 1.f - xv;
      others_false = others_false && ((xv > 0.5f) == neg);
    }
    const int32_t meta = E[k - 1];
    const float w = (float)(meta & 0xffffff);
    const bool own_neg = (meta >> 30) & 1;
    g = fmaf(own_neg ? w : -w, prod, g);
    if (want_eval && ((meta >> 29) & 1) && others_false && (own_true == own_neg))
      unsat += (meta & 0xffffff);
  }
  return g;
}

// 3-SAT occurrence entry in 8 bytes: the other two literals as 16-bit codes
// (position | negated << 15) in the low word, the meta word in the high word.
// Each position's list starts with the clauses it owns, so the count of
// unsatisfied clauses (taken at the owner) is skipped by whole waves in the
// later rounds of a list.
__device__ __forceinline__ void sat3_term(uint64_t en, float xa, float xb, bool own_true,
                                          bool want_eval, float& g, int64_t& unsat) {
  const uint32_t codes = (uint32_t)en;
  const bool na = (codes >> 15) & 1u, nb = (codes >> 31) != 0;
  const float prod = (na ? xa : 1.f - xa) * (nb ? xb : 1.f - xb);
  const int32_t meta = (int32_t)(en >> 32);
  const float w = (float)(meta & 0xffffff);
  const bool own_neg = (meta >> 30) & 1;
  g = fmaf(own_neg ? w : -w, prod, g);
  if (want_eval && ((meta >> 29) & 1) && ((xa > 0.5f) == na) && ((xb > 0.5f) == nb) &&
      (own_true == own_neg))
    unsat += (meta & 0xffffff);
}

// Adjoint of position i from its compact list, four entries per round: their
// loads first (each a contiguous 512-byte read of the wave's slice), then their
// eight gathers, then the arithmetic.
__device__ __forceinline__ float sat3_adjoint(const SatDev& D, const float* __restrict__ xs, int i,
                                              float xi, bool want_eval, int64_t& unsat) {
  const __attribute__((address_space(1))) uint64_t* E =
      (const __attribute__((address_space(1))) uint64_t*)D.pinc3 + D.pinc3_slice[i >> 6] + (i & 63);
  const int len = D.pinc_ptr[i + 1] - D.pinc_ptr[i];
  const bool own_true = xi > 0.5f;
  float g[4] = {0.f, 0.f, 0.f, 0.f};
  int r = 0;
  for (; r + 4 <= len; r += 4) {
    uint64_t en[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) en[u] = E[(r + u) * 64];
    float xa[4], xb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      xa[u] = xs[(uint32_t)en[u] & 0x7fffu];
      xb[u] = xs[((uint32_t)en[u] >> 16) & 0x7fffu];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) sat3_term(en[u], xa[u], xb[u], own_true, want_eval, g[u], unsat);
  }
  for (; r < len; ++r) {
    const uint64_t en = E[r * 64];
    sat3_term(en, xs[(uint32_t)en & 0x7fffu], xs[((uint32_t)en >> 16) & 0x7fffu], own_true, want_eval,
              g[0], unsat);
  }
  return (g[0] + g[1]) + (g[2] + g[3]);
}

// YLDS: y lives in LDS beside x (both n floats), read and written in place by
// the variable's owner, and x^t is read back from LDS; only x^{t+1} is held in
// registers until the barrier.  Used when many variables fall to each thread
// and both arrays fit, so that the per-variable state does not spill.
template <bool K3, int NT, int RMAX, bool YLDS, int GK>
__global__ void __launch_bounds__(NT) sat_persistent(SatDev Dv, int64_t t0, int nsteps) {
  // position space (see SatDev::order): thread tid owns positions tid + j NT
  SatDev D = Dv;
  D.inc_ptr = Dv.pinc_ptr;
  D.inc = Dv.pinc;
  constexpr int NW = NT / 64;
  static_assert(NW <= 16, "the partials of at most 16 waves are summed by one row of lanes");
  extern __shared__ __attribute__((aligned(16))) float xs[];
  __shared__ int64_t red[2][NW];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int b = blockIdx.x, n = D.n;
  float* ys = xs + align16s((size_t)n * 4) / 4;
  float xr[YLDS ? 1 : RMAX], yr[YLDS ? 1 : RMAX], xn[RMAX];
#pragma unroll
  for (int j = 0; j < RMAX; ++j) {
    const int i = tid + j * NT;
    if constexpr (!YLDS) {
      xr[j] = 0.f;
      yr[j] = 0.f;
    }
    if (i < n) {
      const int v = D.order[i];
      const float x = D.X[(size_t)b * D.ld + v], y = D.Y[(size_t)b * D.ld + v];
      xs[i] = x;
      if constexpr (YLDS) {
        ys[i] = y;
      } else {
        xr[j] = x;
        yr[j] = y;
      }
    }
  }
  auto xold = [&](int j, int i) { return YLDS ? xs[i] : xr[j]; };
  int64_t bF = D.rbestF[b], bT = D.rbestT[b];
  uint64_t bTs = D.rbestTs[b];
  int64_t Flast = D.Flast[b];
  GdaP gp = D.gp;
  gp.gkind = GK;  // a constant: only this kind's g and g' are computed
  const float ios = D.ios;
  __syncthreads();
  for (int s = 0; s <= nsteps; ++s) {
    const bool upd = s < nsteps;
    const bool ev = s > 0;
    int64_t S = 0;
    // with y in LDS only x^{t+1} is kept per variable: the loop is not
    // unrolled (twenty copies of the occurrence loop would spill)
#pragma unroll(YLDS ? 1 : RMAX)
    for (int j = 0; j < RMAX; ++j) {
      const int i = tid + j * NT;
      if (i < n) {
        const float xi = xold(j, i);
        const float g = K3 ? sat3_adjoint(D, xs, i, xi, ev, S) : sat_adjoint(D, xs, i, xi, ev, S);
        if (upd) {
          float a, c;
          gda_update(xi, YLDS ? ys[i] : yr[j], g * ios, gp, a, c);
          xn[j] = a;
          if constexpr (YLDS)
            ys[i] = c;
          else
            yr[j] = c;
        }
      }
    }
    if (ev) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) S += __shfl_xor(S, o);
      if (lane == 0) red[s & 1][wid] = S;
    }
    __syncthreads();
    if (ev) {
      // lane l of every wave takes wave (l mod 16)'s partial; a 16-lane row
      // reduction gives the total to every lane (NW <= 16)
      const int64_t F = row16_sum_i64((lane & 15) < NW ? red[s & 1][lane & 15] : 0);
      Flast = F;
      if (F < bF) {
        bF = F;
        bT = t0 + s;
        if (tid == 0) bTs = wall_clock();
        uint8_t* dst = D.best_xr + (size_t)b * n;
#pragma unroll
        for (int j = 0; j < RMAX; ++j) {
          const int i = tid + j * NT;
          if (i < n) dst[D.order[i]] = (uint8_t)(xold(j, i) > 0.5f);
        }
      }
    }
    if (upd) {
#pragma unroll
      for (int j = 0; j < RMAX; ++j) {
        const int i = tid + j * NT;
        if (i < n) {
          xs[i] = xn[j];
          if constexpr (!YLDS) xr[j] = xn[j];
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < RMAX; ++j) {
    const int i = tid + j * NT;
    if (i < n) {
      const int v = D.order[i];
      D.X[(size_t)b * D.ld + v] = xold(j, i);
      D.Y[(size_t)b * D.ld + v] = YLDS ? ys[i] : yr[j];
    }
  }
  if (tid == 0) {
    D.rbestF[b] = bF;
    D.rbestT[b] = bT;
    D.rbestTs[b] = bTs;
    D.Flast[b] = Flast;
  }
}

template <bool K3, int GK, int NT, int RMAX, bool YLDS = false>
static hipError_t launch_sat_k(const SatDev& d, int64_t t0, int nsteps, hipStream_t s) {
  auto kern = sat_persistent<K3, NT, RMAX, YLDS, GK>;
  const size_t lds = align16s((size_t)d.n * 4) * (YLDS ? 2 : 1);
  hipError_t e =
      hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(d.B), dim3(NT), lds, s, d, t0, nsteps);
  return hipGetLastError();
}

// 1024 threads per restart (sixteen waves of gathers in flight) up to 8
// variables per thread in registers, up to 20 with y in LDS (n <= 20000, both
// arrays in the 160 KB); beyond that 512 threads with a larger register budget,
// whose per-variable state partly spills to scratch memory.
template <bool K3, int GK>
static hipError_t launch_sat_r(const SatDev& d, int64_t t0, int nsteps, hipStream_t s) {
  const int r = (d.n + 1023) / 1024;
  if (r <= 4) return launch_sat_k<K3, GK, 1024, 4>(d, t0, nsteps, s);
  if (r <= 8) return launch_sat_k<K3, GK, 1024, 8>(d, t0, nsteps, s);
  if (r <= 20 && 2 * align16s((size_t)d.n * 4) <= kSatYldsBudget)
    return launch_sat_k<K3, GK, 1024, 20, true>(d, t0, nsteps, s);
  const int r2 = (d.n + 511) / 512;
  if (r2 <= 40) return launch_sat_k<K3, GK, 512, 40>(d, t0, nsteps, s);
  if (r2 <= 64) return launch_sat_k<K3, GK, 512, 64>(d, t0, nsteps, s);
  return hipErrorInvalidValue;
}

// One kernel variant per kind of g (GK): read at run time, the kind would make
// the update evaluate both forms of g and g' for every coordinate.
hipError_t launch_sat_persistent(const SatDev& d, int64_t t0, int nsteps, hipStream_t s) {
  if (nsteps <= 0) return hipSuccess;
  if (d.gp.gkind == 0)
    return d.pinc3 ? launch_sat_r<true, 0>(d, t0, nsteps, s)
                  : launch_sat_r<false, 0>(d, t0, nsteps, s);
  return d.pinc3 ? launch_sat_r<true, 1>(d, t0, nsteps, s) : launch_sat_r<false, 1>(d, t0, nsteps, s);
}

// ---- adjoint at given points: gradient (mode 0) or Lagrangian backward (mode 1)

// One workgroup of kAdjNT threads per restart (sixteen waves per CU).
constexpr int kAdjNT = 1024;
template <int MODE>
__global__ void __launch_bounds__(kAdjNT)
    sat_adjoint_kernel(SatDev D, const float* __restrict__ X, int ldx, const float* __restrict__ Yv,
                       const float* __restrict__ dL, float* __restrict__ dx,
                       float* __restrict__ dy, int ldo, int use_lds) {
  extern __shared__ __attribute__((aligned(16))) float xs[];
  const int b = blockIdx.x, tid = threadIdx.x, n = D.n;
  const float* xb = X + (size_t)b * ldx;
  const float scale = MODE == 1 ? dL[b] : 1.f;
  if (use_lds && D.pinc3) {
    // 3-SAT: the persistent kernel's position space and interleaved lists,
    // x permuted into position order in LDS, results written by variable
    for (int p = tid; p < n; p += kAdjNT) xs[p] = xb[D.order[p]];
    __syncthreads();
    for (int p = tid; p < n; p += kAdjNT) {
      int64_t unused = 0;
      const int i = D.order[p];
      const float xi = xs[p];
      const float g = sat3_adjoint(D, xs, p, xi, false, unused) * D.ios;
      if (MODE == 0) {
        dx[(size_t)b * ldo + i] = g;
      } else {
        const float yi = Yv[(size_t)b * ldx + i];
        dx[(size_t)b * ldo + i] = scale * fmaf(yi, g_deriv(xi, D.gp.gkind, D.gp.deg), g);
        dy[(size_t)b * ldo + i] = scale * g_value(xi, D.gp.gkind, D.gp.deg);
      }
    }
    return;
  }
  const float* src = xb;
  if (use_lds) {
    for (int i = tid; i < n; i += kAdjNT) xs[i] = xb[i];
    __syncthreads();
    src = xs;
  }
  for (int i = tid; i < n; i += kAdjNT) {
    int64_t unused = 0;
    const float xi = src[i];
    const float g = sat_adjoint(D, src, i, xi, false, unused) * D.ios;
    if (MODE == 0) {
      dx[(size_t)b * ldo + i] = g;
    } else {
      const float yi = Yv[(size_t)b * ldx + i];
      dx[(size_t)b * ldo + i] = scale * fmaf(yi, g_deriv(xi, D.gp.gkind, D.gp.deg), g);
      dy[(size_t)b * ldo + i] = scale * g_value(xi, D.gp.gkind, D.gp.deg);
    }
  }
}

static hipError_t launch_adjoint(int mode, const SatDev& d, const float* X, int ldx,
                                 const float* Y, const float* dL, float* dx, float* dy, int ldo,
                                 int nb, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  size_t lds = 0;
  const int use_lds = sat_fits(d.n, &lds) ? 1 : 0;
  if (!use_lds) lds = 0;
  hipError_t e;
  if (mode == 0) {
    e = hipFuncSetAttribute((const void*)sat_adjoint_kernel<0>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sat_adjoint_kernel<0>, dim3(nb), dim3(kAdjNT), lds, s, d, X, ldx, Y, dL, dx,
                       dy, ldo, use_lds);
  } else {
    e = hipFuncSetAttribute((const void*)sat_adjoint_kernel<1>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sat_adjoint_kernel<1>, dim3(nb), dim3(kAdjNT), lds, s, d, X, ldx, Y, dL, dx,
                       dy, ldo, use_lds);
  }
  return hipGetLastError();
}

hipError_t launch_sat_grad(const SatDev& d, const float* X, int ldx, float* G, int nb,
                           hipStream_t s) {
  return launch_adjoint(0, d, X, ldx, nullptr, nullptr, G, nullptr, ldx, nb, s);
}

hipError_t launch_sat_bwd(const SatDev& d, const float* x, const float* y, const float* dL,
                          int nb, float* dx, float* dy, hipStream_t s) {
  return launch_adjoint(1, d, x, d.n, y, dL, dx, dy, d.n, nb, s);
}

// ---- clause-major passes: Lagrangian value and exact unsatisfied weight ----

// One workgroup of kFwdNT threads per restart; x of the restart is staged in
// LDS (use_lds) for the clauses' gathers.
constexpr int kFwdNT = 1024;
__global__ void __launch_bounds__(kFwdNT)
    sat_fwd_kernel(SatDev D, const float* __restrict__ x, const float* __restrict__ y,
                   float* __restrict__ L, int use_lds) {
  extern __shared__ __attribute__((aligned(16))) float xs[];
  __shared__ double red[kFwdNT / 64];
  const int b = blockIdx.x, tid = threadIdx.x;
  const float* xb = x + (size_t)b * D.n;
  const float* yb = y + (size_t)b * D.n;
  const float* src = xb;
  if (use_lds) {
    for (int i = tid; i < D.n; i += kFwdNT) xs[i] = xb[i];
    __syncthreads();
    src = xs;
  }
  double acc = 0.0;
  for (int j = tid; j < D.m; j += kFwdNT) {
    float prod = 1.f;
    for (int l = 0; l < D.k; ++l) {
      const int32_t code = D.lits[(size_t)j * D.k + l];
      const float xv = src[code & 0x7fffffff];
      prod *= code < 0 ? xv : 1.f - xv;
    }
    acc += (double)D.w[j] * (double)prod * (double)D.ios;
  }
  for (int i = tid; i < D.n; i += kFwdNT) acc += (double)yb[i] * (double)g_value(xb[i], D.gp.gkind, D.gp.deg);
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    for (int w = 0; w < kFwdNT / 64; ++w) tot += red[w];
    L[b] = (float)tot;
  }
}

hipError_t launch_sat_fwd(const SatDev& d, const float* x, const float* y, int nb, float* L,
                          hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  size_t lds = 0;
  const int use_lds = sat_fits(d.n, &lds) ? 1 : 0;
  if (!use_lds) lds = 0;
  hipError_t e = hipFuncSetAttribute((const void*)sat_fwd_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sat_fwd_kernel, dim3(nb), dim3(kFwdNT), lds, s, d, x, y, L, use_lds);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256)
    sat_eval_kernel(SatDev D, const int8_t* __restrict__ xr, int64_t* __restrict__ F) {
  __shared__ int64_t red[4];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int8_t* xb = xr + (size_t)b * D.ld;
  int64_t acc = 0;
  for (int j = tid; j < D.m; j += 256) {
    bool sat = false;
    for (int l = 0; l < D.k; ++l) {
      const int32_t code = D.lits[(size_t)j * D.k + l];
      sat = sat || ((xb[code & 0x7fffffff] != 0) != (code < 0));
    }
    if (!sat) acc += D.w[j];
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) F[b] = red[0] + red[1] + red[2] + red[3];
}

hipError_t launch_sat_eval(const SatDev& d, const int8_t* xr, int nb, int64_t* F,
                           hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(sat_eval_kernel, dim3(nb), dim3(256), 0, s, d, xr, F);
  return hipGetLastError();
}

}  // namespace pdbo
