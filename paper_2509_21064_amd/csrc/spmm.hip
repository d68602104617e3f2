// Sparse QUBO path without restart residency: one launch per iteration.
//
// The restart-resident kernel of sparse.hip keeps x of one restart in LDS and
// gives each restart a workgroup.  That stops working when x of one restart
// exceeds LDS (n > 32768) and wastes the chip when there are few restarts (the
// paper runs MIS with B = 10 restarts, App. C).  Here every iteration is one
// launch over all rows of the canonical CSR matrix Ahat = offdiag(Q + Q^T)/kappa
// with the iterates node-major ([n][B]): a group of W adjacent lanes owns one
// row i and W restarts, so the gather of x_j reads W contiguous floats for all
// of them, and the update of (x_i, y_i) writes W contiguous floats.
//
// The same gathers give the gradient of x^t (Alg. 1) and the exact objective
// of round(x^t): with E_i = sum_j Ahat_ij [x_j > 1/2] in integers,
// F = (kappa/2) sum_i x_r,i E_i + sum_i c'_i x_r,i.  Each workgroup reduces
// its rows' contributions per restart in LDS (integer atomics, so the order
// does not matter) and stores them once; spmm_best_kernel adds the
// workgroups' partials in a fixed order, takes the first argmin over the
// restarts and updates the incumbent (strict improvement, so the earliest
// iteration wins ties), copying the winning rounded vector from x^t.
#include <climits>

#include "common.h"

namespace pdbo {

constexpr int kSpmmThreads = 256;  // four waves
constexpr int kSpmmUnroll = 8;     // gathers in flight per lane

// PK: the entries are read as packed words (D.packed), one load instead of two.
template <int GK, int MODE, bool PK>
__global__ void __launch_bounds__(kSpmmThreads) spmm_kernel(SpmmDev D, int parity, float* Gout) {
  __shared__ unsigned long long sred[2][64];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int W = D.W, G = D.G, n = D.n, B = D.B;
  const int g = lane / W, bl = lane - g * W;
  const int slice = blockIdx.x % D.nslices;
  const int gpw = D.grid / D.nslices;  // workgroups per slice
  const int b = slice * W + bl;
  const bool bok = g < G && b < B;
  const int rows_per_wg = 4 * G;
  const int nrb = (n + rows_per_wg - 1) / rows_per_wg;
  const float* __restrict__ Xc = D.X[parity];
  float* __restrict__ Xn = D.X[parity ^ 1];
  const int32_t* __restrict__ rp = D.row_ptr;
  const int32_t* __restrict__ col = D.col;
  const int32_t* __restrict__ val = D.val;
  const uint32_t* __restrict__ pk = D.packed;
  if (MODE != 2 && tid < 128) sred[tid >> 6][tid & 63] = 0;
  // the previous iteration's new incumbent, still in Xn (see SpmmDev::win)
  const int win = (MODE == 0 && D.win) ? *D.win : -1;
  GdaP gp = D.gp;
  gp.gkind = GK;
  long long S = 0, C = 0;
  for (int rb = blockIdx.x / D.nslices; rb < nrb; rb += gpw) {
    const int i = rb * rows_per_wg + wid * G + g;
    if (!bok || i >= n) continue;
    const int pe = rp[i + 1];
    int p = rp[i];
    float acc = 0.f;
    int accr = 0;
    for (; p + kSpmmUnroll <= pe; p += kSpmmUnroll) {
      int c[kSpmmUnroll], v[kSpmmUnroll];
      float xk[kSpmmUnroll];
#pragma unroll
      for (int u = 0; u < kSpmmUnroll; ++u) {
        if constexpr (PK) {
          const uint32_t e = pk[p + u];
          c[u] = (int)(e & 0xffffu);
          v[u] = (int)(int16_t)(e >> 16);
        } else {
          c[u] = col[p + u];
          v[u] = val[p + u];
        }
      }
#pragma unroll
      for (int u = 0; u < kSpmmUnroll; ++u) xk[u] = Xc[(size_t)c[u] * B + b];
#pragma unroll
      for (int u = 0; u < kSpmmUnroll; ++u) {
        acc = fmaf((float)v[u], xk[u], acc);
        accr += xk[u] > 0.5f ? v[u] : 0;
      }
    }
    if (p < pe) {  // the rest of the row in one group, padded with its last entry at value 0
      int c[kSpmmUnroll], v[kSpmmUnroll];
      float xk[kSpmmUnroll];
#pragma unroll
      for (int u = 0; u < kSpmmUnroll; ++u) {
        const int q = min(p + u, pe - 1);
        if constexpr (PK) {
          const uint32_t e = pk[q];
          c[u] = (int)(e & 0xffffu);
          v[u] = p + u < pe ? (int)(int16_t)(e >> 16) : 0;
        } else {
          c[u] = col[q];
          v[u] = p + u < pe ? val[q] : 0;
        }
      }
#pragma unroll
      for (int u = 0; u < kSpmmUnroll; ++u) xk[u] = Xc[(size_t)c[u] * B + b];
#pragma unroll
      for (int u = 0; u < kSpmmUnroll; ++u) {
        acc = fmaf((float)v[u], xk[u], acc);
        accr += xk[u] > 0.5f ? v[u] : 0;
      }
    }
    const size_t off = (size_t)i * B + b;
    const float x = Xc[off];
    if constexpr (MODE != 2) {
      if (x > 0.5f) {
        S += accr;
        C += D.cp[i];
      }
    }
    if constexpr (MODE == 0) {
      float xn, yn;
      gda_update(x, D.Y[off], fmaf(D.kos, acc, D.cps[i]), gp, xn, yn);
      if (b == win) D.best_x[i] = (uint8_t)(Xn[off] > 0.5f);  // about to be overwritten
      Xn[off] = xn;
      D.Y[off] = yn;
    } else if constexpr (MODE == 2) {
      Gout[off] = fmaf(D.kos, acc, D.cps[i]);
    }
  }
  if constexpr (MODE != 2) {
    __syncthreads();  // sred is cleared
    if (bok) {
      // two's complement: unsigned addition modulo 2^64 is the signed sum
      if (S) atomicAdd(&sred[0][bl], (unsigned long long)S);
      if (C) atomicAdd(&sred[1][bl], (unsigned long long)C);
    }
    __syncthreads();
    if (tid < W) {  // partials of restart (slice, tid) are contiguous over the workgroups
      const int q = blockIdx.x / D.nslices;
      D.part[((size_t)(slice * 2 + 0) * W + tid) * gpw + q] = (int64_t)sred[0][tid];
      D.part[((size_t)(slice * 2 + 1) * W + tid) * gpw + q] = (int64_t)sred[1][tid];
    }
  }
}

hipError_t launch_spmm(const SpmmDev& d, int mode, int parity, float* G, hipStream_t s) {
  if (d.ndig > 0) return launch_spmm_real(d, mode, parity, G, s);
  const dim3 grid(d.grid), blk(kSpmmThreads);
#define PDBO_S(GK, M)                                                                  \
  if (d.packed)                                                                        \
    hipLaunchKernelGGL((spmm_kernel<GK, M, true>), grid, blk, 0, s, d, parity, G);     \
  else                                                                                 \
    hipLaunchKernelGGL((spmm_kernel<GK, M, false>), grid, blk, 0, s, d, parity, G)
  const int gk = d.gp.gkind;
  if (mode == 1) {
    PDBO_S(0, 1);
  } else if (mode == 2) {
    PDBO_S(0, 2);
  } else if (gk == 0) {
    PDBO_S(0, 0);
  } else if (gk == 1) {
    PDBO_S(1, 0);
  } else {
    PDBO_S(2, 0);
  }
#undef PDBO_S
  return hipGetLastError();
}

constexpr int kBestThreads = 1024;
constexpr int kPartUnroll = 16;  // partials per lane loaded in one batch

__global__ void __launch_bounds__(kBestThreads) spmm_best_kernel(SpmmDev D, int parity,
                                                                 int advance) {
  __shared__ int64_t sF[kBestThreads / 64];
  __shared__ int sb[kBestThreads / 64];
  __shared__ int win, pend;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int64_t t = *D.t_dev;  // the evaluated iterate is x^t
  const int pend0 = D.win ? *D.win : -1;  // a winner no step launch has copied yet
  const int gpw = D.grid / D.nslices;
  int64_t bestF = LLONG_MAX;
  int bestb = INT_MAX;
  // the incumbent and the trace length travel with the partials' loads
  int64_t incF = 0;
  int len = 0;
  if (tid == 0) {
    incF = D.inc->F;
    len = *D.trace_len;
  }
  // one wave per restart: the lanes add the workgroups' partials (contiguous)
  // in a fixed order, so the totals are the same on every run
  for (int b = wid; b < D.B; b += kBestThreads / 64) {
    const int slice = b / D.W, bl = b - slice * D.W;
    const int64_t* pS = D.part + ((size_t)(slice * 2 + 0) * D.W + bl) * gpw;
    const int64_t* pC = D.part + ((size_t)(slice * 2 + 1) * D.W + bl) * gpw;
    int64_t S = 0, C = 0;
    for (int q0 = lane; q0 < gpw; q0 += 64 * kPartUnroll) {  // loads of a batch in flight together
      int64_t a[kPartUnroll], c[kPartUnroll];
#pragma unroll
      for (int u = 0; u < kPartUnroll; ++u) {
        const int q = q0 + u * 64;
        a[u] = q < gpw ? pS[q] : 0;
        c[u] = q < gpw ? pC[q] : 0;
      }
#pragma unroll
      for (int u = 0; u < kPartUnroll; ++u) {
        S += a[u];
        C += c[u];
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      S += __shfl_xor(S, o);
      C += __shfl_xor(C, o);
    }
    const int64_t F = (D.kappa == 2 ? S : S / 2) + C;
    if (lane == 0) D.Flast[b] = F;
    if (F < bestF) {  // increasing b per wave: the first minimum is kept
      bestF = F;
      bestb = b;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int64_t F2 = __shfl_xor(bestF, o);
    const int b2 = __shfl_xor(bestb, o);
    if (F2 < bestF || (F2 == bestF && b2 < bestb)) {
      bestF = F2;
      bestb = b2;
    }
  }
  if (lane == 0) {
    sF[wid] = bestF;
    sb[wid] = bestb;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < kBestThreads / 64; ++w)
      if (sF[w] < bestF || (sF[w] == bestF && sb[w] < bestb)) {
        bestF = sF[w];
        bestb = sb[w];
      }
    int improved = 0;
    if (t >= 1 && bestb != INT_MAX && bestF < incF) {
      const uint64_t ts = wall_clock();
      D.inc->F = bestF;
      D.inc->t = t;
      D.inc->b = bestb;
      D.inc->ts = ts;
      if (len < D.trace_cap) {
        D.trace[len] = TraceRec{t, bestF, (int64_t)bestb, ts};
        *D.trace_len = len + 1;
      }
      improved = 1;
    }
    win = improved ? bestb : -1;
    pend = -1;
    if (advance) *D.t_dev = t + 1;
    if (D.win) {
      if (advance) {  // the next step launch copies the winner while it overwrites X[parity]
        *D.win = win;
        win = -1;
      } else {  // the last launch of a call: a pending winner too
        pend = pend0;
        *D.win = -1;
      }
    }
  }
  __syncthreads();
  // copies made here: first a pending winner of the previous iteration (in the
  // other buffer, which no step launch has overwritten yet), then this one's
  for (int pass = 0; pass < 2; ++pass) {
    const int wb = pass == 0 ? pend : win;
    if (wb < 0) continue;
    const float* X = D.X[pass == 0 ? parity ^ 1 : parity];
    constexpr int U = 8;  // eight strided loads in flight per thread
    for (int i0 = tid; i0 < D.n; i0 += U * kBestThreads) {
      float v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = min(i0 + u * kBestThreads, D.n - 1);
        v[u] = X[(size_t)i * D.B + wb];
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (i0 + u * kBestThreads < D.n) D.best_x[i0 + u * kBestThreads] = (uint8_t)(v[u] > 0.5f);
    }
    __syncthreads();  // the second copy overwrites the first
  }
}

hipError_t launch_spmm_best(const SpmmDev& d, int parity, int advance, hipStream_t s) {
  if (d.ndig > 0) return launch_spmm_real_best(d, parity, advance, nullptr, 0, s);
  hipLaunchKernelGGL(spmm_best_kernel, dim3(1), dim3(kBestThreads), 0, s, d, parity, advance);
  return hipGetLastError();
}

// X^0 (node-major) from the caller's restart-major x0, or drawn by the
// library's generator (same counters as the restart-major paths); Y^0 = y0.
__global__ void spmm_init_kernel(const double* __restrict__ x0, SpmmDev D, float y0,
                                 uint64_t seed) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)D.B * D.n) return;
  const int b = (int)(idx / D.n), i = (int)(idx % D.n);
  const size_t off = (size_t)i * D.B + b;
  D.X[0][off] = x0 ? (float)x0[idx] : philox_start(seed, (uint32_t)b, (uint32_t)i);
  D.Y[off] = y0;
}

hipError_t launch_spmm_init(const double* x0, const SpmmDev& d, float y0, uint64_t seed,
                            hipStream_t s) {
  const size_t tot = (size_t)d.B * d.n;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(spmm_init_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, x0, d,
                     y0, seed);
  return hipGetLastError();
}

}  // namespace pdbo
