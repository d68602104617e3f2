// Float64 weights on the row-parallel CSR path (Eq. 1 with real Q and c).
//
// The gradient is the one of spmm.hip with A/s stored in float32.  The
// objective of a rounded iterate has to be the exact real sum of the selected
// weights, rounded once.  Every finite float64 is an integer multiple of 2^e
// for e its lowest set bit, so with elo the lowest such bit over all weights
// the host writes the canonical A = offdiag(Q + Q^T) and c' = c + diag(Q)
// exactly as integers in units of 2^elo, split into ndig signed base-2^24
// digits.  The two halves of a canonical entry are added digit by digit
// without carries, so |digit| < 2^25 and one digit's sum over a restart's
// selected pairs fits in int64 (2^25 times at most 2^31 nonzeros).  Each digit
// is therefore reduced like the integer path's S and C (per workgroup in LDS,
// partials summed in a fixed order); the best-of-B kernel combines them into
//   N = S + 2 C = sum_d 2^(24 d) (S_d + 2 C_d),   F = N 2^(elo - 1),
// a 256-bit two's complement integer (ndig <= 8: |N| < 2^226), compares those
// exactly (the incumbent is the lexicographic minimum of (F, t, b) as for
// integers) and rounds F to float64 to nearest, ties to even.
#include <climits>

#include "common.h"

namespace pdbo {

constexpr int kRThreads = 256;
constexpr int kRBestThreads = 1024;

template <int GK, int MODE>
__global__ void __launch_bounds__(kRThreads) spmm_real_kernel(SpmmDev D, int parity, float* Gout) {
  __shared__ unsigned long long sred[2 * kMaxDigits][64];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int W = D.W, G = D.G, n = D.n, B = D.B, nd = D.ndig;
  const int g = lane / W, bl = lane - g * W;
  const int slice = blockIdx.x % D.nslices;
  const int gpw = D.grid / D.nslices;
  const int b = slice * W + bl;
  const bool bok = g < G && b < B;
  const int rows_per_wg = 4 * G;
  const int nrb = (n + rows_per_wg - 1) / rows_per_wg;
  const float* __restrict__ Xc = D.X[parity];
  float* __restrict__ Xn = D.X[parity ^ 1];
  if (MODE != 2)
    for (int k = tid; k < 2 * nd * 64; k += kRThreads) sred[k >> 6][k & 63] = 0;
  GdaP gp = D.gp;
  gp.gkind = GK;
  long long S[kMaxDigits], C[kMaxDigits];
#pragma unroll
  for (int d = 0; d < kMaxDigits; ++d) S[d] = C[d] = 0;
  for (int rb = blockIdx.x / D.nslices; rb < nrb; rb += gpw) {
    const int i = rb * rows_per_wg + wid * G + g;
    if (!bok || i >= n) continue;
    const int pe = D.row_ptr[i + 1];
    float acc = 0.f;
    long long r[kMaxDigits];
#pragma unroll
    for (int d = 0; d < kMaxDigits; ++d) r[d] = 0;
    // groups of four entries, the last padded with the row's last entry
    // (masked): their gathers are in flight together
    for (int p = D.row_ptr[i]; p < pe; p += 4) {
      float xk[4], a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = min(p + u, pe - 1);
        xk[u] = Xc[(size_t)D.col[q] * B + b];
        a[u] = D.valf[q];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool in = p + u < pe;
        acc = fmaf(in ? a[u] : 0.f, xk[u], acc);
        if (MODE != 2 && in && xk[u] > 0.5f) {
#pragma unroll
          for (int d = 0; d < kMaxDigits; ++d)
            if (d < nd) r[d] += D.Adig[(size_t)d * D.nnz + p + u];
        }
      }
    }
    const size_t off = (size_t)i * B + b;
    const float x = Xc[off];
    if (MODE != 2 && x > 0.5f) {
#pragma unroll
      for (int d = 0; d < kMaxDigits; ++d)
        if (d < nd) {
          S[d] += r[d];
          C[d] += D.Cdig[(size_t)d * n + i];
        }
    }
    if constexpr (MODE == 0) {
      float xn, yn;
      gda_update(x, D.Y[off], acc + D.cps[i], gp, xn, yn);
      Xn[off] = xn;
      D.Y[off] = yn;
    } else if constexpr (MODE == 2) {
      Gout[off] = acc + D.cps[i];
    }
  }
  if constexpr (MODE != 2) {
    __syncthreads();  // sred is cleared
    if (bok) {
      // two's complement: unsigned addition modulo 2^64 is the signed sum
#pragma unroll
      for (int d = 0; d < kMaxDigits; ++d)
        if (d < nd) {
          if (S[d]) atomicAdd(&sred[d][bl], (unsigned long long)S[d]);
          if (C[d]) atomicAdd(&sred[nd + d][bl], (unsigned long long)C[d]);
        }
    }
    __syncthreads();
    if (tid < W) {
      const int q = blockIdx.x / D.nslices;
      for (int j = 0; j < 2 * nd; ++j)
        D.part[((size_t)(slice * 2 * nd + j) * W + tid) * gpw + q] = (int64_t)sred[j][tid];
    }
  }
}

hipError_t launch_spmm_real(const SpmmDev& d, int mode, int parity, float* G, hipStream_t s) {
  const dim3 grid(d.grid), blk(kRThreads);
#define PDBO_R(GK, M) hipLaunchKernelGGL((spmm_real_kernel<GK, M>), grid, blk, 0, s, d, parity, G)
  const int gk = d.gp.gkind;
  if (mode == 1) {
    PDBO_R(0, 1);
  } else if (mode == 2) {
    PDBO_R(0, 2);
  } else if (gk == 0) {
    PDBO_R(0, 0);
  } else if (gk == 1) {
    PDBO_R(1, 0);
  } else {
    PDBO_R(2, 0);
  }
#undef PDBO_R
  return hipGetLastError();
}

// ---- 256-bit two's complement integers, four 64-bit words, low word first.
// Words are chosen with selects, not indexed, so that they stay in registers.

__device__ __forceinline__ uint64_t wsel(const uint64_t (&w)[4], int k) {
  return k == 0 ? w[0] : k == 1 ? w[1] : k == 2 ? w[2] : k == 3 ? w[3] : 0;
}

// w += v * 2^sh, 0 <= sh < 192
__device__ __forceinline__ void w_add(uint64_t (&w)[4], int64_t v, int sh) {
  const uint64_t ext = v < 0 ? ~0ull : 0ull;
  const int ws = sh >> 6, bs = sh & 63;
  uint64_t carry = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int j = k - ws;  // word j of the sign-extended v lands in word k
    const uint64_t hi = j < 0 ? 0 : (j == 0 ? (uint64_t)v : ext);
    const uint64_t lo = j < 1 ? 0 : (j == 1 ? (uint64_t)v : ext);
    const uint64_t t = bs ? (hi << bs) | (lo >> (64 - bs)) : hi;
    const uint64_t s1 = w[k] + t;
    const uint64_t c1 = s1 < t;
    const uint64_t s2 = s1 + carry;
    const uint64_t c2 = s2 < carry;
    w[k] = s2;
    carry = c1 | c2;
  }
}

__device__ __forceinline__ bool w_less(const uint64_t (&a)[4], const uint64_t (&b)[4]) {
  if (a[3] != b[3]) return (int64_t)a[3] < (int64_t)b[3];
  if (a[2] != b[2]) return a[2] < b[2];
  if (a[1] != b[1]) return a[1] < b[1];
  return a[0] < b[0];
}

__device__ __forceinline__ bool w_equal(const uint64_t (&a)[4], const uint64_t (&b)[4]) {
  return a[0] == b[0] && a[1] == b[1] && a[2] == b[2] && a[3] == b[3];
}

// N 2^E rounded to the nearest float64, ties to even (subnormal results
// rounded at 2^-1074, overflow to infinity).  E >= -1075.
__device__ double w_to_double(const uint64_t (&w)[4], int E) {
  const bool neg = (int64_t)w[3] < 0;
  uint64_t m[4];
  if (neg) {
    uint64_t carry = 1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint64_t t = ~w[k] + carry;
      carry = carry && t == 0;
      m[k] = t;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) m[k] = w[k];
  }
  int top = -1;  // highest set bit of |N|
#pragma unroll
  for (int k = 3; k >= 0; --k)
    if (top < 0 && m[k]) top = 64 * k + 63 - __clzll((long long)m[k]);
  if (top < 0) return 0.0;
  // keep the bits of weight >= 2^r of |N|: 53 significant bits, or down to
  // 2^-1074 for a subnormal result
  int r = top - 52;
  if (top + E < -1022) r = -1074 - E;
  double v;
  if (r <= 0) {
    v = ldexp((double)m[0], E);  // |N| < 2^53 here: exact
  } else {
    const int wr = r >> 6, off = r & 63;
    uint64_t q = wsel(m, wr) >> off;
    if (off) q |= wsel(m, wr + 1) << (64 - off);
    const int h = r - 1;  // the half bit; the sticky bits lie below it
    const uint64_t half = (wsel(m, h >> 6) >> (h & 63)) & 1;
    uint64_t sticky = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (64 * k + 64 <= h)
        sticky |= m[k];
      else if (64 * k < h)
        sticky |= m[k] & ((1ull << (h - 64 * k)) - 1);
    }
    if (half && (sticky || (q & 1))) ++q;
    v = ldexp((double)q, r + E);  // q <= 2^53: exact up to overflow
  }
  return neg ? -v : v;
}

constexpr int kRPartUnroll = 8;

__global__ void __launch_bounds__(kRBestThreads)
    spmm_real_best_kernel(SpmmDev D, int parity, int advance, double* Fout, int nb) {
  constexpr int NW = kRBestThreads / 64;
  __shared__ uint64_t sW[NW][4];
  __shared__ int sb[NW];
  __shared__ int win;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int64_t t = *D.t_dev;
  const int gpw = D.grid / D.nslices;
  const int nd = D.ndig;
  const int Bn = Fout ? nb : D.B;
  uint64_t incw[4] = {0, 0, 0, 0};
  int len = 0;
  if (tid == 0 && !Fout) {
#pragma unroll
    for (int k = 0; k < 4; ++k) incw[k] = D.incw[k];
    len = *D.trace_len;
  }
  uint64_t bw[4] = {~0ull, ~0ull, ~0ull, ~0ull >> 1};  // largest positive
  int bestb = INT_MAX;
  for (int b = wid; b < Bn; b += NW) {  // one wave per restart, fixed order
    const int slice = b / D.W, bl = b - slice * D.W;
    uint64_t w[4] = {0, 0, 0, 0};
    for (int d = 0; d < nd; ++d) {
      const int64_t* pS = D.part + ((size_t)(slice * 2 * nd + d) * D.W + bl) * gpw;
      const int64_t* pC = D.part + ((size_t)(slice * 2 * nd + nd + d) * D.W + bl) * gpw;
      int64_t Sd = 0, Cd = 0;
      for (int q0 = lane; q0 < gpw; q0 += 64 * kRPartUnroll) {
        int64_t a[kRPartUnroll], c[kRPartUnroll];
#pragma unroll
        for (int u = 0; u < kRPartUnroll; ++u) {
          const int q = q0 + u * 64;
          a[u] = q < gpw ? pS[q] : 0;
          c[u] = q < gpw ? pC[q] : 0;
        }
#pragma unroll
        for (int u = 0; u < kRPartUnroll; ++u) {
          Sd += a[u];
          Cd += c[u];
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        Sd += __shfl_xor(Sd, o);
        Cd += __shfl_xor(Cd, o);
      }
      w_add(w, Sd + 2 * Cd, 24 * d);  // every lane holds the same totals
    }
    if (lane == 0) {
      const double F = w_to_double(w, D.elo - 1);
      if (Fout)
        Fout[b] = F;
      else
        D.Fd[b] = F;
    }
    if (w_less(w, bw)) {  // increasing b per wave: the first minimum is kept
#pragma unroll
      for (int k = 0; k < 4; ++k) bw[k] = w[k];
      bestb = b;
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) sW[wid][k] = bw[k];
    sb[wid] = bestb;
  }
  __syncthreads();
  if (tid == 0) {
    for (int v = 1; v < NW; ++v) {
      uint64_t o[4] = {sW[v][0], sW[v][1], sW[v][2], sW[v][3]};
      if (sb[v] != INT_MAX && (w_less(o, bw) || (w_equal(o, bw) && sb[v] < bestb))) {
#pragma unroll
        for (int k = 0; k < 4; ++k) bw[k] = o[k];
        bestb = sb[v];
      }
    }
    int improved = 0;
    if (!Fout && t >= 1 && bestb != INT_MAX && w_less(bw, incw)) {
      const uint64_t ts = wall_clock();
      const double F = w_to_double(bw, D.elo - 1);
      int64_t Fbits;
      __builtin_memcpy(&Fbits, &F, sizeof(F));
#pragma unroll
      for (int k = 0; k < 4; ++k) D.incw[k] = bw[k];
      D.inc->F = Fbits;
      D.inc->t = t;
      D.inc->b = bestb;
      D.inc->ts = ts;
      if (len < D.trace_cap) {
        D.trace[len] = TraceRec{t, Fbits, (int64_t)bestb, ts};
        *D.trace_len = len + 1;
      }
      improved = 1;
    }
    win = improved ? bestb : -1;
    if (!Fout && advance) *D.t_dev = t + 1;
  }
  __syncthreads();
  if (win >= 0) {  // eight strided loads in flight per thread
    const float* X = D.X[parity];
    constexpr int U = 8;
    for (int i0 = tid; i0 < D.n; i0 += U * kRBestThreads) {
      float v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = min(i0 + u * kRBestThreads, D.n - 1);
        v[u] = X[(size_t)i * D.B + win];
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (i0 + u * kRBestThreads < D.n) D.best_x[i0 + u * kRBestThreads] = (uint8_t)(v[u] > 0.5f);
    }
  }
}

hipError_t launch_spmm_real_best(const SpmmDev& d, int parity, int advance, double* Fout, int nb,
                                 hipStream_t s) {
  hipLaunchKernelGGL(spmm_real_best_kernel, dim3(1), dim3(kRBestThreads), 0, s, d, parity, advance,
                     Fout, nb);
  return hipGetLastError();
}

__global__ void real_load_x_kernel(const uint8_t* __restrict__ xr, int nb, SpmmDev D, int parity) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;  // (i, b) node-major
  if (idx >= (size_t)D.n * D.B) return;
  const int i = (int)(idx / D.B), b = (int)(idx % D.B);
  D.X[parity][idx] = (b < nb && xr[(size_t)b * D.n + i]) ? 1.f : 0.f;
}

hipError_t launch_real_load_x(const uint8_t* xr, int nb, const SpmmDev& d, int parity,
                              hipStream_t s) {
  const size_t tot = (size_t)d.n * d.B;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(real_load_x_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, xr,
                     nb, d, parity);
  return hipGetLastError();
}

}  // namespace pdbo
