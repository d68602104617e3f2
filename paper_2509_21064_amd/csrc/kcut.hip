// Max-k-Cut through the softmax reparametrisation (App. B).
//
// Node i of a restart carries k logits Z_{:,i}; its category probabilities are
// X_{:,i} = softmax(Z_{:,i}) on the simplex.  The objective is
// Tr(X W X^T) = sum_{i,j} W_ij X_{:,i} . X_{:,j} (minimised; on one-hot X it is
// twice the weight of the edges inside the parts), with the Lagrangian
// L = Tr(X W X^T)/s + sum_i y_i g(X_{:,i}) for g quadratic (sum_c X_ci^2 - 1)
// or entropy (sum_c X_ci log X_ci).  Simultaneous gradient descent-ascent on
// (Z, y): with G = dL/dX, G_ci = (2/s) (X W)_ci + y_i dg/dX_ci, the chain rule
// through the softmax gives dL/dZ_ci = X_ci (G_ci - sum_c' X_c'i G_c'i), and
// y_i gains beta g(X_{:,i}) at the old X.  The rounded assignment puts node i
// in argmax_c X_ci (the lowest c on ties).
//
// Layout and kernel structure follow the row-parallel CSR path (spmm.hip):
// node-major [n][B][k] arrays, a group of W adjacent lanes owns one row and W
// restarts, each lane holds its restart's k values in registers, and the
// gathers of row i also count the weight of the edges whose ends share the
// rounded category (the exact objective of the rounded X^t).
#include <climits>

#include "common.h"

namespace pdbo {

constexpr int kKcutThreads = 256;
constexpr int kKcutUnroll = 4;  // neighbours whose loads are in flight together

template <int K>
__device__ __forceinline__ int argmax_k(const float (&x)[K]) {
  int c = 0;
#pragma unroll
  for (int u = 1; u < K; ++u)
    if (x[u] > x[c]) c = u;
  return c;
}

template <int K>
__device__ __forceinline__ void softmax_k(const float (&z)[K], float (&x)[K]) {
  float m = z[0];
#pragma unroll
  for (int u = 1; u < K; ++u) m = fmaxf(m, z[u]);
  float t = 0.f;
#pragma unroll
  for (int u = 0; u < K; ++u) {
    x[u] = expf(z[u] - m);
    t += x[u];
  }
  const float r = 1.f / t;
#pragma unroll
  for (int u = 0; u < K; ++u) x[u] *= r;
}

// g of one node's probabilities and its partial derivatives
template <int GK, int K>
__device__ __forceinline__ float kg_value(const float (&x)[K]) {
  float v = 0.f;
#pragma unroll
  for (int u = 0; u < K; ++u) v += GK == 0 ? x[u] * x[u] : (x[u] > 0.f ? x[u] * logf(x[u]) : 0.f);
  return GK == 0 ? v - 1.f : v;
}

template <int GK>
__device__ __forceinline__ float kg_deriv(float x) {
  return GK == 0 ? 2.f * x : logf(fmaxf(x, kEntropyEps)) + 1.f;
}

// MODE 0: gradient, the update of (Z, X, Y) and the objective of round(X^t);
// MODE 1: the objective only; MODE 2: the gradient of f/s with respect to Z
// into Gout (node-major).
template <int K, int GK, int MODE>
__global__ void __launch_bounds__(kKcutThreads) kcut_kernel(KcutDev D, int parity, float* Gout) {
  __shared__ unsigned long long sred[64];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int W = D.W, G = D.G, n = D.n, B = D.B;
  const int g = lane / W, bl = lane - g * W;
  const int slice = blockIdx.x % D.nslices;
  const int gpw = D.grid / D.nslices;
  const int b = slice * W + bl;
  const bool bok = g < G && b < B;
  const int rows_per_wg = 4 * G;
  const int nrb = (n + rows_per_wg - 1) / rows_per_wg;
  const float* __restrict__ Xc = D.X[parity];
  float* __restrict__ Xn = D.X[parity ^ 1];
  if (MODE != 2 && tid < 64) sred[tid] = 0;
  // the previous iteration's new incumbent, still in Xn (see KcutDev::win)
  const int win = MODE == 0 ? *D.win : -1;
  long long S = 0;
  for (int rb = blockIdx.x / D.nslices; rb < nrb; rb += gpw) {
    const int i = rb * rows_per_wg + wid * G + g;
    if (!bok || i >= n) continue;
    const size_t off = ((size_t)i * B + b) * K;
    float xi[K], acc[K];
#pragma unroll
    for (int u = 0; u < K; ++u) {
      xi[u] = Xc[off + u];
      acc[u] = 0.f;
    }
    const int ci = argmax_k<K>(xi);
    int same = 0;
    const int pe = D.row_ptr[i + 1];
    // groups of kKcutUnroll neighbours, the last one padded with the row's
    // last entry at weight 0 (same addresses): their loads are in flight together
    for (int p = D.row_ptr[i]; p < pe; p += kKcutUnroll) {
      int wv[kKcutUnroll];
      float v[kKcutUnroll][K];
#pragma unroll
      for (int e = 0; e < kKcutUnroll; ++e) {
        const int q = min(p + e, pe - 1);
        const int j = D.col[q];
        wv[e] = p + e < pe ? D.w[q] : 0;
        const float* xj = Xc + ((size_t)j * B + b) * K;
#pragma unroll
        for (int u = 0; u < K; ++u) v[e][u] = xj[u];
      }
#pragma unroll
      for (int e = 0; e < kKcutUnroll; ++e) {
#pragma unroll
        for (int u = 0; u < K; ++u) acc[u] = fmaf((float)wv[e], v[e][u], acc[u]);
        same += argmax_k<K>(v[e]) == ci ? wv[e] : 0;
      }
    }
    if constexpr (MODE != 2) S += same;
    if constexpr (MODE == 0) {
      const float y = D.Y[(size_t)i * B + b];
      float gr[K], m = 0.f;
#pragma unroll
      for (int u = 0; u < K; ++u) {
        gr[u] = fmaf(D.tos, acc[u], y * kg_deriv<GK>(xi[u]));
        m = fmaf(xi[u], gr[u], m);
      }
      float z[K], xn[K];
#pragma unroll
      for (int u = 0; u < K; ++u) {
        z[u] = D.Z[off + u];
        z[u] = fmaf(-D.gp.alpha, xi[u] * (gr[u] - m), z[u]);
        D.Z[off + u] = z[u];
      }
      softmax_k<K>(z, xn);
      if (b == win) {  // this lane is about to overwrite the incumbent's probabilities
        float xw[K];
#pragma unroll
        for (int u = 0; u < K; ++u) xw[u] = Xn[off + u];
        D.best_x[i] = (uint8_t)argmax_k<K>(xw);
      }
#pragma unroll
      for (int u = 0; u < K; ++u) Xn[off + u] = xn[u];
      D.Y[(size_t)i * B + b] = fmaf(D.gp.beta, kg_value<GK, K>(xi), y);
    } else if constexpr (MODE == 2) {
      float m = 0.f;
#pragma unroll
      for (int u = 0; u < K; ++u) m = fmaf(xi[u], D.tos * acc[u], m);
#pragma unroll
      for (int u = 0; u < K; ++u) Gout[off + u] = xi[u] * (D.tos * acc[u] - m);
    }
  }
  if constexpr (MODE != 2) {
    __syncthreads();
    if (bok && S) atomicAdd(&sred[bl], (unsigned long long)S);
    __syncthreads();
    if (tid < W) D.part[((size_t)slice * W + tid) * gpw + blockIdx.x / D.nslices] = (int64_t)sred[tid];
  }
}

template <int K>
static void launch_kcut_k(const KcutDev& d, int mode, int parity, float* G, hipStream_t s) {
  const dim3 grid(d.grid), blk(kKcutThreads);
  if (mode == 1)
    hipLaunchKernelGGL((kcut_kernel<K, 0, 1>), grid, blk, 0, s, d, parity, G);
  else if (mode == 2)
    hipLaunchKernelGGL((kcut_kernel<K, 0, 2>), grid, blk, 0, s, d, parity, G);
  else if (d.gp.gkind == 0)
    hipLaunchKernelGGL((kcut_kernel<K, 0, 0>), grid, blk, 0, s, d, parity, G);
  else
    hipLaunchKernelGGL((kcut_kernel<K, 1, 0>), grid, blk, 0, s, d, parity, G);
}

hipError_t launch_kcut(const KcutDev& d, int mode, int parity, float* G, hipStream_t s) {
  switch (d.k) {
    case 2: launch_kcut_k<2>(d, mode, parity, G, s); break;
    case 3: launch_kcut_k<3>(d, mode, parity, G, s); break;
    case 4: launch_kcut_k<4>(d, mode, parity, G, s); break;
    case 5: launch_kcut_k<5>(d, mode, parity, G, s); break;
    case 6: launch_kcut_k<6>(d, mode, parity, G, s); break;
    case 7: launch_kcut_k<7>(d, mode, parity, G, s); break;
    case 8: launch_kcut_k<8>(d, mode, parity, G, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

constexpr int kKBestThreads = 1024;
constexpr int kKPartUnroll = 16;  // partials per lane loaded in one batch

// Objectives F_b = (sum of the rows' same-category weights) / 2 (each edge is
// seen from both ends), first argmin, incumbent with strict improvement, and
// the winner's categories copied from X[parity].
template <int K>
__global__ void __launch_bounds__(kKBestThreads) kcut_best_kernel(KcutDev D, int parity,
                                                                  int advance) {
  __shared__ int64_t sF[kKBestThreads / 64];
  __shared__ int sb[kKBestThreads / 64];
  __shared__ int win, pend;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int64_t t = *D.t_dev;
  const int pend0 = *D.win;  // a winner the step launches have not copied yet
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
  for (int b = wid; b < D.B; b += kKBestThreads / 64) {  // one wave per restart, fixed order
    const int slice = b / D.W, bl = b - slice * D.W;
    const int64_t* pS = D.part + ((size_t)slice * D.W + bl) * gpw;
    int64_t S = 0;
    for (int q0 = lane; q0 < gpw; q0 += 64 * kKPartUnroll) {  // loads of a batch in flight together
      int64_t a[kKPartUnroll];
#pragma unroll
      for (int u = 0; u < kKPartUnroll; ++u) {
        const int q = q0 + u * 64;
        a[u] = q < gpw ? pS[q] : 0;
      }
#pragma unroll
      for (int u = 0; u < kKPartUnroll; ++u) S += a[u];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) S += __shfl_xor(S, o);
    const int64_t F = S / 2;
    if (lane == 0) D.Flast[b] = F;
    if (F < bestF) {
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
    for (int w = 1; w < kKBestThreads / 64; ++w)
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
    if (advance) {
      // the next step launch copies the winner while it overwrites X[parity]
      *D.t_dev = t + 1;
      *D.win = win;
    } else {
      pend = pend0;
      *D.win = -1;
    }
  }
  __syncthreads();
  // the last launch of a call copies at once: first a pending winner of the
  // previous iteration (in the other buffer, which no step launch has
  // overwritten yet), then its own
  for (int pass = 0; pass < 2; ++pass) {
    const int wb = pass == 0 ? pend : win;
    if (advance || wb < 0) continue;
    const float* X = D.X[pass == 0 ? parity ^ 1 : parity];
    constexpr int U = 8;  // eight nodes' K loads in flight per thread
    for (int i0 = tid; i0 < D.n; i0 += U * kKBestThreads) {
      float v[U][K];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const float* x = X + ((size_t)min(i0 + u * kKBestThreads, D.n - 1) * D.B + wb) * K;
#pragma unroll
        for (int c = 0; c < K; ++c) v[u][c] = x[c];
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (i0 + u * kKBestThreads < D.n) D.best_x[i0 + u * kKBestThreads] = (uint8_t)argmax_k<K>(v[u]);
    }
    __syncthreads();  // the second copy overwrites the first
  }
}

hipError_t launch_kcut_best(const KcutDev& d, int parity, int advance, hipStream_t s) {
#define PDBO_KB(KK) \
  hipLaunchKernelGGL(kcut_best_kernel<KK>, dim3(1), dim3(kKBestThreads), 0, s, d, parity, advance)
  switch (d.k) {
    case 2: PDBO_KB(2); break;
    case 3: PDBO_KB(3); break;
    case 4: PDBO_KB(4); break;
    case 5: PDBO_KB(5); break;
    case 6: PDBO_KB(6); break;
    case 7: PDBO_KB(7); break;
    case 8: PDBO_KB(8); break;
    default: return hipErrorInvalidValue;
  }
#undef PDBO_KB
  return hipGetLastError();
}

// Z (node-major) from z, a restart-major (B, n, k) array (device; float64 at
// init, float32 for set_state), or drawn by the library's generator with
// coordinate index i k + c; X = softmax(Z) into X[parity]; Y = y0 unless y
// (restart-major (B, n) float32) is given.
template <typename T>
__global__ void kcut_state_kernel(const T* __restrict__ z, const float* __restrict__ y, KcutDev D,
                                  int parity, float y0, uint64_t seed, int set_y) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;  // (b, i)
  if (idx >= (size_t)D.B * D.n) return;
  const int b = (int)(idx / D.n), i = (int)(idx % D.n);
  const int K = D.k;
  const size_t off = ((size_t)i * D.B + b) * K;
  float zz[8], mx = -INFINITY;
  for (int u = 0; u < K; ++u) {
    zz[u] = z ? (float)z[idx * K + u] : philox_start(seed, (uint32_t)b, (uint32_t)(i * K + u));
    mx = fmaxf(mx, zz[u]);
  }
  float t = 0.f;
  for (int u = 0; u < K; ++u) t += expf(zz[u] - mx);
  const float r = 1.f / t;
  for (int u = 0; u < K; ++u) {
    D.Z[off + u] = zz[u];
    D.X[parity][off + u] = expf(zz[u] - mx) * r;
  }
  if (set_y) D.Y[(size_t)i * D.B + b] = y ? y[idx] : y0;
}

hipError_t launch_kcut_init(const double* z0, const KcutDev& d, float y0, uint64_t seed,
                            hipStream_t s) {
  const size_t tot = (size_t)d.B * d.n;
  hipLaunchKernelGGL((kcut_state_kernel<double>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                     s, z0, (const float*)nullptr, d, 0, y0, seed, 1);
  return hipGetLastError();
}

hipError_t launch_kcut_set(const float* z, const float* y, const KcutDev& d, int parity,
                           hipStream_t s) {
  const size_t tot = (size_t)d.B * d.n;
  hipLaunchKernelGGL((kcut_state_kernel<float>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                     s, z, y, d, parity, 0.f, 0ull, y ? 1 : 0);
  return hipGetLastError();
}

// Exact objective of given category vectors (restart-major (nb, n) bytes):
// the weight of the edges whose ends share a category, each edge once.
__global__ void __launch_bounds__(256) kcut_eval_kernel(KcutDev D, const uint8_t* __restrict__ cat,
                                                        int64_t* __restrict__ F) {
  __shared__ int64_t red[4];
  const int b = blockIdx.x, tid = threadIdx.x;
  const uint8_t* cb = cat + (size_t)b * D.n;
  int64_t acc = 0;
  for (int i = tid; i < D.n; i += 256)
    for (int p = D.row_ptr[i]; p < D.row_ptr[i + 1]; ++p)
      if (D.col[p] > i && cb[D.col[p]] == cb[i]) acc += D.w[p];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) F[b] = red[0] + red[1] + red[2] + red[3];
}

hipError_t launch_kcut_eval(const KcutDev& d, const uint8_t* cat, int nb, int64_t* F,
                            hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(kcut_eval_kernel, dim3(nb), dim3(256), 0, s, d, cat, F);
  return hipGetLastError();
}

}  // namespace pdbo
