// Dual certificate: a lower bound on min F over {0,1}^n (App. D, Dual
// Certificate).
//
// For any y, the minimum of L(., y) over the box [0,1]^n is at most its
// minimum over {0,1}^n, where g vanishes and L = F/s; so s * min_box L(., y)
// bounds min F from below (the weak duality in the proof of Thm. 3.2).  When
// L(., y) is convex (for the quadratic g and y = ybar * 1: A/s + 2 ybar I
// positive semidefinite), any box point x gives a certified value of that
// minimum from below, L(x) + min over z in the box of grad L(x) . (z - x):
// the linearisation of a convex function lies below it, and the linear term is
// minimised coordinate by coordinate at z_i = 0 or 1.
//
// These kernels evaluate that bound at one point x in float64 with the exact
// integer Ahat (int8 limbs or CSR values).  Each row product sum_j Ahat_ij x_j
// carries the classical bound gamma_n sum_j |Ahat_ij x_j| on its rounding
// error (gamma_n = n u / (1 - n u), u = 2^-53), which is propagated to the
// bound together with that of the final sums, so the value returned is below
// the exact one.
#include "common.h"

namespace pdbo {

constexpr double kU = 1.1102230246251565e-16;  // 2^-53

__device__ __forceinline__ double gamma_n(int n) { return (double)n * kU / (1.0 - (double)n * kU); }

// Row i's contributions, in objective units, to the four sums of the bound:
// f_i = x_i (kappa r_i / 2 + c'_i); g_i = x_i^2 - x_i; w_i = s * min(-d_i x_i,
// d_i (1 - x_i)) with d_i the gradient of L; e_i = the rounding bound of r_i
// carried through f_i and w_i.
__device__ __forceinline__ void cert_row(double r, double eabs, int n, double xi, int64_t cpi,
                                         int kappa, double s, double ybar, double* out) {
  const double er = gamma_n(n) * eabs;
  const double d = ((double)kappa * r + (double)cpi) / s + ybar * (2.0 * xi - 1.0);
  out[0] = xi * (0.5 * (double)kappa * r + (double)cpi);
  out[1] = xi * xi - xi;
  out[2] = s * fmin(-d * xi, d * (1.0 - xi));
  out[3] = (double)kappa * er * (0.5 * xi + fmax(xi, 1.0 - xi));
}

// Dense Ahat: one wave per row, lanes over the columns (coalesced limb reads).
__global__ void __launch_bounds__(256)
    cert_rows_dense(const int8_t* __restrict__ A8, int nlimb, int64_t limb_stride, int n, int ld,
                    const float* __restrict__ x, const int64_t* __restrict__ cp, int kappa,
                    double s, double ybar, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  double r = 0.0, ea = 0.0;
  for (int j = lane; j < n; j += 64) {
    int64_t a = 0;
    for (int l = 0; l < nlimb; ++l) a += (int64_t)A8[l * limb_stride + (size_t)i * ld + j] << (8 * l);
    const double t = (double)a * (double)x[j];
    r += t;
    ea += fabs(t);
  }
  for (int o = 32; o > 0; o >>= 1) {
    r += __shfl_xor(r, o);
    ea += __shfl_xor(ea, o);
  }
  if (lane == 0) cert_row(r, ea, n, (double)x[i], cp[i], kappa, s, ybar, out + (size_t)i * 4);
}

// CSR Ahat: one thread per row.
__global__ void __launch_bounds__(256)
    cert_rows_csr(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                  const int32_t* __restrict__ val, int n, const float* __restrict__ x,
                  const int64_t* __restrict__ cp, int kappa, double s, double ybar,
                  double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double r = 0.0, ea = 0.0;
  int deg = 0;
  for (int p = rp[i]; p < rp[i + 1]; ++p, ++deg) {
    const double t = (double)val[p] * (double)x[col[p]];
    r += t;
    ea += fabs(t);
  }
  cert_row(r, ea, deg > 0 ? deg : 1, (double)x[i], cp[i], kappa, s, ybar, out + (size_t)i * 4);
}

// res[0] = certified lower bound; res[1] = s L(x) (the value the descent
// reached, in objective units); res[2] = the Frank-Wolfe gap in objective
// units; res[3] = the total rounding bound subtracted.  Sums in a fixed order.
__global__ void __launch_bounds__(256)
    cert_reduce(const double* __restrict__ rows, int n, double s, double ybar,
                double* __restrict__ res) {
  __shared__ double red[8][256];
  const int tid = threadIdx.x;
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = tid; i < n; i += 256) {
    const double* o = rows + (size_t)i * 4;
    a[0] += o[0];
    a[1] += o[1];
    a[2] += o[2];
    a[3] += o[3];
    a[4] += fabs(o[0]);
    a[5] += fabs(o[1]);
    a[6] += fabs(o[2]);
  }
  for (int k = 0; k < 8; ++k) red[k][tid] = a[k];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h)
      for (int k = 0; k < 8; ++k) red[k][tid] += red[k][tid + h];
    __syncthreads();
  }
  if (tid == 0) {
    const double F = red[0][0], G = s * ybar * red[1][0], W = red[2][0];
    // every term of a sum of n terms is carried with relative error below
    // gamma_{n+2} (the product s * ybar * g included)
    const double gs = gamma_n(n + 2);
    const double err = red[3][0] * (1.0 + gs) +
                       gs * (red[4][0] + s * ybar * red[5][0] + red[6][0]) +
                       2.0 * kU * (fabs(F) + fabs(G) + fabs(W));
    res[0] = F + G + W - err;
    res[1] = F + G;
    res[2] = -W;
    res[3] = err;
  }
}

hipError_t launch_cert_dense(const InstDev& I, const float* x, double s, double ybar, double* rows,
                             double* res, hipStream_t st) {
  hipLaunchKernelGGL(cert_rows_dense, dim3((unsigned)((I.n + 3) / 4)), dim3(256), 0, st, I.A8,
                     I.nlimb, I.limb_stride, I.n, I.ld, x, I.cp, I.kappa, s, ybar, rows);
  hipLaunchKernelGGL(cert_reduce, dim3(1), dim3(256), 0, st, rows, I.n, s, ybar, res);
  return hipGetLastError();
}

hipError_t launch_cert_csr(const CsrDev& d, const float* x, double s, double ybar, double* rows,
                           double* res, hipStream_t st) {
  hipLaunchKernelGGL(cert_rows_csr, dim3((unsigned)((d.n + 255) / 256)), dim3(256), 0, st,
                     d.row_ptr, (const int32_t*)d.col, (const int32_t*)d.val, d.n, x, d.cp, d.kappa,
                     s, ybar, rows);
  hipLaunchKernelGGL(cert_reduce, dim3(1), dim3(256), 0, st, rows, d.n, s, ybar, res);
  return hipGetLastError();
}

__global__ void fill_f32_kernel(float* p, float v, int64_t cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) p[i] = v;
}

hipError_t launch_fill_f32(float* p, float v, int64_t cnt, hipStream_t st) {
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f32_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, p, v,
                     cnt);
  return hipGetLastError();
}

}  // namespace pdbo
