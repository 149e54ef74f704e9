// Kernels of the reverse-mode derivative of the randomized SVD (the sketch
// held fixed) that the forward steps do not provide.  The adjoint walks the
// forward map backwards: a product C = A X gives dA += dC X^T and dX = A^T dC
// (a pass over A); a thin QR Y = Q R (positive diagonal) gives
//   dY = (dQ + Q copyltu(M)) R^{-T},  M = R dR^T - dQ^T Q,
// and the full SVD of the square R_hat = Uh diag(s) Vh^T gives
//   dR_hat = Uh [ (F o (Uh^T dUh - dUh^T Uh)) S + diag(ds)
//                 + S (F o (Vh^T dVh - dVh^T Vh)) ] Vh^T,  F_ij = 1/(s_j^2 - s_i^2).
//  * svd_inner_kernel: the bracket above from Pu = Uh^T dUh, Pv = Vh^T dVh;
//    ds_i = dS_i (i < k) - 2 dres s_i, the second part being the cotangent
//    of ||A - Q Q^T A||_F^2 = ||A||_F^2 - sum_i s_i^2 (all l values).
//  * copyltu_kernel: Mc = copyltu(-P + Q) (P = dQ^T Q, Q = R dR^T or none).
//  * add_kernel, zero_kernel: X += Y, X = 0.
// dA itself, the sum of the 2q + 2 rank-l terms, is formed by the low-rank
// tile kernel.
#include "common.h"
#include "internal.h"

namespace rsvd {
namespace {

constexpr int GNT = 256;

__global__ __launch_bounds__(GNT) void svd_inner_kernel(const double* __restrict__ Pu,
                                                        const double* __restrict__ Pv,
                                                        int64_t ldp, const double* __restrict__ s,
                                                        const double* __restrict__ dS, int k,
                                                        const double* __restrict__ dres, int l,
                                                        double* __restrict__ out, int64_t ldo) {
  const int64_t e = blockIdx.x * (int64_t)GNT + threadIdx.x;
  if (e >= (int64_t)l * l) return;
  const int i = (int)(e / l), j = (int)(e - (e / l) * l);
  double v;
  if (i == j) {
    v = (dS && i < k) ? dS[i] : 0.0;
    if (dres) v -= 2.0 * dres[0] * s[i];
  } else {
    const double f = 1.0 / (s[j] * s[j] - s[i] * s[i]);
    const double au = Pu[(int64_t)i * ldp + j] - Pu[(int64_t)j * ldp + i];
    const double av = Pv[(int64_t)i * ldp + j] - Pv[(int64_t)j * ldp + i];
    v = f * au * s[j] + s[i] * f * av;
  }
  out[(int64_t)i * ldo + j] = v;
}

// Mc = copyltu(N), N = -P (+ Qm): lower triangle of N mirrored to the upper
__global__ __launch_bounds__(GNT) void copyltu_kernel(const double* __restrict__ P,
                                                      const double* __restrict__ Qm, int64_t ld,
                                                      int l, double* __restrict__ Mc,
                                                      int64_t ldm) {
  const int64_t e = blockIdx.x * (int64_t)GNT + threadIdx.x;
  if (e >= (int64_t)l * l) return;
  int i = (int)(e / l), j = (int)(e - (e / l) * l);
  const int a = i >= j ? i : j, b = i >= j ? j : i;   // (a, b) in the lower triangle
  double v = -P[(int64_t)a * ld + b];
  if (Qm) v += Qm[(int64_t)a * ld + b];
  Mc[(int64_t)i * ldm + j] = v;
}

__global__ __launch_bounds__(GNT) void add_kernel(double* __restrict__ X, int64_t ldx,
                                                  const double* __restrict__ Y, int64_t ldy,
                                                  int64_t rows, int cols) {
  const int64_t e = blockIdx.x * (int64_t)GNT + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t r = e / cols, c = e - (e / cols) * cols;
  X[r * ldx + c] += Y[r * ldy + c];
}

__global__ __launch_bounds__(GNT) void zero_kernel(double* __restrict__ X, int64_t ldx,
                                                   int64_t rows, int cols) {
  const int64_t e = blockIdx.x * (int64_t)GNT + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t r = e / cols, c = e - (e / cols) * cols;
  X[r * ldx + c] = 0.0;
}

}  // namespace

hipError_t launch_svd_inner(const double* Pu, const double* Pv, int64_t ldp, const double* s,
                            const double* dS, int k, const double* dres, int l, double* out,
                            int64_t ldo, hipStream_t st) {
  hipLaunchKernelGGL(svd_inner_kernel, dim3((unsigned)cdiv((int64_t)l * l, GNT)), dim3(GNT), 0,
                     st, Pu, Pv, ldp, s, dS, k, dres, l, out, ldo);
  return hipGetLastError();
}

hipError_t launch_copyltu(const double* P, const double* Qm, int64_t ld, int l, double* Mc,
                          int64_t ldm, hipStream_t st) {
  hipLaunchKernelGGL(copyltu_kernel, dim3((unsigned)cdiv((int64_t)l * l, GNT)), dim3(GNT), 0, st,
                     P, Qm, ld, l, Mc, ldm);
  return hipGetLastError();
}

hipError_t launch_add(double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t rows,
                      int cols, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(add_kernel, dim3((unsigned)cdiv(rows * cols, GNT)), dim3(GNT), 0, st, X, ldx,
                     Y, ldy, rows, cols);
  return hipGetLastError();
}

hipError_t launch_zero(double* X, int64_t ldx, int64_t rows, int cols, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)cdiv(rows * cols, GNT)), dim3(GNT), 0, st, X, ldx,
                     rows, cols);
  return hipGetLastError();
}

}  // namespace rsvd
