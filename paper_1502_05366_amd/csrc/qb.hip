// Kernels of the blocked adaptive QB decomposition (Sec. 3.3, Alg. 7) that
// the other steps do not provide:
//  * qb_update_kernel: the deflation A = A - Q_i B_i of one block, with B_i
//    held transposed (Bt = B_i^T, n x b).  A workgroup of 4 waves owns a
//    64 x 64 tile of A; wave w forms rows 16w .. 16w+15 of Q_i B_i on the
//    matrix cores (K = b), subtracts them from A in place and adds the
//    squares of the new entries; the workgroup's sum goes to part[tile].
//    The kernel streams A once in and once out: it is bound by HBM.  Without
//    STORE it only forms ||A - Q_i B_i||_F^2 (the residual of a QB
//    factorization), reading A once.
//  * sum_kernel: ||A||_F^2 = the partial sums added in a fixed order.
//  * transpose_kernel, sub_kernel: B_i rows from Bt, and X -= Y.
#include "common.h"
#include "internal.h"

namespace rsvd {
namespace {

constexpr int QB_NT = 256;

template <bool STORE>
__global__ __launch_bounds__(QB_NT) void qb_update_kernel(double* __restrict__ A, int64_t lda,
                                                          int64_t m, int64_t n,
                                                          const double* __restrict__ Q,
                                                          int64_t ldq,
                                                          const double* __restrict__ Bt,
                                                          int64_t ldbt, int b,
                                                          double* __restrict__ part) {
  __shared__ double red[QB_NT / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.y * 64 + wave * 16;
  const int64_t c0 = (int64_t)blockIdx.x * 64;
  // the wave's 16 x 64 entries of A are loaded first, so that they stream
  // in from HBM while Q_i B_i is formed
  double a0[4][4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int64_t col = c0 + ct * 16 + li;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = r0 + drow(lk, v);
      a0[ct][v] = (row < m && col < n) ? A[row * lda + col] : 0.0;
    }
  }
  d4 acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc[ct] = d4{0.0, 0.0, 0.0, 0.0};
  const int64_t qr = r0 + li;
  for (int k0 = 0; k0 < b; k0 += 4) {
    const int k = k0 + lk;
    const double av = (qr < m && k < b) ? Q[qr * ldq + k] : 0.0;   // Q_i[row][k]
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int64_t col = c0 + ct * 16 + li;
      const double bv = (col < n && k < b) ? Bt[col * ldbt + k] : 0.0;   // B_i[k][col]
      acc[ct] = Mfma<double>::mma(av, bv, acc[ct]);
    }
  }
  double s = 0.0;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int64_t col = c0 + ct * 16 + li;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = r0 + drow(lk, v);
      if (row < m && col < n) {
        const double x = a0[ct][v] - acc[ct][v];
        if (STORE) A[row * lda + col] = x;
        s = fma(x, x, s);
      }
    }
  }
  s = wave_allsum(s);
  if (lane == 0) red[wave] = s;
  __syncthreads();
  if (tid == 0)
    part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// out[0] = sum of part[0 .. np): thread t adds entries t, t + SUM_NT, ... in
// four interleaved chains, then the chains, the waves and the threads are
// added in a fixed order
constexpr int SUM_NT = 1024;

__global__ __launch_bounds__(SUM_NT) void sum_kernel(const double* __restrict__ part, int64_t np,
                                                     double* __restrict__ out) {
  __shared__ double red[SUM_NT / 64];
  const int tid = threadIdx.x;
  double c[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t i = tid;
  for (; i + 3 * SUM_NT < np; i += 4 * SUM_NT) {
#pragma unroll
    for (int u = 0; u < 4; ++u) c[u] += part[i + u * SUM_NT];
  }
  for (; i < np; i += SUM_NT) c[0] += part[i];
  double s = wave_allsum((c[0] + c[1]) + (c[2] + c[3]));
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < SUM_NT / 64; ++w) t += red[w];
    out[0] = t;
  }
}

// B[t][c] = Bt[c][t] for t < b, c < n
__global__ __launch_bounds__(QB_NT) void transpose_kernel(const double* __restrict__ Bt,
                                                          int64_t ldbt, int64_t n, int b,
                                                          double* __restrict__ B, int64_t ldb) {
  const int64_t e = blockIdx.x * (int64_t)QB_NT + threadIdx.x;
  if (e >= n * b) return;
  const int64_t t = e / n, c = e - (e / n) * n;
  B[t * ldb + c] = Bt[c * ldbt + t];
}

// X -= Y (rows x cols)
__global__ __launch_bounds__(QB_NT) void sub_kernel(double* __restrict__ X, int64_t ldx,
                                                    const double* __restrict__ Y, int64_t ldy,
                                                    int64_t rows, int cols) {
  const int64_t e = blockIdx.x * (int64_t)QB_NT + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t r = e / cols, c = e - (e / cols) * cols;
  X[r * ldx + c] -= Y[r * ldy + c];
}

}  // namespace

int64_t qb_update_tiles(int64_t m, int64_t n) { return cdiv(m, 64) * cdiv(n, 64); }

hipError_t launch_qb_update(double* A, int64_t lda, int64_t m, int64_t n, const double* Q,
                            int64_t ldq, const double* Bt, int64_t ldbt, int b, double* part,
                            double* norm2, hipStream_t s) {
  if (m <= 0 || n <= 0 || b < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)cdiv(n, 64), (unsigned)cdiv(m, 64));
  hipLaunchKernelGGL(qb_update_kernel<true>, grid, dim3(QB_NT), 0, s, A, lda, m, n, Q, ldq, Bt,
                     ldbt, b, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(SUM_NT), 0, s, part, qb_update_tiles(m, n), norm2);
  return hipGetLastError();
}

hipError_t launch_resid2(const double* A, int64_t lda, int64_t m, int64_t n, const double* Q,
                         int64_t ldq, const double* Bt, int64_t ldbt, int b, double* part,
                         double* norm2, hipStream_t s) {
  if (m <= 0 || n <= 0 || b < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)cdiv(n, 64), (unsigned)cdiv(m, 64));
  // the kernel does not write A when STORE is false
  hipLaunchKernelGGL(qb_update_kernel<false>, grid, dim3(QB_NT), 0, s, const_cast<double*>(A), lda,
                     m, n, Q, ldq, Bt, ldbt, b, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(SUM_NT), 0, s, part, qb_update_tiles(m, n), norm2);
  return hipGetLastError();
}

hipError_t launch_transpose(const double* Bt, int64_t ldbt, int64_t n, int b, double* B,
                            int64_t ldb, hipStream_t s) {
  if (n <= 0 || b <= 0) return hipSuccess;
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)cdiv(n * b, QB_NT)), dim3(QB_NT), 0, s, Bt,
                     ldbt, n, b, B, ldb);
  return hipGetLastError();
}

hipError_t launch_sub(double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t rows,
                      int cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(sub_kernel, dim3((unsigned)cdiv(rows * cols, QB_NT)), dim3(QB_NT), 0, s, X,
                     ldx, Y, ldy, rows, cols);
  return hipGetLastError();
}

}  // namespace rsvd
