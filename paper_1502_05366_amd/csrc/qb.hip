// Steps of the blocked adaptive QB decomposition (Sec. 3.3, Alg. 7) that the
// other steps do not provide:
//  * the deflation A = A - Q_i B_i of one block with ||A||_F^2 of the result
//    (B_i held transposed, Bt = B_i^T, n x b), and ||A - Q B||_F^2 without
//    writing A: the SUB and NORM modes of the low-rank tile kernel, which
//    stream A once in (and once out): bound by HBM.
//  * transpose_kernel, sub_kernel: B_i rows from Bt, and X -= Y.
#include "common.h"
#include "internal.h"

namespace rsvd {
namespace {

constexpr int QB_NT = 256;

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

int64_t qb_update_tiles(int64_t m, int64_t n) { return lowrank_tiles(m, n); }

hipError_t launch_qb_update(double* A, int64_t lda, int64_t m, int64_t n, const double* Q,
                            int64_t ldq, const double* Bt, int64_t ldbt, int b, double* part,
                            double* norm2, hipStream_t s) {
  if (m <= 0 || n <= 0 || b < 1) return hipErrorInvalidValue;
  LowRank t{};
  t.X[0] = Q; t.W[0] = Bt; t.ldx = ldq; t.ldw = ldbt; t.count = 1; t.l = b;
  return launch_lowrank_sub(t, m, n, A, lda, true, part, norm2, s);
}

hipError_t launch_resid2(const double* A, int64_t lda, int64_t m, int64_t n, const double* Q,
                         int64_t ldq, const double* Bt, int64_t ldbt, int b, double* part,
                         double* norm2, hipStream_t s) {
  if (m <= 0 || n <= 0 || b < 1) return hipErrorInvalidValue;
  LowRank t{};
  t.X[0] = Q; t.W[0] = Bt; t.ldx = ldq; t.ldw = ldbt; t.count = 1; t.l = b;
  // the NORM mode does not write A
  return launch_lowrank_sub(t, m, n, const_cast<double*>(A), lda, false, part, norm2, s);
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
