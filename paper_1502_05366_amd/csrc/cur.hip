// Gathers of the CUR post-processing (Sec. 2.5, Alg. 3; Sec. 3.6):
//   C = A(:, Jc) stored so that its rows are the columns of C^T (the input
//   of the row-selecting pivoted QR), R^T = A(Jr, :)^T (input of the QR that
//   gives R^dagger), rows of an n x k matrix picked by an index list, and
//   M += rows picked from another matrix (the V^T Qt = Qt(Jc,:) + T Qt(Jres,:)
//   product of the CUR factor U).
#include "common.h"
#include "internal.h"

namespace rsvd {
namespace {

// element of A as FP64; BF16 elements are stored as their 16-bit patterns
struct Bf16Bits { uint16_t v; };
__device__ __forceinline__ double as_double(double x) { return x; }
__device__ __forceinline__ double as_double(float x) { return (double)x; }
__device__ __forceinline__ double as_double(Bf16Bits x) {
  return (double)__uint_as_float((uint32_t)x.v << 16);
}

// Crow[i * ldc + t] = A[i, J[t]]  (i < m, t < k)
template <typename TA>
__global__ __launch_bounds__(256) void gather_cols_kernel(const TA* __restrict__ A, int64_t lda,
                                                          int64_t m, int64_t n,
                                                          const int64_t* __restrict__ J, int k,
                                                          double* __restrict__ Crow, int64_t ldc) {
  const int64_t total = m * k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / k;
    const int t = (int)(e - i * k);
    const int64_t j = J[t];
    Crow[i * ldc + t] = (j >= 0 && j < n) ? as_double(A[i * lda + j]) : 0.0;
  }
}

// Rt[j * ldr + t] = A[Jr[t], j]  (j < n, t < k)
template <typename TA>
__global__ __launch_bounds__(256) void gather_rows_t_kernel(const TA* __restrict__ A, int64_t lda,
                                                            int64_t m, int64_t n,
                                                            const int64_t* __restrict__ Jr, int k,
                                                            double* __restrict__ Rt, int64_t ldr) {
  const int64_t total = n * k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int t = (int)(e / n);
    const int64_t j = e - (int64_t)t * n;
    const int64_t r = Jr[t];
    Rt[j * ldr + t] = (r >= 0 && r < m) ? as_double(A[r * lda + j]) : 0.0;
  }
}

// Out[i * ldo + c] = In[J[i] * ldi + c]  (i < rows, c < cols); with add, Out += ...
__global__ __launch_bounds__(256) void pick_rows_kernel(const double* __restrict__ In, int64_t ldi,
                                                        int64_t in_rows,
                                                        const int64_t* __restrict__ J, int64_t rows,
                                                        int cols, double* __restrict__ Out,
                                                        int64_t ldo, int add) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / cols;
    const int c = (int)(e - i * cols);
    const int64_t r = J[i];
    const double v = (r >= 0 && r < in_rows) ? In[r * ldi + c] : 0.0;
    if (add) Out[i * ldo + c] += v;
    else Out[i * ldo + c] = v;
  }
}

__global__ __launch_bounds__(256) void convert_kernel(const float* __restrict__ in, int64_t ldi,
                                                      int64_t rows, int cols,
                                                      double* __restrict__ out, int64_t ldo) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / cols;
    const int c = (int)(e - i * cols);
    out[i * ldo + c] = (double)in[i * ldi + c];
  }
}

int grid_of(int64_t total) {
  int64_t g = cdiv(total, 256);
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t launch_gather_cols(int atype, const void* A, int64_t lda, int64_t m, int64_t n,
                              const int64_t* J, int k, double* Crow, int64_t ldc, hipStream_t s) {
  if (m <= 0 || k <= 0) return hipSuccess;
  const dim3 grid(grid_of(m * k));
  if (atype == 1)
    hipLaunchKernelGGL(gather_cols_kernel<float>, grid, dim3(256), 0, s, (const float*)A, lda, m,
                       n, J, k, Crow, ldc);
  else if (atype == 2)
    hipLaunchKernelGGL(gather_cols_kernel<Bf16Bits>, grid, dim3(256), 0, s, (const Bf16Bits*)A,
                       lda, m, n, J, k, Crow, ldc);
  else
    hipLaunchKernelGGL(gather_cols_kernel<double>, grid, dim3(256), 0, s, (const double*)A, lda,
                       m, n, J, k, Crow, ldc);
  return hipGetLastError();
}

hipError_t launch_gather_rows_t(int atype, const void* A, int64_t lda, int64_t m, int64_t n,
                                const int64_t* Jr, int k, double* Rt, int64_t ldr, hipStream_t s) {
  if (n <= 0 || k <= 0) return hipSuccess;
  const dim3 grid(grid_of(n * k));
  if (atype == 1)
    hipLaunchKernelGGL(gather_rows_t_kernel<float>, grid, dim3(256), 0, s, (const float*)A, lda,
                       m, n, Jr, k, Rt, ldr);
  else if (atype == 2)
    hipLaunchKernelGGL(gather_rows_t_kernel<Bf16Bits>, grid, dim3(256), 0, s,
                       (const Bf16Bits*)A, lda, m, n, Jr, k, Rt, ldr);
  else
    hipLaunchKernelGGL(gather_rows_t_kernel<double>, grid, dim3(256), 0, s, (const double*)A,
                       lda, m, n, Jr, k, Rt, ldr);
  return hipGetLastError();
}

hipError_t launch_pick_rows(const double* In, int64_t ldi, int64_t in_rows, const int64_t* J,
                            int64_t rows, int cols, double* Out, int64_t ldo, bool add,
                            hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(pick_rows_kernel, dim3(grid_of(rows * cols)), dim3(256), 0, s, In, ldi,
                     in_rows, J, rows, cols, Out, ldo, add ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_convert(const float* in, int64_t ldi, int64_t rows, int cols, double* out,
                          int64_t ldo, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(convert_kernel, dim3(grid_of(rows * cols)), dim3(256), 0, s, in, ldi, rows,
                     cols, out, ldo);
  return hipGetLastError();
}

}  // namespace rsvd
