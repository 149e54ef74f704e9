// Storage formats of the mixed-precision path, produced from an FP64 A (the
// paper's arithmetic is FP64; the narrow formats only change how A is held):
//
//  * BF16: each entry rounded to the nearest BF16 value, ties to even,
//    directly from its FP64 value.  With x = f 2^E (f in [0.5, 1)) a BF16
//    number keeps 8 significant bits, so the spacing is 2^(E-8) (2^-133 below
//    the smallest normal); x / spacing is exact, rint rounds to nearest even,
//    and the product is exact in FP32, whose upper half is the BF16 pattern.
//  * FP8 E4M3 (the OCP format without infinities: largest finite 448, NaN
//    S.1111.111, subnormals m/8 2^-6) with one FP32 scale per column:
//    s_j = fl32(max_i |A_ij| / 448) (1 for a zero column), and the code of the
//    FP64 quotient A_ij / s_j, rounded to nearest with ties to even and
//    saturated to +-448.  A is then represented by dec(code) s_j.
// Both are decisions on FP64 values made the same way as the definitions
// state, so they are reproducible bit for bit.
#include "common.h"
#include "internal.h"

namespace rsvd {
namespace {

__device__ __forceinline__ uint16_t bf16_of(double x) {
  if (x != x) return 0x7FC0;
  int E;
  (void)frexp(x, &E);
  if (E < -125) E = -125;
  const double q = ldexp(1.0, E - 8);
  const float r = (float)(rint(x / q) * q);   // exact in FP32
  return (uint16_t)(__float_as_uint(r) >> 16);
}

__device__ __forceinline__ uint8_t e4m3_of(double y) {
  if (y != y) return 0x7F;
  const uint32_t sign = signbit(y) ? 0x80u : 0u;
  double a = fabs(y);
  if (a > 448.0) a = 448.0;
  int E;
  (void)frexp(a, &E);                          // a = f 2^E: exponent E - 1
  int e = E - 1;
  if (e < -6) e = -6;
  const double step = ldexp(1.0, e - 3);
  double q = rint(a / step) * step;
  if (q > 448.0) q = 448.0;
  uint32_t code;
  if (q >= 0x1.0p-6) {
    int E2;
    (void)frexp(q, &E2);
    const int e2 = E2 - 1;
    const uint32_t mant = (uint32_t)rint((ldexp(q, -e2) - 1.0) * 8.0);
    code = ((uint32_t)(e2 + 7) << 3) + mant;
  } else {
    code = (uint32_t)rint(q / 0x1.0p-9);
  }
  return (uint8_t)(code | sign);
}

__global__ __launch_bounds__(256) void to_bf16_kernel(const double* __restrict__ A, int64_t lda,
                                                      int64_t m, int64_t n,
                                                      uint16_t* __restrict__ Q, int64_t ldq) {
  const int64_t total = m * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / n, j = e - i * n;
    Q[i * ldq + j] = bf16_of(A[i * lda + j]);
  }
}

// s_j from the exact column maxima: a workgroup takes 64 columns and every
// row (4 row groups of 64 lanes), so no atomics are needed.
__global__ __launch_bounds__(256) void colscale_f64_kernel(const double* __restrict__ A,
                                                           int64_t lda, int64_t m, int64_t n,
                                                           float* __restrict__ s) {
  __shared__ double part[4][64];
  const int64_t j = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int rg = threadIdx.x >> 6;
  double mx = 0.0;
  if (j < n)
    for (int64_t i = rg; i < m; i += 4) mx = fmax(mx, fabs(A[i * lda + j]));
  part[rg][threadIdx.x & 63] = mx;
  __syncthreads();
  if (rg == 0 && j < n) {
    const double a = fmax(fmax(part[0][threadIdx.x], part[1][threadIdx.x]),
                          fmax(part[2][threadIdx.x], part[3][threadIdx.x]));
    s[j] = a == 0.0 ? 1.0f : (float)(a / 448.0);
  }
}

__global__ __launch_bounds__(256) void to_e4m3_kernel(const double* __restrict__ A, int64_t lda,
                                                      int64_t m, int64_t n,
                                                      const float* __restrict__ s,
                                                      uint8_t* __restrict__ Q, int64_t ldq) {
  const int64_t total = m * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / n, j = e - i * n;
    Q[i * ldq + j] = e4m3_of(A[i * lda + j] / (double)s[j]);
  }
}

int grid_of(int64_t work) {
  int64_t g = cdiv(work, 256);
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t launch_quantize_bf16(const double* A, int64_t lda, int64_t m, int64_t n, uint16_t* Q,
                                int64_t ldq, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_of(m * n)), dim3(256), 0, s, A, lda, m, n, Q, ldq);
  return hipGetLastError();
}

hipError_t launch_quantize_e4m3(const double* A, int64_t lda, int64_t m, int64_t n, uint8_t* Q,
                                int64_t ldq, float* scale, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(colscale_f64_kernel, dim3((unsigned)cdiv(n, 64)), dim3(256), 0, s, A, lda, m,
                     n, scale);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(to_e4m3_kernel, dim3(grid_of(m * n)), dim3(256), 0, s, A, lda, m, n, scale, Q,
                     ldq);
  return hipGetLastError();
}

}  // namespace rsvd
