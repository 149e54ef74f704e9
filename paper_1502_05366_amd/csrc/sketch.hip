// The Gaussian test matrix Omega of the range finder (Fig. 1 step 1; Alg. 5
// line 1: an n x (k+p) matrix with i.i.d. N(0,1) entries).
//
// Generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with
// key = (seed low word, seed high word) and counter (c0, c1, c2, c3) =
// (pair index low, pair index high, stream id, batch), followed by the
// Box-Muller transform in FP64:
//   u1 = ((x0 >> 5) 2^26 + (x1 >> 6) + 1) 2^-53 in (0, 1],
//   u2 = ((x2 >> 5) 2^26 + (x3 >> 6)) 2^-53     in [0, 1),
//   r = sqrt(-2 ln u1), theta = fl(TWO_PI * u2),
//   normal 2t = r cos(theta), normal 2t+1 = r sin(theta)  (t = pair index).
// Omega(i, j) is normal number j*n + i, so a smaller l gives a column prefix.
#include "common.h"
#include "internal.h"
#include "philox_dev.h"

namespace rsvd {
namespace {

template <typename T>
__global__ __launch_bounds__(256) void sketch_kernel(uint32_t k0, uint32_t k1, uint32_t sid,
                                                     uint32_t batch, int64_t n, int64_t l, T* om,
                                                     int64_t ldo) {
  const int64_t total = n * l;
  const int64_t npairs = (total + 1) / 2;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npairs;
       p += (int64_t)gridDim.x * blockDim.x) {
    const Words w = philox10((uint32_t)p, (uint32_t)((uint64_t)p >> 32), sid, batch, k0, k1);
    double z[2];
    box_muller(w, z[0], z[1]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t t = 2 * p + h;
      if (t < total) {
        const int64_t j = t / n, i = t - j * n;
        om[i * ldo + j] = (T)z[h];
      }
    }
  }
  // zero the padding columns l .. ldo-1
  const int64_t pad = ldo - l;
  if (pad > 0) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * pad;
         e += (int64_t)gridDim.x * blockDim.x) {
      const int64_t i = e / pad, j = l + (e - (e / pad) * pad);
      om[i * ldo + j] = T(0);
    }
  }
}

__global__ __launch_bounds__(256) void words_kernel(uint32_t k0, uint32_t k1, uint32_t sid,
                                                    uint32_t batch, uint64_t first, int64_t count,
                                                    uint32_t* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t c = first + (uint64_t)i;
    const Words w = philox10((uint32_t)c, (uint32_t)(c >> 32), sid, batch, k0, k1);
    out[4 * i + 0] = w.x0;
    out[4 * i + 1] = w.x1;
    out[4 * i + 2] = w.x2;
    out[4 * i + 3] = w.x3;
  }
}

int grid_for(int64_t work) {
  int64_t g = cdiv(work, 256);
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t launch_sketch(bool f32, uint64_t seed, uint32_t sid, uint32_t batch, int64_t n,
                         int64_t l, void* Omega, int64_t ldo, hipStream_t s) {
  if (n <= 0 || l <= 0) return hipSuccess;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const int grid = grid_for((n * l + 1) / 2);
  if (f32)
    hipLaunchKernelGGL(sketch_kernel<float>, dim3(grid), dim3(256), 0, s, k0, k1, sid, batch, n,
                       l, static_cast<float*>(Omega), ldo);
  else
    hipLaunchKernelGGL(sketch_kernel<double>, dim3(grid), dim3(256), 0, s, k0, k1, sid, batch, n,
                       l, static_cast<double*>(Omega), ldo);
  return hipGetLastError();
}

hipError_t launch_philox_words(uint64_t seed, uint32_t sid, uint32_t batch, uint64_t first,
                               int64_t count, uint32_t* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(words_kernel, dim3(grid_for(count)), dim3(256), 0, s, (uint32_t)seed,
                     (uint32_t)(seed >> 32), sid, batch, first, count, out);
  return hipGetLastError();
}

}  // namespace rsvd
