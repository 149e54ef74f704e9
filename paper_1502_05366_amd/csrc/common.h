// Shared definitions for the gfx950 kernels of the randomized SVD / ID / CUR
// library: MFMA wrappers, launch helpers and the internal launcher API.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace rsvd {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// 16x16x4 matrix-core products.  Operand layout for a wave of 64 lanes
// (g = l / 16, c = l % 16):
//   A (16 x 4):  lane l holds A[c][g]
//   B (4 x 16):  lane l holds B[g][c]
//   C (16 x 16): lane l, element v holds C[row(g, v)][c] with
//                row = 4 g + v for the FP32 product and row = 4 v + g for the
//                FP64 product (measured on gfx950 with exact integer data).
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef d4 acc_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ int row(int g, int v) { return 4 * v + g; }
};
template <> struct Mfma<float> {
  typedef f4 acc_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ int row(int g, int v) { return 4 * g + v; }
};
// accumulator row of element v in lane group g for the FP64 product
__device__ __forceinline__ int drow(int g, int v) { return 4 * v + g; }

__host__ __device__ __forceinline__ int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ __forceinline__ int64_t rup(int64_t a, int64_t b) { return cdiv(a, b) * b; }

// Bits of the device status word info[0]; info[1] holds the numerical rank
// when bit RANK is set.
enum : int32_t {
  INFO_ORTH_FALLBACK = 1,   // a dependent column was replaced during orth
  INFO_JACOBI_CAP = 2,      // Jacobi stopped at its sweep cap
  INFO_RANK = 4,            // pivoted QR met a residual below the rank tolerance
  INFO_NONFINITE = 8,       // NaN or Inf met in a Gram matrix
  INFO_BARRIER = 16,        // a grid barrier hit its spin cap (internal error)
};

__device__ __forceinline__ void info_or(int32_t* info, int32_t bits) {
  if (info) atomicOr(info, bits);
}

// Cross-workgroup exchange without cache maintenance: data and flags are
// written and read with agent-scope atomic stores / loads (coherent across
// the XCDs without L2 write-back or invalidation), and a writer waits for its
// own stores to complete before it raises a flag.
__device__ __forceinline__ double ld_agent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_agent_u32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent_u32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// all stores issued by this wave have completed
__device__ __forceinline__ void stores_done() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
// flags live 128 bytes apart so that pollers of different flags do not share
// a cache line
constexpr int FLAG_STRIDE = 32;

}  // namespace rsvd
