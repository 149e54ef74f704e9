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
// Wave-wide helpers.  dpp_d moves a double between lanes with a DPP control
// (both 32-bit halves); readlane_d reads one lane's value as a uniform.
template <int CTRL> __device__ __forceinline__ double dpp_d(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double readlane_d(double x, int lane) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// Sum over the 64 lanes of a wave (all lanes active), returned in every lane:
// DPP exchanges inside each row of 16 lanes (xor 1, xor 2, half-row mirror,
// row mirror leave every lane with its row's sum), then the four row sums
// are added in a fixed order.
__device__ __forceinline__ double wave_allsum(double x) {
  x += dpp_d<0xB1>(x);     // quad_perm [1, 0, 3, 2]
  x += dpp_d<0x4E>(x);     // quad_perm [2, 3, 0, 1]
  x += dpp_d<0x141>(x);    // row_half_mirror
  x += dpp_d<0x140>(x);    // row_mirror
  return ((readlane_d(x, 0) + readlane_d(x, 16)) + readlane_d(x, 32)) + readlane_d(x, 48);
}

// 1/x and 1/sqrt(x) from the hardware estimates refined by two Newton steps
// (errors of a few ulps; x > 0 and normal).
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
}

// flags live 128 bytes apart so that pollers of different flags do not share
// a cache line
constexpr int FLAG_STRIDE = 32;

}  // namespace rsvd
