// Narrow passes over A (l <= 64 columns of the skinny operand) in FP32 or
// FP64: with at most 2 l flops per element of A they are bound by HBM, and
// the LDS-staged tile kernel of the wide passes leaves HBM idle between its
// short k-steps.  Here A goes from HBM straight into the matrix-core operands:
// each lane loads 16 contiguous bytes (4 FP32 or 2 FP64 values) of A, and the
// VEC values of one load feed VEC 16x16x4 products, one each.  A product sums
// over its k index in any order, so the k (or column) that a register stands
// for only has to be the same on both operands.
//
//   C = A X  (A M x K): lane (c, g) loads A[r0 + c][k0 + VEC g .. + VEC - 1];
//     product j takes k = k0 + VEC g + j, its B operand X[k][16 b + c] from
//     the transposed copy Xt (L x K, one 16-byte load per lane and 16-column
//     block b); its output is C[r0 + row][16 b + c].
//   C = A^T X (A stored K x M): lane (c, g) loads A[k0 + g][i0 + VEC c .. +
//     VEC - 1] (four rows of a 16 VEC-column strip per load); product j is
//     C^T = X^T A over k = k0 + g, with the A operand X[k0 + g][16 b + c] and
//     the B operand A[k0 + g][i0 + VEC c + j], so its output column c is
//     C[i0 + VEC c + j][16 b + row].
// Loads run PD steps ahead in a ring of registers (no LDS, no barrier).  The
// reduction is split into ks ranges so that every compute unit holds several
// workgroups; each range writes its partial C, and a second kernel adds the
// ranges in a fixed order (deterministic).
#include "common.h"
#include "internal.h"

namespace rsvd {
namespace {

constexpr int NW = 4;          // waves per workgroup
constexpr int RBW = 4;         // 16-row blocks per wave (non-transposed)
// steps of loads in flight (fewer for 3-4 column blocks, for the registers)
template <int CB> constexpr int pdepth() { return CB <= 2 ? 8 : 4; }

struct NArgs {
  const void* A; int64_t lda;
  const void* X; int64_t ldx;    // X (K x L); for the non-transposed pass Xt (L x ldx)
  void* C; int64_t ldc;
  int64_t M, K, L;
  int ks;                        // reduction ranges
  int64_t kchunk;                // steps of the reduction per range
  void* part;                    // ks x M x L partial results (ks > 1)
};

template <typename T> struct V16;
template <> struct V16<float> {
  typedef float4 type;
  static constexpr int N = 4;
};
template <> struct V16<double> {
  typedef double2 type;
  static constexpr int N = 2;
};

template <typename T>
__device__ __forceinline__ typename V16<T>::type load16(const T* p) {
  return *reinterpret_cast<const typename V16<T>::type*>(p);
}
template <typename T>
__device__ __forceinline__ T vget(const typename V16<T>::type& v, int j);
template <> __device__ __forceinline__ float vget<float>(const float4& v, int j) {
  return j == 0 ? v.x : (j == 1 ? v.y : (j == 2 ? v.z : v.w));
}
template <> __device__ __forceinline__ double vget<double>(const double2& v, int j) {
  return j == 0 ? v.x : v.y;
}

// 16 bytes of row `row` from element `col`, elements at or beyond `lim`
// (and rows outside) read as zero
template <typename T>
__device__ __forceinline__ typename V16<T>::type load16_guard(const T* A, int64_t lda, int64_t row,
                                                              bool rok, int64_t col, int64_t lim) {
  constexpr int VEC = V16<T>::N;
  typename V16<T>::type v;
  if (rok && col + VEC <= lim) {
    v = load16(A + row * lda + col);
  } else {
    T e[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) e[j] = (rok && col + j < lim) ? A[row * lda + col + j] : T(0);
    if constexpr (VEC == 4) v = float4{(float)e[0], (float)e[1], (float)e[2], (float)e[3]};
    else v = double2{(double)e[0], (double)e[1]};
  }
  return v;
}

// ---- C = A X ---------------------------------------------------------------
template <typename T, int CB>
__global__ __launch_bounds__(NW * 64) void narrow_n_kernel(NArgs g) {
  constexpr int PD = pdepth<CB>();
  constexpr int VEC = V16<T>::N;
  constexpr int KS = 4 * VEC;                      // k per step
  typedef typename Mfma<T>::acc_t acc_t;
  typedef typename V16<T>::type vec_t;
  const T* __restrict__ A = static_cast<const T*>(g.A);
  const T* __restrict__ Xt = static_cast<const T*>(g.X);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = lane & 15, gq = lane >> 4;
  const int64_t tile = blockIdx.x;                 // NW * RBW * 16 rows
  const int range = blockIdx.y;
  const int64_t r0 = tile * (NW * RBW * 16) + wave * (RBW * 16);
  const int64_t kb = (int64_t)range * g.kchunk * KS;
  const int64_t ke = min(g.K, kb + g.kchunk * KS);
  acc_t acc[RBW][CB];
#pragma unroll
  for (int a = 0; a < RBW; ++a)
#pragma unroll
    for (int b = 0; b < CB; ++b) acc[a][b] = Mfma<T>::zero();
  int64_t arow[RBW];
  bool aok[RBW];
#pragma unroll
  for (int a = 0; a < RBW; ++a) {
    arow[a] = r0 + a * 16 + c;
    aok[a] = arow[a] < g.M;
  }
  int64_t xrow[CB];
#pragma unroll
  for (int b = 0; b < CB; ++b) xrow[b] = b * 16 + c;   // Xt rows >= L are zero padding
  vec_t ra[PD][RBW], rx[PD][CB];
  auto load = [&](int st, int64_t k0) {
    const int64_t kk = k0 + VEC * gq;
#pragma unroll
    for (int a = 0; a < RBW; ++a) ra[st][a] = load16_guard(A, g.lda, arow[a], aok[a], kk, ke);
#pragma unroll
    for (int b = 0; b < CB; ++b) rx[st][b] = load16(Xt + xrow[b] * g.ldx + kk);
  };
  const int64_t nsteps = (ke - kb + KS - 1) / KS;
#pragma unroll
  for (int st = 0; st < PD; ++st)
    if (st < nsteps) load(st, kb + st * KS);
  for (int64_t s0 = 0; s0 < nsteps; s0 += PD) {
#pragma unroll
    for (int st = 0; st < PD; ++st) {
      const int64_t s = s0 + st;
      if (s >= nsteps) break;
#pragma unroll
      for (int j = 0; j < VEC; ++j)
#pragma unroll
        for (int b = 0; b < CB; ++b) {
          const T bv = vget<T>(rx[st][b], j);
#pragma unroll
          for (int a = 0; a < RBW; ++a)
            acc[a][b] = Mfma<T>::mma(vget<T>(ra[st][a], j), bv, acc[a][b]);
        }
      if (s + PD < nsteps) load(st, kb + (s + PD) * KS);
    }
  }
  T* out = g.ks > 1 ? static_cast<T*>(g.part) + (int64_t)range * g.M * g.L : static_cast<T*>(g.C);
  const int64_t ldo = g.ks > 1 ? g.L : g.ldc;
#pragma unroll
  for (int a = 0; a < RBW; ++a)
#pragma unroll
    for (int b = 0; b < CB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = r0 + a * 16 + Mfma<T>::row(gq, v);
        const int64_t col = b * 16 + c;
        if (r < g.M && col < g.L) out[r * ldo + col] = acc[a][b][v];
      }
}

// ---- C = A^T X -------------------------------------------------------------
template <typename T, int CB>
__global__ __launch_bounds__(NW * 64) void narrow_t_kernel(NArgs g) {
  constexpr int PD = pdepth<CB>();
  constexpr int VEC = V16<T>::N;
  constexpr int SW = 16 * VEC;                     // columns of A per wave
  typedef typename Mfma<T>::acc_t acc_t;
  typedef typename V16<T>::type vec_t;
  const T* __restrict__ A = static_cast<const T*>(g.A);
  const T* __restrict__ X = static_cast<const T*>(g.X);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = lane & 15, gq = lane >> 4;
  const int range = blockIdx.y;
  const int64_t i0 = ((int64_t)blockIdx.x * NW + wave) * SW;
  const int64_t kb = (int64_t)range * g.kchunk * 4;
  const int64_t ke = min(g.K, kb + g.kchunk * 4);
  acc_t acc[VEC][CB];
#pragma unroll
  for (int j = 0; j < VEC; ++j)
#pragma unroll
    for (int b = 0; b < CB; ++b) acc[j][b] = Mfma<T>::zero();
  const int64_t icol = i0 + VEC * c;
  vec_t ra[PD];
  T rx[PD][CB];
  auto load = [&](int st, int64_t k0) {
    const int64_t k = k0 + gq;
    const bool kok = k < ke;
    ra[st] = load16_guard(A, g.lda, k, kok, icol, g.M);
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      const int64_t l = b * 16 + c;
      rx[st][b] = (kok && l < g.L) ? X[k * g.ldx + l] : T(0);
    }
  };
  const int64_t nsteps = (ke - kb + 3) / 4;
#pragma unroll
  for (int st = 0; st < PD; ++st)
    if (st < nsteps) load(st, kb + st * 4);
  for (int64_t s0 = 0; s0 < nsteps; s0 += PD) {
#pragma unroll
    for (int st = 0; st < PD; ++st) {
      const int64_t s = s0 + st;
      if (s >= nsteps) break;
#pragma unroll
      for (int j = 0; j < VEC; ++j) {
        const T av = vget<T>(ra[st], j);
#pragma unroll
        for (int b = 0; b < CB; ++b) acc[j][b] = Mfma<T>::mma(rx[st][b], av, acc[j][b]);
      }
      if (s + PD < nsteps) load(st, kb + (s + PD) * 4);
    }
  }
  T* out = g.ks > 1 ? static_cast<T*>(g.part) + (int64_t)range * g.M * g.L : static_cast<T*>(g.C);
  const int64_t ldo = g.ks > 1 ? g.L : g.ldc;
#pragma unroll
  for (int j = 0; j < VEC; ++j)
#pragma unroll
    for (int b = 0; b < CB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = i0 + VEC * c + j;
        const int64_t l = b * 16 + Mfma<T>::row(gq, v);
        if (i < g.M && l < g.L) out[i * ldo + l] = acc[j][b][v];
      }
}

// C = sum over ranges of the partial results, in range order
template <typename T>
__global__ __launch_bounds__(256) void narrow_sum_kernel(const T* __restrict__ part, int ks,
                                                         int64_t M, int64_t L, T* __restrict__ C,
                                                         int64_t ldc) {
  const int64_t total = M * L;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    T s = part[e];
    for (int r = 1; r < ks; ++r) s += part[(int64_t)r * total + e];
    const int64_t i = e / L, l = e - i * L;
    C[i * ldc + l] = s;
  }
}

// Xt[l][k] = X[k][l] for l < rows16 (zero for l >= L) and k < ldt (zero for k >= K)
template <typename T>
__global__ __launch_bounds__(256) void narrow_xt_kernel(const T* __restrict__ X, int64_t ldx,
                                                        int64_t K, int64_t L, int rows16,
                                                        T* __restrict__ Xt, int64_t ldt) {
  const int64_t total = (int64_t)rows16 * ldt;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = e / ldt, k = e - l * ldt;
    Xt[e] = (l < L && k < K) ? X[k * ldx + l] : T(0);
  }
}

struct NPlan {
  int cb, ks;
  int64_t tiles, kchunk, ldt;
};

template <typename T>
NPlan plan_narrow(bool trans, int64_t M, int64_t K, int64_t L, int ncu) {
  constexpr int VEC = V16<T>::N;
  NPlan p;
  p.cb = (int)cdiv(L, 16);
  const int64_t rows_per_wg = trans ? (int64_t)NW * 16 * VEC : (int64_t)NW * RBW * 16;
  p.tiles = cdiv(M, rows_per_wg);
  const int64_t kstep = trans ? 4 : 4 * VEC;
  const int64_t steps = cdiv(K, kstep);
  // about 8 workgroups per compute unit, each with at least 64 steps
  int64_t ks = cdiv((int64_t)8 * ncu, p.tiles);
  if (ks > steps / 64) ks = steps / 64;
  if (ks < 1) ks = 1;
  p.kchunk = cdiv(steps, ks);
  p.ks = (int)cdiv(steps, p.kchunk);
  p.ldt = rup(K, 4 * VEC);
  return p;
}

template <typename T>
size_t narrow_bytes(bool trans, int64_t M, int64_t K, int64_t L, int ncu) {
  const NPlan p = plan_narrow<T>(trans, M, K, L, ncu);
  size_t b = 0;
  if (!trans) b += (size_t)16 * p.cb * p.ldt * sizeof(T) + 256;
  if (p.ks > 1) b += (size_t)p.ks * M * L * sizeof(T) + 256;
  return b;
}

template <typename T, int CB>
hipError_t run_narrow(bool trans, const NArgs& g, int64_t tiles, hipStream_t s) {
  const dim3 grid((unsigned)tiles, (unsigned)g.ks);
  if (trans) hipLaunchKernelGGL((narrow_t_kernel<T, CB>), grid, dim3(NW * 64), 0, s, g);
  else hipLaunchKernelGGL((narrow_n_kernel<T, CB>), grid, dim3(NW * 64), 0, s, g);
  return hipGetLastError();
}

template <typename T>
hipError_t narrow(bool trans, const T* A, int64_t lda, const T* X, int64_t ldx, T* C,
                  int64_t ldc, int64_t M, int64_t K, int64_t L, int ncu, void* work,
                  size_t work_bytes, hipStream_t s) {
  const NPlan p = plan_narrow<T>(trans, M, K, L, ncu);
  if (work_bytes < narrow_bytes<T>(trans, M, K, L, ncu)) return hipErrorInvalidValue;
  char* w = static_cast<char*>(work);
  NArgs g;
  g.A = A; g.lda = lda; g.C = C; g.ldc = ldc;
  g.M = M; g.K = K; g.L = L;
  g.ks = p.ks; g.kchunk = p.kchunk;
  if (!trans) {
    T* Xt = reinterpret_cast<T*>(w);
    w += rup((int64_t)16 * p.cb * p.ldt * sizeof(T) + 256, 256);
    int64_t grid = cdiv((int64_t)16 * p.cb * p.ldt, 256);
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(narrow_xt_kernel<T>, dim3((unsigned)grid), dim3(256), 0, s, X, ldx, K, L,
                       16 * p.cb, Xt, p.ldt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    g.X = Xt; g.ldx = p.ldt;
  } else {
    g.X = X; g.ldx = ldx;
  }
  g.part = w;
  hipError_t e;
  switch (p.cb) {
    case 1: e = run_narrow<T, 1>(trans, g, p.tiles, s); break;
    case 2: e = run_narrow<T, 2>(trans, g, p.tiles, s); break;
    case 3: e = run_narrow<T, 3>(trans, g, p.tiles, s); break;
    case 4: e = run_narrow<T, 4>(trans, g, p.tiles, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess || p.ks == 1) return e;
  int64_t grid = cdiv(M * L, 256);
  if (grid > 8192) grid = 8192;
  hipLaunchKernelGGL(narrow_sum_kernel<T>, dim3((unsigned)grid), dim3(256), 0, s,
                     static_cast<const T*>(g.part), p.ks, M, L, C, ldc);
  return hipGetLastError();
}

}  // namespace

// Used for FP32 A up to 32 columns, where it measured faster than the tiled
// kernel (l = 30 on a 20000 x 10000 A: 2.4 -> 3.1 TB/s for A X, 3.1 -> 3.3 for
// A^T X); FP64 and wider products measured faster in the tiled kernel.
bool narrow_applies(bool f32, int64_t lda, const void* A, int64_t L) {
  const int vec = f32 ? 4 : 2;
  return f32 && L >= 1 && L <= 32 && lda % vec == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0;
}

size_t narrow_work_bytes(bool f32, bool trans, int64_t M, int64_t K, int64_t L, int ncu) {
  return f32 ? narrow_bytes<float>(trans, M, K, L, ncu) : narrow_bytes<double>(trans, M, K, L, ncu);
}

hipError_t launch_narrow(bool f32, bool trans, const void* A, int64_t lda, const void* X,
                         int64_t ldx, void* C, int64_t ldc, int64_t M, int64_t K, int64_t L,
                         int ncu, void* work, size_t work_bytes, hipStream_t s) {
  if (M <= 0 || L <= 0) return hipSuccess;
  if (K <= 0) return hipErrorInvalidValue;
  if (f32)
    return narrow(trans, static_cast<const float*>(A), lda, static_cast<const float*>(X), ldx,
                  static_cast<float*>(C), ldc, M, K, L, ncu, work, work_bytes, s);
  return narrow(trans, static_cast<const double*>(A), lda, static_cast<const double*>(X), ldx,
                static_cast<double*>(C), ldc, M, K, L, ncu, work, work_bytes, s);
}

}  // namespace rsvd
