// Low-rank tile products P = sum_t X_t W_t^T on the matrix cores, with the
// epilogues that the path needs:
//  * OUT:   out = P + 2 dres A        (the rank-l terms of the derivative dA,
//                                      one per product with A, and the direct
//                                      part of d||A||_F^2)
//  * SUB:   A -= P and the partial sums of ||A - P||_F^2   (the deflation
//                                      A = A - Q_i B_i of the blocked QB,
//                                      Sec. 3.3, Alg. 7)
//  * NORM:  the partial sums of ||A - P||_F^2 only          (||A - Q Q^T A||_F^2)
//
// X_t is m x l and W_t is n x l (row-major, leading dimensions ldx / ldw;
// columns >= l are never read).  The reduction runs over the count * l
// columns of the concatenated factors in chunks of KC = 16.
//
// A workgroup of 8 waves owns a 128 x 128 tile of the output; wave w holds
// rows 32 (w & 3) .. +31 and columns 64 (w >> 2) .. +63 as 2 x 4 FP64 MFMA
// 16x16x4 accumulators.  Each chunk of X (128 x 16) and W (128 x 16) is read
// from global memory with 4 consecutive doubles per thread and staged in LDS
// (double buffer, next chunk prefetched into registers during the products),
// so every factor element is read once per tile.  A is read (and for SUB
// written) once, in the epilogue.
#include "common.h"
#include "internal.h"

namespace rsvd {
namespace {

constexpr int LR_NT = 512;
constexpr int LR_BM = 128;
constexpr int LR_BN = 128;
constexpr int LR_KC = 16;
constexpr int LR_LD = LR_KC + 1;    // LDS row length (doubles)

enum : int { LR_OUT = 0, LR_SUB = 1, LR_NORM = 2 };

template <int MODE>
__global__ __launch_bounds__(LR_NT) void lowrank_kernel(LowRank t, int64_t m, int64_t n,
                                                        double* __restrict__ A, int64_t lda,
                                                        const double* __restrict__ dres,
                                                        double* __restrict__ out, int64_t ldo,
                                                        double* __restrict__ part) {
  __shared__ double Xs[2][LR_BM * LR_LD];
  __shared__ double Ws[2][LR_BN * LR_LD];
  __shared__ double red[LR_NT / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.y * LR_BM;
  const int64_t col0 = (int64_t)blockIdx.x * LR_BN;
  const int wr = (wave & 3) * 32, wc = (wave >> 2) * 64;
  // loader: row lr of the X and W chunks, columns lq .. lq+3 of the chunk
  const int lr = tid >> 2, lq = (tid & 3) * 4;
  const int64_t xrow = row0 + lr, wrow = col0 + lr;
  const bool xok = xrow < m, wok = wrow < n;
  const int l = t.l;
  const int kpt = (l + LR_KC - 1) / LR_KC;   // chunks per term
  const int nch = t.count * kpt;

  // Loads are unconditional, from clamped indices; what lies outside the
  // factors or the matrix is zeroed later, when it is used (a branch around a
  // load, or a select right after it, makes the compiler wait for the load
  // there, one load at a time).
  double xv[4], wv[4];
  auto gload = [&](int c) {
    const int term = c / kpt;
    const int k0 = (c - term * kpt) * LR_KC + lq;
    const double* X = t.X[term];
    const double* W = t.W[term];
    const int64_t xr = xok ? xrow : m - 1, wr_ = wok ? wrow : n - 1;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = min(k0 + i, l - 1);
      xv[i] = X[xr * t.ldx + k];
      wv[i] = W[wr_ * t.ldw + k];
    }
  };
  auto sstore = [&](int b, int c) {
    const int term = c / kpt;
    const int k0 = (c - term * kpt) * LR_KC + lq;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool kin = k0 + i < l;
      Xs[b][lr * LR_LD + lq + i] = (xok && kin) ? xv[i] : 0.0;
      Ws[b][lr * LR_LD + lq + i] = (wok && kin) ? wv[i] : 0.0;
    }
  };

  d4 acc[2][4];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[rb][ct] = d4{0.0, 0.0, 0.0, 0.0};

  gload(0);
  sstore(0, 0);
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    // the next chunk (the last one again at the end: unconditional, so the
    // staged registers are not phis); its loads go out before the products
    // and are waited for at the store after them
    const int cn = c + 1 < nch ? c + 1 : c;
    gload(cn);
    __builtin_amdgcn_sched_barrier(0);
    const double* xs = Xs[c & 1];
    const double* ws = Ws[c & 1];
#pragma unroll
    for (int kk = 0; kk < LR_KC / 4; ++kk) {
      const int k = kk * 4 + lk;
      const double a0 = xs[(wr + li) * LR_LD + k];
      const double a1 = xs[(wr + 16 + li) * LR_LD + k];
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const double bv = ws[(wc + ct * 16 + li) * LR_LD + k];
        acc[0][ct] = Mfma<double>::mma(a0, bv, acc[0][ct]);
        acc[1][ct] = Mfma<double>::mma(a1, bv, acc[1][ct]);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    sstore((c + 1) & 1, cn);   // (past the last chunk: a buffer no one reads)
    __syncthreads();
  }

  // the tile's entries of A (for OUT without dres, of out itself, unused),
  // all loads issued before any is used
  const bool needA = (MODE != LR_OUT) || (dres != nullptr);
  const double* Ab = needA ? A : out;
  const int64_t ldb = needA ? lda : ldo;
  double av[2][4][4];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int64_t col = min(col0 + wc + ct * 16 + li, n - 1);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = min(row0 + wr + rb * 16 + drow(lk, v), m - 1);
        av[rb][ct][v] = Ab[row * ldb + col];
      }
    }
  const double alpha = (MODE == LR_OUT && dres) ? 2.0 * dres[0] : 0.0;
  double s = 0.0;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int64_t col = col0 + wc + ct * 16 + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = row0 + wr + rb * 16 + drow(lk, v);
        const bool ok = row < m && col < n;
        const double p = acc[rb][ct][v];
        if (MODE == LR_OUT) {
          if (ok) out[row * ldo + col] = dres ? fma(alpha, av[rb][ct][v], p) : p;
        } else {
          // (a zero outside the matrix leaves the sum as it is)
          const double x = ok ? av[rb][ct][v] - p : 0.0;
          if (MODE == LR_SUB && ok) A[row * lda + col] = x;
          s = fma(x, x, s);
        }
      }
    }
  }
  if (MODE != LR_OUT) {
    s = wave_allsum(s);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (tid == 0) {
      double r = 0.0;
#pragma unroll
      for (int w = 0; w < LR_NT / 64; ++w) r += red[w];
      part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = r;
    }
  }
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
    double r = 0.0;
    for (int w = 0; w < SUM_NT / 64; ++w) r += red[w];
    out[0] = r;
  }
}

bool valid(const LowRank& t) {
  if (t.count < 1 || t.count > LR_MAX || t.l < 1) return false;
  for (int i = 0; i < t.count; ++i)
    if (!t.X[i] || !t.W[i]) return false;
  return true;
}

dim3 grid_of(int64_t m, int64_t n) {
  return dim3((unsigned)cdiv(n, LR_BN), (unsigned)cdiv(m, LR_BM));
}

}  // namespace

int64_t lowrank_tiles(int64_t m, int64_t n) { return cdiv(m, LR_BM) * cdiv(n, LR_BN); }

hipError_t launch_lowrank_out(const LowRank& t, int64_t m, int64_t n, const double* A,
                              int64_t lda, const double* dres, double* out, int64_t ldo,
                              hipStream_t st) {
  if (!valid(t)) return hipErrorInvalidValue;
  if (m <= 0 || n <= 0) return hipSuccess;
  // the OUT epilogue only reads A
  hipLaunchKernelGGL(lowrank_kernel<LR_OUT>, grid_of(m, n), dim3(LR_NT), 0, st, t, m, n,
                     const_cast<double*>(A), lda, dres, out, ldo, nullptr);
  return hipGetLastError();
}

hipError_t launch_lowrank_sub(const LowRank& t, int64_t m, int64_t n, double* A, int64_t lda,
                              bool store, double* part, double* norm2, hipStream_t st) {
  if (!valid(t) || m <= 0 || n <= 0) return hipErrorInvalidValue;
  if (store) {
    hipLaunchKernelGGL(lowrank_kernel<LR_SUB>, grid_of(m, n), dim3(LR_NT), 0, st, t, m, n, A, lda,
                       nullptr, nullptr, 0, part);
  } else {
    hipLaunchKernelGGL(lowrank_kernel<LR_NORM>, grid_of(m, n), dim3(LR_NT), 0, st, t, m, n, A,
                       lda, nullptr, nullptr, 0, part);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(SUM_NT), 0, st, part, lowrank_tiles(m, n), norm2);
  return hipGetLastError();
}

}  // namespace rsvd
