// Batched randomized SVD of many small FP32 matrices in one persistent
// launch: Alg. 5 (RSVD version II) with re-orthonormalization after every
// product (Sec. 3.2, s = 1), applied to each matrix of the batch on its own.
// The matrices are independent, as the blocks of Alg. 8 are, so each one is
// the work of a single workgroup:
//
//   Omega_i (n x l, Philox stream 0, batch = the matrix's index);
//   Y = A Omega; q times { Q = orth(Y); Z = A^T Q; Z = orth(Z); Y = A Z };
//   Q = orth(Y); B^T = A^T Q; Qh = orth(B^T); Rh = Qh^T B^T;
//   Rh = Uh diag(sigma) Vh^T (one-sided Jacobi); U = Q Vh_k, V = Qh Uh_k.
//
// A workgroup of 8 waves pops matrices off a work queue (an atomic counter;
// the host orders the queue by decreasing work) until it is empty, so the
// grid is one workgroup per CU whatever the batch size, and no workgroup
// ever waits for another.  Per matrix:
//  * passes over A (FP32 MFMA 16x16x4, FP32 accumulation): 128-row (or
//    128-column for A^T) tiles of A and 16-deep chunks of the skinny operand
//    staged in LDS with 16-byte loads, double-buffered;
//  * orth = CholeskyQR2 in FP64: Gram X^T X on FP64 MFMA, Cholesky and the
//    inverse of R in LDS, Q = Y R^{-1} on FP64 MFMA; a pivot below
//    1e-13 G_jj marks a dependent column (unit row of R, info bit 1);
//  * the Jacobi SVD of the l x l factor in LDS (the rotations of the
//    single-matrix small SVD);
//  * U and V on FP64 MFMA, written in FP32.
// Skinny matrices live in a per-workgroup slot of the workspace (L2-resident
// for the sizes of a batch), small factors in LDS (l <= 80).
#include "common.h"
#include "internal.h"
#include "jacobi_dev.h"
#include "philox_dev.h"

namespace rsvd {
namespace {

constexpr int BNT = 512;             // 8 waves
constexpr int BLMAX = BATCH_MAX_LP;  // lp <= 80
constexpr int SL = BLMAX + 1;        // LDS row stride of the small FP64 matrices
constexpr int ALD = 17;              // pass: A tile row stride (floats), 128 x 16
constexpr int ATLD = 132;            // pass A^T: A tile row stride (floats), 16 x 128
constexpr int XLD = 84;              // skinny chunk row stride (floats), 16 x lp
constexpr int STAGE_FLOATS = 2 * (128 * ALD + 16 * XLD);   // double buffer
constexpr double ETA_DEP = 1e-13;
constexpr int JAC_MAX_SWEEPS = 40;

struct Lds {
  double a[BLMAX * SL];
  double b[BLMAX * SL];
  float stage[STAGE_FLOATS];         // also the Gram partials (8 x 256 doubles)
  double sig[BLMAX];
  double dgn[BLMAX];
  int flag;
  int item;
};
static_assert(STAGE_FLOATS * sizeof(float) >= 8 * 256 * sizeof(double), "Gram partials");

__device__ __forceinline__ double to_d(float x) { return (double)x; }
__device__ __forceinline__ double to_d(double x) { return x; }
template <typename T> __device__ __forceinline__ T from_d(double x);
template <> __device__ __forceinline__ float from_d<float>(double x) { return (float)x; }
template <> __device__ __forceinline__ double from_d<double>(double x) { return x; }

__device__ __forceinline__ float4 ld4(const float* p) {
  return *reinterpret_cast<const float4*>(p);
}

// Omega (n x lp, FP32): column j < l holds normals j*n .. j*n + n-1 of stream
// 0, batch `batch`; columns l .. lp-1 are zero.
__device__ __noinline__ void b_sketch(float* Om, int64_t n, int l, int lp, uint32_t k0,
                                      uint32_t k1, uint32_t batch) {
  const int tid = threadIdx.x;
  const int64_t total = n * l;
  const int64_t npairs = (total + 1) / 2;
  for (int64_t p = tid; p < npairs; p += BNT) {
    const Words w = philox10((uint32_t)p, (uint32_t)((uint64_t)p >> 32), 0u, batch, k0, k1);
    double z[2];
    box_muller(w, z[0], z[1]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t t = 2 * p + h;
      if (t < total) {
        const int64_t j = t / n, i = t - (t / n) * n;
        Om[i * lp + j] = (float)z[h];
      }
    }
  }
  if (lp > l) {
    const int pad = lp - l;
    for (int64_t e = tid; e < n * pad; e += BNT) {
      const int64_t i = e / pad;
      Om[i * lp + l + (e - i * pad)] = 0.0f;
    }
  }
  __syncthreads();
}

// Y (m x lp) = A X, A m x n (FP32, lda % 4 == 0), X n x lp (FP32).
__device__ __noinline__ void b_pass_n(Lds& s, const float* __restrict__ A, int64_t lda, int64_t m,
                                      int64_t n, const float* __restrict__ X,
                                      float* __restrict__ Y, int lp) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ncb = lp / 16;
  float* As[2] = {s.stage, s.stage + 128 * ALD};
  float* Xs[2] = {s.stage + 2 * 128 * ALD, s.stage + 2 * 128 * ALD + 16 * XLD};
  const int ar = tid >> 2, ac = (tid & 3) * 4;          // A tile: row, 4 columns
  const int xq = lp / 4;                                // float4 per X row
  const int xr = tid / xq, xc = (tid - (tid / xq) * xq) * 4;
  const bool xact = tid < 16 * xq;
  const int64_t nkc = cdiv(n, 16);
  for (int64_t row0 = 0; row0 < m; row0 += 128) {
    f4 acc[5];
#pragma unroll
    for (int cb = 0; cb < 5; ++cb) acc[cb] = f4{0.f, 0.f, 0.f, 0.f};
    float4 av, xv;
    auto gload = [&](int64_t kc) {
      const int64_t k0 = kc * 16;
      const int64_t r = row0 + ar, c = k0 + ac;
      av = make_float4(0.f, 0.f, 0.f, 0.f);
      if (r < m && c < lda) {
        av = ld4(A + r * lda + c);
        if (c + 0 >= n) av.x = 0.f;
        if (c + 1 >= n) av.y = 0.f;
        if (c + 2 >= n) av.z = 0.f;
        if (c + 3 >= n) av.w = 0.f;
      }
      xv = make_float4(0.f, 0.f, 0.f, 0.f);
      if (xact && k0 + xr < n) xv = ld4(X + (k0 + xr) * lp + xc);
    };
    auto sstore = [&](int b) {
      float* a = As[b] + ar * ALD + ac;
      a[0] = av.x; a[1] = av.y; a[2] = av.z; a[3] = av.w;
      if (xact) {
        float* x = Xs[b] + xr * XLD + xc;
        x[0] = xv.x; x[1] = xv.y; x[2] = xv.z; x[3] = xv.w;
      }
    };
    gload(0);
    sstore(0);
    __syncthreads();
    for (int64_t kc = 0; kc < nkc; ++kc) {
      const bool more = kc + 1 < nkc;
      if (more) gload(kc + 1);
      const float* as = As[kc & 1];
      const float* xs = Xs[kc & 1];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const float a = as[(wave * 16 + li) * ALD + kk * 4 + lk];
#pragma unroll
        for (int cb = 0; cb < 5; ++cb)
          if (cb < ncb)
            acc[cb] = Mfma<float>::mma(a, xs[(kk * 4 + lk) * XLD + cb * 16 + li], acc[cb]);
      }
      if (more) sstore((kc + 1) & 1);
      __syncthreads();
    }
#pragma unroll
    for (int cb = 0; cb < 5; ++cb) {
      if (cb < ncb) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t r = row0 + wave * 16 + Mfma<float>::row(lk, v);
          if (r < m) Y[r * lp + cb * 16 + li] = acc[cb][v];
        }
      }
    }
  }
  __syncthreads();
}

// Z (n x lp) = A^T X, A m x n (FP32, lda % 4 == 0), X m x lp (FP32).
__device__ __noinline__ void b_pass_t(Lds& s, const float* __restrict__ A, int64_t lda, int64_t m,
                                      int64_t n, const float* __restrict__ X,
                                      float* __restrict__ Z, int lp) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ncb = lp / 16;
  float* As[2] = {s.stage, s.stage + 16 * ATLD};
  float* Xs[2] = {s.stage + 2 * 16 * ATLD, s.stage + 2 * 16 * ATLD + 16 * XLD};
  const int ar = tid >> 5, ac = (tid & 31) * 4;         // A tile: row of 16, 4 columns of 128
  const int xq = lp / 4;
  const int xr = tid / xq, xc = (tid - (tid / xq) * xq) * 4;
  const bool xact = tid < 16 * xq;
  const int64_t nkc = cdiv(m, 16);
  for (int64_t col0 = 0; col0 < n; col0 += 128) {
    f4 acc[5];
#pragma unroll
    for (int cb = 0; cb < 5; ++cb) acc[cb] = f4{0.f, 0.f, 0.f, 0.f};
    float4 av, xv;
    auto gload = [&](int64_t kc) {
      const int64_t r0 = kc * 16;
      const int64_t r = r0 + ar, c = col0 + ac;
      av = make_float4(0.f, 0.f, 0.f, 0.f);
      if (r < m && c < lda) {
        av = ld4(A + r * lda + c);
        if (c + 0 >= n) av.x = 0.f;
        if (c + 1 >= n) av.y = 0.f;
        if (c + 2 >= n) av.z = 0.f;
        if (c + 3 >= n) av.w = 0.f;
      }
      xv = make_float4(0.f, 0.f, 0.f, 0.f);
      if (xact && r0 + xr < m) xv = ld4(X + (r0 + xr) * lp + xc);
    };
    auto sstore = [&](int b) {
      float* a = As[b] + ar * ATLD + ac;
      a[0] = av.x; a[1] = av.y; a[2] = av.z; a[3] = av.w;
      if (xact) {
        float* x = Xs[b] + xr * XLD + xc;
        x[0] = xv.x; x[1] = xv.y; x[2] = xv.z; x[3] = xv.w;
      }
    };
    gload(0);
    sstore(0);
    __syncthreads();
    for (int64_t kc = 0; kc < nkc; ++kc) {
      const bool more = kc + 1 < nkc;
      if (more) gload(kc + 1);
      const float* as = As[kc & 1];
      const float* xs = Xs[kc & 1];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        // A^T[col][row]: column wave*16 + li of the tile, row kk*4 + lk
        const float a = as[(kk * 4 + lk) * ATLD + wave * 16 + li];
#pragma unroll
        for (int cb = 0; cb < 5; ++cb)
          if (cb < ncb)
            acc[cb] = Mfma<float>::mma(a, xs[(kk * 4 + lk) * XLD + cb * 16 + li], acc[cb]);
      }
      if (more) sstore((kc + 1) & 1);
      __syncthreads();
    }
#pragma unroll
    for (int cb = 0; cb < 5; ++cb) {
      if (cb < ncb) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t c = col0 + wave * 16 + Mfma<float>::row(lk, v);
          if (c < n) Z[c * lp + cb * 16 + li] = acc[cb][v];
        }
      }
    }
  }
  __syncthreads();
}

// out (lp x lp in LDS, stride SL) = X^T Y for X, Y rows x lp (FP32 or FP64),
// on FP64 MFMA.  Tasks (16x16 block, row slice) are spread over the 8 waves;
// with fewer than 8 blocks the rows are cut into slices whose partial blocks
// are added in slice order.
template <typename TX, typename TY>
__device__ __noinline__ void b_xty(Lds& s, const TX* __restrict__ X, const TY* __restrict__ Y, int64_t rows,
                      int lp, double* out) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nb = lp / 16, nblk = nb * nb;
  const int S = nblk >= 8 ? 1 : 8 / nblk;
  const int ntask = nblk * S;
  const int64_t nsteps = cdiv(rows, 4);
  double* part = reinterpret_cast<double*>(s.stage);
  for (int task = wave; task < ntask; task += 8) {
    const int b = task / S, sl = task - (task / S) * S;
    const int bi = b / nb, bj = b - (b / nb) * nb;
    const int64_t st0 = sl * nsteps / S, st1 = (sl + 1) * nsteps / S;
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
    for (int64_t st = st0; st < st1; ++st) {
      const int64_t r = st * 4 + lk;
      const bool ok = r < rows;
      const double a = ok ? to_d(X[r * lp + bi * 16 + li]) : 0.0;
      const double bv = ok ? to_d(Y[r * lp + bj * 16 + li]) : 0.0;
      acc = Mfma<double>::mma(a, bv, acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (S == 1)
        out[(bi * 16 + drow(lk, v)) * SL + bj * 16 + li] = acc[v];
      else
        part[task * 256 + drow(lk, v) * 16 + li] = acc[v];
    }
  }
  __syncthreads();
  if (S > 1) {
    for (int e = tid; e < nblk * 256; e += BNT) {
      const int b = e >> 8, rr = (e >> 4) & 15, cc = e & 15;
      const int bi = b / nb, bj = b - (b / nb) * nb;
      double t = 0.0;
      for (int sl = 0; sl < S; ++sl) t += part[(b * S + sl) * 256 + rr * 16 + cc];
      out[(bi * 16 + rr) * SL + bj * 16 + cc] = t;
    }
    __syncthreads();
  }
}

// Cholesky G = R^T R of the leading l x l block (G, R in LDS, stride SL;
// G is overwritten).  R is upper triangular with zeros below the diagonal
// and the identity in rows / columns l .. lp-1.  A pivot <= ETA_DEP * G_jj
// (or not positive) gives a unit row and sets s.flag.
__device__ __noinline__ void b_chol(Lds& s, double* G, double* R, int l, int lp) {
  const int tid = threadIdx.x;
  for (int e = tid; e < lp * lp; e += BNT) {
    const int r = e / lp, c = e - (e / lp) * lp;
    R[r * SL + c] = (r == c && r >= l) ? 1.0 : 0.0;
  }
  for (int i = tid; i < l; i += BNT) s.dgn[i] = G[i * SL + i];
  __syncthreads();
  for (int j = 0; j < l; ++j) {
    const double d = G[j * SL + j];
    const bool dep = !(d > ETA_DEP * s.dgn[j]);
    const double sq = dep ? 1.0 : sqrt(d);
    for (int t = tid; t < l - j; t += BNT) {
      const int c = j + t;
      R[j * SL + c] = dep ? (t == 0 ? 1.0 : 0.0) : G[j * SL + c] / sq;
    }
    if (dep && tid == 0) s.flag = 1;
    __syncthreads();
    const int nr = l - j - 1;
    for (int e = tid; e < nr * nr; e += BNT) {
      const int r = j + 1 + e / nr, c = j + 1 + (e - (e / nr) * nr);
      if (r <= c) G[r * SL + c] -= R[j * SL + r] * R[j * SL + c];
    }
    __syncthreads();
  }
}

// X = R^{-1} (upper triangular, lp x lp in LDS): thread c solves R x = e_c by
// back substitution for column c < l; rows / columns l .. lp-1 are the identity.
__device__ __noinline__ void b_rinv(const double* R, double* X, int l, int lp) {
  const int tid = threadIdx.x;
  for (int e = tid; e < lp * lp; e += BNT) {
    const int r = e / lp, c = e - (e / lp) * lp;
    X[r * SL + c] = (r == c && r >= l) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int c = tid; c < l; c += BNT) {
    for (int i = c; i >= 0; --i) {
      double t = (i == c) ? 1.0 : 0.0;
      for (int u = i + 1; u <= c; ++u) t -= R[i * SL + u] * X[u * SL + c];
      X[i * SL + c] = t / R[i * SL + i];
    }
  }
  __syncthreads();
}

// Out (rows x ncols, ldo) = In (rows x K, ld lp) B (B in LDS, stride SL, K x N
// with N = rup(ncols, 16) <= 80), on FP64 MFMA.
template <typename TI, typename TO>
__device__ __noinline__ void b_apply(const TI* __restrict__ In, int lp, int64_t rows, int K, const double* B,
                        int ncols, TO* __restrict__ Out, int64_t ldo) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ncb = (ncols + 15) / 16;
  const int64_t nrb = cdiv(rows, 16);
  for (int64_t rb = wave; rb < nrb; rb += 8) {
    d4 acc[5];
#pragma unroll
    for (int cb = 0; cb < 5; ++cb) acc[cb] = d4{0.0, 0.0, 0.0, 0.0};
    const int64_t r = rb * 16 + li;
    const bool ok = r < rows;
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int k = k0 + lk;
      const double a = (ok && k < K) ? to_d(In[r * lp + k]) : 0.0;
#pragma unroll
      for (int cb = 0; cb < 5; ++cb)
        if (cb < ncb) {
          const double bv = k < K ? B[k * SL + cb * 16 + li] : 0.0;
          acc[cb] = Mfma<double>::mma(a, bv, acc[cb]);
        }
    }
#pragma unroll
    for (int cb = 0; cb < 5; ++cb) {
      if (cb < ncb) {
        const int c = cb * 16 + li;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t rr = rb * 16 + drow(lk, v);
          if (rr < rows && c < ncols) Out[rr * ldo + c] = from_d<TO>(acc[cb][v]);
        }
      }
    }
  }
  __syncthreads();
}

// Q (rows x lp) = orth(In) by CholeskyQR2 in FP64; T (rows x lp FP64) holds
// the first pass.
template <typename TI, typename TO>
__device__ void b_orth(Lds& s, const TI* In, int64_t rows, int l, int lp, double* T, TO* Q) {
  b_xty(s, In, In, rows, lp, s.a);
  b_chol(s, s.a, s.b, l, lp);
  b_rinv(s.b, s.a, l, lp);
  b_apply(In, lp, rows, lp, s.a, lp, T, lp);
  b_xty(s, T, T, rows, lp, s.a);
  b_chol(s, s.a, s.b, l, lp);
  b_rinv(s.b, s.a, l, lp);
  b_apply(T, lp, rows, lp, s.a, lp, Q, lp);
}

// One-sided Jacobi on the l x l Rh held in s.a (stride SL): W = Rh (columns
// contiguous, in s.b ... ) -- see the body for the buffer use.  Writes the k
// largest sigma to S and Uh, Vh (l x k, ld lp) to global scratch.
__device__ __noinline__ void b_jacobi(Lds& s, int l, int k, double* S, double* Uh, double* Vh, int lp,
                         int32_t* info) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // W (column j contiguous, ld l) into s.b from Rh in s.a; V = I into s.a
  double* W = s.b;
  double* V = s.a;
  for (int e = tid; e < l * l; e += BNT) {
    const int j = e / l, i = e - (e / l) * l;
    W[j * l + i] = s.a[i * SL + j];
  }
  __syncthreads();
  for (int e = tid; e < l * l; e += BNT) {
    const int j = e / l, i = e - (e / l) * l;
    V[j * l + i] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const double tol = (double)l * 2.220446049250313e-16;
  const int N = l + (l & 1);
  int sweep = 0;
  bool converged = (l < 2);
  while (!converged && sweep < JAC_MAX_SWEEPS) {
    ++sweep;
    if (tid == 0) s.flag = 0;
    __syncthreads();
    for (int r = 0; r < N - 1; ++r) {
      for (int pi = wave; pi < N / 2; pi += BNT / 64) {
        int a = rr_player(pi, r, N), b = rr_player(N - 1 - pi, r, N);
        if (a >= l || b >= l) continue;
        if (a > b) { const int t = a; a = b; b = t; }
        if (rotate_pair(W + a * l, W + b * l, V + a * l, V + b * l, l, lane, tol) && lane == 0)
          s.flag = 1;
      }
      __syncthreads();
    }
    converged = (s.flag == 0);
    __syncthreads();
  }
  if (!converged && tid == 0) info_or(info, INFO_JACOBI_CAP);
  jacobi_finish<BNT>(W, V, l, l, k, s.sig, S, Uh, lp, Vh, lp);
  __syncthreads();
}

// B (in LDS, stride SL, lp x rup(k,16)) = the l x k matrix M (ld lp, global),
// zero elsewhere
__device__ void b_load_small(const double* M, int l, int k, int lp, double* B) {
  const int nc = (int)rup(k, 16);
  for (int e = threadIdx.x; e < lp * nc; e += BNT) {
    const int r = e / nc, c = e - (e / nc) * nc;
    B[r * SL + c] = (r < l && c < k) ? M[r * lp + c] : 0.0;
  }
  __syncthreads();
}

__global__ __launch_bounds__(BNT) void batch_rsvd_kernel(BatchArgs g) {
  __shared__ Lds s;
  const int tid = threadIdx.x;
  char* slot = g.scratch + (int64_t)blockIdx.x * g.slot_bytes;
  float* Om = reinterpret_cast<float*>(slot + g.off_om);
  float* Y = reinterpret_cast<float*>(slot + g.off_y);
  float* Q = reinterpret_cast<float*>(slot + g.off_q);
  float* Z = reinterpret_cast<float*>(slot + g.off_z);
  float* Zq = reinterpret_cast<float*>(slot + g.off_zq);
  double* T = reinterpret_cast<double*>(slot + g.off_t);
  double* Qh = reinterpret_cast<double*>(slot + g.off_qh);
  double* Uh = reinterpret_cast<double*>(slot + g.off_uh);
  double* Vh = reinterpret_cast<double*>(slot + g.off_vh);
  for (;;) {
    if (tid == 0) s.item = atomicAdd(g.counter, 1);
    __syncthreads();
    const int64_t it = s.item;
    __syncthreads();
    if (it >= g.count) break;
    const BatchDesc d = g.desc[it];
    const int64_t m = d.m, n = d.n;
    const int l = d.l, lp = d.lp, k = d.k;
    const float* A = g.A + d.a_off;
    if (tid == 0) s.flag = 0;
    __syncthreads();
    b_sketch(Om, n, l, lp, g.k0, g.k1, (uint32_t)d.index);
    b_pass_n(s, A, d.lda, m, n, Om, Y, lp);
    for (int j = 0; j < g.q; ++j) {
      b_orth(s, Y, m, l, lp, T, Q);
      b_pass_t(s, A, d.lda, m, n, Q, Z, lp);
      b_orth(s, Z, n, l, lp, T, Zq);
      b_pass_n(s, A, d.lda, m, n, Zq, Y, lp);
    }
    b_orth(s, Y, m, l, lp, T, Q);
    b_pass_t(s, A, d.lda, m, n, Q, Z, lp);          // B^T
    b_orth(s, Z, n, l, lp, T, Qh);
    b_xty(s, Qh, Z, n, lp, s.a);                    // Rh = Qh^T B^T
    if (tid == 0 && s.flag) info_or(g.info, INFO_ORTH_FALLBACK);
    b_jacobi(s, l, k, g.S + d.s_off, Uh, Vh, lp, g.info);
    b_load_small(Vh, l, k, lp, s.a);
    b_apply(Q, lp, m, lp, s.a, k, g.U + d.u_off, (int64_t)k);
    b_load_small(Uh, l, k, lp, s.a);
    b_apply(Qh, lp, n, lp, s.a, k, g.V + d.v_off, (int64_t)k);
  }
}

}  // namespace

hipError_t launch_batch_rsvd(const BatchArgs& g, int grid, hipStream_t st) {
  if (grid < 1 || g.count < 1) return hipErrorInvalidValue;
  hipError_t e = launch_set_word(g.counter, 0, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(batch_rsvd_kernel, dim3((unsigned)grid), dim3(BNT), 0, st, g);
  return hipGetLastError();
}

}  // namespace rsvd
