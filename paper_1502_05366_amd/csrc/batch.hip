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
//    128-column for A^T) tiles of A and 64-deep chunks of A and the skinny
//    operand staged in LDS with 16-byte loads, double-buffered;
//  * orth = CholeskyQR2 in FP64: Gram X^T X on FP64 MFMA (upper blocks,
//    rows split over the waves), Cholesky (one barrier per step) and the
//    inverse of R (four lanes per column) in LDS, Q = Y R^{-1} on FP64 MFMA;
//    a pivot below 1e-13 G_jj marks a dependent column (unit row of R, info
//    bit 1), which after the first pass is replaced by a fresh Gaussian
//    column (Philox stream 7) for the second pass to orthonormalize, as the
//    single-matrix orth does; a non-finite pivot sets info bit 8; the second
//    pass is skipped when the first already left ||Q^T Q - I||_F <= 2^-30,
//    far below the FP32 rounding of the bases;
//  * the Jacobi SVD of the l x l factor in LDS (the rotations of the
//    single-matrix small SVD, one column pair per 16 lanes);
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
// Pass shapes (the batch autotuner picks one per matrix): a pass over A
// takes tiles of TM = 128 RPW rows of A (A^T: columns), RPW 16-row blocks
// per wave, and KC-deep chunks of A and of the skinny operand, double
// buffered in LDS.
//   variant 0: TM = 128, KC = 64;  variant 1: TM = 256, KC = 32;
//   variant 2: TM = 128, KC = 32.
// LDS row strides (floats), chosen so that the operand reads of a wave hit
// distinct banks: lane (li, lk) reads row li (stride KC + 4 = 4 or 36 mod
// 64) at column lk of the A tile, and row lk (stride 80 = 16 mod 64, TM + 16
// = 16 mod 64) at column li of the skinny chunk and of the A^T tile.
template <int RPW, int KC> struct PassShape {
  static constexpr int TM = 128 * RPW;
  static constexpr int ALD = KC + 4;           // A tile row stride, TM x KC
  static constexpr int ATLD = TM + 16;         // A^T tile row stride, KC x TM
  static constexpr int STAGE_N = 2 * (TM * ALD + KC * 80);
  static constexpr int STAGE_T = 2 * (KC * ATLD + KC * 80);
  static constexpr int STAGE = STAGE_N > STAGE_T ? STAGE_N : STAGE_T;
};
constexpr int XLD = 80;              // skinny chunk row stride, KC x lp
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int STAGE_FLOATS = cmax(PassShape<1, 64>::STAGE,
                                  cmax(PassShape<2, 32>::STAGE, PassShape<1, 32>::STAGE));
constexpr double ETA_DEP = 1e-13;
constexpr int JAC_MAX_SWEEPS = 40;

// LDS of a workgroup: the passes stage their tiles over the whole union; the
// small factorizations use a, b (lp x lp FP64, stride SL) and the Gram
// partials.  Declared at namespace scope so that every helper addresses it
// as LDS even when it is not inlined.
struct alignas(16) BatchLds {
  union {
    struct {
      double a[BLMAX * SL];
      double b[BLMAX * SL];
      double part[8 * 256];
    } sm;
    float stage[STAGE_FLOATS];
  } u;
  double sig[BLMAX];
  double dgn[BLMAX];
  int depc[BLMAX];     // columns found dependent by the last Cholesky
  int ndep;            // how many
  int nonfinite;       // a non-finite pivot was met (this matrix)
  int flag;
  int item;
};
__shared__ BatchLds g_lds;

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

// A float4 of row r of A at column c (c % 4 == 0, c < lda), entries at
// columns >= n taken as zero
__device__ __forceinline__ float4 ld_a4(const float* A, int64_t lda, int64_t m, int64_t n,
                                        int64_t r, int64_t c) {
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (r < m && c < lda) {
    v = ld4(A + r * lda + c);
    if (c + 0 >= n) v.x = 0.f;
    if (c + 1 >= n) v.y = 0.f;
    if (c + 2 >= n) v.z = 0.f;
    if (c + 3 >= n) v.w = 0.f;
  }
  return v;
}

// 16-byte store (p is 16-byte aligned: every tile stride is a multiple of 4)
__device__ __forceinline__ void st4(float* p, const float4& v) {
  *reinterpret_cast<float4*>(p) = v;
}

// Y (m x lp) = A X, A m x n (FP32, lda % 4 == 0), X n x lp (FP32), lp = 16 NCB.
// Row tiles of TM (16 RPW rows per wave), KC-deep chunks of A and X in LDS.
template <int NCB, int RPW, int KC>
__device__ __noinline__ void b_pass_n(const float* __restrict__ A, int64_t lda, int64_t m,
                                      int64_t n, const float* __restrict__ X,
                                      float* __restrict__ Y) {
  using S = PassShape<RPW, KC>;
  constexpr int lp = 16 * NCB, TM = S::TM, ALD = S::ALD;
  constexpr int AF4 = TM * KC / 4 / BNT;             // float4 of the A tile per thread
  constexpr int KQ = KC / 4;                          // float4 per A tile row
  constexpr int XF4 = (KC * 20 + BNT - 1) / BNT;      // float4 of the X chunk per thread (lp <= 80)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  float* st = g_lds.u.stage;
  const int xq = lp / 4;                                // float4 per X row
  const int xn = KC * xq;                               // float4 per X chunk
  const int64_t nkc = cdiv(n, KC);
  for (int64_t row0 = 0; row0 < m; row0 += TM) {
    f4 acc[RPW][NCB];
#pragma unroll
    for (int rb = 0; rb < RPW; ++rb)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = f4{0.f, 0.f, 0.f, 0.f};
    float4 av[AF4], xv[XF4];
    auto gload = [&](int64_t kc) {
      const int64_t k0 = kc * KC;
#pragma unroll
      for (int u = 0; u < AF4; ++u) {
        const int idx = tid + BNT * u;
        av[u] = ld_a4(A, lda, m, n, row0 + idx / KQ, k0 + (idx % KQ) * 4);
      }
#pragma unroll
      for (int u = 0; u < XF4; ++u) {
        const int idx = tid + BNT * u;
        const int xr = idx / xq, xc = (idx - (idx / xq) * xq) * 4;
        xv[u] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (idx < xn && k0 + xr < n) xv[u] = ld4(X + (k0 + xr) * lp + xc);
      }
    };
    auto sstore = [&](int b) {
      float* as = st + b * (TM * ALD);
      float* xs = st + 2 * TM * ALD + b * (KC * XLD);
#pragma unroll
      for (int u = 0; u < AF4; ++u) {
        const int idx = tid + BNT * u;
        st4(as + (idx / KQ) * ALD + (idx % KQ) * 4, av[u]);
      }
#pragma unroll
      for (int u = 0; u < XF4; ++u) {
        const int idx = tid + BNT * u;
        if (idx < xn) {
          const int xr = idx / xq, xc = (idx - (idx / xq) * xq) * 4;
          st4(xs + xr * XLD + xc, xv[u]);
        }
      }
    };
    gload(0);
    sstore(0);
    __syncthreads();
    for (int64_t kc = 0; kc < nkc; ++kc) {
      const bool more = kc + 1 < nkc;
      if (more) gload(kc + 1);
      const float* as = st + (kc & 1) * (TM * ALD);
      const float* xs = st + 2 * TM * ALD + (kc & 1) * (KC * XLD);
#pragma unroll
      for (int kk = 0; kk < KC / 4; ++kk) {
#pragma unroll
        for (int rb = 0; rb < RPW; ++rb) {
          const float a = as[((wave * RPW + rb) * 16 + li) * ALD + kk * 4 + lk];
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
            acc[rb][cb] =
                Mfma<float>::mma(a, xs[(kk * 4 + lk) * XLD + cb * 16 + li], acc[rb][cb]);
        }
        if (kk % 4 == 3) __builtin_amdgcn_sched_barrier(0);
      }
      if (more) sstore((kc + 1) & 1);
      __syncthreads();
    }
#pragma unroll
    for (int rb = 0; rb < RPW; ++rb)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t r = row0 + (wave * RPW + rb) * 16 + Mfma<float>::row(lk, v);
          if (r < m) Y[r * lp + cb * 16 + li] = acc[rb][cb][v];
        }
      }
  }
  __syncthreads();
}

// Z (n x lp) = A^T X, A m x n (FP32, lda % 4 == 0), X m x lp (FP32), lp = 16 NCB.
// Tiles of TM columns of A (16 RPW per wave), KC-row chunks of A and X in LDS.
template <int NCB, int RPW, int KC>
__device__ __noinline__ void b_pass_t(const float* __restrict__ A, int64_t lda, int64_t m,
                                      int64_t n, const float* __restrict__ X,
                                      float* __restrict__ Z) {
  using S = PassShape<RPW, KC>;
  constexpr int lp = 16 * NCB, TM = S::TM, ATLD = S::ATLD;
  constexpr int AF4 = TM * KC / 4 / BNT;
  constexpr int TQ = TM / 4;                          // float4 per A tile row
  constexpr int XF4 = (KC * 20 + BNT - 1) / BNT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  float* st = g_lds.u.stage;
  const int xq = lp / 4;
  const int xn = KC * xq;
  const int64_t nkc = cdiv(m, KC);
  for (int64_t col0 = 0; col0 < n; col0 += TM) {
    f4 acc[RPW][NCB];
#pragma unroll
    for (int rb = 0; rb < RPW; ++rb)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = f4{0.f, 0.f, 0.f, 0.f};
    float4 av[AF4], xv[XF4];
    auto gload = [&](int64_t kc) {
      const int64_t r0 = kc * KC;
#pragma unroll
      for (int u = 0; u < AF4; ++u) {
        const int idx = tid + BNT * u;
        av[u] = ld_a4(A, lda, m, n, r0 + idx / TQ, col0 + (idx % TQ) * 4);
      }
#pragma unroll
      for (int u = 0; u < XF4; ++u) {
        const int idx = tid + BNT * u;
        const int xr = idx / xq, xc = (idx - (idx / xq) * xq) * 4;
        xv[u] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (idx < xn && r0 + xr < m) xv[u] = ld4(X + (r0 + xr) * lp + xc);
      }
    };
    auto sstore = [&](int b) {
      float* as = st + b * (KC * ATLD);
      float* xs = st + 2 * KC * ATLD + b * (KC * XLD);
#pragma unroll
      for (int u = 0; u < AF4; ++u) {
        const int idx = tid + BNT * u;
        st4(as + (idx / TQ) * ATLD + (idx % TQ) * 4, av[u]);
      }
#pragma unroll
      for (int u = 0; u < XF4; ++u) {
        const int idx = tid + BNT * u;
        if (idx < xn) {
          const int xr = idx / xq, xc = (idx - (idx / xq) * xq) * 4;
          st4(xs + xr * XLD + xc, xv[u]);
        }
      }
    };
    gload(0);
    sstore(0);
    __syncthreads();
    for (int64_t kc = 0; kc < nkc; ++kc) {
      const bool more = kc + 1 < nkc;
      if (more) gload(kc + 1);
      const float* as = st + (kc & 1) * (KC * ATLD);
      const float* xs = st + 2 * KC * ATLD + (kc & 1) * (KC * XLD);
#pragma unroll
      for (int kk = 0; kk < KC / 4; ++kk) {
#pragma unroll
        for (int rb = 0; rb < RPW; ++rb) {
          // A^T[col][row]: column (wave RPW + rb) 16 + li of the tile, row kk*4 + lk
          const float a = as[(kk * 4 + lk) * ATLD + (wave * RPW + rb) * 16 + li];
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
            acc[rb][cb] =
                Mfma<float>::mma(a, xs[(kk * 4 + lk) * XLD + cb * 16 + li], acc[rb][cb]);
        }
        if (kk % 4 == 3) __builtin_amdgcn_sched_barrier(0);
      }
      if (more) sstore((kc + 1) & 1);
      __syncthreads();
    }
#pragma unroll
    for (int rb = 0; rb < RPW; ++rb)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t c = col0 + (wave * RPW + rb) * 16 + Mfma<float>::row(lk, v);
          if (c < n) Z[c * lp + cb * 16 + li] = acc[rb][cb][v];
        }
      }
  }
  __syncthreads();
}

// a (lp x lp, stride SL) = X^T Y for X, Y rows x lp (FP32 or FP64), on FP64
// MFMA.  Tasks (16x16 block, row slice) are spread over the 8 waves; with
// fewer than 8 blocks the rows are cut into slices whose partial blocks are
// added in slice order.  Eight 4-row steps are loaded before their products.
template <typename TX, typename TY>
__device__ __noinline__ void b_xty(const TX* __restrict__ X, const TY* __restrict__ Y,
                                   int64_t rows, int lp) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nb = lp / 16, nblk = nb * nb;
  const int S = nblk >= 8 ? 1 : 8 / nblk;
  const int ntask = nblk * S;
  const int64_t nsteps = cdiv(rows, 4);
  double* out = g_lds.u.sm.a;
  double* part = g_lds.u.sm.part;
  for (int task = wave; task < ntask; task += 8) {
    const int b = task / S, sl = task - (task / S) * S;
    const int bi = b / nb, bj = b - (b / nb) * nb;
    const int64_t st0 = sl * nsteps / S, st1 = (sl + 1) * nsteps / S;
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
    for (int64_t st = st0; st < st1; st += 8) {
      double av[8], bv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t r = (st + u) * 4 + lk;
        const bool ok = st + u < st1 && r < rows;
        av[u] = ok ? to_d(X[r * lp + bi * 16 + li]) : 0.0;
        bv[u] = ok ? to_d(Y[r * lp + bj * 16 + li]) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = Mfma<double>::mma(av[u], bv[u], acc);
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

// a (upper 16x16 blocks, stride SL) = X^T X for X rows x lp (FP32 or FP64)
// on FP64 MFMA.  Wave w forms every upper block over its eighth of the rows
// (two 4-row steps loaded before their products); the eight partial Grams
// are added into a in wave order.
template <int NB, typename TX>
__device__ __noinline__ void b_gram(const TX* __restrict__ X, int64_t rows) {
  constexpr int lp = 16 * NB, nb = NB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  double* out = g_lds.u.sm.a;
  const int64_t nsteps = cdiv(rows, 4);
  const int64_t st0 = wave * nsteps / 8, st1 = (wave + 1) * nsteps / 8;
  d4 acc[NB][NB];
#pragma unroll
  for (int bi = 0; bi < NB; ++bi)
#pragma unroll
    for (int bj = bi; bj < NB; ++bj) acc[bi][bj] = d4{0.0, 0.0, 0.0, 0.0};
  for (int64_t st = st0; st < st1; st += 2) {
    double xv[2][NB];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t r = (st + u) * 4 + lk;
      const bool ok = st + u < st1 && r < rows;
#pragma unroll
      for (int bi = 0; bi < NB; ++bi) xv[u][bi] = ok ? to_d(X[r * lp + bi * 16 + li]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int bi = 0; bi < NB; ++bi)
#pragma unroll
        for (int bj = bi; bj < NB; ++bj)
          acc[bi][bj] = Mfma<double>::mma(xv[u][bi], xv[u][bj], acc[bi][bj]);
  }
  for (int w = 0; w < 8; ++w) {
    if (wave == w) {
#pragma unroll
      for (int bi = 0; bi < NB; ++bi)
#pragma unroll
        for (int bj = bi; bj < NB; ++bj)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double* o = out + (bi * 16 + drow(lk, v)) * SL + bj * 16 + li;
            *o = (w == 0 ? 0.0 : *o) + acc[bi][bj][v];
          }
    }
    __syncthreads();
  }
}

// Cholesky G = R^T R of the leading l x l block (G = a, R = b; only the upper
// triangle of G is read, and G is overwritten).  R is upper triangular with
// zeros below the diagonal and the identity in rows / columns l .. lp-1.  A
// pivot <= ETA_DEP * G_jj (or not positive) gives a unit row and sets the
// flag.  Step j reads only row j of G and updates rows > j, so one barrier
// per step suffices.
__device__ __noinline__ void b_chol(int l, int lp) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* G = g_lds.u.sm.a;
  double* R = g_lds.u.sm.b;
  for (int e = tid; e < lp * lp; e += BNT) {
    const int r = e / lp, c = e - (e / lp) * lp;
    R[r * SL + c] = (r == c && r >= l) ? 1.0 : 0.0;
  }
  for (int i = tid; i < l; i += BNT) g_lds.dgn[i] = G[i * SL + i];
  if (tid == 0) g_lds.ndep = 0;
  __syncthreads();
  for (int j = 0; j < l; ++j) {
    const double d = G[j * SL + j];
    const bool dep = !(d > ETA_DEP * g_lds.dgn[j]);
    if (tid == 0) g_lds.depc[j] = dep ? 1 : 0;
    if (dep) {
      for (int c = j + tid; c < l; c += BNT) R[j * SL + c] = (c == j) ? 1.0 : 0.0;
      if (tid == 0) {
        g_lds.flag = 1;
        ++g_lds.ndep;
        if (!(fabs(d) <= 1.7976931348623157e308)) g_lds.nonfinite = 1;
      }
    } else {
      const double sq = sqrt(d);
      const double inv = 1.0 / d;
      for (int c = j + tid; c < l; c += BNT) R[j * SL + c] = G[j * SL + c] / sq;
      // G[r][c] -= G[j][r] G[j][c] / G[j][j] for j < r <= c < l
      for (int r = j + 1 + wave; r < l; r += BNT / 64) {
        const double gr = G[j * SL + r] * inv;
        for (int c = r + lane; c < l; c += 64) G[r * SL + c] -= gr * G[j * SL + c];
      }
    }
    __syncthreads();
  }
}

// a = R^{-1} with R = b (upper triangular, lp x lp): four lanes per column c
// solve R x = e_c by back substitution, each summing a quarter of every dot
// product; rows / columns l .. lp-1 are the identity.
__device__ __noinline__ void b_rinv(int l, int lp) {
  const int tid = threadIdx.x;
  const double* R = g_lds.u.sm.b;
  double* X = g_lds.u.sm.a;
  for (int e = tid; e < lp * lp; e += BNT) {
    const int r = e / lp, c = e - (e / lp) * lp;
    X[r * SL + c] = (r == c && r >= l) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int grp = tid >> 2, sub = tid & 3;
  for (int c = grp; c < l; c += BNT / 4) {
    for (int i = c; i >= 0; --i) {
      double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
      int u = i + 1 + sub;
      for (; u + 12 <= c; u += 16) {
        t0 += R[i * SL + u] * X[u * SL + c];
        t1 += R[i * SL + u + 4] * X[(u + 4) * SL + c];
        t2 += R[i * SL + u + 8] * X[(u + 8) * SL + c];
        t3 += R[i * SL + u + 12] * X[(u + 12) * SL + c];
      }
      for (; u <= c; u += 4) t0 += R[i * SL + u] * X[u * SL + c];
      double t = (t0 + t1) + (t2 + t3);
      t += __shfl_xor(t, 1, 64);
      t += __shfl_xor(t, 2, 64);
      if (sub == 0) X[i * SL + c] = ((i == c ? 1.0 : 0.0) - t) / R[i * SL + i];
    }
  }
  __syncthreads();
}

// Out (rows x ncols, ldo) = In (rows x lp, lp = 16 NB) a (lp x lp in LDS,
// stride SL; columns >= ncols are formed but not written), on FP64 MFMA; a
// 16-row block's operands are loaded before its products.
template <int NB, typename TI, typename TO>
__device__ __noinline__ void b_apply(const TI* __restrict__ In, int64_t rows, int ncols,
                                     TO* __restrict__ Out, int64_t ldo) {
  constexpr int lp = 16 * NB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const double* B = g_lds.u.sm.a;
  const int64_t nrb = cdiv(rows, 16);
  for (int64_t rb = wave; rb < nrb; rb += 8) {
    const int64_t r = rb * 16 + li;
    const bool ok = r < rows;
    double av[4 * NB];
#pragma unroll
    for (int t = 0; t < 4 * NB; ++t) av[t] = ok ? to_d(In[r * lp + 4 * t + lk]) : 0.0;
    d4 acc[NB];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) acc[cb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < 4 * NB; ++t) {
      const int k = 4 * t + lk;
#pragma unroll
      for (int cb = 0; cb < NB; ++cb)
        acc[cb] = Mfma<double>::mma(av[t], B[k * SL + cb * 16 + li], acc[cb]);
      // keep each step's LDS reads next to its products (bounded registers)
      if (t % 2 == 1) __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const int c = cb * 16 + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t rr = rb * 16 + drow(lk, v);
        if (rr < rows && c < ncols) Out[rr * ldo + c] = from_d<TO>(acc[cb][v]);
      }
    }
  }
  __syncthreads();
}

// Q (rows x lp) = orth(In) by CholeskyQR2 in FP64; T (rows x lp FP64) holds
// the first pass.
// ||G - I||_F^2 of the leading l x l block of the Gram in a (upper blocks:
// diagonal terms once, off-diagonal ones twice), the same value on every
// thread
__device__ double b_gram_offset2(int l) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double* G = g_lds.u.sm.a;
  double t = 0.0;
  for (int e = tid; e < l * l; e += BNT) {
    const int i = e / l, j = e - (e / l) * l;
    if (i == j) {
      const double d = G[i * SL + i] - 1.0;
      t = fma(d, d, t);
    } else if (i < j) {
      const double x = G[i * SL + j];
      t = fma(2.0 * x, x, t);
    }
  }
  t = wave_allsum(t);
  if (lane == 0) g_lds.sig[wave] = t;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < BNT / 64; ++w) r += g_lds.sig[w];
  __syncthreads();
  return r;
}

// Q = T rounded to TO (rows x lp)
template <typename TO>
__device__ void b_copy(const double* T, int64_t rows, int lp, TO* Q) {
  for (int64_t e = threadIdx.x; e < rows * lp; e += BNT) Q[e] = from_d<TO>(T[e]);
  __syncthreads();
}

// Largest ||Q1^T Q1 - I||_F after the first pass for which the second pass
// is skipped: 2^-30, far below the unit roundoff of the FP32 bases (2^-24),
// so the orthogonality of the stored basis is set by its own rounding.
constexpr double ORTH_SKIP2 = 0x1.0p-60;   // (2^-30)^2

// The columns of T (rows x lp) found dependent by the first Cholesky get
// N(0, 1/rows) entries: normal number j*rows + i of Philox stream 7 with
// batch word (orth call << 20 | matrix index), under the call's seed.
__device__ __noinline__ void b_replace(double* T, int64_t rows, int l, int lp, uint32_t k0,
                                       uint32_t k1, uint32_t word) {
  const double scale = 1.0 / sqrt((double)rows);
  for (int j = 0; j < l; ++j) {
    if (!g_lds.depc[j]) continue;
    for (int64_t i2 = threadIdx.x; 2 * i2 < rows; i2 += BNT) {
      const uint64_t t = (uint64_t)j * (uint64_t)rows + 2 * (uint64_t)i2;   // even number
      // normals t and t + 1 come from one counter when t is even; rows may be
      // odd, so each value is computed from its own pair
      double z[2];
      for (int h = 0; h < 2; ++h) {
        const uint64_t th = t + h;
        const uint64_t pr = th >> 1;
        const Words w = philox10((uint32_t)pr, (uint32_t)(pr >> 32), 7u, word, k0, k1);
        double z0, z1;
        box_muller(w, z0, z1);
        z[h] = (th & 1) ? z1 : z0;
      }
      const int64_t i = 2 * i2;
      T[i * lp + j] = z[0] * scale;
      if (i + 1 < rows) T[(i + 1) * lp + j] = z[1] * scale;
    }
  }
  __syncthreads();
}

template <int NB, typename TI, typename TO>
__device__ void b_orth(const TI* In, int64_t rows, int l, double* T, TO* Q, uint32_t k0,
                       uint32_t k1, uint32_t word) {
  constexpr int lp = 16 * NB;
  b_gram<NB>(In, rows);
  b_chol(l, lp);
  b_rinv(l, lp);
  b_apply<NB>(In, rows, lp, T, (int64_t)lp);
  if (g_lds.ndep > 0) b_replace(T, rows, l, lp, k0, k1, word);
  b_gram<NB>(T, rows);
  if (b_gram_offset2(l) <= ORTH_SKIP2) {
    b_copy(T, rows, lp, Q);
    return;
  }
  b_chol(l, lp);
  b_rinv(l, lp);
  b_apply<NB>(T, rows, lp, Q, (int64_t)lp);
}

// One-sided Jacobi on the l x l Rh held in a (stride SL): W (column j
// contiguous, ld l) goes to b and V = I to a.  Round-robin rounds of
// disjoint pairs, one pair per group of 16 lanes (32 groups), NB = lp / 16
// rows per lane.  Writes the k
// largest sigma to S and Uh, Vh (l x k, ld lp) to global scratch.
template <int NB>
__device__ __noinline__ void b_jacobi(int l, int k, double* S, double* Uh, double* Vh, int lp,
                                      int32_t* info) {
  const int tid = threadIdx.x;
  const int grp = tid >> 4, li = tid & 15;
  double* W = g_lds.u.sm.b;
  double* V = g_lds.u.sm.a;
  for (int e = tid; e < l * l; e += BNT) {
    const int j = e / l, i = e - (e / l) * l;
    W[j * l + i] = V[i * SL + j];
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
    if (tid == 0) g_lds.flag = 0;
    __syncthreads();
    for (int r = 0; r < N - 1; ++r) {
      for (int pi = grp; pi < N / 2; pi += BNT / 16) {
        int a = rr_player(pi, r, N), b = rr_player(N - 1 - pi, r, N);
        if (a >= l || b >= l) continue;
        if (a > b) { const int t = a; a = b; b = t; }
        if (rotate_pair16<NB>(W + a * l, W + b * l, V + a * l, V + b * l, l, li, tol) && li == 0)
          g_lds.flag = 1;
      }
      __syncthreads();
    }
    converged = (g_lds.flag == 0);
    __syncthreads();
  }
  if (!converged && tid == 0) info_or(info, INFO_JACOBI_CAP);
  jacobi_finish<BNT>(W, V, l, l, k, g_lds.sig, S, Uh, lp, Vh, lp);
  __syncthreads();
}

// a (stride SL, lp x lp) = the l x k matrix M (ld lp, global), zero elsewhere
__device__ void b_load_small(const double* M, int l, int k, int lp) {
  double* B = g_lds.u.sm.a;
  const int nc = lp;
  for (int e = threadIdx.x; e < lp * nc; e += BNT) {
    const int r = e / nc, c = e - (e / nc) * nc;
    B[r * SL + c] = (r < l && c < k) ? M[r * lp + c] : 0.0;
  }
  __syncthreads();
}

// The decomposition of one matrix after its sketch, for lp = 16 NB.
template <int NB, int RPW, int KC>
__device__ __noinline__ void b_one(const BatchArgs& g, const BatchDesc& d, const float* A,
                                   const float* Om,
                      float* Y, float* Q, float* Z, float* Zq, double* T, double* Qh,
                      double* Uh, double* Vh) {
  constexpr int lp = 16 * NB;
  const int64_t m = d.m, n = d.n;
  const int l = d.l, k = d.k;
  // batch word of the replacement columns: orth call (high bits), matrix
  const uint32_t mw = (uint32_t)d.index & 0xFFFFFu;
  uint32_t call = 0;
  b_pass_n<NB, RPW, KC>(A, d.lda, m, n, Om, Y);
  for (int j = 0; j < g.q; ++j) {
    b_orth<NB>(Y, m, l, T, Q, g.k0, g.k1, (call++ << 20) | mw);
    b_pass_t<NB, RPW, KC>(A, d.lda, m, n, Q, Z);
    b_orth<NB>(Z, n, l, T, Zq, g.k0, g.k1, (call++ << 20) | mw);
    b_pass_n<NB, RPW, KC>(A, d.lda, m, n, Zq, Y);
  }
  b_orth<NB>(Y, m, l, T, Q, g.k0, g.k1, (call++ << 20) | mw);
  b_pass_t<NB, RPW, KC>(A, d.lda, m, n, Q, Z);   // B^T
  b_orth<NB>(Z, n, l, T, Qh, g.k0, g.k1, (call++ << 20) | mw);
  b_xty(Qh, Z, n, lp);                         // Rh = Qh^T B^T
  if (threadIdx.x == 0 && g_lds.flag) info_or(g.info, INFO_ORTH_FALLBACK);
  if (threadIdx.x == 0 && g_lds.nonfinite) info_or(g.info, INFO_NONFINITE);
  b_jacobi<NB>(l, k, g.S + d.s_off, Uh, Vh, lp, g.info);
  b_load_small(Vh, l, k, lp);
  b_apply<NB>(Q, m, k, g.U + d.u_off, (int64_t)k);
  b_load_small(Uh, l, k, lp);
  b_apply<NB>(Qh, n, k, g.V + d.v_off, (int64_t)k);
}

__global__ __launch_bounds__(BNT) void batch_rsvd_kernel(BatchArgs g) {
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
    if (tid == 0) g_lds.item = atomicAdd(g.counter, 1);
    __syncthreads();
    const int64_t it = g_lds.item;
    __syncthreads();
    if (it >= g.count) break;
    const BatchDesc d = g.desc[it];
    const int lp = d.lp;
    const float* A = g.A + d.a_off;
    if (tid == 0) {
      g_lds.flag = 0;
      g_lds.nonfinite = 0;
    }
    __syncthreads();
    b_sketch(Om, d.n, d.l, lp, g.k0, g.k1, (uint32_t)d.index);
    // (lp / 16, pass shape) -> one instantiation
#define RSVD_B1(NBV)                                                                     \
  switch (d.variant) {                                                                   \
    case 1: b_one<NBV, 2, 32>(g, d, A, Om, Y, Q, Z, Zq, T, Qh, Uh, Vh); break;           \
    case 2: b_one<NBV, 1, 32>(g, d, A, Om, Y, Q, Z, Zq, T, Qh, Uh, Vh); break;           \
    default: b_one<NBV, 1, 64>(g, d, A, Om, Y, Q, Z, Zq, T, Qh, Uh, Vh); break;          \
  }
    switch (lp / 16) {
      case 1: RSVD_B1(1); break;
      case 2: RSVD_B1(2); break;
      case 3: RSVD_B1(3); break;
      case 4: RSVD_B1(4); break;
      default: RSVD_B1(5); break;
    }
#undef RSVD_B1
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
