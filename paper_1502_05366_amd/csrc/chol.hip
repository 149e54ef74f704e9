// orth(Y) by CholeskyQR (the unpivoted QR `[Q, ~] = qr(Y, 0)` of Sec. 2.1,
// used between the products of the power scheme of Sec. 3.2 and in Alg. 5):
//   G = Y^T Y (FP64),  G = R^T R (Cholesky),  Q = Y R^{-1}  (triangular solve),
// applied twice (CholeskyQR2) so that Q is orthonormal to working precision.
//
// Kernels here:
//  * chol_kernel: one workgroup of 8 waves factors an lp x lp Gram matrix
//    (lp <= 256) held in 16x16 matrix-core accumulator tiles (right-looking,
//    block size 16).  It writes R (upper triangular, zero below), the inverses
//    of its 16x16 diagonal blocks, and a flag per column.  A column whose
//    Schur pivot is not above eta * G_jj (numerically dependent on the
//    columns before it) gets a unit row in R, so it is removed from the
//    factorization of the later columns and can be replaced afterwards.
//  * chol_ni_kernel: the factor of the second pass's Gram matrix, which is
//    I + E with E of the order of the unit roundoff times cond(Y)^2.  With
//    R = I + F (F upper triangular), R^T R = I + E reads F = Phi(E - F^T F),
//    Phi taking the strict upper triangle and half the diagonal, so
//    F = Phi(E) + O(||E||^2) and R^{-1} = I - F + O(||F||^2).  When
//    ||E||_F^2 <= NI_TAU2 (a quarter of the unit roundoff) both truncations
//    sit below rounding.  The kernel writes R = I + Phi(E) with the inverses
//    of its diagonal blocks and the parts of ||E||_F^2; chol_kernel adds the
//    parts and returns at once when the test passes, and otherwise factors G
//    as in the first pass, overwriting R.
//  * trsm_kernel: Q = Y R^{-1} for a tall Y, one wave per 16 rows, column
//    block by column block (Q_c = (Y_c - sum_{b<c} Q_b R_bc) R_cc^{-1}).
//  * replace_kernel: overwrites flagged columns of Q with fresh Gaussian
//    vectors (Philox stream 7) scaled to unit expected norm.
//  * trmm_kernel: R = R2 R1 for the two passes.
#include "common.h"
#include "internal.h"

namespace rsvd {
namespace {

constexpr int NI_NT = 256;
constexpr double NI_TAU2 = 2.5e-17;   // bound on ||G - I||_F^2 (about a quarter of 2^-52)
// ||G - I||_F^2 of the second Gram below which an FP32 basis is the first
// pass rounded to FP32: (2^-30)^2, far below the FP32 unit roundoff 2^-24
constexpr double TRSM_SKIP2 = 0x1.0p-60;
constexpr int CH_NT = 512;
constexpr int CH_NW = CH_NT / 64;  // waves
constexpr int MAXNB = 16;          // lp <= 256
constexpr int MAXT = MAXNB * (MAXNB + 1) / 2;

__device__ __forceinline__ double shfl_d(double v, int src) { return __shfl(v, src, 64); }

// Tile t of the row-major enumeration of the upper triangle of an nb x nb
// tile grid: row a starts at t = a*nb - a*(a-1)/2.  Arguments are uniform.
__device__ __forceinline__ int tile_row(int t, int nb) {
  int a = 0;
  while (a + 1 < nb && (a + 1) * nb - (a + 1) * a / 2 <= t) ++a;
  return a;
}
__device__ __forceinline__ int tile_col(int t, int nb) {
  const int a = tile_row(t, nb);
  return a + (t - (a * nb - a * (a - 1) / 2));
}

// Load tile (a, b) of the symmetric G (upper triangle read; padding rows and
// columns >= l are those of the identity) in accumulator layout.
__device__ __forceinline__ d4 load_gtile(const double* G, int64_t ldg, int l, int a, int b,
                                         int lane) {
  d4 t;
  const int col = b * 16 + (lane & 15);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = a * 16 + drow(lane >> 4, v);
    double x;
    if (row < l && col < l) {
      x = (row <= col) ? G[(int64_t)row * ldg + col] : G[(int64_t)col * ldg + row];
    } else {
      x = (row == col) ? 1.0 : 0.0;
    }
    t[v] = x;
  }
  return t;
}

template <int TPW>   // tiles per wave: ceil(nb (nb + 1) / 2 / 16)
__global__ __launch_bounds__(CH_NT) void chol_kernel(const double* __restrict__ G, int64_t ldg,
                                                     int l, int lp, double eta,
                                                     double* __restrict__ R, int64_t ldr,
                                                     double* __restrict__ Rdinv,
                                                     int32_t* __restrict__ dep, int32_t* info,
                                                     const double* __restrict__ ni_part) {
  const int nb = lp / 16;
  if (ni_part != nullptr) {
    // the near-identity test: the blocks' parts of ||G - I||_F^2, added in a
    // fixed order by every wave (each lane holds at most one part)
    const int ln = threadIdx.x & 63;
    const double e2 = wave_allsum(ln < nb ? ni_part[ln] : 0.0);
    if (e2 <= NI_TAU2) return;   // false for NaN
  }
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;

  __shared__ double Dss[16 * 17];        // diagonal block being factored
  __shared__ double Xss[16 * 16];        // its inverse
  __shared__ double P[16 * 256];         // row panel of R (rows s*16 .. s*16+15)
  __shared__ double Tw[CH_NW][16 * 16]; // per-wave transpose scratch
  __shared__ int depblk[16];
  __shared__ double diag0[256];
  __shared__ double rowb[16];           // row j of R_ss (diagonal-block step j)
  __shared__ double xcb[16];            // column j of R_ss^{-1}

  for (int j = tid; j < lp; j += CH_NT) diag0[j] = (j < l) ? G[(int64_t)j * ldg + j] : 1.0;
  // zero the strictly lower part of R
  for (int r = 1 + (tid >> 6); r < lp; r += CH_NT / 64)
    for (int c = tid & 63; c < r; c += 64) R[(int64_t)r * ldr + c] = 0.0;
  __syncthreads();
  const int ntiles = nb * (nb + 1) / 2;

  d4 acc[TPW];
  int ta[TPW], tb[TPW];      // tile coordinates (wave-uniform); ta = nb marks no tile
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    const int t = wave + CH_NW * q;
    ta[q] = (t < ntiles) ? tile_row(t, nb) : nb;
    tb[q] = (t < ntiles) ? tile_col(t, nb) : nb;
    if (t < ntiles) acc[q] = load_gtile(G, ldg, l, ta[q], tb[q], lane);
    else acc[q] = d4{0.0, 0.0, 0.0, 0.0};
  }

  for (int s = 0; s < nb; ++s) {
    // (a) the owner of tile (s, s) hands it to LDS
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      if (ta[q] == s && tb[q] == s) {
#pragma unroll
        for (int v = 0; v < 4; ++v) Dss[drow(lk, v) * 17 + li] = acc[q][v];
      }
    }
    __syncthreads();
    // (b) wave 0 factors the 16x16 block held in its 64 lanes (accumulator
    // layout: lane (g, c) element v is row 4v + g, column c) and builds
    // X = R_ss^{-1} alongside, column by column:
    //   X[r][j] = (delta_rj - S_r[j]) / R[j][j],  S_r[b] += X[r][j] R[j][b] (b > j),
    // where S_r[b] = sum_{a<b} X[r][a] R[a][b] waits in element (r, b) of y.
    // Row j of R and column j of X reach every lane through two 16-entry
    // LDS buffers; the pivot is read as a uniform value.
    if (wave == 0) {
      const int g = lk, c = li;
      double x[4], y[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) { x[v] = Dss[drow(g, v) * 17 + c]; y[v] = 0.0; }
      // lane c holds the dependence threshold of column c of the block; the
      // column flags are collected in two wave-uniform masks and written
      // after the block
      const double thr = eta * diag0[s * 16 + c];
      uint32_t okm = 0u, nfm = 0u;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int vj = j >> 2, gj = j & 3;
        const double d = readlane_d(x[vj], 16 * gj + j);      // Schur pivot G'[j][j]
        const bool finite = isfinite(d);
        const bool ok = finite && d > readlane_d(thr, j);
        okm |= ok ? (1u << j) : 0u;
        nfm |= finite ? 0u : (1u << j);
        const double inv = ok ? rsq_nr(d) : 1.0;             // 1 / R[j][j]
        const double rjj = ok ? d * inv : 1.0;
        if (g == gj) {
          // this lane holds G'[j][c]: row j of R, and (lane c == j) column j of X
          double rj;
          if (c == j) rj = rjj;
          else if (c > j) rj = ok ? x[vj] * inv : 0.0;
          else rj = 0.0;
          rowb[c] = rj;
        }
        if (c == j) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = drow(g, v);
            y[v] = ((r == j ? 1.0 : 0.0) - y[v]) * inv;
            xcb[r] = y[v];
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const double rjc = rowb[c];                           // R[j][c]
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = drow(g, v);
          const double rja = rowb[a];                         // R[j][a]
          const double xaj = xcb[a];                          // X[a][j]
          if (a > j && a <= c) x[v] = fma(-rja, rjc, x[v]);
          if (a == j) x[v] = rjc;
          if (c > j) y[v] = fma(xaj, rjc, y[v]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      if (lane < 16) {
        const int gcol = s * 16 + lane;
        const int dj = ((okm >> lane) & 1u) ? 0 : 1;
        depblk[lane] = dj;
        if (gcol < l) dep[gcol] = dj;
      }
      if (lane == 0) {
        // columns of the block below l that failed the test
        const uint32_t lmask = (l - s * 16 >= 16) ? 0xFFFFu : ((1u << (l - s * 16)) - 1u);
        const uint32_t bad = ~okm & lmask;
        if ((bad & nfm) != 0u) info_or(info, INFO_NONFINITE);
        if ((bad & ~nfm) != 0u) info_or(info, INFO_ORTH_FALLBACK);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = drow(g, v);
        if (a > c) x[v] = 0.0;
        R[(int64_t)(s * 16 + a) * ldr + s * 16 + c] = x[v];
        Xss[a * 16 + c] = y[v];
        Rdinv[(int64_t)s * 256 + a * 16 + c] = y[v];
      }
    }
    __syncthreads();
    // (c) panel: R_sb = R_ss^{-T} G_sb for b > s, zero rows of dependent columns
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      if (ta[q] == s && tb[q] > s && tb[q] < nb) {
        const int b = tb[q];
#pragma unroll
        for (int v = 0; v < 4; ++v) Tw[wave][drow(lk, v) * 16 + li] = acc[q][v];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        d4 r = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int k = 4 * kk + lk;
          const double av = Xss[k * 16 + li];          // (R_ss^{-T})[li][k]
          const double bv = Tw[wave][k * 16 + li];     // G_sb[k][li]
          r = Mfma<double>::mma(av, bv, r);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = drow(lk, v);
          const double x = depblk[row] ? 0.0 : r[v];
          r[v] = x;
          P[row * 256 + b * 16 + li] = x;
          R[(int64_t)(s * 16 + row) * ldr + b * 16 + li] = x;
        }
        acc[q] = r;
      }
    }
    __syncthreads();
    // (d) trailing update: G_ab -= R_sa^T R_sb for s < a <= b; the k-steps
    // run outermost so that consecutive products go to different tiles
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int k = 4 * kk + lk;
#pragma unroll
      for (int q = 0; q < TPW; ++q) {
        if (ta[q] > s && ta[q] < nb) {
          const double av = -P[k * 256 + ta[q] * 16 + li];
          const double bv = P[k * 256 + tb[q] * 16 + li];
          acc[q] = Mfma<double>::mma(av, bv, acc[q]);
        }
      }
    }
    __syncthreads();
  }
}


// Workgroup c takes rows 16c .. 16c+15: it writes those rows of R = I + Phi(G - I)
// (zero below the diagonal, identity in the padding), the inverse
// I - F_cc + F_cc^2 of the diagonal block, clear flags for those columns, and
// its part of ||G - I||_F^2 (upper triangle, off-diagonal entries twice) to
// part[c].  The writes are speculative: chol_kernel adds the parts in order
// and, when the sum exceeds NI_TAU2, overwrites all of them.
__global__ __launch_bounds__(NI_NT) void chol_ni_kernel(const double* __restrict__ G, int64_t ldg,
                                                        int l, int lp, double* __restrict__ R,
                                                        int64_t ldr, double* __restrict__ Rdinv,
                                                        int32_t* __restrict__ dep,
                                                        double* __restrict__ part) {
  constexpr int NW = NI_NT / 64;
  __shared__ double red[NW];
  __shared__ double Fd[16 * 17];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c = blockIdx.x;
  double s = 0.0;
  // wave w takes rows 16c + w, 16c + w + NW, ...; lanes run along the row
  for (int ii = wave; ii < 16; ii += NW) {
    const int i = c * 16 + ii;
    const double* gr = G + (int64_t)i * ldg;
    double* rr = R + (int64_t)i * ldr;
    for (int j = lane; j < lp; j += 64) {
      double f = 0.0;
      if (i < l && j < l && i <= j) {
        const double x = gr[j] - (i == j ? 1.0 : 0.0);
        s = fma((i == j ? 1.0 : 2.0) * x, x, s);
        f = (i == j) ? 0.5 * x : x;
      }
      rr[j] = (i == j ? 1.0 : 0.0) + f;
      if ((j >> 4) == c) Fd[ii * 17 + (j & 15)] = f;
    }
  }
  s = wave_allsum(s);
  if (lane == 0) red[wave] = s;
  if (tid < 16 && c * 16 + tid < l) dep[c * 16 + tid] = 0;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < NW; ++w) t += red[w];
    part[c] = t;
  }
  // inverse of the diagonal block: I - F_cc + F_cc^2
  {
    const int x = tid >> 4, y = tid & 15;
    double f2 = 0.0;
    for (int t = x; t <= y; ++t) f2 = fma(Fd[x * 17 + t], Fd[t * 17 + y], f2);
    Rdinv[(int64_t)c * 256 + x * 16 + y] = ((x == y) ? 1.0 : 0.0) - Fd[x * 17 + y] + f2;
  }
}

// Q = Y R^{-1}: one wave per 16 rows of Y, column block by column block, in
// transposed form Q_c^T = R_cc^{-T} (Y_c^T - sum_{b<c} R_bc^T Q_b^T).  The
// accumulator layout of a 16x16 product (lane (j, g) holds rows 4v + g of
// column j) is also the B-operand layout of the next products, so every
// Q_b^T stays in registers (4 doubles per lane) from the step that makes it
// to the last column block, and the wave needs no LDS and no barrier.
// R_bc^T and R_cc^{-T} are read as A operands straight from memory (L2).
template <typename TY, typename TQ, int NB>
__global__ __launch_bounds__(256) void trsm_kernel(const TY* __restrict__ Y, int64_t ldy,
                                                   int64_t M, int l, int lp,
                                                   const double* __restrict__ R, int64_t ldr,
                                                   const double* __restrict__ Rdinv,
                                                   TQ* __restrict__ Q, int64_t ldq,
                                                   const double* __restrict__ skip_part) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  if (row0 >= M) return;
  const int nb = lp / 16;
  const int64_t r = row0 + li;
  const bool rok = r < M;
  const TY* yr = Y + (rok ? r : 0) * ldy;
  TQ* qr = Q + (rok ? r : 0) * ldq;
  if (skip_part) {
    // ||Y^T Y - I||_F^2 from its parts (the same order on every thread): when
    // Y is orthonormal to within TRSM_SKIP2, Q = Y rounded to TQ
    double e2 = 0.0;
    for (int c = 0; c < nb; ++c) e2 += skip_part[c];
    if (e2 <= TRSM_SKIP2) {
      for (int c = 0; c < nb; ++c) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int col = c * 16 + 4 * v + lk;
          if (rok && col < l) qr[col] = (TQ)yr[col];
        }
      }
      return;
    }
  }
  d4 qt[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c < nb) {
      d4 acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = c * 16 + 4 * v + lk;
        acc[v] = (rok && col < l) ? (double)yr[col] : 0.0;
      }
#pragma unroll
      for (int b = 0; b < c; ++b) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const double av = -R[(int64_t)(b * 16 + 4 * kk + lk) * ldr + c * 16 + li];  // R_bc[k][i]
          acc = Mfma<double>::mma(av, qt[b][kk], acc);
        }
      }
      d4 out = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const double av = Rdinv[(int64_t)c * 256 + (4 * kk + lk) * 16 + li];  // Rinv_cc[k][i]
        out = Mfma<double>::mma(av, acc[kk], out);
      }
      qt[c] = out;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = c * 16 + 4 * v + lk;
        if (rok && col < l) qr[col] = (TQ)out[v];
      }
    }
  }
}

// Replace every flagged column j of Q (M rows) by N(0, 1/M) entries from
// Philox stream 7, counter pair index = j*M + i for normal (i, j), batch = call.
__device__ __forceinline__ double normal_at(uint32_t k0, uint32_t k1, uint32_t sid, uint32_t batch,
                                            uint64_t t) {
  uint32_t c0 = (uint32_t)(t >> 1), c1 = (uint32_t)(t >> 33), c2 = sid, c3 = batch;
  const uint32_t PM0 = 0xD2511F53u, PM1 = 0xCD9E8D57u, PW0 = 0x9E3779B9u, PW1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += PW0; k1 += PW1; }
    const uint32_t hi0 = __umulhi(PM0, c0), lo0 = PM0 * c0;
    const uint32_t hi1 = __umulhi(PM1, c2), lo1 = PM1 * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  const double a = (double)(c0 >> 5) * 67108864.0 + (double)(c1 >> 6);
  const double b = (double)(c2 >> 5) * 67108864.0 + (double)(c3 >> 6);
  const double u1 = (a + 1.0) * 0x1.0p-53, u2 = b * 0x1.0p-53;
  const double r = sqrt(-2.0 * log(u1)), th = 6.283185307179586 * u2;
  return (t & 1) ? r * sin(th) : r * cos(th);
}

template <typename TQ>
__global__ __launch_bounds__(256) void replace_kernel(TQ* __restrict__ Q, int64_t ldq, int64_t M,
                                                      int l, const int32_t* __restrict__ dep,
                                                      uint64_t seed, uint32_t call) {
  // the flagged columns, listed once per workgroup (usually none)
  __shared__ int list[256];
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int j = threadIdx.x; j < l; j += blockDim.x)
    if (dep[j]) list[atomicAdd(&cnt, 1)] = j;
  __syncthreads();
  const int nd = cnt;
  if (nd == 0) return;
  const double scale = 1.0 / sqrt((double)M);
  for (int q = 0; q < nd; ++q) {
    const int j = list[q];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < M;
         i += (int64_t)gridDim.x * blockDim.x) {
      const double z = normal_at((uint32_t)seed, (uint32_t)(seed >> 32), 7u, call,
                                 (uint64_t)j * (uint64_t)M + (uint64_t)i);
      Q[i * ldq + j] = (TQ)(z * scale);
    }
  }
}

// C = A B for upper-triangular lp x lp A, B (C upper triangular, zero below);
// rows k of B with bdep[k] != 0 count as zero (the unit rows that the
// Cholesky gives dependent columns stand for a zero residual, so the product
// is the R of Y = Q R).  One wave per 16 x 16 tile of C, on the matrix cores.
__global__ __launch_bounds__(256) void trmm_kernel(const double* __restrict__ Am, int64_t lda,
                                                   const double* __restrict__ Bm, int64_t ldb,
                                                   const int32_t* __restrict__ bdep,
                                                   double* __restrict__ C, int64_t ldc, int lp) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nb = lp / 16;
  const int t = blockIdx.x * 4 + wave;
  if (t >= nb * nb) return;
  const int a = t / nb, b = t - (t / nb) * nb;
  d4 acc = d4{0.0, 0.0, 0.0, 0.0};
  for (int q = a; q <= b; ++q) {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int kx = q * 16 + 4 * kk + lk;
      const double av = Am[(int64_t)(a * 16 + li) * lda + kx];
      const double bv = (bdep != nullptr && bdep[kx] != 0) ? 0.0 : Bm[(int64_t)kx * ldb + b * 16 + li];
      acc = Mfma<double>::mma(av, bv, acc);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = a * 16 + drow(lk, v), col = b * 16 + li;
    C[(int64_t)row * ldc + col] = (row <= col) ? acc[v] : 0.0;
  }
}

__global__ void set_word_kernel(int32_t* w, int32_t v) { *w = v; }

// T = Y - T: the residual of a projection of Y (block orthonormalization)
template <typename TY>
__global__ __launch_bounds__(256) void rsub_kernel(const TY* __restrict__ Y, int64_t ldy,
                                                   double* __restrict__ T, int64_t ldt,
                                                   int64_t rows, int cols) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / cols, c = e - r * cols;
    T[r * ldt + c] = (double)Y[r * ldy + c] - T[r * ldt + c];
  }
}

// rows of R that belong to dependent columns, zeroed (their unit rows are
// placeholders, not part of Y = Q R)
__global__ __launch_bounds__(64) void zero_dep_rows_kernel(double* __restrict__ R, int64_t ldr,
                                                           int lp, const int32_t* __restrict__ dep) {
  const int j = blockIdx.x;
  if (!dep[j]) return;
  for (int c = threadIdx.x; c < lp; c += blockDim.x) R[(int64_t)j * ldr + c] = 0.0;
}

// Gram matrix G = Y^T Y (FP64) of a tall Y (rows x l), upper 16x16 tiles only.
// The column blocks are cut into segments of 4; a tile group is a pair of
// segments (sa <= sb) and holds the at most 16 upper tiles between them, so a
// workgroup of the group needs only the <= 128 columns of its two segments.
// Each group owns a number of workgroups proportional to its tiles per wave
// (1 or 2), and workgroup j of the group reduces the j-th of that many equal
// row ranges.  16-row chunks of the group's columns are staged in LDS (row
// stride 144 doubles, so the four row groups of a wave fall on different bank
// halves), the next chunk is fetched into registers while the current one is
// multiplied, and each tile accumulates on one wave's matrix cores.  Partial
// tiles go to part[workgroup][slot]; gram_reduce_kernel adds a tile's
// partials in workgroup order (deterministic).
constexpr int GR_NT = 512;
constexpr int GR_NW = GR_NT / 64;
constexpr int GR_SEG = 4;                   // column blocks per segment
constexpr int GR_MAXSEG = MAXNB / GR_SEG;   // 4
constexpr int GR_MAXG = GR_MAXSEG * (GR_MAXSEG + 1) / 2;
constexpr int GR_LDS = 144;                 // LDS row stride (doubles)

struct GramPlan {
  int nb, nseg, ngroups, total;
  int sa[GR_MAXG], sb[GR_MAXG];
  int off[GR_MAXG + 1];                     // first workgroup of each group
};

template <typename TY>
__global__ __launch_bounds__(GR_NT) void gram_kernel(const TY* __restrict__ Y, int64_t ldy,
                                                     int64_t rows, int l, GramPlan gp,
                                                     double* __restrict__ part) {
  __shared__ double Ys[2][16 * GR_LDS];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int x = blockIdx.x;
  int g = 0;
  while (g + 1 < gp.ngroups && gp.off[g + 1] <= x) ++g;
  const int sa = gp.sa[g], sb = gp.sb[g];
  const int ng = gp.off[g + 1] - gp.off[g], j = x - gp.off[g];
  const int64_t r0 = ((int64_t)j * rows) / ng, r1 = ((int64_t)(j + 1) * rows) / ng;
  const bool diag = sa == sb;
  const int ncol = diag ? 64 : 128;
  const int sh = diag ? 6 : 7;
  // the (up to) two tiles of this wave: slot u = 4 * (ta - 4 sa) + (tb - 4 sb)
  bool tv[2];
  int ca[2], cb[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int u = wave + GR_NW * q;
    const int ta = GR_SEG * sa + (u >> 2), tb = GR_SEG * sb + (u & 3);
    tv[q] = ta < gp.nb && tb < gp.nb && ta <= tb;
    ca[q] = (u >> 2) * 16;
    cb[q] = (diag ? 0 : 64) + (u & 3) * 16;
  }
  d4 acc[2];
  acc[0] = d4{0.0, 0.0, 0.0, 0.0};
  acc[1] = d4{0.0, 0.0, 0.0, 0.0};
  const int nch = (int)cdiv(r1 - r0, 16);
  double pre[4];
  auto fetch = [&](int ch) {
    const int64_t base = r0 + (int64_t)ch * 16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = tid + GR_NT * i;
      const int rr = e >> sh, cc = e & (ncol - 1);
      const int gcol = (cc < 64) ? sa * 64 + cc : sb * 64 + (cc - 64);
      const int64_t r = base + rr;
      pre[i] = (e < 16 * ncol && r < r1 && gcol < l) ? (double)Y[r * ldy + gcol] : 0.0;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = tid + GR_NT * i;
      if (e < 16 * ncol) Ys[buf][(e >> sh) * GR_LDS + (e & (ncol - 1))] = pre[i];
    }
  };
  if (nch > 0) {
    fetch(0);
    stash(0);
  }
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nch) fetch(ch + 1);
    const double* ys = Ys[buf];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (tv[q]) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int k = 4 * kk + lk;
          acc[q] = Mfma<double>::mma(ys[k * GR_LDS + ca[q] + li], ys[k * GR_LDS + cb[q] + li],
                                     acc[q]);
        }
      }
    }
    if (ch + 1 < nch) stash(buf ^ 1);
    __syncthreads();
  }
  double* P = part + (int64_t)x * 16 * 256;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    if (tv[q]) {
      const int u = wave + GR_NW * q;
#pragma unroll
      for (int v = 0; v < 4; ++v) P[u * 256 + drow(lk, v) * 16 + li] = acc[q][v];
    }
  }
}

// G_ab = sum over the workgroups of the group of (a, b) of their partial
// tile, in workgroup order (four interleaved chains added in a fixed order).
__global__ __launch_bounds__(256) void gram_reduce_kernel(const double* __restrict__ part,
                                                          GramPlan gp, double* __restrict__ Gm,
                                                          int64_t ldg) {
  const int t = blockIdx.x, e = threadIdx.x;
  const int a = tile_row(t, gp.nb), b = tile_col(t, gp.nb);
  const int sa = a / GR_SEG, sb = b / GR_SEG;
  const int g = sa * gp.nseg - sa * (sa - 1) / 2 + (sb - sa);
  const int u = 4 * (a - GR_SEG * sa) + (b - GR_SEG * sb);
  const int w0 = gp.off[g], ng = gp.off[g + 1] - w0;
  const double* p = part + ((int64_t)w0 * 16 + u) * 256 + e;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int w = 0;
  for (; w + 4 <= ng; w += 4) {
    s0 += p[(int64_t)(w + 0) * 4096];
    s1 += p[(int64_t)(w + 1) * 4096];
    s2 += p[(int64_t)(w + 2) * 4096];
    s3 += p[(int64_t)(w + 3) * 4096];
  }
  for (; w < ng; ++w) s0 += p[(int64_t)w * 4096];
  Gm[(int64_t)(a * 16 + (e >> 4)) * ldg + b * 16 + (e & 15)] = (s0 + s1) + (s2 + s3);
}

GramPlan plan_gram(int64_t rows, int lp, int ncu) {
  GramPlan gp;
  gp.nb = lp / 16;
  gp.nseg = (int)cdiv(gp.nb, GR_SEG);
  gp.ngroups = 0;
  int wsum = 0;
  int wt[GR_MAXG];
  for (int sa = 0; sa < gp.nseg; ++sa)
    for (int sb = sa; sb < gp.nseg; ++sb) {
      const int na = std::min(GR_SEG, gp.nb - GR_SEG * sa);
      const int nbb = std::min(GR_SEG, gp.nb - GR_SEG * sb);
      const int tiles = (sa == sb) ? na * (na + 1) / 2 : na * nbb;
      gp.sa[gp.ngroups] = sa;
      gp.sb[gp.ngroups] = sb;
      wt[gp.ngroups] = (int)cdiv(tiles, GR_NW);   // tiles per wave: 1 or 2
      wsum += wt[gp.ngroups];
      ++gp.ngroups;
    }
  // about two workgroups per CU in all, at least 64 rows per workgroup
  const int64_t budget = 2 * (int64_t)ncu;
  int64_t unit = budget / wsum;
  const int64_t maxunit = std::max<int64_t>(1, rows / (64 * 2));
  unit = std::max<int64_t>(1, std::min(unit, maxunit));
  gp.off[0] = 0;
  for (int g = 0; g < gp.ngroups; ++g) gp.off[g + 1] = gp.off[g] + (int)(unit * wt[g]);
  gp.total = gp.off[gp.ngroups];
  return gp;
}

}  // namespace

size_t gram_part_bytes(int lp, int ncu) {
  (void)lp;
  return (size_t)2 * ncu * 16 * 256 * sizeof(double);
}

hipError_t launch_gram(bool y_f32, const void* Y, int64_t ldy, int64_t rows, int l, int lp,
                       double* Gm, int64_t ldg, double* part, int ncu, hipStream_t s) {
  if (lp > 256 || lp % 16) return hipErrorInvalidValue;
  const GramPlan gp = plan_gram(rows, lp, ncu);
  if (y_f32)
    hipLaunchKernelGGL(gram_kernel<float>, dim3(gp.total), dim3(GR_NT), 0, s, (const float*)Y,
                       ldy, rows, l, gp, part);
  else
    hipLaunchKernelGGL(gram_kernel<double>, dim3(gp.total), dim3(GR_NT), 0, s, (const double*)Y,
                       ldy, rows, l, gp, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int ntiles = gp.nb * (gp.nb + 1) / 2;
  hipLaunchKernelGGL(gram_reduce_kernel, dim3(ntiles), dim3(256), 0, s, part, gp, Gm, ldg);
  return hipGetLastError();
}

hipError_t launch_chol(const double* G, int64_t ldg, int l, int lp, double eta, double* R,
                       int64_t ldr, double* Rdinv, int32_t* dep, int32_t* info, hipStream_t s,
                       double* ni_part) {
  if (lp > 256 || lp % 16) return hipErrorInvalidValue;
  const int nb = lp / 16;
  const int tpw = (int)cdiv(nb * (nb + 1) / 2, CH_NW);
  if (ni_part != nullptr) {
    hipLaunchKernelGGL(chol_ni_kernel, dim3(nb), dim3(NI_NT), 0, s, G, ldg, l, lp, R, ldr, Rdinv,
                       dep, ni_part);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
#define RSVD_CHOL(T)                                                                          \
  hipLaunchKernelGGL(chol_kernel<T>, dim3(1), dim3(CH_NT), 0, s, G, ldg, l, lp, eta, R, ldr, \
                     Rdinv, dep, info, ni_part)
  if (tpw <= 1) RSVD_CHOL(1);
  else if (tpw <= 2) RSVD_CHOL(2);
  else if (tpw <= 4) RSVD_CHOL(4);
  else if (tpw <= 7) RSVD_CHOL(7);
  else if (tpw <= 10) RSVD_CHOL(10);
  else if (tpw <= 14) RSVD_CHOL(14);
  else RSVD_CHOL(17);
#undef RSVD_CHOL
  return hipGetLastError();
}

template <int NB>
hipError_t launch_trsm_nb(bool y_f32, bool q_f32, const void* Y, int64_t ldy, int64_t M, int l,
                          int lp, const double* R, int64_t ldr, const double* Rdinv, void* Q,
                          int64_t ldq, const double* skip_part, hipStream_t s) {
  const dim3 grid((unsigned)cdiv(M, 64));
  if (!y_f32 && !q_f32)
    hipLaunchKernelGGL((trsm_kernel<double, double, NB>), grid, dim3(256), 0, s,
                       (const double*)Y, ldy, M, l, lp, R, ldr, Rdinv, (double*)Q, ldq, skip_part);
  else if (y_f32 && q_f32)
    hipLaunchKernelGGL((trsm_kernel<float, float, NB>), grid, dim3(256), 0, s,
                       (const float*)Y, ldy, M, l, lp, R, ldr, Rdinv, (float*)Q, ldq, skip_part);
  else if (y_f32 && !q_f32)
    hipLaunchKernelGGL((trsm_kernel<float, double, NB>), grid, dim3(256), 0, s,
                       (const float*)Y, ldy, M, l, lp, R, ldr, Rdinv, (double*)Q, ldq, skip_part);
  else
    hipLaunchKernelGGL((trsm_kernel<double, float, NB>), grid, dim3(256), 0, s,
                       (const double*)Y, ldy, M, l, lp, R, ldr, Rdinv, (float*)Q, ldq, skip_part);
  return hipGetLastError();
}

hipError_t launch_trsm(bool y_f32, bool q_f32, const void* Y, int64_t ldy, int64_t M, int l,
                       int lp, const double* R, int64_t ldr, const double* Rdinv, void* Q,
                       int64_t ldq, hipStream_t s, const double* skip_part) {
  if (M <= 0) return hipSuccess;
  if (lp > 256 || lp % 16) return hipErrorInvalidValue;
  const int nb = lp / 16;
  if (nb <= 2) 
    return launch_trsm_nb<2>(y_f32, q_f32, Y, ldy, M, l, lp, R, ldr, Rdinv, Q, ldq,
                              skip_part, s);
  if (nb <= 4) 
    return launch_trsm_nb<4>(y_f32, q_f32, Y, ldy, M, l, lp, R, ldr, Rdinv, Q, ldq,
                              skip_part, s);
  if (nb <= 8) 
    return launch_trsm_nb<8>(y_f32, q_f32, Y, ldy, M, l, lp, R, ldr, Rdinv, Q, ldq,
                              skip_part, s);
  if (nb <= 12)
    return launch_trsm_nb<12>(y_f32, q_f32, Y, ldy, M, l, lp, R, ldr, Rdinv, Q, ldq,
                              skip_part, s);
  return launch_trsm_nb<16>(y_f32, q_f32, Y, ldy, M, l, lp, R, ldr, Rdinv, Q, ldq, skip_part,
                            s);
}

hipError_t launch_replace(bool q_f32, void* Q, int64_t ldq, int64_t M, int l, const int32_t* dep,
                          uint64_t seed, uint32_t call, hipStream_t s) {
  if (l > 256) return hipErrorInvalidValue;
  const int grid = (int)(cdiv(M, 256) < 1024 ? cdiv(M, 256) : 1024);
  if (q_f32)
    hipLaunchKernelGGL(replace_kernel<float>, dim3(grid), dim3(256), 0, s, (float*)Q, ldq, M, l,
                       dep, seed, call);
  else
    hipLaunchKernelGGL(replace_kernel<double>, dim3(grid), dim3(256), 0, s, (double*)Q, ldq, M, l,
                       dep, seed, call);
  return hipGetLastError();
}

hipError_t launch_trmm_upper(const double* A, int64_t lda, const double* B, int64_t ldb,
                             const int32_t* bdep, double* C, int64_t ldc, int lp, hipStream_t s) {
  if (lp > 256 || lp % 16) return hipErrorInvalidValue;
  const int nb = lp / 16;
  hipLaunchKernelGGL(trmm_kernel, dim3((unsigned)cdiv(nb * nb, 4)), dim3(256), 0, s, A, lda, B,
                     ldb, bdep, C, ldc, lp);
  return hipGetLastError();
}

hipError_t launch_set_word(int32_t* w, int32_t v, hipStream_t s) {
  hipLaunchKernelGGL(set_word_kernel, dim3(1), dim3(1), 0, s, w, v);
  return hipGetLastError();
}

hipError_t launch_rsub(bool y_f32, const void* Y, int64_t ldy, double* T, int64_t ldt,
                       int64_t rows, int cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  int64_t grid = cdiv(rows * cols, 256);
  if (grid > 16384) grid = 16384;
  if (y_f32)
    hipLaunchKernelGGL(rsub_kernel<float>, dim3((unsigned)grid), dim3(256), 0, s,
                       (const float*)Y, ldy, T, ldt, rows, cols);
  else
    hipLaunchKernelGGL(rsub_kernel<double>, dim3((unsigned)grid), dim3(256), 0, s,
                       (const double*)Y, ldy, T, ldt, rows, cols);
  return hipGetLastError();
}

hipError_t launch_zero_dep_rows(double* R, int64_t ldr, int l, int lp, const int32_t* dep,
                                hipStream_t s) {
  if (l <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_dep_rows_kernel, dim3(l), dim3(64), 0, s, R, ldr, lp, dep);
  return hipGetLastError();
}

}  // namespace rsvd
