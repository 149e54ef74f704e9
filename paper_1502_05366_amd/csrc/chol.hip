// orth(Y) by CholeskyQR (the unpivoted QR `[Q, ~] = qr(Y, 0)` of Sec. 2.1,
// used between the products of the power scheme of Sec. 3.2 and in Alg. 5):
//   G = Y^T Y (FP64),  G = R^T R (Cholesky),  Q = Y R^{-1}  (triangular solve),
// applied twice (CholeskyQR2) so that Q is orthonormal to working precision.
//
// Kernels here:
//  * chol_kernel: one workgroup factors an lp x lp Gram matrix (lp <= 256)
//    held in 16x16 matrix-core accumulator tiles (right-looking, block size
//    16, one-step lookahead).  It writes R (upper triangular, zero below), the inverses
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
#include <type_traits>

#include "common.h"
#include "internal.h"

namespace rsvd {
namespace {

constexpr int NI_NT = 256;
constexpr double NI_TAU2 = 2.5e-17;   // bound on ||G - I||_F^2 (about a quarter of 2^-52)
// ||G - I||_F^2 of the second Gram below which an FP32 basis is the first
// pass rounded to FP32: (2^-30)^2, far below the FP32 unit roundoff 2^-24
constexpr double TRSM_SKIP2 = 0x1.0p-60;
constexpr int MAXNB = 16;          // lp <= 256
// LDS row stride of the Cholesky's panel row (doubles): rows k and k+1 fall
// on different halves of the banks
constexpr int CH_LDP = 272;

// f(integral_constant<int, i>) for i = 0 .. N-1 (compile-time indices)
template <int I, int N, typename F> __device__ __forceinline__ void static_for_(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>());
    static_for_<I + 1, N>(f);
  }
}
template <int N, typename F> __device__ __forceinline__ void static_for(F&& f) {
  static_for_<0, N>(f);
}

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
    // one load per element (clamped address), no branches
    const bool in = row < l && col < l;
    const int64_t off = in ? (int64_t)min(row, col) * ldg + max(row, col) : 0;
    const double g = G[off];
    t[v] = in ? g : ((row == col) ? 1.0 : 0.0);
  }
  return t;
}

// Right-looking block Cholesky with a one-step lookahead, one workgroup of
// NW waves.  Waves 1 .. NW-1 hold the upper 16x16 tiles of G in matrix-core
// accumulator layout (tile t of the row-major enumeration of the upper
// triangle lives in slot t / (NW-1) of wave 1 + t % (NW-1)); wave 0 owns no
// tile and factors the diagonal blocks.  Block step s has two phases:
//   1. wave 0 takes the diagonal tile (s, s), which its owner handed over in
//      the previous step with the panels 0 .. s-2 applied, applies panel
//      s-1 and factors it (R_ss and X = R_ss^{-1}); meanwhile the other waves
//      apply panel s-1 to every tile of rows >= s, and the owner of
//      (s+1, s+1) hands that tile over for the next step;
//   2. the owners of the tiles (s, b), b > s, form the panel row
//      R_sb = X^T G_sb (rows of dependent columns zeroed) in LDS and in R.
// The panel lives in LDS (16 x lp, one buffer: phase 2 of a step writes it
// after phase 1 has read the previous one).
template <int NW, int TPW>
__global__ __launch_bounds__(64 * NW) void chol_kernel(const double* __restrict__ G, int64_t ldg,
                                                       int l, int lp, double eta,
                                                       double* __restrict__ R, int64_t ldr,
                                                       double* __restrict__ Rdinv,
                                                       int32_t* __restrict__ dep, int32_t* info,
                                                       const double* __restrict__ ni_part) {
  constexpr int NT = 64 * NW, NU = NW - 1;
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

  __shared__ double P[16 * CH_LDP];     // panel row of R (rows 16s .. 16s+15)
  __shared__ double Dn[2][16 * 17];     // diagonal tile handed to wave 0
  __shared__ double Dw[16 * 17];        // wave 0: the updated diagonal tile
  __shared__ double Rs[16 * 16];        // R_ss, row-major
  __shared__ double Xs[16 * 16];        // R_ss^{-1}, row-major
  __shared__ double dinvs[16];          // 1 / R_ss[j][j]
  __shared__ double diag0[256];
  __shared__ int depblk[16];

  for (int j = tid; j < lp; j += NT) diag0[j] = (j < l) ? G[(int64_t)j * ldg + j] : 1.0;
  // zero the strictly lower part of R
  for (int r = 1 + wave; r < lp; r += NW)
    for (int c = lane; c < r; c += 64) R[(int64_t)r * ldr + c] = 0.0;

  // slot table of an update wave: lane q holds (a | b << 8) of slot q's tile
  // (a = 255: no tile)
  const int ntiles = nb * (nb + 1) / 2;
  int coord = 255;
  if (wave > 0 && lane < TPW) {
    const int t = (wave - 1) + NU * lane;
    if (t < ntiles) {
      int a = 0;
      while (a + 1 < nb && (a + 1) * nb - (a + 1) * a / 2 <= t) ++a;
      const int b = a + (t - (a * nb - a * (a - 1) / 2));
      coord = a | (b << 8);
    }
  }
  d4 acc[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    const int ab = __builtin_amdgcn_readlane(coord, q);
    const int a = ab & 255, b = ab >> 8;
    // (a slot without a tile reads identity values: no branch around the loads)
    acc[q] = load_gtile(G, ldg, l, a, b, lane);
    if (a == 0 && b == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) Dn[0][drow(lk, v) * 17 + li] = acc[q][v];
    }
  }
  __syncthreads();

  // Wave 0 and the update waves run separate loops over s that meet at the
  // same two barriers per step, so the tiles' registers are live only in the
  // update waves' loop.
  if (wave == 0) {
    for (int s = 0; s < nb; ++s) {
      // (1, wave 0) the diagonal tile with panel s-1 applied, in accumulator
      // layout, then as columns: lane c (all four row groups alike) holds
      // x[a] = G'[a][c]
      d4 t;
#pragma unroll
      for (int v = 0; v < 4; ++v) t[v] = Dn[s & 1][drow(lk, v) * 17 + li];
      if (s > 0) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const double pv = P[(4 * kk + lk) * CH_LDP + s * 16 + li];
          t = Mfma<double>::mma(-pv, pv, t);
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) Dw[drow(lk, v) * 17 + li] = t[v];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // c = li through an opaque move, so that the per-lane constants derived
      // from it are formed here and not kept live across the whole s loop
      int c;
      asm volatile("v_mov_b32 %0, %1" : "=v"(c) : "v"(li));
      double x[16];
#pragma unroll
      for (int a = 0; a < 16; ++a) x[a] = Dw[a * 17 + c];
      // right-looking elimination inside the block: step j takes the pivot
      // d = G'[j][j] from lane j and turns x[j] into row j of R (lane c >= j
      // gets x[j] / sqrt(d), which is sqrt(d) itself in lane j), then
      // subtracts R[j][a] R[j][c] from the rows a > j.  Lanes c < j compute
      // values that are never read (rows below the diagonal are dropped at
      // the end).  A column whose pivot is not above eta * G_jj gets a unit
      // row.
      const double thr = eta * diag0[s * 16 + c];
      uint32_t okm = 0u, nfm = 0u;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const double d = readlane_d(x[j], j);
        const bool finite = __builtin_isfinite(d);
        const bool ok = finite && d > readlane_d(thr, j);
        okm |= ok ? (1u << j) : 0u;
        nfm |= finite ? 0u : (1u << j);
        // branch-free: the estimate is formed for any d and then selected
        const double inv0 = rsq_nr(d);
        const double inv = ok ? inv0 : 1.0;
        const double r = ok ? x[j] * inv0 : ((c == j) ? 1.0 : 0.0);
        x[j] = r;
        if (lane == 0) dinvs[j] = inv;
#pragma unroll
        for (int a = j + 1; a < 16; ++a) x[a] = fma(-readlane_d(r, a), r, x[a]);
      }
      // R_ss to LDS (the four row groups of the wave hold the same columns
      // and store the same values); the update waves copy it to R in phase 2
#pragma unroll
      for (int a = 0; a < 16; ++a) Rs[a * 16 + c] = (a <= c) ? x[a] : 0.0;
      if (lane < 16) {
        const int dj = ((okm >> c) & 1u) ? 0 : 1;
        depblk[c] = dj;
        if (s * 16 + c < l) dep[s * 16 + c] = dj;
      }
      if (lane == 0) {
        // columns of the block below l that failed the test
        const uint32_t lmask = (l - s * 16 >= 16) ? 0xFFFFu : ((1u << (l - s * 16)) - 1u);
        const uint32_t bad = ~okm & lmask;
        if ((bad & nfm) != 0u) info_or(info, INFO_NONFINITE);
        if ((bad & ~nfm) != 0u) info_or(info, INFO_ORTH_FALLBACK);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // X = R_ss^{-1}, column c in lane c by back substitution (the entries
      // below the diagonal come out zero).  Row a of R is read from LDS (the
      // same address in every lane); the terms of rows b > a+1 are summed in
      // two chains before X[a+1] is known, so each row adds one product to
      // the dependent chain.
      double X[16];
#pragma unroll
      for (int a = 15; a >= 0; --a) {
        double u0 = (a == c) ? 1.0 : 0.0, u1 = 0.0;
#pragma unroll
        for (int b = 15; b > a + 1; --b) {
          if ((b & 1) == 0) u0 = fma(-Rs[a * 16 + b], X[b], u0);
          else u1 = fma(-Rs[a * 16 + b], X[b], u1);
        }
        double u = u0 + u1;
        if (a < 15) u = fma(-Rs[a * 16 + a + 1], X[a + 1], u);
        X[a] = u * dinvs[a];
      }
#pragma unroll
      for (int a = 0; a < 16; ++a) Xs[a * 16 + c] = X[a];
      __syncthreads();
      __syncthreads();   // (2) the update waves form the panel row
    }
  } else {
    for (int s = 0; s < nb; ++s) {
      // (1, update waves) panel s-1 on every tile of rows >= s but (s, s);
      // the k-steps run outermost so that consecutive products go to
      // different tiles
      if (s > 0) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int k = 4 * kk + lk;
#pragma unroll
          for (int q = 0; q < TPW; ++q) {
            const int ab = __builtin_amdgcn_readlane(coord, q);
            const int a = ab & 255, b = ab >> 8;
            if (a >= s && a < nb && b > s) {
              const double av = -P[k * CH_LDP + a * 16 + li];
              const double bv = P[k * CH_LDP + b * 16 + li];
              acc[q] = Mfma<double>::mma(av, bv, acc[q]);
            }
          }
          // (operands of one k-step at a time in registers)
          __builtin_amdgcn_sched_barrier(0);
        }
      }
#pragma unroll
      for (int q = 0; q < TPW; ++q) {
        const int ab = __builtin_amdgcn_readlane(coord, q);
        if (ab == ((s + 1) | ((s + 1) << 8))) {
#pragma unroll
          for (int v = 0; v < 4; ++v) Dn[(s + 1) & 1][drow(lk, v) * 17 + li] = acc[q][v];
        }
      }
      __syncthreads();
      // (2) panel row s: R_sb = X^T G_sb.  The accumulator layout of G_sb is
      // the B-operand layout of the k-steps (element kk of lane (i, g) is
      // row 4 kk + g, column i).  The update waves also copy R_ss and its
      // inverse from LDS to R and Rdinv.
      for (int e = tid - 64; e < 512; e += NT - 64) {
        if (e < 256) R[(int64_t)(s * 16 + (e >> 4)) * ldr + s * 16 + (e & 15)] = Rs[e];
        else Rdinv[(int64_t)s * 256 + (e - 256)] = Xs[e - 256];
      }
#pragma unroll
      for (int q = 0; q < TPW; ++q) {
        const int ab = __builtin_amdgcn_readlane(coord, q);
        const int a = ab & 255, b = ab >> 8;
        if (a == s && b > s) {
          d4 r = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int kk = 0; kk < 4; ++kk)
            r = Mfma<double>::mma(Xs[(4 * kk + lk) * 16 + li], acc[q][kk], r);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = drow(lk, v);
            const double x = depblk[row] ? 0.0 : r[v];
            P[row * CH_LDP + b * 16 + li] = x;
            R[(int64_t)(s * 16 + row) * ldr + b * 16 + li] = x;
          }
        }
      }
      __syncthreads();
    }
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

// Q = Y R^{-1}: a workgroup of 4 waves takes 64 rows of Y (a wave 16),
// column block by column block, in transposed form
// Q_c^T = R_cc^{-T} (Y_c^T - sum_{b<c} R_bc^T Q_b^T).  The accumulator layout
// of a 16x16 product (lane (j, g) holds rows 4v + g of column j) is also the
// B-operand layout of the next products, so every Q_b^T stays in registers
// (4 doubles per lane) from the step that makes it to the last column block.
// The A operands of column block c (-R_bc for b < c, then R_cc^{-1}) are
// staged in LDS in operand order, shared by the four waves and double
// buffered: thread (kk, lane) fetches the k-step kk operands of the next
// column (and each wave its next Y values) into registers while the current
// column is multiplied, and one barrier per column block separates the two.
template <typename TY, typename TQ, int NB>
__global__ __launch_bounds__(256) void trsm_kernel(const TY* __restrict__ Y, int64_t ldy,
                                                   int64_t M, int l, int lp,
                                                   const double* __restrict__ R, int64_t ldr,
                                                   const double* __restrict__ Rdinv,
                                                   TQ* __restrict__ Q, int64_t ldq,
                                                   const double* __restrict__ skip_part) {
  __shared__ double Rb[2][NB * 256];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int nb = lp / 16;
  // (a wave past the last row still stages its share of the operands)
  const int64_t r = ((int64_t)blockIdx.x * 4 + wave) * 16 + li;
  const bool rok = r < M;
  const TY* yr = Y + (rok ? r : 0) * ldy;
  TQ* qr = Q + (rok ? r : 0) * ldq;
  if (skip_part) {
    // ||Y^T Y - I||_F^2 from its parts (the same order on every thread, so
    // the whole workgroup takes the same branch): when Y is orthonormal to
    // within TRSM_SKIP2, Q = Y rounded to TQ
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
  double pre[NB], ypre[4];
  // operands of column block c (compile-time slot count) read at column cf
  // (equal to c but past the last block, where the values go unused); no
  // branches around the loads, so they stay in flight across the products
  auto fetch = [&](auto cc, int cf) {
    constexpr int c = decltype(cc)::value;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      if (i < c) pre[i] = -R[(int64_t)(i * 16 + 4 * wave + lk) * ldr + cf * 16 + li];
      else if (i == c) pre[i] = Rdinv[(int64_t)cf * 256 + (4 * wave + lk) * 16 + li];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int col = cf * 16 + 4 * v + lk;
      const bool ok = rok && col < l;
      const double y = (double)yr[ok ? col : 0];
      ypre[v] = ok ? y : 0.0;
    }
  };
  auto stash = [&](int c) {
    double* rb = Rb[c & 1];
#pragma unroll
    for (int i = 0; i < NB; ++i)
      if (i <= c) rb[i * 256 + wave * 64 + lane] = pre[i];
  };
  fetch(std::integral_constant<int, 0>(), 0);
  stash(0);
  __syncthreads();
  d4 qt[NB];
  static_for<NB>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    if (c < nb) {
      d4 acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = ypre[v];
      if constexpr (c + 1 < NB) fetch(std::integral_constant<int, c + 1>(), min(c + 1, nb - 1));
      // (the loads issue before the products)
      __builtin_amdgcn_sched_barrier(0);
      const double* rb = Rb[c & 1];
#pragma unroll
      for (int b = 0; b < c; ++b) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
          acc = Mfma<double>::mma(rb[b * 256 + kk * 64 + lane], qt[b][kk], acc);  // -R_bc[k][i]
      }
      d4 out = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
        out = Mfma<double>::mma(rb[c * 256 + kk * 64 + lane], acc[kk], out);  // Rinv_cc[k][i]
      qt[c] = out;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = c * 16 + 4 * v + lk;
        if (rok && col < l) qr[col] = (TQ)out[v];
      }
      if (c + 1 < nb) stash(c + 1);
      __syncthreads();
    }
  });
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
  const int tiles = nb * (nb + 1) / 2;
  if (ni_part != nullptr) {
    hipLaunchKernelGGL(chol_ni_kernel, dim3(nb), dim3(NI_NT), 0, s, G, ldg, l, lp, R, ldr, Rdinv,
                       dep, ni_part);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // 8 waves: wave 0 factors the diagonal blocks, 7 hold the tiles (2 waves
  // per SIMD leave each up to 256 registers)
#define RSVD_CHOL(T)                                                                        \
  hipLaunchKernelGGL((chol_kernel<8, T>), dim3(1), dim3(512), 0, s, G, ldg, l, lp, eta, R, ldr, \
                     Rdinv, dep, info, ni_part)
  const int tpw = (int)cdiv(tiles, 7);
  if (tpw <= 1) RSVD_CHOL(1);
  else if (tpw <= 2) RSVD_CHOL(2);
  else if (tpw <= 4) RSVD_CHOL(4);
  else if (tpw <= 8) RSVD_CHOL(8);
  else if (tpw <= 15) RSVD_CHOL(15);
  else RSVD_CHOL(20);
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
