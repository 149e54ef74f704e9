// Tall-skinny products against A on the matrix cores (the passes over A of
// the range finder: Y = A Omega, Z = A^T Q, Y = A Z, B^T = A^T Q), also used
// for Gram matrices and the small products of the post-processing.
//
//   C[M x L] = op(A) X,  op(A) = A (M x K, row-major, lda)  or
//                        op(A) = A^T with A stored K x M row-major (lda)
//   X is K x L row-major (ldx), C is M x L row-major (ldc).
//
// Work decomposition ("stream-K"): the output is cut into BM x BN tiles and
// the reduction into BK-deep steps; the T * KI (tile, step) units are split
// into G contiguous ranges, one per workgroup, so every workgroup gets the
// same number of matrix-core steps whatever T is.  A range that covers a whole
// tile writes C directly; a range that covers part of a tile writes its
// partial sum to a slot of the workspace, and a fix-up kernel adds the
// partial sums of each split tile in workgroup order (deterministic).
//
// Tiles: 8 waves per workgroup (4 along M x 2 along L), BM = 128 rows,
// BN = 32 * CBW columns, BK = 16.  Each wave owns 2 x CBW 16x16 accumulator
// blocks.  A and X tiles are staged in LDS (double-buffered) with coalesced
// global loads: rows of A (or of A^T's storage) are read along their
// contiguous dimension, so every byte of A is read from HBM once per pass.
#include "common.h"
#include "internal.h"

namespace rsvd {

namespace {

constexpr int BM = 128;
constexpr int BK = 16;
constexpr int NT = 512;

struct GemmArgs {
  const void* A; int64_t lda;
  const void* X; int64_t ldx;
  void* C; int64_t ldc;
  int64_t M, K, L;
  int64_t nct, KI, U;
  int64_t G;
  void* part;
};

__device__ __forceinline__ int64_t range_begin(int64_t w, int64_t U, int64_t G) {
  return (w * U) / G;
}

template <typename TA, typename TX, typename TC, typename TO, bool TRANS, int CBW>
__global__ __launch_bounds__(NT) void gemm_sk_kernel(GemmArgs g) {
  constexpr int BN = 32 * CBW;
  constexpr int ALD = TRANS ? (BM + 1) : (BK + 1);   // LDS row length of the A tile
  constexpr int AROWS = TRANS ? BK : BM;
  typedef typename Mfma<TC>::acc_t acc_t;

  __shared__ TC As[2][AROWS * ALD];
  __shared__ TC Xs[2][BK * BN];

  const TA* __restrict__ A = static_cast<const TA*>(g.A);
  const TX* __restrict__ X = static_cast<const TX*>(g.X);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave & 3;        // row-wave: rows wr*32 .. wr*32+31 of the tile
  const int wc = wave >> 2;       // col-wave: cols wc*16*CBW .. of the tile
  const int li = lane & 15;
  const int lk = lane >> 4;

  const int64_t w = blockIdx.x;
  int64_t u = range_begin(w, g.U, g.G);
  const int64_t uend = range_begin(w + 1, g.U, g.G);

  // per-thread global->LDS assignment
  // A, not transposed: row ai, 4 consecutive k starting at ak
  // A, transposed:     k-row ak, 4 consecutive i starting at ai
  const int a_r = TRANS ? (tid >> 5) : (tid >> 2);
  const int a_c = TRANS ? ((tid & 31) * 4) : ((tid & 3) * 4);
  // X: k-row x_r, CBW consecutive columns from x_c
  const int x_r = tid >> 5;
  const int x_c = (tid & 31) * CBW;

  while (u < uend) {
    const int64_t tile = u / g.KI;
    const int64_t kb = u - tile * g.KI;
    const int64_t ke = min(g.KI, kb + (uend - u));
    u += ke - kb;
    const int64_t row0 = (tile / g.nct) * BM;
    const int64_t col0 = (tile % g.nct) * BN;

    acc_t acc[2][CBW];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < CBW; ++j) acc[i][j] = Mfma<TC>::zero();

    // One step's loads in registers (a stage).  FP64 (CLAMP): clamped
    // addresses, so every load is issued without a branch around it, and
    // out-of-range elements are zeroed only when they are written to LDS (no
    // wait for the loads comes before that).  FP32: guarded loads, which
    // measured faster there.
    constexpr bool CLAMP = sizeof(TC) == 8;
    struct Stage {
      TC ra[4];
      TC rx[CBW];
      bool oka[4], okx[CBW];
    };
    auto gload = [&](Stage& st, int64_t kt) {
      const int64_t k0 = kt * BK;
      if (!TRANS) {
        const int64_t gi = row0 + a_r;
        const bool rok = gi < g.M;
        const int64_t gic = rok ? gi : g.M - 1;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int64_t gk = k0 + a_c + c;
          st.oka[c] = rok && gk < g.K;
          if (CLAMP) st.ra[c] = (TC)A[gic * g.lda + (gk < g.K ? gk : g.K - 1)];
          else st.ra[c] = st.oka[c] ? (TC)A[gi * g.lda + gk] : TC(0);
        }
      } else {
        const int64_t gk = k0 + a_r;
        const bool kok = gk < g.K;
        const int64_t gkc = kok ? gk : g.K - 1;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int64_t gi = row0 + a_c + c;
          st.oka[c] = kok && gi < g.M;
          if (CLAMP) st.ra[c] = (TC)A[gkc * g.lda + (gi < g.M ? gi : g.M - 1)];
          else st.ra[c] = st.oka[c] ? (TC)A[gk * g.lda + gi] : TC(0);
        }
      }
      const int64_t gk = k0 + x_r;
      const bool kok = gk < g.K;
      const int64_t gkc = kok ? gk : g.K - 1;
#pragma unroll
      for (int c = 0; c < CBW; ++c) {
        const int64_t gj = col0 + x_c + c;
        st.okx[c] = kok && gj < g.L;
        if (CLAMP) st.rx[c] = (TC)X[gkc * g.ldx + (gj < g.L ? gj : g.L - 1)];
        else st.rx[c] = st.okx[c] ? (TC)X[gk * g.ldx + gj] : TC(0);
      }
    };
    auto sstore = [&](const Stage& st, int buf) {
#pragma unroll
      for (int c = 0; c < 4; ++c)
        As[buf][a_r * ALD + a_c + c] = (CLAMP && !st.oka[c]) ? TC(0) : st.ra[c];
#pragma unroll
      for (int c = 0; c < CBW; ++c)
        Xs[buf][x_r * BN + x_c + c] = (CLAMP && !st.okx[c]) ? TC(0) : st.rx[c];
    };
    // the products of one k-step from LDS buffer b; at_kk0 runs inside the
    // unrolled k loop before its first products (the scheduler spreads the
    // next loads among them: measured Y = AX 1.75 -> 1.62 ms)
    auto compute = [&](int b, auto&& at_kk0) {
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        if (kk == 0) at_kk0();
        const int k = kk * 4 + lk;
        TC av[2];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
          const int i = wr * 32 + rb * 16 + li;
          av[rb] = TRANS ? As[b][k * ALD + i] : As[b][i * ALD + k];
        }
#pragma unroll
        for (int cb = 0; cb < CBW; ++cb) {
          const TC bv = Xs[b][k * BN + wc * 16 * CBW + cb * 16 + li];
#pragma unroll
          for (int rb = 0; rb < 2; ++rb) acc[rb][cb] = Mfma<TC>::mma(av[rb], bv, acc[rb][cb]);
        }
      }
    };

    if constexpr (CLAMP && CBW <= 7) {
      // FP64: two stages, so that a step's loads are issued two steps before
      // they are stored to LDS (the latency of loads under the pass's
      // traffic exceeds one step's products).  Two steps per iteration keep
      // each stage in its own registers.  Loads past the range re-read its
      // last step; their stores are skipped.  (CBW = 8 keeps one stage: the
      // second does not fit its registers; measured slower.)
      Stage s0, s1;
      gload(s0, kb);
      sstore(s0, 0);
      gload(s1, min(kb + 1, ke - 1));
      __syncthreads();
      for (int64_t kt = kb; kt < ke; kt += 2) {
        // step kt (buffer 0): s1 holds step kt + 1, s0 receives kt + 2
        compute(0, [&]() { gload(s0, min(kt + 2, ke - 1)); });
        if (kt + 1 < ke) sstore(s1, 1);
        __syncthreads();
        if (kt + 1 >= ke) break;
        // step kt + 1 (buffer 1): s0 holds step kt + 2, s1 receives kt + 3
        compute(1, [&]() { gload(s1, min(kt + 3, ke - 1)); });
        if (kt + 2 < ke) sstore(s0, 0);
        __syncthreads();
      }
    } else {
      Stage s0;
      gload(s0, kb);
      sstore(s0, 0);
      __syncthreads();
      int buf = 0;
      for (int64_t kt = kb; kt < ke; ++kt) {
        const bool more = kt + 1 < ke;
        if (!CLAMP && more) gload(s0, kt + 1);
        compute(buf, [&]() {
          if (CLAMP && more) gload(s0, kt + 1);
        });
        if (more) sstore(s0, buf ^ 1);
        __syncthreads();
        buf ^= 1;
      }
    }

    const bool full = (kb == 0) && (ke == g.KI);
    if (full) {
      TO* C = static_cast<TO*>(g.C);
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < CBW; ++cb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t r = row0 + wr * 32 + rb * 16 + Mfma<TC>::row(lk, v);
            const int64_t c = col0 + wc * 16 * CBW + cb * 16 + li;
            if (r < g.M && c < g.L) C[r * g.ldc + c] = (TO)acc[rb][cb][v];
          }
    } else {
      const int64_t slot = 2 * w + (kb == 0 ? 1 : 0);
      TC* P = static_cast<TC*>(g.part) + slot * (int64_t)(BM * BN);
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < CBW; ++cb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = wr * 32 + rb * 16 + Mfma<TC>::row(lk, v);
            const int c = wc * 16 * CBW + cb * 16 + li;
            P[r * BN + c] = acc[rb][cb][v];
          }
    }
  }
}

// Adds the partial sums of every tile that was split between workgroups.
// Grid: (tile, chunk of the tile's elements); each thread sums its elements
// over the workgroups that covered the tile, in a fixed order (eight
// interleaved chains, then their pairwise sums).  Chunks of FIX_CHUNK
// elements, or of FIX_CHUNK_FEW (one element per thread) when there are too
// few tiles to fill the chip: a reduction over a tall K splits each of a few
// small output tiles across ~100 workgroups, and its latency then sets the
// time.
constexpr int FIX_CHUNK = 1024;
constexpr int FIX_CHUNK_FEW = 256;

template <typename TC, typename TO, int CBW>
__global__ __launch_bounds__(256) void gemm_fixup_kernel(GemmArgs g) {
  constexpr int BN = 32 * CBW;
  const int64_t tile = blockIdx.x;
  const int64_t ufirst = tile * g.KI;
  const int64_t ulast = ufirst + g.KI - 1;
  // the workgroup whose range holds unit u: the largest w with begin(w) <= u
  const int64_t wf = ((ufirst + 1) * g.G + g.U - 1) / g.U - 1;
  const int64_t wl = ((ulast + 1) * g.G + g.U - 1) / g.U - 1;
  if (wf == wl) return;
  const int64_t row0 = (tile / g.nct) * BM;
  const int64_t col0 = (tile % g.nct) * BN;
  const TC* P = static_cast<const TC*>(g.part);
  TO* C = static_cast<TO*>(g.C);
  const int chunk = (BM * BN + (int)gridDim.y - 1) / (int)gridDim.y;
  const int e0 = blockIdx.y * chunk;
  const int e1 = min(e0 + chunk, BM * BN);
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int64_t r = row0 + e / BN;
    const int64_t c = col0 + e % BN;
    if (r >= g.M || c >= g.L) continue;
    // eight independent chains (workgroups w .. w+7), added in a fixed order:
    // the loads of eight partial tiles are in flight at once
    TC s[8] = {TC(0), TC(0), TC(0), TC(0), TC(0), TC(0), TC(0), TC(0)};
    int64_t w = wf;
    for (; w + 7 <= wl; w += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t wu = w + u;
        const bool ok = range_begin(wu, g.U, g.G) != range_begin(wu + 1, g.U, g.G);
        const int64_t slot = 2 * wu + (wu == wf ? 1 : 0);
        s[u] += ok ? P[slot * (int64_t)(BM * BN) + e] : TC(0);
      }
    }
    for (; w <= wl; ++w) {
      if (range_begin(w, g.U, g.G) == range_begin(w + 1, g.U, g.G)) continue;
      const int64_t slot = 2 * w + (w == wf ? 1 : 0);
      s[0] += P[slot * (int64_t)(BM * BN) + e];
    }
    C[r * g.ldc + c] = (TO)(((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7])));
  }
}

template <typename TA, typename TX, typename TC, typename TO, bool TRANS, int CBW>
hipError_t run(const GemmArgs& g, hipStream_t s) {
  hipLaunchKernelGGL((gemm_sk_kernel<TA, TX, TC, TO, TRANS, CBW>), dim3(g.G), dim3(NT), 0, s, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // with one workgroup per tile every range is a whole tile: no fix-up
  const int64_t T = g.U / g.KI;
  if (g.G != T) {
    unsigned nch = (unsigned)cdiv(BM * 32 * CBW, FIX_CHUNK);
    if (T * nch < 4 * 256) nch = (unsigned)cdiv(BM * 32 * CBW, FIX_CHUNK_FEW);
    hipLaunchKernelGGL((gemm_fixup_kernel<TC, TO, CBW>), dim3((unsigned)T, nch), dim3(256), 0, s,
                       g);
    e = hipGetLastError();
  }
  return e;
}

template <typename TA, typename TX, typename TC, typename TO, bool TRANS>
hipError_t dispatch_cbw(const GemmArgs& g, int cbw, hipStream_t s) {
  switch (cbw) {
    case 1: return run<TA, TX, TC, TO, TRANS, 1>(g, s);
    case 2: return run<TA, TX, TC, TO, TRANS, 2>(g, s);
    case 3: return run<TA, TX, TC, TO, TRANS, 3>(g, s);
    case 4: return run<TA, TX, TC, TO, TRANS, 4>(g, s);
    case 5: return run<TA, TX, TC, TO, TRANS, 5>(g, s);
    case 6: return run<TA, TX, TC, TO, TRANS, 6>(g, s);
    case 7: return run<TA, TX, TC, TO, TRANS, 7>(g, s);
    case 8: return run<TA, TX, TC, TO, TRANS, 8>(g, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename TA, typename TX, typename TC, typename TO>
hipError_t dispatch_trans(const GemmArgs& g, bool trans, int cbw, hipStream_t s) {
  return trans ? dispatch_cbw<TA, TX, TC, TO, true>(g, cbw, s)
               : dispatch_cbw<TA, TX, TC, TO, false>(g, cbw, s);
}

}  // namespace

GemmPlan plan_gemm(int64_t M, int64_t K, int64_t L, int ncu, int force_G) {
  GemmPlan p;
  // the fewest column tiles of at most 256 columns, as even as 32-column
  // steps allow (l = 576: three tiles of 192, not 256 + 256 + 64 with a
  // quarter of the products on padding)
  const int64_t ncb = cdiv(L, 16);
  const int64_t nct = cdiv(ncb, 16);
  p.cbw = (int)cdiv(ncb, 2 * nct);
  if (p.cbw < 1) p.cbw = 1;
  const int64_t BN = 32 * p.cbw;
  p.nrt = cdiv(M, BM);
  p.nct = cdiv(L, BN);
  p.KI = cdiv(K, BK);
  if (p.KI < 1) p.KI = 1;
  const int64_t T = p.nrt * p.nct;
  p.U = T * p.KI;
  if (force_G > 0) {
    p.G = force_G < p.U ? force_G : p.U;
  } else if (p.KI <= 32 && T >= ncu / 2) {
    p.G = T;                        // short reductions: one whole tile each
  } else {
    // at least ~16 k-steps per workgroup, so that few output tiles over a
    // long reduction do not leave a fix-up of hundreds of partial tiles
    int64_t G = p.U / 16;
    if (G < T) G = T;
    // narrow products (l <= 64) are bound by HBM latency: two workgroups per
    // compute unit keep more loads in flight (measured at l = 30 on a
    // 20000 x 10000 FP64 A: 3.0 -> 3.5 TB/s for A X, 3.2 -> 4.0 for A^T X)
    const int64_t gmax = p.cbw <= 2 ? 2 * (int64_t)ncu : ncu;
    if (G > gmax) G = gmax;
    p.G = G;
  }
  p.bm = BM;
  p.bn = BN;
  return p;
}

size_t gemm_part_bytes(const GemmPlan& p, size_t tc_size) {
  if (p.G == p.nrt * p.nct) return 0;
  return (size_t)(2 * p.G) * (size_t)(p.bm * p.bn) * tc_size;
}

hipError_t launch_gemm(GemmTypes ty, bool trans, const void* A, int64_t lda, const void* X,
                       int64_t ldx, void* C, int64_t ldc, int64_t M, int64_t K, int64_t L,
                       const GemmPlan& plan, void* part, size_t part_cap, hipStream_t s) {
  if (M <= 0 || L <= 0) return hipSuccess;
  if (K <= 0) return hipErrorInvalidValue;   // the clamped loads need one element of A and X
  GemmPlan p = plan;
  const size_t tc = (ty == GEMM_FFFF) ? sizeof(float) : sizeof(double);
  if (gemm_part_bytes(p, tc) > part_cap) p.G = p.nrt * p.nct;   // whole tiles: no partials
  GemmArgs g;
  g.A = A; g.lda = lda; g.X = X; g.ldx = ldx; g.C = C; g.ldc = ldc;
  g.M = M; g.K = K; g.L = L;
  g.nct = p.nct; g.KI = p.KI; g.U = p.U; g.G = p.G; g.part = part;
  switch (ty) {
    case GEMM_DDDD: return dispatch_trans<double, double, double, double>(g, trans, p.cbw, s);
    case GEMM_FFFF: return dispatch_trans<float, float, float, float>(g, trans, p.cbw, s);
    case GEMM_FFDD: return dispatch_trans<float, float, double, double>(g, trans, p.cbw, s);
    case GEMM_FDDF: return dispatch_trans<float, double, double, float>(g, trans, p.cbw, s);
    case GEMM_DDDF: return dispatch_trans<double, double, double, float>(g, trans, p.cbw, s);
    case GEMM_FDDD: return dispatch_trans<float, double, double, double>(g, trans, p.cbw, s);
    case GEMM_DFDD: return dispatch_trans<double, float, double, double>(g, trans, p.cbw, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rsvd
