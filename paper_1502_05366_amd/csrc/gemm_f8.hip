// Passes over an FP8 A on the matrix cores (mixed-precision range finder with
// A stored as FP8 E4M3 codes and one FP32 scale per column, A ~ A8 diag(s)).
//
//   Y = A X    = A8 (diag(s) X)          : the column scales sit on the
//                                          reduction index, so they are folded
//                                          into the skinny operand before it is
//                                          quantized;
//   Z = A^T X  = diag(s) (A8^T X)        : they are an epilogue row scale.
// The skinny operand X' (diag(s) X, or X) is quantized per output column:
// t_j = max_k |X'_kj| / 448, X8 = e4m3(X' / t) (nearest, ties to even), and
// the product is (op(A8) X8) diag(t) (diag(s) in the transposed case), with
// v_mfma_scale_f32_16x16x128_f8f6f4 on E4M3 x E4M3 (unit block scales) and
// FP32 accumulation.  A two-term split X' ~ t X8 + t2 X8lo (X8lo the codes of
// the residual with their own column scales t2) keeps about twice the
// significand bits in the last projection, as the BF16 passes do.
//
// Work decomposition as the BF16 passes: stream-K over (tile, k-step) units,
// deterministic partial tiles and a fix-up kernel that applies the scales;
// BM = 128 rows, BN = 32 * CBW columns (CBW <= 9, so l = 576 takes two column
// tiles), BK = 128 bytes (one matrix-core depth), 8 waves (4 along M x 2
// along L), each wave 2 x CBW accumulator tiles (72 accumulator registers per
// lane at CBW = 9, within the 256 of two waves per SIMD).
//
// MFMA operand layout (16 x 16 x 128, lane l, g = l / 16, c = l % 16): lane
// l holds 32 consecutive k of row c of the A operand and the same 32 k of
// column c of the B operand (k = 32 g .. 32 g + 31); D: lane l element v
// holds D[4 g + v][c].  Both operands sit in LDS with k contiguous ([row][k]
// for A, [col][k] for Xt): staged through registers with rows padded to 144
// bytes, or (Y = A X with K a multiple of 128, gemm_f8_dma_kernel) loaded
// straight into LDS in unpadded rows with rotated 16-byte chunks.  A
// transposed pass (A stored K x M) transposes 4 x 4 byte blocks in registers
// on the way into LDS.
#include "common.h"
#include "internal.h"

namespace rsvd {
namespace {

typedef int i8v __attribute__((ext_vector_type(8)));       // 32 bytes: one MFMA operand
typedef unsigned int u4v __attribute__((ext_vector_type(4)));  // 16 bytes

constexpr int BM = 128;
constexpr int BK = 128;            // bytes (= elements) of k per step
constexpr int KP = BK + 16;        // padded LDS row (bytes)
constexpr int NT = 512;
constexpr int RB = BM / 64;        // 16-row accumulator tiles per wave (2)
constexpr int MAX_CBW = 9;
constexpr int SCALE_ONE = 127;     // E8M0 block scale 2^0

struct F8Args {
  const uint8_t* A; int64_t lda;
  const uint8_t* X; int64_t ldx;      // Xt: L x K codes, row c holds column c of X'
  float* C; int64_t ldc;
  int64_t M, K, L;
  int64_t nct, KI, U, G;
  float* part;
  const float* xs;                    // L column scales t of the skinny operand
  const float* rs;                    // M row scales (transposed pass) or null
  int accumulate;
};

__device__ __forceinline__ int64_t range_begin(int64_t w, int64_t U, int64_t G) {
  return (w * U) / G;
}

__device__ __forceinline__ float out_scale(const F8Args& g, int64_t r, int64_t c) {
  return g.rs ? g.xs[c] * g.rs[r] : g.xs[c];
}

// bytes b of the four words w[0..3], packed into one word (byte r from w[r])
__device__ __forceinline__ uint32_t gather_byte(const uint32_t (&w)[4], int b) {
  const int sh = 8 * b;
  return ((w[0] >> sh) & 0xFFu) | (((w[1] >> sh) & 0xFFu) << 8) | (((w[2] >> sh) & 0xFFu) << 16) |
         (((w[3] >> sh) & 0xFFu) << 24);
}

// mask of the first n bytes of a word (n clamped to 0..4)
__device__ __forceinline__ uint32_t byte_mask(int64_t n) {
  return n >= 4 ? 0xFFFFFFFFu : n <= 0 ? 0u : (0xFFFFFFFFu >> (32 - 8 * (int)n));
}

template <bool TRANS, int CBW>
__global__ __launch_bounds__(NT) void gemm_f8_kernel(F8Args g) {
  constexpr int BN = 32 * CBW;
  __shared__ __attribute__((aligned(16))) uint8_t As[2][BM * KP];
  // Xs rows up to the staging's last chunk: the chunks past BN rows (zero)
  // are stored unconditionally, a branch there would split the loop body
  constexpr int XROWS = ((32 * CBW * BK / 16 + NT - 1) / NT) * NT / 8;
  __shared__ __attribute__((aligned(16))) uint8_t Xs[2][XROWS * KP];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave & 3;
  const int wc = wave >> 2;
  const int li = lane & 15;
  const int lk = lane >> 4;

  const int64_t w = blockIdx.x;
  int64_t u = range_begin(w, g.U, g.G);
  const int64_t uend = range_begin(w + 1, g.U, g.G);

  // staging: A in 16-byte chunks (APT per thread; transposed: 4 APT words per
  // thread, k rows KR kq .. KR kq + KR - 1 of the i quad 4 ir .. 4 ir + 3);
  // Xt in 16-byte chunks, XPT per thread (the last one partial)
  constexpr int APT = BM * BK / 16 / NT;
  constexpr int XCH = BN * BK / 16;
  constexpr int XPT = (XCH + NT - 1) / NT;
  static_assert(XPT * NT / 8 == XROWS, "staged Xs rows");
  constexpr int IQ = BM / 4;                 // i quads of a transposed tile
  constexpr int KR = BK / (NT / IQ);         // k rows per thread (= 4 APT)
  static_assert(KR == 4 * APT, "transposed staging covers the tile");
  const int ir = tid % IQ, kq = tid / IQ;

  while (u < uend) {
    const int64_t tile = u / g.KI;
    const int64_t kb = u - tile * g.KI;
    const int64_t ke = min(g.KI, kb + (uend - u));
    u += ke - kb;
    const int64_t row0 = (tile / g.nct) * BM;
    const int64_t col0 = (tile % g.nct) * BN;

    f4 acc[RB][CBW];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < CBW; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

      u4v ra[APT];                 // A chunks (transposed: 4 k rows of one i quad each)
    u4v rx[XPT];

    // Loads are unconditional, from a clamped address; what lies outside the
    // operands is zeroed when the staged step is stored (a branch around a
    // load makes the compiler wait for it at the join, and so does a select
    // right after it).  Rows of A are 16-byte aligned with a leading
    // dimension of 16k bytes and Xt rows are zero-padded to 16k, so a word or
    // chunk that starts inside a row lies inside its storage; the bytes of A
    // past the last column (row padding) are masked.
    auto gload = [&](int64_t kt) {
      const int64_t k0 = kt * BK;
      if (!TRANS) {
#pragma unroll
        for (int q = 0; q < APT; ++q) {
          const int ch = tid + q * NT;
          const int64_t gi = row0 + (ch >> 3);
          const int64_t gk = k0 + (ch & 7) * 16;
          const bool ok = gi < g.M && gk < g.K;
          ra[q] = *reinterpret_cast<const u4v*>(g.A + (ok ? gi * g.lda + gk : 0));
        }
      } else {
        // word r of chunk q: k row KR kq + 4 q + r, bytes i = 4 ir .. 4 ir + 3
        const int64_t gi = row0 + 4 * ir;
#pragma unroll
        for (int q = 0; q < APT; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t gk = k0 + KR * kq + 4 * q + r;
            const bool ok = gk < g.K && gi < g.M;
            ra[q][r] = *reinterpret_cast<const uint32_t*>(g.A + (ok ? gk * g.lda + gi : 0));
          }
      }
#pragma unroll
      for (int q = 0; q < XPT; ++q) {
        const int ch = tid + q * NT;
        const int64_t gj = col0 + (ch >> 3);
        const int64_t gk = k0 + (ch & 7) * 16;
        const bool ok = ch < XCH && gj < g.L && gk < g.K;
        rx[q] = *reinterpret_cast<const u4v*>(g.X + (ok ? gj * g.ldx + gk : 0));
      }
    };
    // zero what the loads of k-step kt read from outside the operands
    auto gmask = [&](int64_t kt) {
      const int64_t k0 = kt * BK;
      if (!TRANS) {
#pragma unroll
        for (int q = 0; q < APT; ++q) {
          const int ch = tid + q * NT;
          const int64_t gi = row0 + (ch >> 3);
          const int64_t gk = k0 + (ch & 7) * 16;
          const bool ok = gi < g.M && gk < g.K;
          const int64_t nb = g.K - gk;          // bytes of the chunk inside the row
#pragma unroll
          for (int w = 0; w < 4; ++w) ra[q][w] &= ok ? byte_mask(nb - 4 * w) : 0u;
        }
      } else {
        const int64_t gi = row0 + 4 * ir;
        const uint32_t im = byte_mask(g.M - gi);
#pragma unroll
        for (int q = 0; q < APT; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t gk = k0 + KR * kq + 4 * q + r;
            ra[q][r] &= gk < g.K ? im : 0u;
          }
      }
#pragma unroll
      for (int q = 0; q < XPT; ++q) {
        const int ch = tid + q * NT;
        const int64_t gj = col0 + (ch >> 3);
        const int64_t gk = k0 + (ch & 7) * 16;
        const bool ok = ch < XCH && gj < g.L && gk < g.K;
        rx[q] = ok ? rx[q] : u4v{0u, 0u, 0u, 0u};
      }
    };
    auto sstore = [&](int buf, int64_t kt) {
      gmask(kt);
      if (!TRANS) {
#pragma unroll
        for (int q = 0; q < APT; ++q) {
          const int ch = tid + q * NT;
          *reinterpret_cast<u4v*>(&As[buf][(ch >> 3) * KP + (ch & 7) * 16]) = ra[q];
        }
      } else {
#pragma unroll
        for (int q = 0; q < APT; ++q) {
          const uint32_t wv[4] = {ra[q][0], ra[q][1], ra[q][2], ra[q][3]};
          const int kc = KR * kq + 4 * q;
#pragma unroll
          for (int b = 0; b < 4; ++b)
            *reinterpret_cast<uint32_t*>(&As[buf][(4 * ir + b) * KP + kc]) = gather_byte(wv, b);
        }
      }
#pragma unroll
      for (int q = 0; q < XPT; ++q) {
        const int ch = tid + q * NT;
        *reinterpret_cast<u4v*>(&Xs[buf][(ch >> 3) * KP + (ch & 7) * 16]) = rx[q];
      }
    };

    gload(kb);
    sstore(0, kb);
    __syncthreads();
    int buf = 0;
    for (int64_t kt = kb; kt < ke; ++kt) {
      const int64_t kn = kt + 1 < ke ? kt + 1 : kt;
      // unconditional (the last step loads its own k-step again): under a
      // branch the staged registers would become phis that the compiler
      // fills by copies, waiting for the loads before the products
      gload(kn);
      // the loads go out before the products (left alone, the compiler sinks
      // them to the stores that use them)
      __builtin_amdgcn_sched_barrier(0);
      i8v av[RB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const int i = wr * 16 * RB + rb * 16 + li;
        const u4v lo = *reinterpret_cast<const u4v*>(&As[buf][i * KP + lk * 32]);
        const u4v hi = *reinterpret_cast<const u4v*>(&As[buf][i * KP + lk * 32 + 16]);
        av[rb] = i8v{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3],
                     (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
      }
#pragma unroll
      for (int cb = 0; cb < CBW; ++cb) {
        const int j = wc * 16 * CBW + cb * 16 + li;
        const u4v lo = *reinterpret_cast<const u4v*>(&Xs[buf][j * KP + lk * 32]);
        const u4v hi = *reinterpret_cast<const u4v*>(&Xs[buf][j * KP + lk * 32 + 16]);
        const i8v bv = i8v{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3],
                           (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
          acc[rb][cb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
              av[rb], bv, acc[rb][cb], 0, 0, 0, SCALE_ONE, 0, SCALE_ONE);
      }
      // the staged step goes to the other buffer after every product (on the
      // last step too, where no one reads it): the wait for its loads goes here
      __builtin_amdgcn_sched_barrier(0);
      sstore(buf ^ 1, kn);
      __syncthreads();
      buf ^= 1;
    }

    const bool full = (kb == 0) && (ke == g.KI);
    if (full) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CBW; ++cb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t r = row0 + wr * 16 * RB + rb * 16 + 4 * lk + v;
            const int64_t c = col0 + wc * 16 * CBW + cb * 16 + li;
            if (r < g.M && c < g.L) {
              float* cp = g.C + r * g.ldc + c;
              const float x = acc[rb][cb][v] * out_scale(g, r, c);
              *cp = g.accumulate ? *cp + x : x;
            }
          }
    } else {
      const int64_t slot = 2 * w + (kb == 0 ? 1 : 0);
      float* P = g.part + slot * (int64_t)(BM * BN);
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CBW; ++cb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = wr * 16 * RB + rb * 16 + 4 * lk + v;
            const int c = wc * 16 * CBW + cb * 16 + li;
            P[r * BN + c] = acc[rb][cb][v];
          }
    }
  }
}

// ---- Y = A X with both operands streamed straight into LDS -----------------
//
// The same tiles, work ranges and partial slots as gemm_f8_kernel, for the
// pass whose operands both hold k contiguously (A rows and Xt rows) and K a
// multiple of BK: the direct-to-LDS loads (global_load_lds_dwordx4) move
// each 128-byte k-step row from HBM into LDS without staging registers,
// three LDS stages deep (two k-steps in flight while the third is
// multiplied).  Staged rows are unpadded; the 16-byte chunk c of staged row
// r sits in slot c ^ (r & 7), so that the 8 lanes of one operand read
// (8 rows, one chunk) hit 8 different slots.  Rows past M or L are clamped
// to the last one (their products are discarded).
typedef __attribute__((address_space(3))) void* lds_vp;
typedef __attribute__((address_space(1))) void* gbl_vp;

template <int CBW> struct F8Dma {
  static constexpr int BN = 32 * CBW;
  static constexpr int ROWS = BM + BN;                 // staged rows per k-step
  static constexpr int NI = ROWS / 8;                  // 1 KB wave loads per k-step
  static constexpr int LPW = (NI + NT / 64 - 1) / (NT / 64);   // per wave (a few repeated)
  static constexpr int STAGE = ROWS * BK;              // bytes
  static constexpr int NS = 3;
  static constexpr size_t LDS = (size_t)NS * STAGE;
  static_assert(LDS <= 160 * 1024, "three stages fit the LDS");
};

// s_waitcnt that waits until at most n vector-memory operations are in
// flight (lgkm and exp counters left alone)
template <int N> __device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

template <int CBW>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2))) void gemm_f8_dma_kernel(F8Args g) {
  using D = F8Dma<CBW>;
  constexpr int BN = D::BN;
  constexpr int NS = D::NS;
  extern __shared__ __attribute__((aligned(16))) uint8_t dsm[];   // NS x ROWS x BK

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave & 3;
  const int wc = wave >> 2;
  const int li = lane & 15;
  const int lk = lane >> 4;

  const int64_t w = blockIdx.x;
  int64_t u = range_begin(w, g.U, g.G);
  const int64_t uend = range_begin(w + 1, g.U, g.G);

  while (u < uend) {
    const int64_t tile = u / g.KI;
    const int64_t kb = u - tile * g.KI;
    const int64_t ke = min(g.KI, kb + (uend - u));
    u += ke - kb;
    const int64_t row0 = (tile / g.nct) * BM;
    const int64_t col0 = (tile % g.nct) * BN;

    f4 acc[RB][CBW];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < CBW; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    // the loads of k-step kt into stage b: wave load j fills staged rows
    // 8 j .. 8 j + 7, lane l the slot l % 8 of row 8 j + l / 8
    auto issue = [&](int64_t kt, int b) {
      const int64_t k0 = kt * BK;
#pragma unroll
      for (int q = 0; q < D::LPW; ++q) {
        int j = wave + (NT / 64) * q;
        if (j >= D::NI) j -= D::NI;               // (a repeated load: same data, same slots)
        const int r = j * 8 + (lane >> 3);
        const int sch = (lane & 7) ^ (r & 7);     // the chunk this slot holds
        const uint8_t* src;
        if (r < BM) {
          const int64_t gi = min(row0 + r, g.M - 1);
          src = g.A + gi * g.lda + k0 + 16 * sch;
        } else {
          const int64_t gj = min(col0 + (r - BM), g.L - 1);
          src = g.X + gj * g.ldx + k0 + 16 * sch;
        }
        uint8_t* dst = dsm + (size_t)b * D::STAGE + (size_t)j * 8 * BK;
        __builtin_amdgcn_global_load_lds((gbl_vp)src, (lds_vp)dst, 16, 0, 0);
      }
    };

    const int64_t nst = ke - kb;
#pragma unroll
    for (int p = 0; p < NS - 1; ++p) issue(min(kb + p, ke - 1), p);
    for (int64_t t = 0; t < nst; ++t) {
      // this wave's loads of step t are done when at most the later NS - 2
      // steps' loads are in flight; the barrier makes every wave's visible
      // and frees the stage read at step t - 1
      wait_vm<(NS - 2) * D::LPW>();
      // a plain barrier: __syncthreads' release fence would wait for every
      // load in flight (the direct-to-LDS loads count as LDS writes)
      asm volatile("s_barrier" ::: "memory");
      issue(min(kb + t + NS - 1, ke - 1), (int)((t + NS - 1) % NS));
      const uint8_t* st = dsm + (size_t)(t % NS) * D::STAGE;
      auto oread = [&](int r) {
        const int x = r & 7;
        const u4v lo = *reinterpret_cast<const u4v*>(st + r * BK + 16 * ((2 * lk) ^ x));
        const u4v hi = *reinterpret_cast<const u4v*>(st + r * BK + 16 * ((2 * lk + 1) ^ x));
        return i8v{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3],
                   (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
      };
      i8v av[RB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) av[rb] = oread(wr * 16 * RB + rb * 16 + li);
      // every operand read before the first product: read one column block
      // at a time, the compiler waits for each read just before its products
      i8v bv[CBW];
#pragma unroll
      for (int cb = 0; cb < CBW; ++cb) bv[cb] = oread(BM + wc * 16 * CBW + cb * 16 + li);
#pragma unroll
      for (int cb = 0; cb < CBW; ++cb)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
          acc[rb][cb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
              av[rb], bv[cb], acc[rb][cb], 0, 0, 0, SCALE_ONE, 0, SCALE_ONE);
    }
    // no load may still be writing LDS when the next tile's first loads go out
    wait_vm<0>();
    __syncthreads();

    const bool full = (kb == 0) && (ke == g.KI);
    if (full) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CBW; ++cb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t r = row0 + wr * 16 * RB + rb * 16 + 4 * lk + v;
            const int64_t c = col0 + wc * 16 * CBW + cb * 16 + li;
            if (r < g.M && c < g.L) {
              float* cp = g.C + r * g.ldc + c;
              const float x = acc[rb][cb][v] * out_scale(g, r, c);
              *cp = g.accumulate ? *cp + x : x;
            }
          }
    } else {
      const int64_t slot = 2 * w + (kb == 0 ? 1 : 0);
      float* P = g.part + slot * (int64_t)(BM * BN);
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CBW; ++cb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = wr * 16 * RB + rb * 16 + 4 * lk + v;
            const int c = wc * 16 * CBW + cb * 16 + li;
            P[r * BN + c] = acc[rb][cb][v];
          }
    }
  }
}

// Sums the partial tiles of every split tile in workgroup order, then scales.
constexpr int FIX_CHUNK = 1024;

template <int CBW>
__global__ __launch_bounds__(256) void f8_fixup_kernel(F8Args g) {
  constexpr int BN = 32 * CBW;
  const int64_t tile = blockIdx.x;
  const int64_t ufirst = tile * g.KI;
  const int64_t ulast = ufirst + g.KI - 1;
  const int64_t wf = ((ufirst + 1) * g.G + g.U - 1) / g.U - 1;
  const int64_t wl = ((ulast + 1) * g.G + g.U - 1) / g.U - 1;
  if (wf == wl) return;
  const int64_t row0 = (tile / g.nct) * BM;
  const int64_t col0 = (tile % g.nct) * BN;
  const int e0 = blockIdx.y * FIX_CHUNK;
  const int e1 = min(e0 + FIX_CHUNK, BM * BN);
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int64_t r = row0 + e / BN;
    const int64_t c = col0 + e % BN;
    if (r >= g.M || c >= g.L) continue;
    float s = 0.f;
    for (int64_t w = wf; w <= wl; ++w) {
      if (range_begin(w, g.U, g.G) == range_begin(w + 1, g.U, g.G)) continue;
      const int64_t slot = 2 * w + (w == wf ? 1 : 0);
      s += g.part[slot * (int64_t)(BM * BN) + e];
    }
    float* cp = g.C + r * g.ldc + c;
    const float x = s * out_scale(g, r, c);
    *cp = g.accumulate ? *cp + x : x;
  }
}

// the direct-to-LDS kernel takes Y = A X when K is a multiple of BK (its
// k-steps then never leave the rows); the leading dimensions and the
// operands' 16-byte alignment hold for every FP8 pass
template <bool TRANS> bool f8_dma_ok(const F8Args& g) {
  return !TRANS && g.K % BK == 0 && g.lda % 16 == 0 && g.ldx % 16 == 0 &&
         (reinterpret_cast<uintptr_t>(g.A) & 15) == 0 && (reinterpret_cast<uintptr_t>(g.X) & 15) == 0;
}

template <bool TRANS, int CBW>
hipError_t run_f8(const F8Args& g, hipStream_t s) {
  hipError_t e;
  if (f8_dma_ok<TRANS>(g)) {
    const size_t shm = F8Dma<CBW>::LDS;
    e = hipFuncSetAttribute((const void*)gemm_f8_dma_kernel<CBW>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((gemm_f8_dma_kernel<CBW>), dim3((unsigned)g.G), dim3(NT), shm, s, g);
  } else {
    hipLaunchKernelGGL((gemm_f8_kernel<TRANS, CBW>), dim3((unsigned)g.G), dim3(NT), 0, s, g);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t T = g.U / g.KI;
  if (g.G != T) {
    const unsigned nch = (unsigned)cdiv(BM * 32 * CBW, FIX_CHUNK);
    hipLaunchKernelGGL((f8_fixup_kernel<CBW>), dim3((unsigned)T, nch), dim3(256), 0, s, g);
    e = hipGetLastError();
  }
  return e;
}

template <bool TRANS>
hipError_t dispatch_f8(const F8Args& g, int cbw, hipStream_t s) {
  switch (cbw) {
    case 1: return run_f8<TRANS, 1>(g, s);
    case 2: return run_f8<TRANS, 2>(g, s);
    case 3: return run_f8<TRANS, 3>(g, s);
    case 4: return run_f8<TRANS, 4>(g, s);
    case 5: return run_f8<TRANS, 5>(g, s);
    case 6: return run_f8<TRANS, 6>(g, s);
    case 7: return run_f8<TRANS, 7>(g, s);
    case 8: return run_f8<TRANS, 8>(g, s);
    case 9: return run_f8<TRANS, 9>(g, s);
    default: return hipErrorInvalidValue;
  }
}

// ---- the skinny operand in FP8 ---------------------------------------------
//
// E4M3 code of an FP32 value (nearest, ties to even, saturated to +-448; NaN
// to 0x7F): with e the binary exponent of |y| (at least -6, the smallest
// normal), the spacing is 2^(e-3); the rounded magnitude is re-read as
// (exponent, significand) fields.
__device__ __forceinline__ uint8_t e4m3_from_float(float y) {
  if (y != y) return 0x7F;
  const uint32_t sign = y < 0.f ? 0x80u : 0u;
  const float a = fabsf(y);
  uint32_t code;
  if (a >= 448.f) {
    code = 0x7E;
  } else {
    int e;
    (void)frexpf(a, &e);                       // a = f 2^e, f in [0.5, 1)
    const int E = max(e - 1, -6);
    const float step = ldexpf(1.f, E - 3);
    const float q = fminf(rintf(a / step) * step, 448.f);
    if (q >= 0x1.0p-6f) {
      int e2;
      (void)frexpf(q, &e2);
      const int E2 = e2 - 1;
      const uint32_t mant = (uint32_t)rintf((ldexpf(q, -E2) - 1.f) * 8.f);
      code = ((uint32_t)(E2 + 7) << 3) | mant;
    } else {
      code = (uint32_t)rintf(q * 512.f);
    }
  }
  return (uint8_t)(code | sign);
}

__device__ __forceinline__ float e4m3_to_float(uint8_t c) {
  const int e = (c >> 3) & 0xF, m = c & 7;
  const float v = e == 0 ? (float)m * 0x1.0p-9f : ldexpf(1.f + (float)m * 0.125f, e - 7);
  return (c & 0x80) ? -v : v;
}

// Element (k, c) of the operand being quantized: X'(k, c) = s_k X(k, c) (s may
// be null), or in residual mode the part that the first term leaves,
// X'(k, c) - t0_c dec(X8_0[c][k]).
template <typename TX>
__device__ __forceinline__ float xval(const TX* X, int64_t ldx, const float* s, int64_t k, int c,
                                      const uint8_t* prev, int64_t ldp, const float* t0) {
  float v = (float)X[k * ldx + c];
  if (s) v *= s[k];
  if (prev) v -= t0[c] * e4m3_to_float(prev[(int64_t)c * ldp + k]);
  return v;
}

// tmax[c] = max_k |X'(k, c)| as FP32 bits (non-negative floats order as
// integers); tmax zeroed beforehand.  Block: 64 columns x 4 row groups.
template <typename TX>
__global__ __launch_bounds__(256) void colmax_kernel(const TX* __restrict__ X, int64_t ldx,
                                                     int64_t rows, int cols, const float* s,
                                                     const uint8_t* prev, int64_t ldp,
                                                     const float* t0, uint32_t* tmax) {
  __shared__ float part[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int rg = threadIdx.x >> 6;
  // four independent maxima (a maximum does not depend on the order), so
  // that four loads per thread are in flight
  float m0 = 0.f, m1 = 0.f, m2 = 0.f, m3 = 0.f;
  if (c < cols) {
    const int64_t st = (int64_t)gridDim.y * 4;
    int64_t k = blockIdx.y * 4 + rg;
    for (; k + 3 * st < rows; k += 4 * st) {
      m0 = fmaxf(m0, fabsf(xval(X, ldx, s, k, c, prev, ldp, t0)));
      m1 = fmaxf(m1, fabsf(xval(X, ldx, s, k + st, c, prev, ldp, t0)));
      m2 = fmaxf(m2, fabsf(xval(X, ldx, s, k + 2 * st, c, prev, ldp, t0)));
      m3 = fmaxf(m3, fabsf(xval(X, ldx, s, k + 3 * st, c, prev, ldp, t0)));
    }
    for (; k < rows; k += st) m0 = fmaxf(m0, fabsf(xval(X, ldx, s, k, c, prev, ldp, t0)));
  }
  part[rg][threadIdx.x & 63] = fmaxf(fmaxf(m0, m1), fmaxf(m2, m3));
  __syncthreads();
  // one atomic per column and workgroup
  if (rg == 0 && c < cols) {
    const int i = threadIdx.x;
    const float m = fmaxf(fmaxf(part[0][i], part[1][i]), fmaxf(part[2][i], part[3][i]));
    atomicMax(tmax + c, __float_as_uint(m));
  }
}

// t[c] = tmax[c] / 448 (1 for a zero column)
__global__ __launch_bounds__(256) void colscale_kernel(const uint32_t* tmax, int cols, float* t) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= cols) return;
  const float m = __uint_as_float(tmax[c]);
  t[c] = m > 0.f ? m / 448.f : 1.f;
}

// Xt[c][k] = e4m3(X'(k, c) / t[c]); padding k in [rows, ldo) zero.  One 64 x
// 64 tile per workgroup: s_k X(k, c) goes through LDS (read with c
// contiguous), the residual term and the code are formed with k contiguous
// (the reads of prev and the writes of Xt), so all three are coalesced.  The
// arithmetic is xval's, in its order.
constexpr int TT = 64;

template <typename TX>
__global__ __launch_bounds__(256) void encode_kernel(const TX* __restrict__ X, int64_t ldx,
                                                     int64_t rows, int cols, const float* s,
                                                     const uint8_t* prev, int64_t ldp,
                                                     const float* t0, const float* t,
                                                     uint8_t* __restrict__ Xt, int64_t ldo) {
  __shared__ float tile[TT][TT + 1];
  const int64_t k0 = (int64_t)blockIdx.x * TT;
  const int c0 = blockIdx.y * TT;
  const int lo = threadIdx.x & 63, hi = threadIdx.x >> 6;
  for (int i = hi; i < TT; i += 4) {
    const int64_t k = k0 + i;
    const int c = c0 + lo;
    float v = 0.f;
    if (k < rows && c < cols) {
      v = (float)X[k * ldx + c];
      if (s) v *= s[k];
    }
    tile[i][lo] = v;
  }
  __syncthreads();
  for (int i = hi; i < TT; i += 4) {
    const int c = c0 + i;
    const int64_t k = k0 + lo;
    if (c >= cols || k >= ldo) continue;
    uint8_t code = 0;
    if (k < rows) {
      float v = tile[lo][i];
      if (prev) v -= t0[c] * e4m3_to_float(prev[(int64_t)c * ldp + k]);
      code = e4m3_from_float(v / t[c]);
    }
    Xt[(int64_t)c * ldo + k] = code;
  }
}

__global__ void zero_u32_kernel(uint32_t* p, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0u;
}

template <typename TX>
hipError_t quant_x(const TX* X, int64_t ldx, int64_t rows, int cols, const float* s,
                   const uint8_t* prev, int64_t ldp, const float* t0, uint8_t* Xt, int64_t ldo,
                   float* t, uint32_t* tmax, hipStream_t st) {
  const unsigned cb = (unsigned)cdiv(cols, 256);
  hipLaunchKernelGGL(zero_u32_kernel, dim3(cb), dim3(256), 0, st, tmax, cols);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned gx = (unsigned)cdiv(cols, 64);
  int64_t gy = cdiv(rows, 256);
  if (gy > 256) gy = 256;
  if (gy < 1) gy = 1;
  hipLaunchKernelGGL(colmax_kernel<TX>, dim3(gx, (unsigned)gy), dim3(256), 0, st, X, ldx, rows,
                     cols, s, prev, ldp, t0, tmax);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(colscale_kernel, dim3(cb), dim3(256), 0, st, tmax, cols, t);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const dim3 grid((unsigned)cdiv(ldo, TT), (unsigned)cdiv(cols, TT));
  hipLaunchKernelGGL(encode_kernel<TX>, grid, dim3(256), 0, st, X, ldx, rows, cols, s, prev, ldp,
                     t0, t, Xt, ldo);
  return hipGetLastError();
}

}  // namespace

GemmPlan plan_gemm_f8(int64_t M, int64_t K, int64_t L, int ncu) {
  GemmPlan p;
  const int64_t ncb = cdiv(L, 16);
  p.cbw = ncb <= 2 * MAX_CBW ? (int)cdiv(ncb, 2) : MAX_CBW;
  if (p.cbw < 1) p.cbw = 1;
  const int64_t BN = 32 * p.cbw;
  p.nrt = cdiv(M, BM);
  p.nct = cdiv(L, BN);
  p.KI = cdiv(K, BK);
  if (p.KI < 1) p.KI = 1;
  const int64_t T = p.nrt * p.nct;
  p.U = T * p.KI;
  if (p.KI <= 4 && T >= ncu / 2) p.G = T;
  else p.G = p.U < ncu ? p.U : ncu;
  p.bm = BM;
  p.bn = (int)BN;
  return p;
}

size_t gemm_f8_part_bytes(const GemmPlan& p) {
  if (p.G == p.nrt * p.nct) return 0;
  return (size_t)(2 * p.G) * (size_t)(p.bm * p.bn) * sizeof(float);
}

hipError_t launch_gemm_f8(bool trans, const uint8_t* A, int64_t lda, const uint8_t* Xt,
                          int64_t ldx, const float* xscale, const float* rscale, float* C,
                          int64_t ldc, int64_t M, int64_t K, int64_t L, const GemmPlan& plan,
                          void* part, size_t part_cap, bool accumulate, hipStream_t s) {
  if (M <= 0 || L <= 0) return hipSuccess;
  GemmPlan p = plan;
  if (gemm_f8_part_bytes(p) > part_cap) p.G = p.nrt * p.nct;
  F8Args g;
  g.A = A; g.lda = lda; g.X = Xt; g.ldx = ldx; g.C = C; g.ldc = ldc;
  g.M = M; g.K = K; g.L = L;
  g.nct = p.nct; g.KI = p.KI; g.U = p.U; g.G = p.G;
  g.part = static_cast<float*>(part);
  g.xs = xscale;
  g.rs = rscale;
  g.accumulate = accumulate ? 1 : 0;
  return trans ? dispatch_f8<true>(g, p.cbw, s) : dispatch_f8<false>(g, p.cbw, s);
}

hipError_t launch_quant_x_f8(bool x_f32, const void* X, int64_t ldx, int64_t rows, int cols,
                             const float* rowscale, const uint8_t* prev, int64_t ldp,
                             const float* t0, uint8_t* Xt, int64_t ldo, float* t, uint32_t* tmax,
                             hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  if (x_f32)
    return quant_x(static_cast<const float*>(X), ldx, rows, cols, rowscale, prev, ldp, t0, Xt, ldo,
                   t, tmax, s);
  return quant_x(static_cast<const double*>(X), ldx, rows, cols, rowscale, prev, ldp, t0, Xt, ldo,
                 t, tmax, s);
}

}  // namespace rsvd
