// Passes over a BF16 A on the matrix cores (mixed-precision range finder):
// C[M x L] (FP32) = op(A) Xb with A and Xb in BF16 and FP32 accumulation,
// v_mfma_f32_16x16x32_bf16.  The skinny operand arrives in FP32 or FP64 and is
// rounded to BF16 (to nearest even) and transposed (Xt = X^T, L x K, k
// contiguous) by convert_bf16_kernel before the pass; everything after the
// pass (CholeskyQR, Jacobi, pivoted QR) stays in FP64.
//
// Work decomposition as in the FP64 pass: stream-K over (tile, k-step) units
// with deterministic partial sums and a fix-up kernel; BM = 256 rows, BN =
// 32 * CBW columns, BK = 64 (two MFMA depths), 8 waves (4 along M x 2 along
// L), each wave 4 x CBW accumulator tiles.  The large BM halves the re-reads
// of the skinny operand per byte of A; the deep k-step keeps enough bytes of
// A in flight per workgroup for a pass that is bound by HBM, not by the
// matrix cores.
//
// MFMA operand layout (16 x 16 x 32, lane l, g = l / 16, c = l % 16):
//   A: lane l holds A[c][8 g .. 8 g + 7]; B: lane l holds B[8 g .. 8 g + 7][c];
//   D: lane l element v holds D[4 g + v][c].
// Both operands are staged in LDS with k contiguous ([row][k] for A, [col][k]
// for Xt), rows padded to 40 elements, so each lane reads its 8 values with
// one 16-byte LDS load.  A transposed pass (A stored K x M) transposes its
// tile on the way into LDS.
#include "common.h"
#include "internal.h"

namespace rsvd {
namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

constexpr int BM = 256;
constexpr int BK = 64;
constexpr int KP = BK + 8;         // padded k extent of an LDS row
constexpr int NT = 512;
constexpr int RB = BM / 64;        // 16-row accumulator tiles per wave

struct Bf16Args {
  const uint16_t* A; int64_t lda;
  const uint16_t* X; int64_t ldx;     // Xt: L x K, row c holds column c of X
  float* C; int64_t ldc;
  int64_t M, K, L;
  int64_t nct, KI, U, G;
  float* part;
  int accumulate;                     // C += op(A) Xt instead of C = op(A) Xt
  // S > 0 (the direct-to-LDS pass only): workgroup w takes one (row tile,
  // column tile, k split) in an XCD-aware order instead of a stream-K range
  int S;
  int64_t nrt;
};

__device__ __forceinline__ int64_t range_begin(int64_t w, int64_t U, int64_t G) {
  return (w * U) / G;
}

// RNE rounding of an FP32 value to BF16 bits (NaN kept quiet)
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// RBW row blocks per wave (tile rows 64 * RBW), k-steps BKW deep: <TRANS, 4,
// CBW, 64> for the 256-row tiles, <true, 2, CBW, 32> for the whole-width tiles
// of the transposed pass at l > 256.  EX: every 16-byte chunk of A that starts
// inside the matrix lies wholly inside it (the chunks' direction a multiple
// of 8 long, lda a multiple of 8, A 16-byte aligned).  The loads of the next
// k-step are then unconditional, from a clamped address, and go out before
// the products (scheduling barriers hold the order); the select that zeroes
// chunks outside the operands is taken when they are stored after the
// products.  A branch around a load, or a select right after it, makes the
// compiler wait for the load there.  Without EX, chunks that cross the edge
// are read element by element.
template <bool TRANS, int RBW, int CBW, int BKW, bool EX>
__global__ __launch_bounds__(NT) void gemm_bf16_kernel(Bf16Args g) {
  constexpr int BN = 32 * CBW;
  constexpr int BMv = 64 * RBW;
  constexpr int KPv = BKW + 8;         // padded k extent of an LDS row
  constexpr int KCH = BKW / 8;         // 16-byte k chunks per row
  __shared__ __attribute__((aligned(16))) uint16_t As[2][BMv * KPv];
  __shared__ __attribute__((aligned(16))) uint16_t Xs[2][BN * KPv];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave & 3;
  const int wc = wave >> 2;
  const int li = lane & 15;
  const int lk = lane >> 4;

  const int64_t w = blockIdx.x;
  int64_t u = 0, uend = 0;
  int64_t sp_tile = 0, sp_s = 0;
  if (g.S == 0) {
    u = range_begin(w, g.U, g.G);
    uend = range_begin(w + 1, g.U, g.G);
  } else {
    // split mode, as in the direct-to-LDS kernel: the workgroups of one XCD
    // share the column tile and k split
    const int64_t x = w % 8, j = w / 8;
    const int64_t rq_n = (g.nrt + 7) / 8;
    const int64_t rq = j % rq_n, cs = j / rq_n;
    const int64_t ct = cs / g.S, rt = x + 8 * rq;
    if (rt >= g.nrt || ct >= g.nct) return;   // (the whole workgroup)
    sp_tile = rt * g.nct + ct;
    sp_s = cs - ct * g.S;
    u = 0;
    uend = 1;
  }

  // staging in 8-element (16-byte) chunks: APT per thread for A, XPT (the
  // last one partial) for Xt
  constexpr int ACH = BMv * BKW / 8;
  constexpr int APT = ACH / NT;
  static_assert(APT >= 1 && APT * NT == ACH, "A staging");
  constexpr int XCH = BKW * BN / 8;
  constexpr int XPT = (XCH + NT - 1) / NT;

  while (u < uend) {
    int64_t tile, kb, ke;
    if (g.S == 0) {
      tile = u / g.KI;
      kb = u - tile * g.KI;
      ke = min(g.KI, kb + (uend - u));
      u += ke - kb;
    } else {
      tile = sp_tile;
      kb = (sp_s * g.KI) / g.S;
      ke = ((sp_s + 1) * g.KI) / g.S;
      u = uend;
    }
    const int64_t row0 = (tile / g.nct) * BMv;
    const int64_t col0 = (tile % g.nct) * BN;

    f4 acc[RBW][CBW];
#pragma unroll
    for (int i = 0; i < RBW; ++i)
#pragma unroll
      for (int j = 0; j < CBW; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    us8 ra[APT];
    us8 rx[XPT];
    // EX: whether each staged chunk lies inside its operand (the zeroing
    // select waits for the load, so it is taken when the chunk is stored)
    bool aok[APT], xok[XPT];

    auto gload_ex = [&](int64_t kt) {
      const int64_t k0 = kt * BKW;
#pragma unroll
      for (int q = 0; q < APT; ++q) {
        const int ch = tid + q * NT;
        int64_t gi, gk;
        if (!TRANS) {
          gi = row0 + ch / KCH;
          gk = k0 + (ch % KCH) * 8;
        } else {
          gk = k0 + (ch % BKW);
          gi = row0 + (ch / BKW) * 8;
        }
        const bool ok = gi < g.M && gk < g.K;
        const int64_t off = !TRANS ? gi * g.lda + gk : gk * g.lda + gi;
        ra[q] = *reinterpret_cast<const us8*>(g.A + (ok ? off : 0));
        aok[q] = ok;
      }
#pragma unroll
      for (int q = 0; q < XPT; ++q) {
        // Xt rows are zero-padded to whole k-steps: a chunk that starts
        // below K lies inside its row
        const int ch = tid + q * NT;
        const int64_t gj = col0 + ch / KCH;
        const int64_t gk = k0 + (ch % KCH) * 8;
        const bool ok = ch < XCH && gj < g.L && gk < g.K;
        rx[q] = *reinterpret_cast<const us8*>(g.X + (ok ? gj * g.ldx + gk : 0));
        xok[q] = ok;
      }
    };
    auto gload = [&](int64_t kt) {
      if constexpr (EX) {
        gload_ex(kt);
        return;
      }
      const int64_t k0 = kt * BKW;
#pragma unroll
      for (int q = 0; q < APT; ++q) {
        const int ch = tid + q * NT;
        us8 v;
        if (!TRANS) {
          // row ch / KCH, k chunk (ch % KCH) * 8
          const int64_t gi = row0 + ch / KCH;
          const int64_t gk = k0 + (ch % KCH) * 8;
          const uint16_t* p = g.A + gi * g.lda + gk;
          if (gi < g.M && gk + 8 <= g.K) {
            v = *reinterpret_cast<const us8*>(p);
          } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = (gi < g.M && gk + j < g.K) ? p[j] : (uint16_t)0;
          }
        } else {
          // k row ch % BKW, i chunk (ch / BKW) * 8: consecutive lanes take
          // consecutive k, so the transposing LDS writes do not collide
          const int64_t gk = k0 + (ch % BKW);
          const int64_t gi = row0 + (ch / BKW) * 8;
          const uint16_t* p = g.A + gk * g.lda + gi;
          if (gk < g.K && gi + 8 <= g.M) {
            v = *reinterpret_cast<const us8*>(p);
          } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = (gk < g.K && gi + j < g.M) ? p[j] : (uint16_t)0;
          }
        }
        ra[q] = v;
      }
#pragma unroll
      for (int q = 0; q < XPT; ++q) {
        const int ch = tid + q * NT;
        us8 v = us8{0, 0, 0, 0, 0, 0, 0, 0};
        if (ch < XCH) {
          // column ch / KCH of the tile, k chunk (ch % KCH) * 8
          const int64_t gj = col0 + ch / KCH;
          const int64_t gk = k0 + (ch % KCH) * 8;
          const uint16_t* p = g.X + gj * g.ldx + gk;
          if (gj < g.L && gk + 8 <= g.K) {
            v = *reinterpret_cast<const us8*>(p);
          } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = (gj < g.L && gk + j < g.K) ? p[j] : (uint16_t)0;
          }
        }
        rx[q] = v;
      }
    };
    auto sstore = [&](int buf) {
      if constexpr (EX) {
        const us8 z = us8{0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < APT; ++q) ra[q] = aok[q] ? ra[q] : z;
#pragma unroll
        for (int q = 0; q < XPT; ++q) rx[q] = xok[q] ? rx[q] : z;
      }
#pragma unroll
      for (int q = 0; q < APT; ++q) {
        const int ch = tid + q * NT;
        if (!TRANS) {
          *reinterpret_cast<us8*>(&As[buf][(ch / KCH) * KPv + (ch % KCH) * 8]) = ra[q];
        } else {
          const int kr = ch % BKW, i0 = (ch / BKW) * 8;
#pragma unroll
          for (int j = 0; j < 8; ++j) As[buf][(i0 + j) * KPv + kr] = ra[q][j];
        }
      }
#pragma unroll
      for (int q = 0; q < XPT; ++q) {
        const int ch = tid + q * NT;
        if (ch < XCH) *reinterpret_cast<us8*>(&Xs[buf][(ch / KCH) * KPv + (ch % KCH) * 8]) = rx[q];
      }
    };

    gload(kb);
    sstore(0);
    __syncthreads();
    int buf = 0;
    for (int64_t kt = kb; kt < ke; ++kt) {
      const bool more = kt + 1 < ke;
      if constexpr (EX) {
        // unconditional (the last step loads its own k-step again): under a
        // branch the staged registers become phis filled by copies, which
        // wait for the loads before the products
        gload(more ? kt + 1 : kt);
        // the loads go out before the products (left alone, the compiler
        // sinks them to the stores that use them)
        __builtin_amdgcn_sched_barrier(0);
      } else {
        if (more) gload(kt + 1);
      }
#pragma unroll
      for (int kk = 0; kk < BKW / 32; ++kk) {
        bf8 av[RBW];
#pragma unroll
        for (int rb = 0; rb < RBW; ++rb) {
          const int i = wr * 16 * RBW + rb * 16 + li;
          av[rb] = *reinterpret_cast<const bf8*>(&As[buf][i * KPv + kk * 32 + lk * 8]);
        }
#pragma unroll
        for (int cb = 0; cb < CBW; ++cb) {
          const int j = wc * 16 * CBW + cb * 16 + li;
          const bf8 bv = *reinterpret_cast<const bf8*>(&Xs[buf][j * KPv + kk * 32 + lk * 8]);
#pragma unroll
          for (int rb = 0; rb < RBW; ++rb)
            acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[rb], bv, acc[rb][cb], 0, 0, 0);
        }
      }
      if constexpr (EX) {
        // (on the last step too: the stage written is read by no one), after
        // every product, where the wait for the staged loads goes
        __builtin_amdgcn_sched_barrier(0);
        sstore(buf ^ 1);
      } else {
        if (more) sstore(buf ^ 1);
      }
      __syncthreads();
      buf ^= 1;
    }

    const bool full = (kb == 0) && (ke == g.KI);
    if (full) {
#pragma unroll
      for (int rb = 0; rb < RBW; ++rb)
#pragma unroll
        for (int cb = 0; cb < CBW; ++cb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t r = row0 + wr * 16 * RBW + rb * 16 + 4 * lk + v;
            const int64_t c = col0 + wc * 16 * CBW + cb * 16 + li;
            if (r < g.M && c < g.L) {
              float* cp = g.C + r * g.ldc + c;
              *cp = g.accumulate ? *cp + acc[rb][cb][v] : acc[rb][cb][v];
            }
          }
    } else {
      const int64_t slot = (g.S > 0) ? tile * g.S + sp_s : 2 * w + (kb == 0 ? 1 : 0);
      float* P = g.part + slot * (int64_t)(BMv * BN);
#pragma unroll
      for (int rb = 0; rb < RBW; ++rb)
#pragma unroll
        for (int cb = 0; cb < CBW; ++cb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = wr * 16 * RBW + rb * 16 + 4 * lk + v;
            const int c = wc * 16 * CBW + cb * 16 + li;
            P[r * BN + c] = acc[rb][cb][v];
          }
    }
  }
}

// Y = A Xt for a row-major A (the non-transposed pass) with both operands
// moved from HBM to LDS by the direct-to-LDS loads (global_load_lds_dwordx4),
// so that several k-steps are in flight without staging registers: four LDS
// stages of 32-deep k-steps, three of them loading while the fourth is
// multiplied; one barrier per k-step.  A wave's 16-byte load writes 64
// consecutive 16-byte slots of LDS, so a staged row (32 k, 64 bytes) holds
// its four 16-byte chunks in a rotated order (chunk s of row r in slot
// s ^ ((r >> 2) & 3)): the 16 lanes that read one chunk of 16 consecutive
// rows then hit 16 different 4-bank groups.  Rows past M or L re-read the last
// row; k past K re-reads A's last chunk against the zero padding of Xt (so
// the launch needs K and lda multiples of 8, A 16-byte aligned and
// ldx >= 32 * ceil(K / 32), Xt zero beyond K).
constexpr int DK = 32;
constexpr int DNS = 4;
typedef __attribute__((address_space(3))) void* lds_vp;
typedef __attribute__((address_space(1))) void* gbl_vp;

template <int RBW, int CBW> struct DmaDims {
  static constexpr int BMv = 64 * RBW;                 // tile rows (4 waves of 16 * RBW)
  static constexpr int BN = 32 * CBW;
  static constexpr int ROWS = BMv + BN;                // staged rows per k-step
  static constexpr int NI = ROWS / 16;                 // 1 KB wave loads per k-step
  static constexpr int LPW = (NI + NT / 64 - 1) / (NT / 64);   // per wave (a few repeated)
  static constexpr int STAGE = ROWS * DK;              // elements
  static constexpr int NS = (RBW == 4) ? DNS : 3;     // LDS stages (wide tiles: three)
  static constexpr size_t LDS = (size_t)NS * STAGE * sizeof(uint16_t);
};

// s_waitcnt that waits until at most n vector-memory operations are in
// flight (lgkm and exp counters left alone)
template <int N> __device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

template <int RBW, int CBW>
__global__ __launch_bounds__(NT) void gemm_bf16_dma_kernel(Bf16Args g) {
  using D = DmaDims<RBW, CBW>;
  constexpr int BN = D::BN;
  constexpr int BMv = D::BMv;
  constexpr int NS = D::NS;
  extern __shared__ __attribute__((aligned(16))) uint16_t dsm[];   // DNS x ROWS x DK

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave & 3;
  const int wc = wave >> 2;
  const int li = lane & 15;
  const int lk = lane >> 4;

  const int64_t w = blockIdx.x;
  int64_t u = 0, uend = 0;
  int64_t sp_tile = 0, sp_s = 0;
  if (g.S == 0) {
    u = range_begin(w, g.U, g.G);
    uend = range_begin(w + 1, g.U, g.G);
  } else {
    // split mode.  Workgroups are dealt to the XCDs in turn (w % 8), so the
    // workgroups of one XCD that run at the same time take the same column
    // tile and k split of different row tiles: their operand Xt k-slices are
    // the same lines of that XCD's L2.
    const int64_t x = w % 8, j = w / 8;
    const int64_t rq_n = (g.nrt + 7) / 8;
    const int64_t rq = j % rq_n, cs = j / rq_n;
    const int64_t ct = cs / g.S, rt = x + 8 * rq;
    if (rt >= g.nrt || ct >= g.nct) return;   // (the whole workgroup)
    sp_tile = rt * g.nct + ct;
    sp_s = cs - ct * g.S;
    u = 0;
    uend = 1;
  }

  while (u < uend) {
    int64_t tile, kb, ke;
    if (g.S == 0) {
      tile = u / g.KI;
      kb = u - tile * g.KI;
      ke = min(g.KI, kb + (uend - u));
      u += ke - kb;
    } else {
      tile = sp_tile;
      kb = (sp_s * g.KI) / g.S;
      ke = ((sp_s + 1) * g.KI) / g.S;
      u = uend;
    }
    const int64_t row0 = (tile / g.nct) * BMv;
    const int64_t col0 = (tile % g.nct) * BN;

    f4 acc[RBW][CBW];
#pragma unroll
    for (int i = 0; i < RBW; ++i)
#pragma unroll
      for (int j = 0; j < CBW; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    // the loads of k-step kt into stage b
    auto issue = [&](int64_t kt, int b) {
      const int64_t k0 = kt * DK;
#pragma unroll
      for (int q = 0; q < D::LPW; ++q) {
        int j = wave + (NT / 64) * q;
        if (j >= D::NI) j -= D::NI;               // (a repeated load: same data, same slots)
        const int r = j * 16 + (lane >> 2);       // staged row
        const int sch = (lane & 3) ^ ((r >> 2) & 3);   // the chunk this slot holds
        const uint16_t* src;
        if (r < BMv) {
          const int64_t gi = min(row0 + r, g.M - 1);
          const int64_t gk = min(k0 + 8 * sch, g.K - 8);
          src = g.A + gi * g.lda + gk;
        } else {
          const int64_t gj = min(col0 + (r - BMv), g.L - 1);
          src = g.X + gj * g.ldx + k0 + 8 * sch;
        }
        uint16_t* dst = dsm + (size_t)b * D::STAGE + (size_t)j * 16 * DK;
        __builtin_amdgcn_global_load_lds((gbl_vp)src, (lds_vp)dst, 16, 0, 0);
      }
    };

    const int64_t nst = ke - kb;
#pragma unroll
    for (int p = 0; p < NS - 1; ++p) issue(min(kb + p, ke - 1), p);
    for (int64_t t = 0; t < nst; ++t) {
      // this wave's loads of step t are done when at most the later
      // DNS - 2 steps' loads are in flight; the barrier makes every wave's
      // visible and frees the stage read at step t - 1
      wait_vm<(NS - 2) * D::LPW>();
      // a plain barrier: __syncthreads' release fence would wait for every
      // load in flight (the direct-to-LDS loads count as LDS writes)
      asm volatile("s_barrier" ::: "memory");
      issue(min(kb + t + NS - 1, ke - 1), (int)((t + NS - 1) % NS));
      const uint16_t* st = dsm + (size_t)(t % NS) * D::STAGE;
      bf8 av[RBW];
#pragma unroll
      for (int rb = 0; rb < RBW; ++rb) {
        const int r = wr * 16 * RBW + rb * 16 + li;
        av[rb] = *reinterpret_cast<const bf8*>(st + r * DK + 8 * (lk ^ ((r >> 2) & 3)));
      }
#pragma unroll
      for (int cb = 0; cb < CBW; ++cb) {
        const int r = BMv + wc * 16 * CBW + cb * 16 + li;
        const bf8 bv = *reinterpret_cast<const bf8*>(st + r * DK + 8 * (lk ^ ((r >> 2) & 3)));
#pragma unroll
        for (int rb = 0; rb < RBW; ++rb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[rb], bv, acc[rb][cb], 0, 0, 0);
      }
    }
    // no load may still be writing LDS when the next tile's first loads go out
    wait_vm<0>();
    __syncthreads();

    const bool full = (kb == 0) && (ke == g.KI);
    if (full) {
#pragma unroll
      for (int rb = 0; rb < RBW; ++rb)
#pragma unroll
        for (int cb = 0; cb < CBW; ++cb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t r = row0 + wr * 16 * RBW + rb * 16 + 4 * lk + v;
            const int64_t c = col0 + wc * 16 * CBW + cb * 16 + li;
            if (r < g.M && c < g.L) {
              float* cp = g.C + r * g.ldc + c;
              *cp = g.accumulate ? *cp + acc[rb][cb][v] : acc[rb][cb][v];
            }
          }
    } else {
      const int64_t slot = (g.S > 0) ? tile * g.S + sp_s : 2 * w + (kb == 0 ? 1 : 0);
      float* P = g.part + slot * (int64_t)(BMv * BN);
#pragma unroll
      for (int rb = 0; rb < RBW; ++rb)
#pragma unroll
        for (int cb = 0; cb < CBW; ++cb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = wr * 16 * RBW + rb * 16 + 4 * lk + v;
            const int c = wc * 16 * CBW + cb * 16 + li;
            P[r * BN + c] = acc[rb][cb][v];
          }
    }
  }
}

// Sums the partial tiles of every split tile in workgroup order.
constexpr int FIX_CHUNK = 1024;

template <int CBW>
__global__ __launch_bounds__(256) void bf16_fixup_kernel(Bf16Args g) {
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
    *cp = g.accumulate ? *cp + s : s;
  }
}

// Split mode: C = the sum of the S partial tiles of each tile, in split order.
template <int CBW>
__global__ __launch_bounds__(256) void bf16_split_fixup_kernel(Bf16Args g) {
  constexpr int BN = 32 * CBW;
  const int64_t tile = blockIdx.x;
  const int64_t row0 = (tile / g.nct) * BM;
  const int64_t col0 = (tile % g.nct) * BN;
  const int e0 = blockIdx.y * FIX_CHUNK;
  const int e1 = min(e0 + FIX_CHUNK, BM * BN);
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int64_t r = row0 + e / BN;
    const int64_t c = col0 + e % BN;
    if (r >= g.M || c >= g.L) continue;
    float sum = 0.f;
    for (int sp = 0; sp < g.S; ++sp) sum += g.part[(tile * g.S + sp) * (int64_t)(BM * BN) + e];
    float* cp = g.C + r * g.ldc + c;
    *cp = g.accumulate ? *cp + sum : sum;
  }
}

template <bool TRANS, int CBW, int RBW = 4, int BKW = BK>
hipError_t run_bf16(const Bf16Args& g, hipStream_t s) {
  // chunks run along k (A X) or along the rows of the result (A^T X).  The
  // 256-row tiles keep the conditional loads: with 4 row blocks per wave
  // their registers do not hold a step's loads in flight across the products
  const int64_t run = TRANS ? g.M : g.K;
  const bool ex = RBW == 2 && run % 8 == 0 && g.lda % 8 == 0 &&
                  (reinterpret_cast<uintptr_t>(g.A) & 15) == 0 && g.ldx % 8 == 0 &&
                  (reinterpret_cast<uintptr_t>(g.X) & 15) == 0;
  if constexpr (RBW == 2) {
    if (ex) {
      hipLaunchKernelGGL((gemm_bf16_kernel<TRANS, RBW, CBW, BKW, true>), dim3((unsigned)g.G),
                         dim3(NT), 0, s, g);
    } else {
      hipLaunchKernelGGL((gemm_bf16_kernel<TRANS, RBW, CBW, BKW, false>), dim3((unsigned)g.G),
                         dim3(NT), 0, s, g);
    }
  } else {
    (void)ex;
    hipLaunchKernelGGL((gemm_bf16_kernel<TRANS, RBW, CBW, BKW, false>), dim3((unsigned)g.G),
                       dim3(NT), 0, s, g);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t T = g.U / g.KI;
  if (g.S > 1) {
    const unsigned nch = (unsigned)cdiv(BM * 32 * CBW, FIX_CHUNK);
    hipLaunchKernelGGL((bf16_split_fixup_kernel<CBW>), dim3((unsigned)T, nch), dim3(256), 0, s,
                       g);
    return hipGetLastError();
  }
  if (g.S == 0 && g.G != T) {
    const unsigned nch = (unsigned)cdiv(BM * 32 * CBW, FIX_CHUNK);
    hipLaunchKernelGGL((bf16_fixup_kernel<CBW>), dim3((unsigned)T, nch), dim3(256), 0, s, g);
    e = hipGetLastError();
  }
  return e;
}

template <int RBW, int CBW>
hipError_t run_bf16_dma(const Bf16Args& g, hipStream_t s) {
  const size_t shm = DmaDims<RBW, CBW>::LDS;
  hipError_t e = hipFuncSetAttribute((const void*)gemm_bf16_dma_kernel<RBW, CBW>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((gemm_bf16_dma_kernel<RBW, CBW>), dim3((unsigned)g.G), dim3(NT), shm, s, g);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t T = g.U / g.KI;
  if (g.S > 1) {
    // (the 256-row tiles only: the wide tiles run with S = 1)
    const unsigned nch = (unsigned)cdiv(BM * 32 * CBW, FIX_CHUNK);
    hipLaunchKernelGGL((bf16_split_fixup_kernel<CBW>), dim3((unsigned)T, nch), dim3(256), 0, s,
                       g);
    return hipGetLastError();
  }
  if (g.S == 0 && g.G != T) {
    const unsigned nch = (unsigned)cdiv(BM * 32 * CBW, FIX_CHUNK);
    hipLaunchKernelGGL((bf16_fixup_kernel<CBW>), dim3((unsigned)T, nch), dim3(256), 0, s, g);
    e = hipGetLastError();
  }
  return e;
}

hipError_t dispatch_bf16_dma(const Bf16Args& g, int cbw, hipStream_t s) {
  switch (cbw) {
    case 1: return run_bf16_dma<4, 1>(g, s);
    case 2: return run_bf16_dma<4, 2>(g, s);
    case 3: return run_bf16_dma<4, 3>(g, s);
    case 4: return run_bf16_dma<4, 4>(g, s);
    case 5: return run_bf16_dma<4, 5>(g, s);
    case 6: return run_bf16_dma<4, 6>(g, s);
    case 7: return run_bf16_dma<4, 7>(g, s);
    case 8: return run_bf16_dma<4, 8>(g, s);
    default: return hipErrorInvalidValue;
  }
}

// the transposed pass in whole-width tiles (128 rows, 32-deep k-steps)
hipError_t dispatch_bf16_wide_t(const Bf16Args& g, int cbw, hipStream_t s) {
  switch (cbw) {
    case 12: return run_bf16<true, 12, 2, 32>(g, s);
    case 16: return run_bf16<true, 16, 2, 32>(g, s);
    case 18: return run_bf16<true, 18, 2, 32>(g, s);
    default: return hipErrorInvalidValue;
  }
}

// wide tiles: 128 rows x 32 * cbw columns (cbw 12, 16 or 18), the whole L
hipError_t dispatch_bf16_dma_wide(const Bf16Args& g, int cbw, hipStream_t s) {
  switch (cbw) {
    case 12: return run_bf16_dma<2, 12>(g, s);
    case 16: return run_bf16_dma<2, 16>(g, s);
    case 18: return run_bf16_dma<2, 18>(g, s);
    default: return hipErrorInvalidValue;
  }
}

template <bool TRANS>
hipError_t dispatch_bf16(const Bf16Args& g, int cbw, hipStream_t s) {
  switch (cbw) {
    case 1: return run_bf16<TRANS, 1>(g, s);
    case 2: return run_bf16<TRANS, 2>(g, s);
    case 3: return run_bf16<TRANS, 3>(g, s);
    case 4: return run_bf16<TRANS, 4>(g, s);
    case 5: return run_bf16<TRANS, 5>(g, s);
    case 6: return run_bf16<TRANS, 6>(g, s);
    case 7: return run_bf16<TRANS, 7>(g, s);
    case 8: return run_bf16<TRANS, 8>(g, s);
    default: return hipErrorInvalidValue;
  }
}

// Xt[c * ldo + k] = bf16(x) (MODE 0) or bf16(x - bf16(x)) (MODE 1: the low
// part of a two-term BF16 split; the subtraction is exact in FP32), x =
// X[k][c] rounded to FP32, for c < cols, k < rows; the padding k in [rows,
// ldo) is zero.  One 64 x 64 tile per workgroup passes through LDS, so that
// the reads (c contiguous) and the writes (k contiguous) are both coalesced.
constexpr int TT = 64;

template <typename T, int MODE>
__global__ __launch_bounds__(256) void convert_bf16_kernel(const T* __restrict__ in, int64_t ldi,
                                                           int64_t rows, int cols,
                                                           uint16_t* __restrict__ out,
                                                           int64_t ldo) {
  __shared__ uint16_t tile[TT][TT + 2];
  const int64_t k0 = (int64_t)blockIdx.x * TT;
  const int c0 = blockIdx.y * TT;
  const int lo = threadIdx.x & 63, hi = threadIdx.x >> 6;
  for (int i = hi; i < TT; i += 4) {
    const int64_t k = k0 + i;
    const int c = c0 + lo;
    uint16_t v = 0;
    if (k < rows && c < cols) {
      const float x = (float)in[k * ldi + c];
      if (MODE == 0) {
        v = to_bf16(x);
      } else {
        const float h = __uint_as_float((uint32_t)to_bf16(x) << 16);
        v = to_bf16(x - h);
      }
    }
    tile[i][lo] = v;
  }
  __syncthreads();
  for (int i = hi; i < TT; i += 4) {
    const int c = c0 + i;
    const int64_t k = k0 + lo;
    if (c < cols && k < ldo) out[(int64_t)c * ldo + k] = tile[lo][i];
  }
}

}  // namespace

GemmPlan plan_gemm_bf16(int64_t M, int64_t K, int64_t L, int ncu) {
  GemmPlan p;
  const int64_t ncb = cdiv(L, 16);
  p.cbw = ncb <= 16 ? (int)cdiv(ncb, 2) : 8;
  if (p.cbw < 1) p.cbw = 1;
  const int64_t BN = 32 * p.cbw;
  p.nrt = cdiv(M, BM);
  p.nct = cdiv(L, BN);
  p.KI = cdiv(K, BK);
  if (p.KI < 1) p.KI = 1;
  const int64_t T = p.nrt * p.nct;
  p.U = T * p.KI;
  if (p.KI <= 8 && T >= ncu / 2) p.G = T;
  else p.G = p.U < ncu ? p.U : ncu;
  p.bm = BM;
  p.bn = (int)BN;
  return p;
}

size_t gemm_bf16_part_bytes(const GemmPlan& p) {
  if (p.G == p.nrt * p.nct) return 0;
  return (size_t)(2 * p.G) * (size_t)(p.bm * p.bn) * sizeof(float);
}

namespace {
hipError_t gemm_bf16(bool trans, const uint16_t* A, int64_t lda, const uint16_t* Xt, int64_t ldx,
                     float* C, int64_t ldc, int64_t M, int64_t K, int64_t L, const GemmPlan& plan,
                     void* part, size_t part_cap, bool accumulate, hipStream_t s) {
  if (M <= 0 || L <= 0) return hipSuccess;
  GemmPlan p = plan;
  if (gemm_bf16_part_bytes(p) > part_cap) p.G = p.nrt * p.nct;
  Bf16Args g;
  g.A = A; g.lda = lda; g.X = Xt; g.ldx = ldx; g.C = C; g.ldc = ldc;
  g.M = M; g.K = K; g.L = L;
  g.nct = p.nct; g.KI = p.KI; g.U = p.U; g.G = p.G;
  g.part = static_cast<float*>(part);
  g.accumulate = accumulate ? 1 : 0;
  g.S = 0;
  g.nrt = p.nrt;
  // the direct-to-LDS kernel (32-deep k-steps) where its alignment and
  // padding conditions hold, in split mode: S = the splits per tile that keep
  // the tiles x splits within the CUs (one tile per workgroup when there are
  // more tiles than CUs), the partial tiles within the workspace
  const int64_t kid = cdiv(K, DK);
  const bool dma_ok = !trans && K >= 8 && K % 8 == 0 && lda % 8 == 0 && ldx % 8 == 0 &&
                      ldx >= kid * DK && (reinterpret_cast<uintptr_t>(A) & 15) == 0 &&
                      (reinterpret_cast<uintptr_t>(Xt) & 15) == 0;
  // wide tiles (l > 256): 128 rows x all columns per workgroup, so that A is
  // read once instead of once per 256-column tile; one tile per workgroup
  // (no partial sums) when the row tiles fill the CUs
  if (dma_ok && p.nct > 1 && L <= 576 && cdiv(M, 128) >= p.G) {
    const int cw = (L <= 384) ? 12 : (L <= 512) ? 16 : 18;
    const int64_t nrt = cdiv(M, 128);
    g.nct = 1;
    g.nrt = nrt;
    g.KI = kid;
    g.U = nrt * kid;
    g.S = 1;
    g.G = 8 * cdiv(nrt, 8);
    return dispatch_bf16_dma_wide(g, cw, s);
  }
  if (dma_ok) {
    const int64_t T = p.nrt * p.nct;
    int64_t S = std::max<int64_t>(1, std::min<int64_t>(kid / 8, (int64_t)p.G / T));
    while (S > 1 && (size_t)(T * S) * (size_t)(BM * 32 * p.cbw) * sizeof(float) > part_cap) --S;
    g.KI = kid;
    g.U = T * kid;
    g.S = (int)S;
    g.G = 8 * p.nct * S * cdiv(p.nrt, 8);
    return dispatch_bf16_dma(g, p.cbw, s);
  }
  // the transposed pass at l > 256 in whole-width tiles as well (A
  // transposed on its way into LDS, 32-deep k-steps), one tile per workgroup
  if (trans && p.nct > 1 && L <= 576 && cdiv(M, 128) >= p.G) {
    const int cw = (L <= 384) ? 12 : (L <= 512) ? 16 : 18;
    const int64_t nrt = cdiv(M, 128), kiw = cdiv(K, 32);
    g.nct = 1;
    g.nrt = nrt;
    g.KI = kiw;
    g.U = nrt * kiw;
    g.S = 1;
    g.G = 8 * cdiv(nrt, 8);
    return dispatch_bf16_wide_t(g, cw, s);
  }
  // the register-staged kernel (64-deep k-steps; the transposed pass) in the
  // same split mode when the tiles are fewer than the CUs
  {
    const int64_t T = p.nrt * p.nct;
    int64_t S = std::min<int64_t>(p.KI / 4, (int64_t)p.G / T);
    while (S > 1 && (size_t)(T * S) * (size_t)(BM * 32 * p.cbw) * sizeof(float) > part_cap) --S;
    if (S >= 2) {
      g.S = (int)S;
      g.G = 8 * p.nct * S * cdiv(p.nrt, 8);
    }
  }
  return trans ? dispatch_bf16<true>(g, p.cbw, s) : dispatch_bf16<false>(g, p.cbw, s);
}
}  // namespace

hipError_t launch_gemm_bf16(bool trans, const uint16_t* A, int64_t lda, const uint16_t* Xt,
                            int64_t ldx, float* C, int64_t ldc, int64_t M, int64_t K, int64_t L,
                            const GemmPlan& plan, void* part, size_t part_cap, hipStream_t s) {
  return gemm_bf16(trans, A, lda, Xt, ldx, C, ldc, M, K, L, plan, part, part_cap, false, s);
}

hipError_t launch_gemm_bf16_acc(bool trans, const uint16_t* A, int64_t lda, const uint16_t* Xt,
                                int64_t ldx, float* C, int64_t ldc, int64_t M, int64_t K,
                                int64_t L, const GemmPlan& plan, void* part, size_t part_cap,
                                hipStream_t s) {
  return gemm_bf16(trans, A, lda, Xt, ldx, C, ldc, M, K, L, plan, part, part_cap, true, s);
}

hipError_t launch_bf16_residual(const float* X, int64_t ldx, int64_t rows, int cols,
                                uint16_t* out, int64_t ldo, hipStream_t s) {
  if (cols <= 0 || ldo <= 0) return hipSuccess;
  const dim3 grid((unsigned)cdiv(ldo, TT), (unsigned)cdiv(cols, TT));
  hipLaunchKernelGGL((convert_bf16_kernel<float, 1>), grid, dim3(256), 0, s, X, ldx, rows, cols,
                     out, ldo);
  return hipGetLastError();
}

hipError_t launch_convert_bf16(bool in_f32, const void* in, int64_t ldi, int64_t rows, int cols,
                               uint16_t* out, int64_t ldo, hipStream_t s) {
  if (cols <= 0 || ldo <= 0) return hipSuccess;
  const dim3 grid((unsigned)cdiv(ldo, TT), (unsigned)cdiv(cols, TT));
  if (in_f32)
    hipLaunchKernelGGL((convert_bf16_kernel<float, 0>), grid, dim3(256), 0, s, (const float*)in,
                       ldi, rows, cols, out, ldo);
  else
    hipLaunchKernelGGL((convert_bf16_kernel<double, 0>), grid, dim3(256), 0, s,
                       (const double*)in, ldi, rows, cols, out, ldo);
  return hipGetLastError();
}

}  // namespace rsvd
