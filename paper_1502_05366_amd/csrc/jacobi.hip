// The small SVD of Alg. 5 (RSVD Version II): svd(R_hat) of the l x l factor
// from the QR of B^T, by one-sided (Hestenes) Jacobi rotations in FP64.
//
// Columns a_p, a_q of W (initially R_hat) are rotated until every pair is
// orthogonal to within tol = l * eps relative to their norms:
//   alpha = a_p.a_p, beta = a_q.a_q, gamma = a_p.a_q,
//   zeta = (beta - alpha) / (2 gamma), t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
//   c = 1 / sqrt(1 + t^2), s = c t,
//   a_p <- c a_p - s a_q, a_q <- s a_p + c a_q  (and the same on V = I).
// On exit R_hat V = W with orthogonal columns: sigma_j = ||w_j||,
// Uh_j = w_j / sigma_j, Vh_j = v_j, so R_hat = Uh diag(sigma) Vh^T.
//
// Pairs are scheduled in round-robin rounds of disjoint pairs (circle
// method).  Small factors (l <= 64) run in one workgroup with W and V in LDS,
// one pair per group of 16 lanes (16-lane sums); larger ones run as a block
// Jacobi over several workgroups (below).
// Output: the k largest sigma in descending order (stable for ties) and the
// matching columns of Uh and Vh.
#include <algorithm>

#include "common.h"
#include "internal.h"
#include "jacobi_dev.h"

namespace rsvd {
namespace {

constexpr int JNT = 1024;
// One workgroup up to l = 64 (2 * 64 * 64 * 8 B = 64 KB of LDS); larger
// factors take the block iteration.
constexpr int LDS_MAX_L = 64;

// l <= LDS_MAX_L: the whole iteration in one workgroup, W and V in LDS.
__global__ __launch_bounds__(JNT) void jacobi_lds_kernel(const double* __restrict__ Rh, int64_t ldr,
                                                         int l, int k, double* __restrict__ S,
                                                         double* __restrict__ Uh, int64_t lduh,
                                                         double* __restrict__ Vh, int64_t ldvh,
                                                         int max_sweeps, double tol, int32_t* info) {
  extern __shared__ double smem[];
  __shared__ int rotated;
  __shared__ double sig[256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t ld = l;
  double* W = smem;
  double* V = smem + (int64_t)l * l;
  for (int j = wave; j < l; j += JNT / 64)
    for (int i = lane; i < l; i += 64) {
      W[j * ld + i] = Rh[(int64_t)i * ldr + j];
      V[j * ld + i] = (i == j) ? 1.0 : 0.0;
    }
  __syncthreads();
  const int N = l + (l & 1);
  int sweep = 0;
  bool converged = (l < 2);
  while (!converged && sweep < max_sweeps) {
    ++sweep;
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < N - 1; ++r) {
      // one pair per group of 16 lanes (64 groups: every pair of a round at once)
      for (int pi = tid >> 4; pi < N / 2; pi += JNT / 16) {
        int a = rr_player(pi, r, N), b = rr_player(N - 1 - pi, r, N);
        if (a >= l || b >= l) continue;
        if (a > b) { const int t = a; a = b; b = t; }
        if (rotate_pair16<LDS_MAX_L / 16>(W + a * ld, W + b * ld, V + a * ld, V + b * ld, l,
                                          tid & 15, tol) &&
            (tid & 15) == 0)
          rotated = 1;
      }
      __syncthreads();
    }
    converged = (rotated == 0);
    __syncthreads();
  }
  if (!converged && tid == 0) info_or(info, INFO_JACOBI_CAP);
  jacobi_finish<JNT>(W, V, ld, l, k, sig, S, Uh, lduh, Vh, ldvh);
}

// ---- block one-sided Jacobi over several workgroups (l > LDS_MAX_L) -------
//
// The l columns are cut into blocks of BS; blocks are paired by the same
// round-robin schedule as columns, and each of the NB/2 workgroups of one
// launch takes one block pair per round: it rotates every cross pair (x from
// the first block, y from the second; in round 0 also the pairs inside each
// block) and writes the 2*BS columns of W and V back.  Between rounds the
// workgroups exchange progress through per-workgroup tags (agent-scope
// release / acquire); a sweep over all rounds visits every column pair
// exactly once.  The iteration stops after the first sweep without a
// rotation.
constexpr int BS = 16;

struct JacArgs {
  double* W; double* V; int64_t ld;
  int l, nbp, G, max_sweeps;
  double tol;
  uint32_t* tags;       // [G] rounds completed by each workgroup (FLAG_STRIDE apart)
  uint32_t* rot;        // [2][G] rotation flag of the current / previous sweep
  uint32_t* abort_flag;
  uint32_t wait_bias;   // 0; 1 in the forced give-up test mode (waits for a value never posted)
  uint32_t spin_cap;
  int32_t* info;
  int32_t* sweeps_out;
};

// spin until workgroup v has completed `target` rounds (bounded: past the cap
// the wait gives up, raises the abort flag and INFO_BARRIER)
__device__ void jac_wait_tag(const JacArgs& a, int v, uint32_t target) {
  uint32_t spins = 0;
  while (ld_agent_u32(a.tags + v * FLAG_STRIDE) < target + a.wait_bias) {
    if ((++spins & 63) == 0) {
      if (ld_agent_u32(a.abort_flag)) break;
      if (spins > a.spin_cap) {
        st_agent_u32(a.abort_flag, 1u);
        info_or(a.info, INFO_BARRIER);
        break;
      }
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

__device__ void jac_wait_all(const JacArgs& a, uint32_t target) {
  const int tid = threadIdx.x;
  if (tid < a.G) jac_wait_tag(a, tid, target);
  __syncthreads();
}

// Before round r + 1 of a sweep, workgroup w needs only its two blocks of
// that round, written back by the workgroups that held them in round r: it
// waits for those (so the workgroups drift apart by a few rounds instead of
// all waiting for the slowest one every round).  A block's owners follow
// each other round by round, so every block is read after the previous
// owner's writes and written after its reads.
__device__ void jac_wait_owners(const JacArgs& a, uint32_t target, int r, int w) {
  const int tid = threadIdx.x;
  if (tid < a.G) {
    const int nb = a.nbp;
    const int b1 = rr_player(w, r + 1, nb), b2 = rr_player(nb - 1 - w, r + 1, nb);
    const int p1 = rr_player(tid, r, nb), p2 = rr_player(nb - 1 - tid, r, nb);
    if (p1 == b1 || p1 == b2 || p2 == b1 || p2 == b2) jac_wait_tag(a, tid, target);
  }
  __syncthreads();
}

// The block kernel takes the rotation parameters from the Gram matrix of its
// block pair instead of from the columns.  At the start of a round the
// workgroup forms G = X^T X (X = W(:, pair blocks), 2BS columns) on the matrix
// cores from fresh columns; each step of the round then reads alpha, beta,
// gamma of its BS disjoint pairs from G, updates the touched entries of G by
// the same rotations applied from both sides (on a rotated pair the diagonal
// becomes alpha - t gamma, beta + t gamma and the pair entry 0), and
// accumulates the rotations in a 2BS x 2BS orthogonal J.  The round ends with
// W(:, pair) <- W(:, pair) J and V(:, pair) <- V(:, pair) J on the matrix
// cores.  The pairs, their order and the rotation formulas are those of the
// column iteration; only where alpha, beta, gamma come from differs, and the
// test of a pair that has not moved in the round reads fresh inner products,
// so the final sweep (no rotation) checks every pair on the columns
// themselves.  A step touches 2BS x 2BS entries of G and J instead of the
// 2 l entries of two columns, and the l-long work moves to the products.
//
// W and V are held padded, ROWS x (nbp BS) with ROWS = 16 JRPL rows (zero
// beyond l rows and l columns), so that every tile access is in range.
// Lane layout (g = lane / 16, c = lane % 16): row tile t of wave w covers
// rows 16 (w RTW + t) + c; the lane holds W(row, col 4 kk + g), kk = 0..7, of
// the block pair, the B operand of W_new^T = J^T W^T.  The Gram product needs
// the rows along the reduction instead: each wave passes its tiles through a
// small LDS area of its own and reads them back as W(16 t + 4 k + g, col c),
// so W is read from memory once, coalesced, for both products.
constexpr int JJ = 2 * BS;   // columns of a block pair
constexpr int GLD = JJ + 1;  // LDS stride of G and J
constexpr int TLD = 17;      // LDS stride of a wave's transposition area
constexpr int JACOBI_MAX_L = 576;
// JRPL: 16-row tiles of a column; NW: waves (2 per SIMD).  The products
// keep their operands in registers: W's are loaded at the start of the round
// and kept through the steps; V's are loaded with them at JRPL = 16
// (l <= 256) and after W's product at JRPL = 40 (l <= 576, register budget).
template <int JRPL, int NW> struct JacDims {
  static constexpr int NT = 64 * NW;
  static constexpr int ROWS = 16 * JRPL;
  static constexpr int RTW = JRPL / NW;        // row tiles per wave
  static constexpr bool PRE = JRPL <= 16;      // V operands loaded at the start
  static_assert(JRPL % NW == 0, "row tiles must split evenly over the waves");
  static constexpr size_t LDS =
      ((size_t)NW * 3 * 256 + (size_t)NW * JJ * TLD + 3 * (size_t)JJ * GLD) * sizeof(double);
};

// Rotation of jacobi_rotation with t = s / c returned as well.
__device__ __forceinline__ bool jacobi_rotation_t(double al, double be, double ga, double tol,
                                                  double& cs, double& sn, double& tt) {
  if (!(ga * ga > (tol * tol) * (al * be))) return false;
  const double zeta = (be - al) * (0.5 * rcp_nr1(ga));
  const double az = fabs(zeta);
  double t;
  if (az < 1e150) {
    const double z2 = fma(zeta, zeta, 1.0);
    t = rcp_nr1(az + z2 * rsq_nr(z2));
  } else {
    t = 0.5 * rcp_nr1(az);
  }
  t = zeta >= 0.0 ? t : -t;
  cs = rsq_nr(fma(t, t, 1.0));
  sn = cs * t;
  tt = t;
  return true;
}

// Columns (p, q) of pair P in step t: round 0 first visits the pairs inside
// each block (BS - 1 round-robin steps, both blocks at once), then every
// round visits the cross pairs (x_P, y_{(P + t) mod BS}), t = 0 .. BS - 1.
__device__ __forceinline__ void pair_cols(bool inner, int t, int P, int& p, int& q) {
  if (inner) {
    const int half = P / (BS / 2), pi = P % (BS / 2);
    p = rr_player(pi, t, BS);
    q = rr_player(BS - 1 - pi, t, BS);
    if (p > q) { const int x = p; p = q; q = x; }
    p += half * BS;
    q += half * BS;
  } else {
    p = P;
    q = BS + (P + t) % BS;
  }
}

template <int JRPL, int NW>
__global__ __launch_bounds__(64 * NW) void jacobi_block_kernel(JacArgs a) {
  using D = JacDims<JRPL, NW>;
  constexpr int NT = D::NT, RTW = D::RTW;
  extern __shared__ double smem[];
  __shared__ int rotated, rround;
  __shared__ int ptab[(BS - 1) * BS];       // inner steps: p | q << 8 of pair P in step t
  double* Gp = smem;                        // [NW][3][16 x 16] partial Gram tiles
  double* Ts = Gp + NW * 3 * 256;           // [NW][JJ][TLD] transposition areas
  double* G = Ts + NW * JJ * TLD;           // [2][JJ][GLD], G(i, j) at i GLD + j, two copies
  double* Jm = G + 2 * JJ * GLD;            // [JJ][GLD], J(c, j) at c GLD + j
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int w = blockIdx.x;
  const int64_t ld = a.ld;
  uint32_t done = 0;
  int sweep = 0;
  bool converged = false;
  if (tid == 0) rotated = 0;
  for (int e = tid; e < (BS - 1) * BS; e += NT) {
    int p, q;
    pair_cols(true, e / BS, e % BS, p, q);
    ptab[e] = p | (q << 8);
  }
  while (!converged && sweep < a.max_sweeps) {
    for (int r = 0; r < a.nbp - 1; ++r) {
      const int bi = rr_player(w, r, a.nbp), bj = rr_player(a.nbp - 1 - w, r, a.nbp);
      auto gcol_of = [&](int c) { return (c < BS) ? bi * BS + c : bj * BS + (c - BS); };
      // the block pair's rows of W (and at JRPL = 16 of V), coalesced
      double wu[RTW][8], vu[RTW][8];
      // the lane's rows of column c start at M + col_off(c); the tiles of a
      // wave follow each other (16 rows apart)
      const int64_t row0 = 16 * wave * RTW + li;
      auto col_off = [&](int c) { return (int64_t)gcol_of(c) * ld + row0; };
      auto load_upd = [&](const double* M, double (&u)[RTW][8]) {
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
          const double* pc = M + col_off(4 * kk + lg);
#pragma unroll
          for (int t = 0; t < RTW; ++t) u[t][kk] = ld_agent(pc + 16 * t);
        }
      };
      load_upd(a.W, wu);
      if (D::PRE) load_upd(a.V, vu);
      for (int e = tid; e < JJ * JJ; e += NT)
        Jm[(e / JJ) * GLD + e % JJ] = (e / JJ == e % JJ) ? 1.0 : 0.0;
      if (tid == 0) rround = 0;
      // G = X^T X: every wave sums its rows, the partial tiles are added in
      // wave order
      {
        double* T = Ts + wave * JJ * TLD;
        d4 axx = Mfma<double>::zero(), axy = Mfma<double>::zero(), ayy = Mfma<double>::zero();
        // (the area is the wave's own and one wave's LDS accesses complete in
        // order: a wave barrier keeps the compiler from moving them)
#pragma unroll
        for (int t = 0; t < RTW; ++t) {
#pragma unroll
          for (int kk = 0; kk < 8; ++kk) T[(4 * kk + lg) * TLD + li] = wu[t][kk];
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const double x = T[li * TLD + 4 * k + lg], y = T[(BS + li) * TLD + 4 * k + lg];
            axx = Mfma<double>::mma(x, x, axx);
            axy = Mfma<double>::mma(x, y, axy);
            ayy = Mfma<double>::mma(y, y, ayy);
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int e = drow(lg, v) * 16 + li;
          Gp[(wave * 3 + 0) * 256 + e] = axx[v];
          Gp[(wave * 3 + 1) * 256 + e] = axy[v];
          Gp[(wave * 3 + 2) * 256 + e] = ayy[v];
        }
      }
      __syncthreads();
      for (int e = tid; e < 256; e += NT) {
        // partials read CH waves at a time, added in wave order
        constexpr int CH = NW % 4 == 0 ? 4 : 2;
        static_assert(NW % CH == 0, "");
        double sxx = 0.0, sxy = 0.0, syy = 0.0;
#pragma unroll
        for (int v0 = 0; v0 < NW; v0 += CH) {
          double px[CH], py[CH], pz[CH];
#pragma unroll
          for (int v = 0; v < CH; ++v) {
            px[v] = Gp[((v0 + v) * 3 + 0) * 256 + e];
            py[v] = Gp[((v0 + v) * 3 + 1) * 256 + e];
            pz[v] = Gp[((v0 + v) * 3 + 2) * 256 + e];
          }
#pragma unroll
          for (int v = 0; v < CH; ++v) {
            sxx += px[v];
            sxy += py[v];
            syy += pz[v];
          }
        }
        const int i = e / 16, j = e % 16;
        G[i * GLD + j] = sxx;
        G[(BS + i) * GLD + BS + j] = syy;
        G[i * GLD + BS + j] = sxy;
        G[(BS + j) * GLD + i] = sxy;
      }
      __syncthreads();
      // the steps of the round on G and J.  Thread (I, K) of the first BS^2
      // (I = tid / BS, K = lane % BS) owns the 2 x 2 blocks of G and of J on
      // the rows of pair I and the columns of pair K (the pairs of a step
      // partition the 2BS columns, so the blocks partition G and J).  Every
      // lane computes the rotation of its pair K and takes that of pair I
      // from a lane of its own row of 16 whose K is I, so one barrier per
      // step suffices: G is read from one copy and written to the other,
      // each J block is read and written by its owner only.
      // A round in which no pair of the block pair passes the rotation test
      // on the fresh G rotates nothing (G never changes), so its steps are
      // skipped: the same decisions as running them.  Every sweep's last
      // round set is such a check.
      int any_pair = 0;
      for (int e = tid; e < BS * BS; e += NT) {
        const double tol2 = a.tol * a.tol;
        const int i = e / BS, j = e % BS;
        const double gc = G[i * GLD + BS + j];
        int need = gc * gc > tol2 * (G[i * GLD + i] * G[(BS + j) * GLD + BS + j]);
        if (r == 0 && i < j) {
          const double gx = G[i * GLD + j], gy = G[(BS + i) * GLD + BS + j];
          need |= gx * gx > tol2 * (G[i * GLD + i] * G[j * GLD + j]);
          need |= gy * gy > tol2 * (G[(BS + i) * GLD + BS + i] * G[(BS + j) * GLD + BS + j]);
        }
        any_pair |= need;
      }
      const int ninner = (r == 0) ? BS - 1 : 0;
      const int I = tid / BS, K = tid % BS;
      const int srcI = (lane & ~(BS - 1)) | I;
      // one step on the pairs (pI, qI) of thread row I and (pK, qK) of
      // thread column K, G read from copy st & 1
      auto step = [&](int st, int pI, int qI, int pK, int qK) {
        const double* Gc = G + (st & 1) * JJ * GLD;
        double* Gn = G + ((st + 1) & 1) * JJ * GLD;
        const double aK = Gc[pK * GLD + pK], bK = Gc[qK * GLD + qK], gK = Gc[pK * GLD + qK];
        const double gpp = Gc[pI * GLD + pK], gpq = Gc[pI * GLD + qK];
        const double gqp = Gc[qI * GLD + pK], gqq = Gc[qI * GLD + qK];
        const double jpp = Jm[pI * GLD + pK], jpq = Jm[pI * GLD + qK];
        const double jqp = Jm[qI * GLD + pK], jqq = Jm[qI * GLD + qK];
        double cK = 1.0, sK = 0.0, tK = 0.0;
        const bool rK = jacobi_rotation_t(aK, bK, gK, a.tol, cK, sK, tK);
        if (!rK) { cK = 1.0; sK = 0.0; }
        // (1, 0) for a pair that does not turn: the products below are then
        // exact copies
        const double cI = __shfl(cK, srcI, 64), sI = __shfl(sK, srcI, 64);
        if (I == K) {
          if (rK) { rotated = 1; rround = 1; }
          Gn[pK * GLD + pK] = rK ? aK - tK * gK : aK;
          Gn[qK * GLD + qK] = rK ? bK + tK * gK : bK;
          Gn[pK * GLD + qK] = rK ? 0.0 : gK;
          Gn[qK * GLD + pK] = rK ? 0.0 : gK;
        } else {
          // rows by the rotation of pair I, then columns by that of pair K
          const double rpp = cI * gpp - sI * gqp, rqp = sI * gpp + cI * gqp;
          const double rpq = cI * gpq - sI * gqq, rqq = sI * gpq + cI * gqq;
          Gn[pI * GLD + pK] = cK * rpp - sK * rpq;
          Gn[pI * GLD + qK] = sK * rpp + cK * rpq;
          Gn[qI * GLD + pK] = cK * rqp - sK * rqq;
          Gn[qI * GLD + qK] = sK * rqp + cK * rqq;
        }
        // J <- J J_t on the block: its columns pK, qK turn by pair K
        if (rK) {
          Jm[pI * GLD + pK] = cK * jpp - sK * jpq;
          Jm[pI * GLD + qK] = sK * jpp + cK * jpq;
          Jm[qI * GLD + pK] = cK * jqp - sK * jqq;
          Jm[qI * GLD + qK] = sK * jqp + cK * jqq;
        }
      };
      if (__syncthreads_or(any_pair)) {
#pragma unroll 1
        for (int st = 0; st < ninner + BS; ++st) {
          if (tid < BS * BS) {
            int pI, qI, pK, qK;
            if (st < ninner) {
              const int eI = ptab[st * BS + I], eK = ptab[st * BS + K];
              pI = eI & 0xFF; qI = eI >> 8; pK = eK & 0xFF; qK = eK >> 8;
            } else {
              const int t = st - ninner;
              pI = I; qI = BS + ((I + t) & (BS - 1));
              pK = K; qK = BS + ((K + t) & (BS - 1));
            }
            step(st, pI, qI, pK, qK);
          }
          __syncthreads();
        }
      }
      // W(:, pair) <- W(:, pair) J and V(:, pair) <- V(:, pair) J as
      // W_new^T = J^T W^T (A operand J^T from LDS, B operand the row tiles);
      // lane (c, g) receives rows r0 + c of columns 16 jh + 4 v + g
      if (rround) {
        double ja[2][8];
#pragma unroll
        for (int jh = 0; jh < 2; ++jh)
#pragma unroll
          for (int kk = 0; kk < 8; ++kk) ja[jh][kk] = Jm[(4 * kk + lg) * GLD + 16 * jh + li];
        // TG row tiles at a time: 2 TG independent accumulator chains
        constexpr int TG = RTW <= 2 ? RTW : 1;
        auto apply = [&](const double (&u)[RTW][8], double* M) {
#pragma unroll
          for (int t0 = 0; t0 < RTW; t0 += TG) {
            d4 acc[TG][2];
#pragma unroll
            for (int t = 0; t < TG; ++t)
#pragma unroll
              for (int jh = 0; jh < 2; ++jh) acc[t][jh] = Mfma<double>::zero();
#pragma unroll
            for (int kk = 0; kk < 8; ++kk)
#pragma unroll
              for (int t = 0; t < TG; ++t)
#pragma unroll
                for (int jh = 0; jh < 2; ++jh)
                  acc[t][jh] = Mfma<double>::mma(ja[jh][kk], u[t0 + t][kk], acc[t][jh]);
#pragma unroll
            for (int jh = 0; jh < 2; ++jh)
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                double* pc = M + col_off(16 * jh + drow(lg, v)) + 16 * t0;
#pragma unroll
                for (int t = 0; t < TG; ++t) st_agent(pc + 16 * t, acc[t][jh][v]);
              }
          }
        };
        apply(wu, a.W);
        if (!D::PRE) load_upd(a.V, vu);
        apply(vu, a.V);
      }
      const bool last = (r == a.nbp - 2);
      if (last && tid == 0)
        st_agent_u32(a.rot + ((sweep & 1) * a.G + w) * FLAG_STRIDE, (uint32_t)rotated);
      stores_done();
      __syncthreads();
      ++done;
      if (tid == 0) st_agent_u32(a.tags + w * FLAG_STRIDE, done);
      // the sweep's end needs every workgroup's rotation flag
      if (last) jac_wait_all(a, done);
      else jac_wait_owners(a, done, r, w);
    }
    // every workgroup reads the same flags, so all take the same decision
    uint32_t any = 0;
    for (int v = 0; v < a.G; ++v)
      any |= ld_agent_u32(a.rot + ((sweep & 1) * a.G + v) * FLAG_STRIDE);
    ++sweep;
    converged = (any == 0);
    __syncthreads();
    if (tid == 0) rotated = 0;
    __syncthreads();
  }
  if (w == 0 && tid == 0) {
    if (!converged) info_or(a.info, INFO_JACOBI_CAP);
    if (a.sweeps_out) *a.sweeps_out = sweep;
  }
}

// W = Rh (column j of W is row j of the row-major Rh), V = I, both padded
// with zeros to ld rows and ncols columns
__global__ __launch_bounds__(256) void jacobi_init_kernel(const double* __restrict__ Rh,
                                                          int64_t ldr, int l, int ncols,
                                                          double* __restrict__ W,
                                                          double* __restrict__ V, int64_t ld,
                                                          uint32_t* ctl, int nctl) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < nctl) ctl[e] = 0;
  if (e >= ld * ncols) return;
  const int j = (int)(e / ld), i = (int)(e - (int64_t)j * ld);
  const bool in = i < l && j < l;
  W[e] = in ? Rh[(int64_t)i * ldr + j] : 0.0;
  V[e] = (in && i == j) ? 1.0 : 0.0;
}

// The output of the block iteration spread over the chip (one wave per
// column; the single-workgroup jacobi_finish took ~0.6 ms at l = 576, its
// row-strided writes of Uh and Vh issued from one compute unit).  First
// sigma_j = ||w_j|| into sig, then each column's rank among the sigma
// (descending, ties by index) and, for the k largest, S, Uh and Vh.  The
// arithmetic is jacobi_finish's.
constexpr int JOW = 8;   // waves (columns) per workgroup

__global__ __launch_bounds__(64 * JOW) void jacobi_sig_kernel(const double* __restrict__ W,
                                                              int64_t ld, int l,
                                                              double* __restrict__ sig) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * JOW + (threadIdx.x >> 6);
  if (j >= l) return;   // (a whole wave)
  double s2 = 0.0;
  for (int i = lane; i < l; i += 64) {
    const double x = W[j * ld + i];
    s2 += x * x;
  }
  s2 = wave_sum(s2);
  if (lane == 0) sig[j] = sqrt(s2);
}

__global__ __launch_bounds__(64 * JOW) void jacobi_out_kernel(
    const double* __restrict__ W, const double* __restrict__ V, int64_t ld, int l, int k,
    const double* __restrict__ sig, double* __restrict__ S, double* __restrict__ Uh, int64_t lduh,
    double* __restrict__ Vh, int64_t ldvh) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * JOW + (threadIdx.x >> 6);
  if (j >= l) return;   // (a whole wave)
  const double sj = sig[j];
  int rank = 0;
  for (int i = lane; i < l; i += 64) {
    const double si = sig[i];
    rank += (si > sj || (si == sj && i < j)) ? 1 : 0;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) rank += __shfl_xor(rank, off, 64);
  if (rank >= k) return;
  if (lane == 0) S[rank] = sj;
  const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
  for (int i = lane; i < l; i += 64) {
    Uh[(int64_t)i * lduh + rank] = W[j * ld + i] * inv;
    Vh[(int64_t)i * ldvh + rank] = V[j * ld + i];
  }
}

}  // namespace

// control words of the block iteration: tags [64], rotation flags [2][64],
// the abort flag (FLAG_STRIDE apart; at most 64 workgroups)
constexpr int JCTL = 200;

// padded shape of W and V in the block iteration
static int jac_rows(int l) { return l <= 256 ? 16 * 16 : 16 * 40; }
static int jac_cols(int l) {
  const int nb = (int)cdiv(l, BS);
  return (nb + (nb & 1)) * BS;
}

size_t jacobi_work_bytes(int l) {
  // W, V (padded), the control words of the block iteration and the l sigma
  return 2 * (size_t)jac_rows(l) * jac_cols(l) * sizeof(double) +
         JCTL * FLAG_STRIDE * sizeof(uint32_t) + (size_t)l * sizeof(double) + 256;
}

template <int JRPL, int NW>
hipError_t launch_block(JacArgs& a, hipStream_t s) {
  const size_t shm = JacDims<JRPL, NW>::LDS;
  hipError_t e = hipFuncSetAttribute((const void*)jacobi_block_kernel<JRPL, NW>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  void* args[] = {&a};
  return hipLaunchKernel((const void*)jacobi_block_kernel<JRPL, NW>, dim3(a.G),
                         dim3(JacDims<JRPL, NW>::NT), args, shm, s);
}

hipError_t launch_jacobi(const double* Rh, int64_t ldr, int l, int k, double* work, double* S,
                         double* Uh, int64_t lduh, double* Vh, int64_t ldvh, int max_sweeps,
                         int32_t* info, int32_t* sweeps_out, bool giveup_test, hipStream_t s) {
  if (l > JACOBI_MAX_L) return hipErrorInvalidValue;
  const double tol = (double)l * 2.220446049250313e-16;
  if (l <= LDS_MAX_L) {
    const size_t shm = 2 * (size_t)l * l * sizeof(double);
    if (shm > 65536) {
      const hipError_t e = hipFuncSetAttribute((const void*)jacobi_lds_kernel,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)shm);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(jacobi_lds_kernel, dim3(1), dim3(JNT), shm, s, Rh, ldr, l, k, S, Uh, lduh,
                       Vh, ldvh, max_sweeps, tol, info);
    return hipGetLastError();
  }
  const int64_t ld = jac_rows(l);
  const int ncols = jac_cols(l);
  double* W = work;
  double* V = work + (size_t)ld * ncols;
  uint32_t* ctl = reinterpret_cast<uint32_t*>(V + (size_t)ld * ncols);
  const int nbp = ncols / BS;
  JacArgs a;
  a.W = W; a.V = V; a.ld = ld; a.l = l; a.nbp = nbp; a.G = nbp / 2; a.max_sweeps = max_sweeps;
  a.tol = tol;
  a.tags = ctl;                                   // 64 flags
  a.rot = ctl + 64 * FLAG_STRIDE;                 // 2 x 64 flags
  a.abort_flag = ctl + 192 * FLAG_STRIDE;
  a.wait_bias = giveup_test ? 1u : 0u;
  a.spin_cap = giveup_test ? (1u << 10) : (1u << 22);
  a.info = info;
  a.sweeps_out = sweeps_out;
  // one thread per element of W and per control word
  const int64_t ninit = std::max<int64_t>(ld * ncols, (int64_t)JCTL * FLAG_STRIDE);
  hipLaunchKernelGGL(jacobi_init_kernel, dim3((unsigned)cdiv(ninit, 256)), dim3(256), 0, s, Rh,
                     ldr, l, ncols, W, V, ld, ctl, JCTL * FLAG_STRIDE);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = (l <= 256) ? launch_block<16, 8>(a, s) : launch_block<40, 8>(a, s);
  if (e != hipSuccess) return e;
  double* sig = reinterpret_cast<double*>(ctl + JCTL * FLAG_STRIDE);
  const unsigned nwg = (unsigned)cdiv(l, JOW);
  hipLaunchKernelGGL(jacobi_sig_kernel, dim3(nwg), dim3(64 * JOW), 0, s, W, ld, l, sig);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(jacobi_out_kernel, dim3(nwg), dim3(64 * JOW), 0, s, W, V, ld, l, k, sig, S,
                     Uh, lduh, Vh, ldvh);
  return hipGetLastError();
}

}  // namespace rsvd
