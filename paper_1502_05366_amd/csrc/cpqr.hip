// k steps of the column-pivoted QR (Sec. 2.3) of the short, wide B = Q^T A
// (l x n), which selects the skeleton columns of the ID computed from B
// (Sec. 3.5, last part) and, applied to C^T, the rows of the CUR (Sec. 2.5,
// Sec. 3.6).  Then T = S11^{-1} S12 (Sec. 2.4) by back substitution.
//
// One launch of G <= (compute units) workgroups that wait for each other with
// bounded spins (below); workgroup g keeps columns
// [g*cs, (g+1)*cs) of B in LDS for the whole factorization.  Step s:
//   1. each workgroup finds its unchosen column with the largest residual
//      norm ||B(s:, j)|| (FP64, lowest column index on ties) and publishes
//      the norm, the index and rows s.. of that column;
//   2. grid barrier;
//   3. every workgroup reads the G candidates, picks the global pivot the
//      same way, builds the Householder reflector H = I - beta v v^T of the
//      pivot column (v = x + sign(x_0)||x|| e_1, beta = 2 / v^T v) from the
//      published values, and applies it to rows s.. of its unchosen columns;
//   4. residual norms are recomputed exactly over rows s+1.. .
// Chosen columns keep their place; the remaining columns are listed in
// ascending index order.  The rank tolerance is max(r, c) * eps * ||B||_F.
#include "common.h"
#include "internal.h"

namespace rsvd {
namespace {

constexpr int CQ_NT = 512;
constexpr double DEPS = 2.220446049250313e-16;

struct CpqrArgs {
  const void* Bt; int64_t ldb;     // column j of B at Bt + j * ldb
  int r; int64_t c; int k;
  int G; int64_t cs; int rp;
  double* slots;                   // [2][G][slot_len]: norm^2, index, ||.||_F^2 part, column
  int64_t slot_len;
  uint32_t* tags;                  // [2][G] (FLAG_STRIDE apart) step + 1 of the last post
  uint32_t* abort_flag;            // set when a wait exceeds its spin cap
  uint32_t wait_bias;              // 0; 1 only in the forced give-up test mode
  uint32_t spin_cap;
  int64_t* J;                      // [c]
  double* S11t;                    // column t = top k rows of pivot column t (ld = lds)
  double* S12t;                    // column rho = top k rows of residual column rho
  int64_t lds;
  double* pivn;                    // [k] pivot norms
  int32_t* info;                   // [2]
};

// Exchange between the workgroups of one step: every workgroup posts its
// candidate into its own slot and then raises the slot's tag to step + 1
// (release); readers wait for each tag (acquire) and read the slot with
// agent-scope loads.  No counter is shared, so no atomic is contended.  A wait
// longer than its spin cap raises the abort flag and INFO_BARRIER; all later
// waits then return at once, so the kernel always runs to its end (its
// results are then flagged invalid).  In the forced give-up test mode the
// host sets wait_bias = 1, so every wait is for a value that no workgroup
// posts, and a small spin cap.
constexpr uint32_t SPIN_CAP = 1u << 22;
constexpr uint32_t SPIN_CAP_TEST = 1u << 10;

// Called by every thread of the workgroup after the slot data has been stored
// with agent-scope stores: each wave waits for its stores, then thread 0
// raises the tag.
__device__ __forceinline__ void post_tag(uint32_t* tag, uint32_t value) {
  stores_done();
  __syncthreads();
  if (threadIdx.x == 0) st_agent_u32(tag, value);
}

// Relaxed polling; the slot data is then read with agent-scope loads.
__device__ __forceinline__ void wait_tag(const uint32_t* tag, uint32_t value, uint32_t* abort_flag,
                                         uint32_t spin_cap, int32_t* info) {
  uint32_t spins = 0;
  while (ld_agent_u32(tag) != value) {
    if ((++spins & 63) == 0) {
      if (ld_agent_u32(abort_flag) != 0) break;
      if (spins > spin_cap) {
        st_agent_u32(abort_flag, 1u);
        info_or(info, INFO_BARRIER);
        break;
      }
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// argmax of (val, idx): larger val wins, lower idx on equal val
__device__ __forceinline__ bool better(double v1, int64_t i1, double v2, int64_t i2) {
  return v1 > v2 || (v1 == v2 && i1 < i2);
}

// Selection key of a squared residual norm: NaN (from non-finite entries of
// B) maps to -0.5, below every finite norm and above the empty-candidate
// value -1, so such columns are still chosen, last and lowest index first:
// the k pivots are always k distinct columns and the index bookkeeping
// below stays a permutation.  The step then reports INFO_NONFINITE.
__device__ __forceinline__ double sel_key(double s2) { return s2 == s2 ? s2 : -0.5; }

constexpr int CQ_NW = CQ_NT / 64;
// A column is handled by one row of 16 lanes, RPL rows per lane (rows
// rl + 16 e, e < RPL); the plan takes the smallest instantiated RPL with
// 16 RPL >= r and a column stride rp >= 16 RPL, so every row a lane touches is
// in its column (rows r .. 16 RPL - 1 hold zeros) and no access needs a
// per-lane test.
constexpr int CQ_RPLS[] = {2, 4, 8, 12, 13, 14, 16};

// sum over the 16 lanes of a row, returned in each of them
__device__ __forceinline__ double row16_sum(double x) {
  x += dpp_d<0xB1>(x);
  x += dpp_d<0x4E>(x);
  x += dpp_d<0x141>(x);
  x += dpp_d<0x140>(x);
  return x;
}

template <typename TB, int RPL>
__global__ __launch_bounds__(CQ_NT) void cpqr_kernel(CpqrArgs a) {
  extern __shared__ double smem[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cg = lane >> 4, rl = lane & 15;
  const int g = blockIdx.x;
  const int64_t j0 = (int64_t)g * a.cs;
  int64_t ncols = a.c - j0;
  if (ncols > a.cs) ncols = a.cs;
  if (ncols < 0) ncols = 0;
  const int r = a.r, rp = a.rp;

  double* slab = smem;                         // [cs][rp]
  double* nrm = slab + a.cs * rp;              // [cs]
  double* v = nrm + a.cs;                      // [rp]
  int* chosen_at = (int*)(v + rp);             // [cs] step at which chosen, -1 if not
  int64_t* piv = (int64_t*)(chosen_at + a.cs + (a.cs & 1));  // [k]
  __shared__ double redv[2][CQ_NW];
  __shared__ int64_t redi[2][CQ_NW];
  __shared__ int redg[2][CQ_NW];
  __shared__ double redf[CQ_NW];
  __shared__ double sh_beta, sh_alpha, sh_gv;
  __shared__ int64_t sh_gi;
  __shared__ int sh_gg;

  const TB* Bt = static_cast<const TB*>(a.Bt);
  for (int64_t e = tid; e < ncols * rp; e += CQ_NT) {
    const int64_t jj = e / rp;
    const int i = (int)(e - jj * rp);
    slab[e] = (i < r) ? (double)Bt[(j0 + jj) * a.ldb + i] : 0.0;
  }
  // the reflector's rows >= r stay zero (the steps write rows s .. r-1)
  for (int i = tid; i < rp; i += CQ_NT) v[i] = 0.0;
  __syncthreads();
  // initial norms, the workgroup's share of ||B||_F^2 and each lane's best
  // column (largest norm, lowest index on ties).  A column is handled by one
  // row of 16 lanes (rows rl + 16 e of the column), four columns per wave.
  double fpart = 0.0;
  double bv = -1.0;
  int64_t bi = INT64_MAX;
  for (int64_t jb = 0; jb < ncols; jb += CQ_NW * 4) {
    const int64_t jj = jb + wave * 4 + cg;
    const bool act = jj < ncols;
    const double* col = slab + (act ? jj : 0) * rp;
    double s2 = 0.0;
#pragma unroll
    for (int e = 0; e < RPL; ++e) {
      const double x = col[rl + 16 * e];
      s2 = fma(x, x, s2);
    }
    s2 = row16_sum(s2);
    if (act) {
      if (rl == 0) {
        nrm[jj] = s2; chosen_at[jj] = -1; fpart += s2;
        if (!(s2 <= 1.7976931348623157e308)) info_or(a.info, INFO_NONFINITE);   // NaN or Inf in B
      }
      if (better(sel_key(s2), j0 + jj, bv, bi)) { bv = sel_key(s2); bi = j0 + jj; }
    }
  }
  fpart = wave_allsum(fpart);
  if (lane == 0) redf[wave] = fpart;
  double tol = 0.0;
  int frank = a.k;

  for (int s = 0; s < a.k; ++s) {
    const int par = s & 1;
    // 1. the workgroup's candidate (lanes' bests, fixed order), posted
#pragma unroll
    for (int off = 16; off < 64; off <<= 1) {
      const double ov = __shfl_xor(bv, off, 64);
      const int64_t oi = __shfl_xor(bi, off, 64);
      if (better(ov, oi, bv, bi)) { bv = ov; bi = oi; }
    }
    if (lane == 0) { redv[par][wave] = bv; redi[par][wave] = bi; }
    __syncthreads();
    double* myslot = a.slots + ((int64_t)par * a.G + g) * a.slot_len;
    double cv = redv[par][0];
    int64_t ci = redi[par][0];
    for (int w = 1; w < CQ_NW; ++w)
      if (better(redv[par][w], redi[par][w], cv, ci)) { cv = redv[par][w]; ci = redi[par][w]; }
    if (tid == 0) {
      double f = 0.0;
      if (s == 0)
        for (int w = 0; w < CQ_NW; ++w) f += redf[w];
      st_agent(myslot + 0, cv);
      st_agent(myslot + 1, (double)(ci == INT64_MAX ? -1 : ci));
      st_agent(myslot + 2, f);
    }
    if (ci != INT64_MAX) {
      const int64_t jj = ci - j0;
      for (int i = s + tid; i < r; i += CQ_NT) st_agent(myslot + 3 + i, slab[jj * rp + i]);
    }
    post_tag(a.tags + (par * a.G + g) * FLAG_STRIDE, (uint32_t)s + 1u);
    // 2./3. thread w waits for workgroup w's tag and reads its candidate; the
    // global pivot is the best candidate (lowest index on ties)
    double gv = -1.0;
    int64_t gi = INT64_MAX;
    int gg = 0;
    double fro_part = 0.0;
    for (int w = tid; w < a.G; w += CQ_NT) {
      wait_tag(a.tags + (par * a.G + w) * FLAG_STRIDE, (uint32_t)s + 1u + a.wait_bias,
               a.abort_flag, a.spin_cap, a.info);
      const double* sl = a.slots + ((int64_t)par * a.G + w) * a.slot_len;
      const double vv = ld_agent(sl + 0);
      const double iv = ld_agent(sl + 1);
      if (s == 0) fro_part += ld_agent(sl + 2);
      if (iv >= 0.0) {
        const int64_t ii = (int64_t)iv;
        if (better(vv, ii, gv, gi)) { gv = vv; gi = ii; gg = w; }
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(gv, off, 64);
      const int64_t oi = __shfl_xor(gi, off, 64);
      const int og = __shfl_xor(gg, off, 64);
      if (better(ov, oi, gv, gi)) { gv = ov; gi = oi; gg = og; }
    }
    if (s == 0) fro_part = wave_allsum(fro_part);
    const int rb = par ^ 1;                // the other half of the reduction buffers
    if (lane == 0) { redv[rb][wave] = gv; redi[rb][wave] = gi; redg[rb][wave] = gg; }
    if (s == 0 && lane == 0) redf[wave] = fro_part;
    __syncthreads();
    gv = redv[rb][0]; gi = redi[rb][0]; gg = redg[rb][0];
    for (int w = 1; w < CQ_NW; ++w)
      if (better(redv[rb][w], redi[rb][w], gv, gi)) { gv = redv[rb][w]; gi = redi[rb][w]; gg = redg[rb][w]; }
    if (s == 0) {
      double fro2 = 0.0;
      for (int w = 0; w < CQ_NW; ++w) fro2 += redf[w];
      tol = (double)(r > a.c ? r : a.c) * DEPS * sqrt(fro2);
    }
    // without a valid candidate (possible only after an aborted wait, whose
    // results are flagged invalid) column 0 stands in, so that every index
    // stays in range
    if (gi < 0 || gi >= a.c) { gi = 0; gg = 0; }
    // the pivot's posted norm^2 is ||x||^2 of its rows s..r-1; a non-finite
    // pivot (NaN key -0.5, or Inf) is taken with a zero reflector
    const bool pfin = gv >= 0.0 && gv <= 1.7976931348623157e308;
    if (!pfin && g == 0 && tid == 0) info_or(a.info, INFO_NONFINITE);
    const double pnorm = pfin ? sqrt(gv) : 0.0;
    if (frank == a.k && pnorm <= tol) frank = s;
    const double* psl = a.slots + ((int64_t)par * a.G + gg) * a.slot_len;
    for (int i = s + tid; i < r; i += CQ_NT) v[i] = ld_agent(psl + 3 + i);
    __syncthreads();
    if (tid == 0) {
      const double normx = pnorm;
      const double x0 = v[s];
      if (normx == 0.0) {
        sh_beta = 0.0;
        sh_alpha = 0.0;
      } else {
        const double sg = x0 >= 0.0 ? 1.0 : -1.0;
        v[s] = x0 + sg * normx;
        sh_alpha = -sg * normx;
        // v^T v = 2 ||x|| (||x|| + |x_0|)
        sh_beta = 1.0 / (normx * (normx + fabs(x0)));
      }
      if (g == 0) {
        a.J[s] = gi;
        a.pivn[s] = pnorm;
      }
      piv[s] = gi;
    }
    __syncthreads();
    const double beta = sh_beta, alpha = sh_alpha;
    // apply H to the unchosen owned columns, recompute their norms over rows
    // s+1.. and track each lane's best column.  Rows above s enter as exact
    // zeros through v (selected per lane), rows r .. 16 RPL - 1 are zero in
    // the slab and in v; a column's stores run under one test.
    bv = -1.0;
    bi = INT64_MAX;
    double vr[RPL];
#pragma unroll
    for (int e = 0; e < RPL; ++e) {
      const int i = rl + 16 * e;
      const double vv = v[i];
      vr[e] = i >= s ? vv : 0.0;
    }
    for (int64_t jb = 0; jb < ncols; jb += CQ_NW * 4) {
      const int64_t jj = jb + wave * 4 + cg;
      const bool inr = jj < ncols;
      const int64_t jc = inr ? jj : 0;       // a column of the slab for the loads
      const bool act = inr && chosen_at[jc] < 0;
      const bool is_piv = act && (j0 + jj == gi);
      double* col = slab + jc * rp;
      double x[RPL];
      double dp[4] = {0.0, 0.0, 0.0, 0.0};   // four partial sums: short FMA chains
#pragma unroll
      for (int e = 0; e < RPL; ++e) {
        x[e] = col[rl + 16 * e];
        dp[e & 3] = fma(vr[e], x[e], dp[e & 3]);
      }
      const double wdot = beta * row16_sum((dp[0] + dp[1]) + (dp[2] + dp[3]));
      const bool upd = act && !is_piv && beta != 0.0;
#pragma unroll
      for (int e = 0; e < RPL; ++e) {
        const int i = rl + 16 * e;
        const double y = fma(-wdot, vr[e], x[e]);
        x[e] = (upd && i >= s) ? y : x[e];
      }
      if (upd) {
#pragma unroll
        for (int e = 0; e < RPL; ++e) col[rl + 16 * e] = x[e];
      }
      if (is_piv) {
#pragma unroll
        for (int e = 0; e < RPL; ++e) {
          const int i = rl + 16 * e;
          col[i] = (i == s) ? alpha : (i > s ? 0.0 : x[e]);
        }
        if (rl == 0) { chosen_at[jj] = s; nrm[jj] = 0.0; }
      }
      double sp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int e = 0; e < RPL; ++e) {
        const int i = rl + 16 * e;
        const double f = fma(x[e], x[e], sp[e & 3]);
        sp[e & 3] = i > s ? f : sp[e & 3];
      }
      const double s2 = row16_sum((sp[0] + sp[1]) + (sp[2] + sp[3]));
      if (act && !is_piv) {
        if (rl == 0) nrm[jj] = s2;
        if (better(sel_key(s2), j0 + jj, bv, bi)) { bv = sel_key(s2); bi = j0 + jj; }
      }
    }
  }
  __syncthreads();
  if (g == 0 && tid == 0 && frank < a.k) {
    info_or(a.info, INFO_RANK);
    a.info[1] = frank;
  }
  // After an aborted wait the workgroups may disagree on the pivots, so the
  // positions below would not be a permutation: then J lists the columns in
  // order and the factors are not written (the call reports INFO_BARRIER).
  if (ld_agent_u32(a.abort_flag) != 0) {
    for (int64_t jj = tid; jj < ncols; jj += CQ_NT) a.J[j0 + jj] = j0 + jj;
    return;
  }
  // outputs: top k rows of every owned column
  for (int64_t jj = wave; jj < ncols; jj += CQ_NW) {
    const int64_t j = j0 + jj;
    const int t = chosen_at[jj];
    double* dst;
    if (t >= 0) {
      dst = a.S11t + (int64_t)t * a.lds;
    } else {
      int64_t before = 0;
      for (int q = lane; q < a.k; q += 64) before += (piv[q] < j) ? 1 : 0;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) before += __shfl_xor(before, off, 64);
      const int64_t rho = j - before;
      dst = a.S12t + rho * a.lds;
      if (lane == 0) a.J[a.k + rho] = j;
    }
    for (int i = lane; i < a.k; i += 64) dst[i] = (i < r) ? slab[jj * rp + i] : 0.0;
  }
}

// Upper-triangular solve X = S^{-1} B with many right-hand sides (k <= 256),
// by block back substitution over 16 x 16 blocks:
//   X_c = M_c (B_c - sum_{b>c} S_cb X_b),  c = nb-1 .. 0,
// where M_c is the solve with the diagonal block S_cc under the rule that a
// zero pivot gives a zero unknown (x_i = 0 when S_ii = 0); that rule is
// linear in the right-hand side, so M_c is the matrix of 16 such solves with
// the unit vectors, formed in LDS by every workgroup.  One wave takes 16
// right-hand sides; as in the orth triangular solve, the 16 x 16 product
// in accumulator layout (lane (j, g) holds rows 4v + g of column j) is the
// B operand of the later products, so each X_b stays in registers.  Strided
// access: S(i, j) = S[i*s_r + j*s_c], right-hand side `col` element i =
// Bm[col*b_c + i*b_r], X(i, col) = X[i*x_r + col*x_c].
constexpr int BSB_MAXNB = 16;

template <int NB>
__global__ __launch_bounds__(256) void backsub_kernel(const double* __restrict__ S, int64_t s_r,
                                                      int64_t s_c, const double* __restrict__ Bm,
                                                      int64_t b_r, int64_t b_c, int k,
                                                      int64_t nrhs, double* __restrict__ X,
                                                      int64_t x_r, int64_t x_c) {
  __shared__ double Sd[BSB_MAXNB][16 * 17];   // diagonal blocks of S
  __shared__ double Md[BSB_MAXNB][16 * 17];   // their solve matrices M_c
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nb = (int)cdiv(k, 16);
  for (int e = tid; e < nb * 256; e += 256) {
    const int c = e >> 8, i = (e >> 4) & 15, j = e & 15;
    const int gi = c * 16 + i, gj = c * 16 + j;
    Sd[c][i * 17 + j] = (gi < k && gj < k && i <= j) ? S[gi * s_r + gj * s_c] : 0.0;
  }
  __syncthreads();
  if (tid < nb * 16) {
    // column j of M_c: back substitution with the unit vector e_j
    const int c = tid >> 4, j = tid & 15;
    const double* sd = Sd[c];
    double x[16];
#pragma unroll
    for (int i = 15; i >= 0; --i) {
      double t = (i == j) ? 1.0 : 0.0;
#pragma unroll
      for (int q = i + 1; q < 16; ++q) t -= sd[i * 17 + q] * x[q];
      const double sii = sd[i * 17 + i];
      x[i] = (sii != 0.0) ? t / sii : 0.0;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) Md[c][i * 17 + j] = x[i];
  }
  __syncthreads();
  const int64_t col0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  if (col0 >= nrhs) return;
  const int64_t col = col0 + li;
  const bool cok = col < nrhs;
  const double* bc = Bm + (cok ? col : 0) * b_c;
  double* xc = X + (cok ? col : 0) * x_c;
  // The loads of a block step are unconditional, from clamped indices, with
  // a select after them (under a branch each load was waited for at once);
  // blocks past nb contribute zeros (their X blocks start at zero).
  d4 xt[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) xt[c] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int c = NB - 1; c >= 0; --c) {
    if (c < nb) {
      d4 acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = c * 16 + 4 * v + lk;
        const double bv = bc[min(i, k - 1) * b_r];
        acc[v] = (cok && i < k) ? bv : 0.0;
      }
#pragma unroll
      for (int b = c + 1; b < NB; ++b) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int i = c * 16 + li, j = b * 16 + 4 * kk + lk;
          const double sv = S[min(i, k - 1) * s_r + min(j, k - 1) * s_c];
          const double av = (i < k && j < k) ? -sv : 0.0;   // S_cb[li][k]
          acc = Mfma<double>::mma(av, xt[b][kk], acc);
        }
      }
      d4 out = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
        out = Mfma<double>::mma(Md[c][li * 17 + 4 * kk + lk], acc[kk], out);
      xt[c] = out;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = c * 16 + 4 * v + lk;
        if (cok && i < k) xc[i * x_r] = out[v];
      }
    }
  }
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace

size_t cpqr_lds_bytes(int64_t cs, int rp, int k) {
  return (size_t)(cs * rp + cs + rp) * sizeof(double) + (size_t)(cs + (cs & 1)) * sizeof(int) +
         (size_t)k * sizeof(int64_t);
}

CpqrPlan plan_cpqr(int r, int64_t c, int k, int ncu) {
  CpqrPlan p;
  // rows per lane: the smallest instantiated RPL with 16 RPL >= r
  p.rpl = 0;
  for (int v : CQ_RPLS)
    if (p.rpl == 0 && 16 * v >= r) p.rpl = v;
  // column stride of the LDS slab: rp = 16 (mod 32) doubles puts consecutive
  // columns on opposite halves of the LDS banks; rp >= 16 RPL
  p.rp = (int)(rup(std::max(r, 16 * p.rpl) + 16, 32) - 16);
  int64_t G = cdiv(c, 32);
  if (G > ncu) G = ncu;
  if (G < 1) G = 1;
  p.G = (int)G;
  p.cs = cdiv(c, G);
  p.lds = cpqr_lds_bytes(p.cs, p.rp, k);
  p.slot_len = 3 + p.rp;
  p.ok = p.lds <= 150 * 1024 && r <= 256 && k <= 256 && k <= r && k <= c && p.rpl > 0;
  return p;
}

size_t cpqr_work_bytes(const CpqrPlan& p) {
  return (size_t)(2 * p.G * p.slot_len) * sizeof(double) +
         (size_t)(2 * p.G + 1) * FLAG_STRIDE * sizeof(uint32_t) + 64;
}

hipError_t launch_cpqr(bool b_f32, const void* Bt, int64_t ldb, int r, int64_t c, int k,
                       const CpqrPlan& p, void* work, int64_t* J, double* S11t, double* S12t,
                       int64_t lds, double* pivn, int32_t* info, bool giveup_test,
                       hipStream_t s) {
  if (!p.ok) return hipErrorInvalidValue;
  CpqrArgs a;
  a.Bt = Bt; a.ldb = ldb; a.r = r; a.c = c; a.k = k;
  a.G = p.G; a.cs = p.cs; a.rp = p.rp;
  double* w = static_cast<double*>(work);
  a.slots = w;
  a.slot_len = p.slot_len;
  a.tags = reinterpret_cast<uint32_t*>(w + 2 * p.G * p.slot_len);
  a.abort_flag = a.tags + 2 * p.G * FLAG_STRIDE;
  a.J = J; a.S11t = S11t; a.S12t = S12t; a.lds = lds; a.pivn = pivn; a.info = info;
  a.wait_bias = giveup_test ? 1u : 0u;
  a.spin_cap = giveup_test ? SPIN_CAP_TEST : SPIN_CAP;
  hipError_t e = launch_fill_u32(a.tags, 0u, (2 * p.G + 1) * FLAG_STRIDE, s);
  if (e != hipSuccess) return e;
  void* args[] = {&a};
  const void* fn = nullptr;
#define RSVD_CQ(V)                                                                       \
  if (p.rpl == V)                                                                        \
    fn = b_f32 ? (const void*)cpqr_kernel<float, V> : (const void*)cpqr_kernel<double, V>;
  RSVD_CQ(2) RSVD_CQ(4) RSVD_CQ(8) RSVD_CQ(12) RSVD_CQ(13) RSVD_CQ(14) RSVD_CQ(16)
#undef RSVD_CQ
  if (!fn) return hipErrorInvalidValue;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds);
  if (e != hipSuccess) return e;
  e = hipLaunchKernel(fn, dim3(p.G), dim3(CQ_NT), args, p.lds, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_backsub(const double* S, int64_t s_r, int64_t s_c, const double* Bm,
                          int64_t b_r, int64_t b_c, int k, int64_t nrhs, double* X, int64_t x_r,
                          int64_t x_c, hipStream_t s) {
  if (nrhs <= 0 || k <= 0) return hipSuccess;
  if (k > 256) return hipErrorInvalidValue;
  const dim3 grid((unsigned)cdiv(nrhs, 64));
  const int nb = (int)cdiv(k, 16);
#define RSVD_BSB(NBV)                                                                           \
  hipLaunchKernelGGL(backsub_kernel<NBV>, grid, dim3(256), 0, s, S, s_r, s_c, Bm, b_r, b_c, k, \
                     nrhs, X, x_r, x_c)
  if (nb <= 2) RSVD_BSB(2);
  else if (nb <= 4) RSVD_BSB(4);
  else if (nb <= 8) RSVD_BSB(8);
  else if (nb <= 13) RSVD_BSB(13);
  else RSVD_BSB(16);
#undef RSVD_BSB
  return hipGetLastError();
}

}  // namespace rsvd
