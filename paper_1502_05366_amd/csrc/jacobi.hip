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
// One workgroup up to l = 64 (2 * 64 * 64 * 8 B = 64 KB of LDS).  At l = 80 the
// one-workgroup iteration measured 1.09 ms against 1.00 ms for the block
// iteration on three workgroups, so larger factors take the block iteration.
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
// launch takes one block pair per round: it loads the 2*BS
// columns of W and V into LDS, rotates every cross pair (x from the first
// block, y from the second; in round 0 also the pairs inside each block),
// and writes the columns back.  Between rounds the workgroups exchange
// progress through per-workgroup tags (agent-scope release / acquire); a
// sweep over all rounds visits every column pair exactly once.  The
// iteration stops after the first sweep without a rotation.
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

__device__ void jac_wait_all(const JacArgs& a, uint32_t target) {
  const int tid = threadIdx.x;
  if (tid < a.G) {
    uint32_t spins = 0;
    while (ld_agent_u32(a.tags + tid * FLAG_STRIDE) < target + a.wait_bias) {
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
  __syncthreads();
}

// The block kernel gives each column pair to one row of 16 lanes, so a wave
// works on four pairs at once: lane (row g, position c) holds rows c + 16 e
// (e = 0..15) of both W columns of its pair.  Sums over a pair are DPP
// exchanges inside the row; the rotation is computed by every lane of the row
// (rows whose pair is already orthogonal apply the identity).  V is not
// rotated column by column: the rotations of a round are accumulated in a
// 2BS x 2BS orthogonal J (two rows per lane), and the round ends with
// V(:, pair blocks) <- V(:, pair blocks) J on the matrix cores.
constexpr int JB_NT = 256;   // 4 waves x 4 pairs = BS pairs per step
constexpr int JJ = 2 * BS;   // order of J
// Rows per lane JRPL: 16 for l <= 256, 36 for l <= 576 (a column of W is
// 16 JRPL rows, rows >= l zero).  LDS column stride of W: the rows + 16
// doubles, so columns q and q+1 start on opposite halves of the LDS banks;
// J's column stride alternates bank halves too.  At JRPL = 36 the two W blocks
// and J fill 158 KB of the 160 KB of LDS.
constexpr int JACOBI_MAX_L = 576;
template <int JRPL> struct JacDims {
  static constexpr int ROWS = 16 * JRPL;
  static constexpr int JLD = ROWS + 16;
  static constexpr int JJS = JRPL > 16 ? 40 : 48;
  static constexpr size_t LDS = (2 * (size_t)BS * JLD + (size_t)JJ * JJS) * sizeof(double);
};

__device__ __forceinline__ double row16_sum(double x) {
  x += dpp_d<0xB1>(x);     // quad_perm [1, 0, 3, 2]
  x += dpp_d<0x4E>(x);     // quad_perm [2, 3, 0, 1]
  x += dpp_d<0x141>(x);    // row_half_mirror
  x += dpp_d<0x140>(x);    // row_mirror
  return x;
}

template <int JRPL>
__device__ __forceinline__ bool rotate_row16(double (&xw)[JRPL], double (&xj)[2],
                                             double (&yw)[JRPL], double (&yj)[2], double tol) {
  double al[2] = {0.0, 0.0}, be[2] = {0.0, 0.0}, ga[2] = {0.0, 0.0};   // two chains each
#pragma unroll
  for (int e = 0; e < JRPL; ++e) {
    al[e & 1] = fma(xw[e], xw[e], al[e & 1]);
    be[e & 1] = fma(yw[e], yw[e], be[e & 1]);
    ga[e & 1] = fma(xw[e], yw[e], ga[e & 1]);
  }
  const double alpha = row16_sum(al[0] + al[1]);
  const double beta = row16_sum(be[0] + be[1]);
  const double gamma = row16_sum(ga[0] + ga[1]);
  double cs, sn;
  const bool rot = jacobi_rotation(alpha, beta, gamma, tol, cs, sn);
  if (!rot) { cs = 1.0; sn = 0.0; }
#pragma unroll
  for (int e = 0; e < JRPL; ++e) {
    const double a = xw[e], b = yw[e];
    xw[e] = cs * a - sn * b;
    yw[e] = sn * a + cs * b;
  }
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const double c = xj[e], d = yj[e];
    xj[e] = cs * c - sn * d;
    yj[e] = sn * c + cs * d;
  }
  return rot;
}

template <int JRPL>
__device__ __forceinline__ void lds_col_load(const double* base, int rl, double (&v)[JRPL]) {
#pragma unroll
  for (int e = 0; e < JRPL; ++e) v[e] = base[rl + 16 * e];
}
template <int JRPL>
__device__ __forceinline__ void lds_col_store(double* base, int rl, const double (&v)[JRPL]) {
#pragma unroll
  for (int e = 0; e < JRPL; ++e) base[rl + 16 * e] = v[e];
}
template <int JJS>
__device__ __forceinline__ void lds_j_load(const double* Jl, int col, int rl, double (&v)[2]) {
  v[0] = Jl[col * JJS + rl];
  v[1] = Jl[col * JJS + rl + 16];
}
template <int JJS>
__device__ __forceinline__ void lds_j_store(double* Jl, int col, int rl, const double (&v)[2]) {
  Jl[col * JJS + rl] = v[0];
  Jl[col * JJS + rl + 16] = v[1];
}

template <int JRPL>
__global__ __launch_bounds__(JB_NT) void jacobi_block_kernel(JacArgs a) {
  constexpr int ROWS = JacDims<JRPL>::ROWS;
  constexpr int JLD = JacDims<JRPL>::JLD;
  constexpr int JJS = JacDims<JRPL>::JJS;
  extern __shared__ double smem[];
  __shared__ int rotated;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rl = lane & 15;
  const int ps = wave * 4 + (lane >> 4);    // pair slot 0 .. BS-1
  const int w = blockIdx.x;
  const int l = a.l;
  double* Wl = smem;                        // [2*BS][JLD]
  double* Jl = smem + 2 * BS * JLD;         // [JJ][JJS], column-major
  uint32_t done = 0;
  int sweep = 0;
  bool converged = false;
  if (tid == 0) rotated = 0;
  while (!converged && sweep < a.max_sweeps) {
    for (int r = 0; r < a.nbp - 1; ++r) {
      const int bi = rr_player(w, r, a.nbp), bj = rr_player(a.nbp - 1 - w, r, a.nbp);
      auto gcol_of = [&](int c) { return (c < BS) ? bi * BS + c : bj * BS + (c - BS); };
      // load the two W blocks (columns >= l and rows >= l read as zero), each
      // thread issuing all its loads before its LDS writes; J = I
      {
        // wave w takes columns w, w+4, .. of the 2 BS; lanes run down the
        // rows (one column's loads per batch)
        for (int cc = 0; cc < 2 * BS / 4; ++cc) {
          const int c = wave + 4 * cc;
          const int gcol = gcol_of(c);
          double vv[ROWS / 64];
#pragma unroll
          for (int t = 0; t < ROWS / 64; ++t) {
            const int i = lane + 64 * t;
            vv[t] = (i < l && gcol < l) ? ld_agent(a.W + (int64_t)gcol * a.ld + i) : 0.0;
          }
#pragma unroll
          for (int t = 0; t < ROWS / 64; ++t) Wl[c * JLD + lane + 64 * t] = vv[t];
        }
#pragma unroll
        for (int e = 0; e < JJ * JJ / JB_NT; ++e) {
          const int idx = tid + e * JB_NT;
          Jl[(idx / JJ) * JJS + idx % JJ] = (idx / JJ == idx % JJ) ? 1.0 : 0.0;
        }
      }
      __syncthreads();
      bool rot = false;
      double xw[JRPL], yw[JRPL], xj[2], yj[2];
      if (r == 0) {
        // pairs inside each block: BS-1 round-robin rounds, both blocks at once
        for (int t = 0; t < BS - 1; ++t) {
          const int half = ps / (BS / 2), pi = ps % (BS / 2);
          int p = rr_player(pi, t, BS), q = rr_player(BS - 1 - pi, t, BS);
          if (p > q) { const int x = p; p = q; q = x; }
          p += half * BS; q += half * BS;
          lds_col_load<JRPL>(Wl + p * JLD, rl, xw); lds_j_load<JJS>(Jl, p, rl, xj);
          lds_col_load<JRPL>(Wl + q * JLD, rl, yw); lds_j_load<JJS>(Jl, q, rl, yj);
          rot |= rotate_row16<JRPL>(xw, xj, yw, yj, a.tol);
          lds_col_store<JRPL>(Wl + p * JLD, rl, xw); lds_j_store<JJS>(Jl, p, rl, xj);
          lds_col_store<JRPL>(Wl + q * JLD, rl, yw); lds_j_store<JJS>(Jl, q, rl, yj);
          __syncthreads();
        }
      }
      // cross pairs (x_p, y_{(p+t) mod BS}), t = 0 .. BS-1: pair slot p keeps
      // x_p in registers, the y columns move between slots through LDS
      {
        const int p = ps;
        lds_col_load<JRPL>(Wl + p * JLD, rl, xw); lds_j_load<JJS>(Jl, p, rl, xj);
        for (int t = 0; t < BS; ++t) {
          const int q = BS + (p + t) % BS;
          lds_col_load<JRPL>(Wl + q * JLD, rl, yw); lds_j_load<JJS>(Jl, q, rl, yj);
          rot |= rotate_row16<JRPL>(xw, xj, yw, yj, a.tol);
          lds_col_store<JRPL>(Wl + q * JLD, rl, yw); lds_j_store<JJS>(Jl, q, rl, yj);
          __syncthreads();
        }
        lds_col_store<JRPL>(Wl + p * JLD, rl, xw); lds_j_store<JJS>(Jl, p, rl, xj);
      }
      if (rot) rotated = 1;
      __syncthreads();
      // W back to memory
      {
        for (int cc = 0; cc < 2 * BS / 4; ++cc) {
          const int c = wave + 4 * cc;
          const int gcol = gcol_of(c);
#pragma unroll
          for (int t = 0; t < ROWS / 64; ++t) {
            const int i = lane + 64 * t;
            if (i < l && gcol < l) st_agent(a.W + (int64_t)gcol * a.ld + i, Wl[c * JLD + i]);
          }
        }
      }
      // V(:, pair) <- V(:, pair) J: wave v takes row tiles v, v+4, v+8, ..
      // (16 rows each, in groups of RG tiles) and both 16-column halves; it
      // reads all rows of a group before it writes any, and no other wave
      // touches them
      {
        constexpr int RT = JRPL / 4;           // row tiles per wave
        constexpr int RG = RT % 3 == 0 ? 3 : RT;
        const int li = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int q0 = 0; q0 < RT; q0 += RG) {
          double av[RG][JJ / 4];
#pragma unroll
          for (int q = 0; q < RG; ++q) {
            const int row = (wave + 4 * (q0 + q)) * 16 + li;
#pragma unroll
            for (int kk = 0; kk < JJ / 4; ++kk) {
              const int gcol = gcol_of(kk * 4 + lk);
              av[q][kk] =
                  (row < l && gcol < l) ? ld_agent(a.V + (int64_t)gcol * a.ld + row) : 0.0;
            }
          }
#pragma unroll
          for (int ct = 0; ct < JJ / 16; ++ct) {
            double bv[JJ / 4];
#pragma unroll
            for (int kk = 0; kk < JJ / 4; ++kk) bv[kk] = Jl[(ct * 16 + li) * JJS + kk * 4 + lk];
#pragma unroll
            for (int q = 0; q < RG; ++q) {
              d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
              for (int kk = 0; kk < JJ / 4; ++kk)
                acc = Mfma<double>::mma(av[q][kk], bv[kk], acc);
              const int gcol = gcol_of(ct * 16 + li);
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int row = (wave + 4 * (q0 + q)) * 16 + drow(lk, v);
                if (row < l && gcol < l) st_agent(a.V + (int64_t)gcol * a.ld + row, acc[v]);
              }
            }
          }
        }
      }
      const bool last = (r == a.nbp - 2);
      if (last && tid == 0)
        st_agent_u32(a.rot + ((sweep & 1) * a.G + w) * FLAG_STRIDE, (uint32_t)rotated);
      stores_done();
      __syncthreads();
      ++done;
      if (tid == 0) st_agent_u32(a.tags + w * FLAG_STRIDE, done);
      jac_wait_all(a, done);
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

__global__ __launch_bounds__(256) void jacobi_init_kernel(const double* __restrict__ Rh,
                                                          int64_t ldr, int l,
                                                          double* __restrict__ W,
                                                          double* __restrict__ V, int64_t ld,
                                                          uint32_t* ctl, int nctl) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < nctl) ctl[e] = 0;
  if (e >= (int64_t)l * l) return;
  const int j = (int)(e / l), i = (int)(e - (int64_t)j * l);
  W[(int64_t)j * ld + i] = Rh[(int64_t)i * ldr + j];
  V[(int64_t)j * ld + i] = (i == j) ? 1.0 : 0.0;
}

__global__ __launch_bounds__(JNT) void jacobi_finish_kernel(const double* __restrict__ W,
                                                            const double* __restrict__ V,
                                                            int64_t ld, int l, int k,
                                                            double* __restrict__ S,
                                                            double* __restrict__ Uh, int64_t lduh,
                                                            double* __restrict__ Vh,
                                                            int64_t ldvh) {
  __shared__ double sig[JACOBI_MAX_L];
  jacobi_finish<JNT>(W, V, ld, l, k, sig, S, Uh, lduh, Vh, ldvh);
}

}  // namespace

// control words of the block iteration: tags [64], rotation flags [2][64],
// the abort flag (FLAG_STRIDE apart; at most 64 workgroups)
constexpr int JCTL = 200;

size_t jacobi_work_bytes(int l) {
  // W, V (l x l each) and the control words of the block iteration
  return 2 * (size_t)l * l * sizeof(double) + JCTL * FLAG_STRIDE * sizeof(uint32_t) + 256;
}

template <int JRPL>
hipError_t launch_block(JacArgs& a, hipStream_t s) {
  const size_t shm = JacDims<JRPL>::LDS;
  hipError_t e = hipFuncSetAttribute((const void*)jacobi_block_kernel<JRPL>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  void* args[] = {&a};
  return hipLaunchKernel((const void*)jacobi_block_kernel<JRPL>, dim3(a.G), dim3(JB_NT), args,
                         shm, s);
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
  double* W = work;
  double* V = work + (size_t)l * l;
  uint32_t* ctl = reinterpret_cast<uint32_t*>(V + (size_t)l * l);
  const int nb = (int)cdiv(l, BS);
  const int nbp = nb + (nb & 1);
  JacArgs a;
  a.W = W; a.V = V; a.ld = l; a.l = l; a.nbp = nbp; a.G = nbp / 2; a.max_sweeps = max_sweeps;
  a.tol = tol;
  a.tags = ctl;                                   // 64 flags
  a.rot = ctl + 64 * FLAG_STRIDE;                 // 2 x 64 flags
  a.abort_flag = ctl + 192 * FLAG_STRIDE;
  a.wait_bias = giveup_test ? 1u : 0u;
  a.spin_cap = giveup_test ? (1u << 10) : (1u << 22);
  a.info = info;
  a.sweeps_out = sweeps_out;
  // one thread per element of W and per control word
  const int64_t ninit = std::max<int64_t>((int64_t)l * l, (int64_t)JCTL * FLAG_STRIDE);
  hipLaunchKernelGGL(jacobi_init_kernel, dim3((unsigned)cdiv(ninit, 256)), dim3(256), 0, s, Rh,
                     ldr, l, W, V, (int64_t)l, ctl, JCTL * FLAG_STRIDE);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = (l <= 256) ? launch_block<16>(a, s) : launch_block<36>(a, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(jacobi_finish_kernel, dim3(1), dim3(JNT), 0, s, W, V, (int64_t)l, l, k, S, Uh,
                     lduh, Vh, ldvh);
  return hipGetLastError();
}

}  // namespace rsvd
