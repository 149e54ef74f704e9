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
// One workgroup of 16 waves; pairs are scheduled in round-robin rounds of
// disjoint pairs (circle method), one pair per wave at a time; the dot
// products are wave reductions.  W and V live in LDS when they fit and in
// global memory (L2-resident) otherwise.  Output: the k largest sigma in
// descending order (stable for ties) and the matching columns of Uh and Vh.
#include "common.h"
#include "internal.h"

namespace rsvd {
namespace {

constexpr int JNT = 1024;
constexpr int LDS_MAX_L = 64;     // 2 * 64 * 64 * 8 B = 64 KB

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ int rr_player(int pos, int r, int N) {
  return pos == 0 ? 0 : ((pos - 1 + r) % (N - 1)) + 1;
}

// W, V: column-major, column j at base + j * ld (ld >= l)
template <bool IN_LDS>
__global__ __launch_bounds__(JNT) void jacobi_kernel(const double* __restrict__ Rh, int64_t ldr,
                                                     int l, int k, double* Wg, double* Vg,
                                                     int64_t ldw, double* __restrict__ S,
                                                     double* __restrict__ Uh, int64_t lduh,
                                                     double* __restrict__ Vh, int64_t ldvh,
                                                     int max_sweeps, double tol, int32_t* info) {
  extern __shared__ double smem[];
  __shared__ int rotated;
  __shared__ double sig[256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* W;
  double* V;
  int64_t ld;
  if (IN_LDS) {
    ld = l;
    W = smem;
    V = smem + (int64_t)l * l;
  } else {
    ld = ldw;
    W = Wg;
    V = Vg;
  }
  // W = R_hat (column-major), V = I
  for (int64_t e = tid; e < (int64_t)l * l; e += JNT) {
    const int j = (int)(e / l), i = (int)(e % l);
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
      for (int pi = wave; pi < N / 2; pi += JNT / 64) {
        int a = rr_player(pi, r, N), b = rr_player(N - 1 - pi, r, N);
        if (a >= l || b >= l) continue;
        if (a > b) { const int t = a; a = b; b = t; }
        double* wa = W + a * ld;
        double* wb = W + b * ld;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = lane; i < l; i += 64) {
          const double x = wa[i], y = wb[i];
          al += x * x; be += y * y; ga += x * y;
        }
        al = wave_sum(al); be = wave_sum(be); ga = wave_sum(ga);
        if (!(fabs(ga) > tol * sqrt(al * be))) continue;
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + t * t);
        const double sn = cs * t;
        for (int i = lane; i < l; i += 64) {
          const double x = wa[i], y = wb[i];
          wa[i] = cs * x - sn * y;
          wb[i] = sn * x + cs * y;
        }
        double* va = V + a * ld;
        double* vb = V + b * ld;
        for (int i = lane; i < l; i += 64) {
          const double x = va[i], y = vb[i];
          va[i] = cs * x - sn * y;
          vb[i] = sn * x + cs * y;
        }
        if (lane == 0) rotated = 1;
      }
      __syncthreads();
    }
    converged = (rotated == 0);
    __syncthreads();
  }
  if (!converged && tid == 0) info_or(info, INFO_JACOBI_CAP);

  // singular values = column norms
  for (int j = wave; j < l; j += JNT / 64) {
    double s2 = 0.0;
    for (int i = lane; i < l; i += 64) { const double x = W[j * ld + i]; s2 += x * x; }
    s2 = wave_sum(s2);
    if (lane == 0) sig[j] = sqrt(s2);
  }
  __syncthreads();
  // stable descending rank, then write the first k
  for (int j = wave; j < l; j += JNT / 64) {
    const double sj = sig[j];
    int rank = 0;
    for (int i = lane; i < l; i += 64) {
      const double si = sig[i];
      rank += (si > sj || (si == sj && i < j)) ? 1 : 0;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) rank += __shfl_xor(rank, off, 64);
    if (rank < k) {
      if (lane == 0) S[rank] = sj;
      const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
      for (int i = lane; i < l; i += 64) {
        Uh[(int64_t)i * lduh + rank] = W[j * ld + i] * inv;
        Vh[(int64_t)i * ldvh + rank] = V[j * ld + i];
      }
    }
  }
}

}  // namespace

hipError_t launch_jacobi(const double* Rh, int64_t ldr, int l, int k, double* Wwork, double* Vwork,
                         int64_t ldw, double* S, double* Uh, int64_t lduh, double* Vh,
                         int64_t ldvh, int max_sweeps, int32_t* info, hipStream_t s) {
  if (l > 256) return hipErrorInvalidValue;
  const double tol = (double)l * 2.220446049250313e-16;
  if (l <= LDS_MAX_L) {
    const size_t shm = 2 * (size_t)l * l * sizeof(double);
    hipLaunchKernelGGL(jacobi_kernel<true>, dim3(1), dim3(JNT), shm, s, Rh, ldr, l, k, Wwork,
                       Vwork, ldw, S, Uh, lduh, Vh, ldvh, max_sweeps, tol, info);
  } else {
    hipLaunchKernelGGL(jacobi_kernel<false>, dim3(1), dim3(JNT), 0, s, Rh, ldr, l, k, Wwork,
                       Vwork, ldw, S, Uh, lduh, Vh, ldvh, max_sweeps, tol, info);
  }
  return hipGetLastError();
}

}  // namespace rsvd
