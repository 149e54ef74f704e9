// Device pieces of the one-sided (Hestenes) Jacobi SVD shared by the
// single-matrix and the batched small SVD: the rotation of a column pair,
// the round-robin pair schedule and the sorted output.
#pragma once

#include "common.h"

namespace rsvd {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Rotation (c, s) that orthogonalizes a column pair with squared norms al, be
// and inner product ga (the formulas in the header); false when the pair is
// already orthogonal to within tol.
// 1/x with one Newton step: enough for quantities that only set the rotation
// angle (c and s are made consistent afterwards)
__device__ __forceinline__ double rcp_nr1(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

__device__ __forceinline__ bool jacobi_rotation(double al, double be, double ga, double tol,
                                                double& cs, double& sn) {
  // |ga| > tol sqrt(al be), compared in squares
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
  // c = 1 / sqrt(1 + t^2) to full precision, so that c^2 + s^2 = 1 to rounding
  cs = rsq_nr(fma(t, t, 1.0));
  sn = cs * t;
  return true;
}

__device__ __forceinline__ int rr_player(int pos, int r, int N) {
  return pos == 0 ? 0 : ((pos - 1 + r) % (N - 1)) + 1;
}

// Sum over a row of 16 lanes (a DPP row), returned in every lane of the
// row: exchanges xor 1 and xor 2 inside quads, then the half-row and the
// row mirror.  All 16 lanes of the row must be active.
__device__ __forceinline__ double dpp_row16_sum(double x) {
  x += dpp_d<0xB1>(x);     // quad_perm [1, 0, 3, 2]
  x += dpp_d<0x4E>(x);     // quad_perm [2, 3, 0, 1]
  x += dpp_d<0x141>(x);    // row_half_mirror
  x += dpp_d<0x140>(x);    // row_mirror
  return x;
}

// Rotation of the column pair (a, b) of W and V (columns contiguous, length
// l <= 16 RPL) by one group of 16 lanes, a DPP row: lane li holds rows li,
// li + 16, ...; the dot products are DPP row sums (the same value on every
// lane of the group).  Returns true when a rotation was applied.
template <int RPL>
__device__ __forceinline__ bool rotate_pair16(double* wa, double* wb, double* va, double* vb,
                                              int l, int li, double tol) {
  double xa[RPL], xb[RPL];
  double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int i = li + 16 * t;
    xa[t] = i < l ? wa[i] : 0.0;
    xb[t] = i < l ? wb[i] : 0.0;
    al = fma(xa[t], xa[t], al);
    be = fma(xb[t], xb[t], be);
    ga = fma(xa[t], xb[t], ga);
  }
  al = dpp_row16_sum(al);
  be = dpp_row16_sum(be);
  ga = dpp_row16_sum(ga);
  double cs, sn;
  if (!jacobi_rotation(al, be, ga, tol, cs, sn)) return false;
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int i = li + 16 * t;
    if (i < l) {
      wa[i] = cs * xa[t] - sn * xb[t];
      wb[i] = sn * xa[t] + cs * xb[t];
    }
  }
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int i = li + 16 * t;
    if (i < l) {
      const double y = va[i], z = vb[i];
      va[i] = cs * y - sn * z;
      vb[i] = sn * y + cs * z;
    }
  }
  return true;
}

// Singular values = column norms of W; the k largest (stable descending
// order) go to S with Uh(:, rank) = w_j / sigma_j and Vh(:, rank) = v_j.
// Called by every thread of a workgroup of NTH threads; sig has l entries.
template <int NTH>
__device__ void jacobi_finish(const double* W, const double* V, int64_t ld, int l, int k,
                              double* sig, double* __restrict__ S, double* __restrict__ Uh,
                              int64_t lduh, double* __restrict__ Vh, int64_t ldvh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j = wave; j < l; j += NTH / 64) {
    double s2 = 0.0;
    for (int i = lane; i < l; i += 64) { const double x = W[j * ld + i]; s2 += x * x; }
    s2 = wave_sum(s2);
    if (lane == 0) sig[j] = sqrt(s2);
  }
  __syncthreads();
  for (int j = wave; j < l; j += NTH / 64) {
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

// Rotate the column pair (a, b) of W (and V) if it is not yet orthogonal;
// executed by one wave.  Returns true when a rotation was applied.
__device__ __forceinline__ bool rotate_pair(double* wa, double* wb, double* va, double* vb, int l,
                                            int lane, double tol) {
  double al = 0.0, be = 0.0, ga = 0.0;
  for (int i = lane; i < l; i += 64) {
    const double x = wa[i], y = wb[i];
    al += x * x; be += y * y; ga += x * y;
  }
  al = wave_allsum(al); be = wave_allsum(be); ga = wave_allsum(ga);
  double cs, sn;
  if (!jacobi_rotation(al, be, ga, tol, cs, sn)) return false;
  for (int i = lane; i < l; i += 64) {
    const double x = wa[i], y = wb[i];
    wa[i] = cs * x - sn * y;
    wb[i] = sn * x + cs * y;
  }
  for (int i = lane; i < l; i += 64) {
    const double x = va[i], y = vb[i];
    va[i] = cs * x - sn * y;
    vb[i] = sn * x + cs * y;
  }
  return true;
}

}  // namespace
}  // namespace rsvd
