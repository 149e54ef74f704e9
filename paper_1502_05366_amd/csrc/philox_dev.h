// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the FP64
// Box-Muller transform used for every Gaussian matrix of the path: key =
// (seed low word, seed high word), counter = (pair index low, pair index
// high, stream id, batch); normals 2t and 2t+1 come from pair t:
//   u1 = ((x0 >> 5) 2^26 + (x1 >> 6) + 1) 2^-53,  u2 = ((x2 >> 5) 2^26 + (x3 >> 6)) 2^-53,
//   r = sqrt(-2 ln u1), theta = 2 pi u2, (r cos theta, r sin theta).
#pragma once

#include "common.h"

namespace rsvd {
namespace {

constexpr uint32_t PM0 = 0xD2511F53u, PM1 = 0xCD9E8D57u;
constexpr uint32_t PW0 = 0x9E3779B9u, PW1 = 0xBB67AE85u;
constexpr double TWO_PI = 6.283185307179586;

struct Words { uint32_t x0, x1, x2, x3; };

__device__ __forceinline__ Words philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += PW0; k1 += PW1; }
    const uint32_t hi0 = __umulhi(PM0, c0), lo0 = PM0 * c0;
    const uint32_t hi1 = __umulhi(PM1, c2), lo1 = PM1 * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return Words{c0, c1, c2, c3};
}

__device__ __forceinline__ void box_muller(const Words& w, double& z0, double& z1) {
  const double a = (double)(w.x0 >> 5) * 67108864.0 + (double)(w.x1 >> 6);
  const double b = (double)(w.x2 >> 5) * 67108864.0 + (double)(w.x3 >> 6);
  const double u1 = (a + 1.0) * 0x1.0p-53;
  const double u2 = b * 0x1.0p-53;
  const double r = sqrt(-2.0 * log(u1));
  const double th = TWO_PI * u2;
  z0 = r * cos(th);
  z1 = r * sin(th);
}

}  // namespace
}  // namespace rsvd
