// fmc_device.hpp -- device-side arithmetic shared by the gfx950 kernels.
//
// Counter-based random numbers (Philox-4x64-10, Salmon et al. SC'11), the
// Feistel stratum permutation of the LHS design (Sec. IV-B), the inverse
// normal CDF (Wichura AS 241, PPND16) and the KLE basis (eq. 7).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fmc {

// ---------------------------------------------------------------------------
// Philox-4x64-10: ten rounds of two 64x64->128 multiplies with xor mixing; the
// key advances by the Weyl constants (golden ratio, sqrt(3)-1) between rounds.
// ---------------------------------------------------------------------------
struct u64x4 {
  uint64_t v[4];
};

__device__ __forceinline__ u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
  constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ULL;
  constexpr uint64_t kM1 = 0xCA5A826395121157ULL;
  constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ULL;
  constexpr uint64_t kW1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(kM0, c0), lo0 = kM0 * c0;
    const uint64_t hi1 = __umul64hi(kM1, c2), lo1 = kM1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += kW0;
    k1 += kW1;
  }
  u64x4 o;
  o.v[0] = c0;
  o.v[1] = c1;
  o.v[2] = c2;
  o.v[3] = c3;
  return o;
}

// Stream tags of the method's draws (counter word 3).
constexpr uint64_t kTagPerm = 1, kTagJitter = 2, kTagSrs = 3;

__device__ __forceinline__ uint64_t draw64(uint64_t seed, uint64_t a, uint64_t b, uint64_t c,
                                           uint64_t tag) {
  return philox4x64_10(a, b, c, tag, seed, 0).v[0];
}

// Uniform strictly inside (0,1) from the top 52 bits, centred; exact.
__device__ __forceinline__ double u01(uint64_t x) {
  return ((double)(x >> 12) + 0.5) * 0x1.0p-52;
}

// ---------------------------------------------------------------------------
// Stratum permutation of one LHS row: an 8-round balanced Feistel network on
// 2h bits, cycle-walked into [0, N).  Round r of row i xors the right half
// with the low h bits of the splitmix64 finaliser (Steele, Lea and Flood 2014)
// of R ^ k_{i,r}, where the round keys k_{i,r} are Philox draws keyed on
// (i, r).  A bijection of [0, N) computed per element, so no permutation is
// stored; the eight keys of a row are drawn once per workgroup.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ int feistel_half_bits(int64_t N) {
  int b = 0;
  while (b < 62 && ((int64_t)1 << b) < N) ++b;
  const int h = (b + 1) >> 1;
  return h < 1 ? 1 : h;
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

__device__ __forceinline__ int64_t lhs_stratum(const uint64_t (&key)[8], int64_t N, int h,
                                               int64_t n) {
  const uint64_t mask = (1ULL << h) - 1ULL;
  uint64_t x = (uint64_t)n;
  do {
    uint64_t L = x >> h, R = x & mask;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const uint64_t f = mix64(R ^ key[r]) & mask;
      const uint64_t t = L ^ f;
      L = R;
      R = t;
    }
    x = (L << h) | R;
  } while (x >= (uint64_t)N);
  return (int64_t)x;
}

// ---------------------------------------------------------------------------
// Inverse standard normal CDF, Wichura's AS 241 (PPND16): rational
// approximations of degree 7/7 on the central range |p - 1/2| <= 0.425 and in
// the variable r = sqrt(-log(min(p, 1-p))) on two tail ranges.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double ppnd16(double p) {
  const double q = p - 0.5;
  if (fabs(q) <= 0.425) {
    const double r = 0.180625 - q * q;
    const double num =
        ((((((2.5090809287301226727e+3 * r + 3.3430575583588128105e+4) * r +
             6.7265770927008700853e+4) * r + 4.5921953931549871457e+4) * r +
           1.3731693765509461125e+4) * r + 1.9715909503065514427e+3) * r +
         1.3314166789178437745e+2) * r + 3.3871328727963666080e0;
    const double den =
        ((((((5.2264952788528545610e+3 * r + 2.8729085735721942674e+4) * r +
             3.9307895800092710610e+4) * r + 2.1213794301586595867e+4) * r +
           5.3941960214247511077e+3) * r + 6.8718700749205790830e+2) * r +
         4.2313330701600911252e+1) * r + 1.0;
    return q * (num / den);
  }
  double r = q < 0.0 ? p : 1.0 - p;
  r = sqrt(-log(r));
  double v;
  if (r <= 5.0) {
    r -= 1.6;
    const double num =
        ((((((7.74545014278341407640e-4 * r + 2.27238449892691845833e-2) * r +
             2.41780725177450611770e-1) * r + 1.27045825245236838258e0) * r +
           3.64784832476320460504e0) * r + 5.76949722146069140550e0) * r +
         4.63033784615654529590e0) * r + 1.42343711074968357734e0;
    const double den =
        ((((((1.05075007164441684324e-9 * r + 5.47593808499534494600e-4) * r +
             1.51986665636164571966e-2) * r + 1.48103976427480074590e-1) * r +
           6.89767334985100004550e-1) * r + 1.67638483018380384940e0) * r +
         2.05319162663775882187e0) * r + 1.0;
    v = num / den;
  } else {
    r -= 5.0;
    const double num =
        ((((((2.01033439929228813265e-7 * r + 2.71155556874348757815e-5) * r +
             1.24266094738807843860e-3) * r + 2.65321895265761230930e-2) * r +
           2.96560571828504891230e-1) * r + 1.78482653991729133580e0) * r +
         5.46378491116411436990e0) * r + 6.65790464350110377720e0;
    const double den =
        ((((((2.04426310338993978564e-15 * r + 1.42151175831644588870e-7) * r +
             1.84631831751005468180e-5) * r + 7.86869131145613259100e-4) * r +
           1.48753612908506148525e-2) * r + 1.36929880922735805310e-1) * r +
         5.99832206555887937690e-1) * r + 1.0;
    v = num / den;
  }
  return q < 0.0 ? -v : v;
}

// Probability inside stratum s of N: (s + U)/N, kept below 1.
__device__ __forceinline__ double stratum_prob(int64_t s, double U, int64_t N) {
  double p = ((double)s + U) / (double)N;
  return p >= 1.0 ? 0x1.fffffffffffffp-1 : p;
}

}  // namespace fmc
