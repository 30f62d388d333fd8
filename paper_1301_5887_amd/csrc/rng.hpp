// Device random numbers of the sampler.
//
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11): ten rounds of two 64x64->128 multiplies with a Weyl
// key schedule.  Uniform integers on [0, N) by Lemire's nearly-divisionless
// method (ACM TOMACS 2019): accept high64(x*N) unless low64(x*N) falls below
// 2^64 mod N, in which case the same word of the next retry round is used.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wedge {

struct U64x4 {
  uint64_t w[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
    const uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  return U64x4{{c0, c1, c2, c3}};
}

// Key domains (the key's second word): 1 plain sampling; 2, 3, 4 the
// training, auxiliary and evaluation streams of the control variate.
constexpr uint64_t kDomainSample = 1;

// Finish a uniform-below draw whose round-0 word was x: accept or walk the
// retry rounds of word t for counter (s, bword, g) under key (seed, domain).
__device__ __forceinline__ uint64_t below_from(uint64_t x, uint64_t N, uint64_t seed,
                                               uint64_t domain, uint64_t s, uint64_t bword,
                                               uint64_t g, int t) {
  uint64_t lo = x * N;
  if (lo < N) {
    const uint64_t thr = (0 - N) % N;
    uint64_t r = 0;
    while (lo < thr) {
      ++r;
      U64x4 o = philox4x64_10(s, bword, g, r, seed, domain);
      x = o.w[t];
      lo = x * N;
    }
  }
  return __umul64hi(x, N);
}

}  // namespace wedge
