// Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11): ten rounds of the 4x64 Philox bijection with the
// published multipliers and Weyl key increments.  Shared by the sampler and
// the fused DEANN value-and-gradient pass, which draw the same rows.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace deann {

struct Philox4x64 {
  uint64_t v[4];
};

__device__ __forceinline__ Philox4x64 philox4x64_10(uint64_t k0, uint64_t k1, uint64_t c0,
                                                    uint64_t c1, uint64_t c2, uint64_t c3) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  Philox4x64 o;
  o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
  return o;
}

// The r-th smallest row of X2 = X minus the k neighbours: r + #{t : gaps[t]
// <= r}, gaps[t] = nn_t - t over the neighbours sorted ascending
// (non-decreasing).
__device__ __forceinline__ int64_t rank_to_row(uint64_t r, const int32_t* __restrict__ gaps,
                                               int64_t k) {
  int64_t lo = 0, hi = k;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((uint64_t)(int64_t)gaps[mid] <= r) lo = mid + 1; else hi = mid;
  }
  return (int64_t)(r + (uint64_t)lo);
}

// A draw with repetition from X2 (n - k = size2 rows): the rank
// floor(word size2 / 2^64) of a uniform 64-bit word.
__device__ __forceinline__ int64_t draw_row(uint64_t word, uint64_t size2,
                                            const int32_t* __restrict__ gaps, int64_t k) {
  return rank_to_row(__umul64hi(word, size2), gaps, k);
}

}  // namespace deann
