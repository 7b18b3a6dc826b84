// Device helpers of the entropy stage (Sec. 3.2, Eq. 12).
//
// The per-displacement sums use S = sum c log2 c over integer counts; with
// N = sum of the joint counts, Eq. 12 and Eq. 2 give
//   MI = log2 N + (S_AB - S_A - S_B) / N,
// which equals H_A + H_B - H_AB exactly (the relative frequencies c/N have
// log2(c/N) = log2 c - log2 N and the counts of each histogram sum to N).
//
// log2 of a count is evaluated in FP64 without a library call: with
// c = 2^e (1 + f), j = the top 8 bits of f and m_j = 1 + j/256,
//   log2 c = e + log2 m_j + ln(1 + r) / ln 2,  r = (1 + f - m_j) / m_j,
// where 0 <= r < 2^-8 and ln(1 + r) is summed to r^6 (truncation below
// 1e-17).  log2 m_j and 1/m_j come from a 512-entry FP64 table.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cmif {

__device__ __forceinline__ double log2_u32(uint32_t n, const double* tab) {
  const int e = 31 - __clz((int)n);
  const uint32_t j = e >= 8 ? (n >> (e - 8)) & 0xFFu : (n << (8 - e)) & 0xFFu;
  const double m = ldexp((double)n, -e);
  const double mj = 1.0 + (double)j * (1.0 / 256.0);
  const double r = (m - mj) * tab[256 + j];
  double p = -1.0 / 6.0;
  p = fma(p, r, 1.0 / 5.0);
  p = fma(p, r, -1.0 / 4.0);
  p = fma(p, r, 1.0 / 3.0);
  p = fma(p, r, -1.0 / 2.0);
  p = fma(p, r, 1.0);
  const double ln1p = p * r;
  return ((double)e + tab[j]) + ln1p * 1.4426950408889634074;
}

// c log2 c with 0 log 0 = 0 (and 1 log 1 = 0)
__device__ __forceinline__ double xlog2x_u32(uint32_t n, const double* tab) {
  return n <= 1u ? 0.0 : (double)n * log2_u32(n, tab);
}

// Vigna's splitmix64 output function applied to a counter.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

}  // namespace cmif
