// Device helpers shared by the LAMG kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lamg {
namespace dev {

// splitmix64 finaliser of x + golden gamma (Steele, Lea & Flood 2014), used
// as a counter-based hash.
__device__ __host__ inline uint64_t sm64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
__device__ __host__ inline uint64_t hash5(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b, uint64_t c) {
  uint64_t h = sm64(seed);
  h = sm64(h ^ stream);
  h = sm64(h ^ a);
  h = sm64(h ^ b);
  return sm64(h ^ c);
}
// U[-1,1): the top 53 bits times 2^-52, minus one; exact in binary64.
__device__ __host__ inline double unit_pm1(uint64_t h) {
  return (double)(h >> 11) * (1.0 / 4503599627370496.0) - 1.0;
}

// xor-butterfly fold of 64 lane partial sums: after the offsets 32..1 every
// lane holds the same total; lane j adds its partner j^off at each step.
template <class T>
__device__ inline T wave_fold(T s) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s = s + __shfl_xor(s, off, 64);
  return s;
}

// Row reduction in the fixed order: a single thread sums a short row
// (<= 64 terms) left to right.
template <class T, class F>
__device__ inline T row_sum_seq(int len, F term) {
  T s = 0;
  for (int t = 0; t < len; ++t) s += term(t);
  return s;
}
// Long rows (> 64 terms), one wavefront: chunks of CHUNK consecutive terms;
// in each chunk lane j sums terms j, j+64, ... left to right, the butterfly
// folds the chunk, and chunk sums are added left to right.
constexpr int CHUNK = 512;
template <class T, class F>
__device__ inline T row_sum_wave(int len, int lane, F term) {
  T total = 0;
  for (int c0 = 0; c0 < len; c0 += CHUNK) {
    T s = 0;
#pragma unroll
    for (int q = 0; q < CHUNK / 64; ++q) {
      const int t = c0 + lane + 64 * q;
      if (t < len) s += term(t);
    }
    total += wave_fold(s);
  }
  return total;
}

}  // namespace dev
}  // namespace lamg
