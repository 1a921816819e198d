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

// The value of lane j ^ OFF, one 32-bit word.  Partners inside a row of 16
// lanes come through DPP moves (register to register): xor 1 and xor 2 as
// quad permutations [1,0,3,2] and [2,3,0,1], xor 8 as a rotation of the row
// by 8, xor 4 as the half-row mirror (lane i of 8 reads 7 - i) followed by
// the quad reversal [3,2,1,0] (i ^ 3), whose composition reads i ^ 4.  The
// offsets 16 and 32 cross rows and go through ds_bpermute.
template <int OFF>
__device__ __attribute__((always_inline)) inline int lane_xor32(int v) {
  if constexpr (OFF == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
  else if constexpr (OFF == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);
  else if constexpr (OFF == 4)
    return __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false), 0x1B, 0xF, 0xF, false);
  else if constexpr (OFF == 8) return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false);
  else return __shfl_xor(v, OFF, 64);
}
template <int OFF>
__device__ __attribute__((always_inline)) inline float lane_xor(float v) {
  return __builtin_bit_cast(float, lane_xor32<OFF>(__builtin_bit_cast(int, v)));
}
template <int OFF>
__device__ __attribute__((always_inline)) inline double lane_xor(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = lane_xor32<OFF>((int)(uint32_t)u), hi = lane_xor32<OFF>((int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// xor-butterfly fold of 64 lane partial sums: after the offsets 32..1 every
// lane holds the same total; lane j adds its partner j^off at each step (the
// two partners add the same pair, so they stay equal bit for bit).
template <class T>
__device__ inline T wave_fold(T s) {
  s = s + lane_xor<32>(s);
  s = s + lane_xor<16>(s);
  s = s + lane_xor<8>(s);
  s = s + lane_xor<4>(s);
  s = s + lane_xor<2>(s);
  s = s + lane_xor<1>(s);
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

// Iterate recombination (eq. recomb), y = x + sum_i alpha_i (X_i - x) over
// th <= 2 saved iterates.  With D_i = X_i - x and d_i = R_i - r = -A D_i, the
// six running sums of one element are, for
//   norm 0 (the residual 2-norm, as printed): d0.d0, d0.d1, d1.d1, d0.r, d1.r, r.r
//   norm 1 (the energy norm of the error):   -D0.d0, -D0.d1, -D1.d1, -D0.r, -D1.r, -D1.d0
// so that in both cases alpha solves G alpha = -g with G from the first three
// (norm 1: the off-diagonal averaged over its two products) and g from the
// next two.
template <class T>
__device__ inline void recomb_terms(int norm, int th, T ru, T R0, T R1, T xu, T X0, T X1, double (&v)[6]) {
  const double r = (double)ru;
  const double d0 = (double)(R0 - ru);
  const double d1 = th > 1 ? (double)(R1 - ru) : 0.0;
  if (norm == 0) {
    v[0] += d0 * d0; v[1] += d0 * d1; v[2] += d1 * d1; v[3] += d0 * r; v[4] += d1 * r; v[5] += r * r;
  } else {
    const double e0 = (double)(X0 - xu);
    const double e1 = th > 1 ? (double)(X1 - xu) : 0.0;
    v[0] += -(e0 * d0); v[1] += -(e0 * d1); v[2] += -(e1 * d1); v[3] += -(e0 * r); v[4] += -(e1 * r);
    v[5] += -(e1 * d0);
  }
}
// The th x th normal equations from the six totals; a direction is dropped
// (alpha_i = 0) when its Gram entry is not above 1e-28 r.r (norm 0) or 0
// (norm 1), or when the 2 x 2 determinant is at most 1e-12 G00 G11.
__host__ __device__ inline void recomb_alpha(int norm, int th, const double (&t)[6], double* a0, double* a1) {
  const double G00 = t[0], G11 = t[2], g0 = t[3], g1 = t[4];
  const double G01 = norm == 0 ? t[1] : 0.5 * (t[1] + t[5]);
  const double tiny = norm == 0 ? 1e-28 * t[5] : 0.0;
  *a0 = 0;
  *a1 = 0;
  if (th == 1) {
    if (G00 > tiny) *a0 = -g0 / G00;
    return;
  }
  const double det = G00 * G11 - G01 * G01;
  if (G00 > tiny && G11 > tiny && det > 1e-12 * G00 * G11) {
    *a0 = (-g0 * G11 + g1 * G01) / det;
    *a1 = (-g1 * G00 + g0 * G01) / det;
  } else if (G00 >= G11) {
    if (G00 > tiny) *a0 = -g0 / G00;
  } else {
    if (G11 > tiny) *a1 = -g1 / G11;
  }
}

}  // namespace dev
}  // namespace lamg
