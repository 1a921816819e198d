// Stable LSD radix sort and exclusive scan for the setup's sparse assembly
// (Galerkin and Schur products summed by key, colour-major renumbering,
// aggregate member lists, the stage-1 affinity quantile).  Integer work only,
// so the results are exact and independent of the launch shape.
//
// Sort: 8-bit digits from bit 0 up to the caller's end bit.  Each pass is a
// per-tile digit histogram, an exclusive scan of the histograms in digit-major
// order (so tile b's digit d lands after every digit < d and after digit d of
// tiles < b), and a scatter in which each element's rank among the equal
// digits of its tile comes from wavefront ballots (stable: tile order is
// round-major, then wavefront, then lane, i.e. element order).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <type_traits>

#include "lamg_internal.hpp"

namespace lamg {
namespace sortk {
// internal linkage: each translation unit that sorts holds its own kernels
namespace {

constexpr int RS_THREADS = 256;                   // 4 wavefronts
constexpr int RS_WAVES = RS_THREADS / 64;
constexpr int RS_ROUNDS = 16;                     // rounds of RS_THREADS elements per tile
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;   // 4096 elements per tile
constexpr int RS_BINS = 256;
constexpr int SC_THREADS = 256;
constexpr int SC_ITEMS = 8;
constexpr int SC_TILE = SC_THREADS * SC_ITEMS;    // 2048 elements per scan block

// Keys as unsigned integers whose order is the sort order.  Doubles: the sign
// bit set flips every bit, else the sign bit alone is set (ascending order,
// -0 before +0).
template <class K>
struct KeyBits {
  using U = K;
  __device__ static U enc(K k) { return k; }
  __device__ static K dec(U u) { return u; }
};
template <>
struct KeyBits<double> {
  using U = uint64_t;
  __device__ static U enc(double k) {
    const U u = (U)__double_as_longlong(k);
    return (u >> 63) ? ~u : (u | (1ull << 63));
  }
  __device__ static double dec(U u) {
    return __longlong_as_double((long long)((u >> 63) ? (u & ~(1ull << 63)) : ~u));
  }
};

struct NoVal {};

// counts[d * ntiles + tile] = elements of the tile whose digit is d (ENC:
// the keys are raw and encoded here, on the first pass)
template <class K, bool ENC>
__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const K* __restrict__ kin, int64_t n, int shift,
                                                        int* __restrict__ counts, int ntiles) {
  __shared__ int h[RS_BINS];
  for (int d = threadIdx.x; d < RS_BINS; d += RS_THREADS) h[d] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = base + (int64_t)r * RS_THREADS + threadIdx.x;
    if (i < n) {
      typename KeyBits<K>::U u;
      if constexpr (ENC) u = KeyBits<K>::enc(kin[i]);
      else u = kin[i];
      atomicAdd(&h[(int)((u >> shift) & (RS_BINS - 1))], 1);
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < RS_BINS; d += RS_THREADS) counts[(int64_t)d * ntiles + blockIdx.x] = h[d];
}

// Scatter of one pass.  kin holds encoded keys except on the first pass
// (pass0: raw keys, encoded here); the last pass (last) decodes on the way out.
template <class K, class V>
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const void* __restrict__ kin_, const V* __restrict__ vin,
                                                           void* __restrict__ kout_, V* __restrict__ vout, int64_t n,
                                                           int shift, int pass0, int last,
                                                           const int* __restrict__ offs, int ntiles) {
  using U = typename KeyBits<K>::U;
  constexpr bool HAS_V = !std::is_same<V, NoVal>::value;
  __shared__ int run[RS_BINS];
  __shared__ int wc[RS_WAVES][RS_BINS];
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  for (int d = tid; d < RS_BINS; d += RS_THREADS) run[d] = offs[(int64_t)d * ntiles + blockIdx.x];
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    for (int w = 0; w < RS_WAVES; ++w) wc[w][tid] = 0;  // RS_THREADS == RS_BINS
    __syncthreads();
    const int64_t i = base + (int64_t)r * RS_THREADS + tid;
    const bool in = i < n;
    U u = 0;
    if (in) u = pass0 ? KeyBits<K>::enc(((const K*)kin_)[i]) : ((const U*)kin_)[i];
    const int d = (int)((u >> shift) & (RS_BINS - 1));
    // lanes of this wavefront holding the same digit
    uint64_t same = __ballot(in);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bb = __ballot((d >> b) & 1);
      same &= ((d >> b) & 1) ? bb : ~bb;
    }
    const int rank = __popcll(same & lt);
    if (in && rank == 0) wc[wv][d] = __popcll(same);
    __syncthreads();
    {  // digit tid: wavefront offsets within the round, then the running offset
      int o = run[tid];
#pragma unroll
      for (int w = 0; w < RS_WAVES; ++w) {
        const int t = wc[w][tid];
        wc[w][tid] = o;
        o += t;
      }
      run[tid] = o;
    }
    __syncthreads();
    if (in) {
      const int p = wc[wv][d] + rank;
      if (last) ((K*)kout_)[p] = KeyBits<K>::dec(u);
      else ((U*)kout_)[p] = u;
      if constexpr (HAS_V) vout[p] = vin[i];
    }
    __syncthreads();
  }
}

// Exclusive scan of m = n + 1 ints (element n reads as 0): block sums, the
// scan of the block sums (recursively), then each block's scan plus offset.
__device__ inline int scan_in(const int* in, int64_t n, int64_t i) { return i < n ? in[i] : 0; }
__global__ __launch_bounds__(SC_THREADS) void k_scan_sums(const int* __restrict__ in, int64_t n, int* __restrict__ bs) {
  __shared__ int sh[SC_THREADS / 64];
  const int64_t b0 = (int64_t)blockIdx.x * SC_TILE;
  int s = 0;
  for (int q = 0; q < SC_ITEMS; ++q) {
    const int64_t i = b0 + (int64_t)q * SC_THREADS + threadIdx.x;
    if (i <= n) s += scan_in(in, n, i);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < SC_THREADS / 64; ++w) t += sh[w];
    bs[blockIdx.x] = t;
  }
}
// out[i] = boff[block] + sum of in[j] for block's j < i (exclusive)
__global__ __launch_bounds__(SC_THREADS) void k_scan_apply(const int* __restrict__ in, int64_t n,
                                                           const int* __restrict__ boff, int* __restrict__ out) {
  __shared__ int sh[SC_THREADS / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t b0 = (int64_t)blockIdx.x * SC_TILE + (int64_t)tid * SC_ITEMS;
  int v[SC_ITEMS];
  int s = 0;
#pragma unroll
  for (int q = 0; q < SC_ITEMS; ++q) {
    const int64_t i = b0 + q;
    v[q] = i <= n ? scan_in(in, n, i) : 0;
    s += v[q];
  }
  // inclusive scan of the thread sums within the wavefront
  int inc = s;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(inc, off, 64);
    if (lane >= off) inc += t;
  }
  if (lane == 63) sh[wv] = inc;
  __syncthreads();
  int before = boff ? boff[blockIdx.x] : 0;
  for (int w = 0; w < wv; ++w) before += sh[w];
  int o = before + inc - s;
#pragma unroll
  for (int q = 0; q < SC_ITEMS; ++q) {
    const int64_t i = b0 + q;
    if (i <= n) out[i] = o;
    o += v[q];
  }
}


// Scratch ints needed by exclusive_scan for n inputs (the block sums of
// every recursion level and their scans).
inline size_t scan_scratch(int64_t n) {
  size_t t = 0;
  int64_t m = n + 1;
  while (m > SC_TILE) {
    const int64_t nb = (m + SC_TILE - 1) / SC_TILE;
    t += 2 * (size_t)(nb + 1);
    m = nb + 1;
  }
  return t + 1;
}
// out[0..n]: out[0] = 0, out[i + 1] = in[0] + ... + in[i]
inline void exclusive_scan(hipStream_t s, const int* in, int* out, int64_t n, int* scratch) {
  const int64_t m = n + 1;
  const int64_t nb = (m + SC_TILE - 1) / SC_TILE;
  if (nb <= 1) {
    hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(SC_THREADS), 0, s, in, n, (const int*)nullptr, out);
    return;
  }
  int* bs = scratch;
  int* bo = scratch + nb + 1;
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(SC_THREADS), 0, s, in, n, bs);
  exclusive_scan(s, bs, bo, nb, scratch + 2 * (nb + 1));
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(SC_THREADS), 0, s, in, n, (const int*)bo, out);
}

// Temporary bytes of radix_sort for n elements (keys and values of one
// ping-pong buffer, the histograms and their scan).
template <class K, class V>
inline size_t sort_scratch_bytes(int64_t n) {
  const int64_t nt = (n + RS_TILE - 1) / RS_TILE;
  const int64_t nc = nt * RS_BINS;
  size_t b = 0;
  b += ((size_t)n * sizeof(typename KeyBits<K>::U) + 255) & ~(size_t)255;
  if (!std::is_same<V, NoVal>::value) b += ((size_t)n * sizeof(V) + 255) & ~(size_t)255;
  b += (((size_t)nc + 1) * sizeof(int) + 255) & ~(size_t)255;
  b += (((size_t)nc + 1) * sizeof(int) + 255) & ~(size_t)255;
  b += (scan_scratch(nc) * sizeof(int) + 255) & ~(size_t)255;
  return b;
}
// Stable ascending sort of (key, value) pairs by the key bits [0, endbit)
// (all bits of a double key).  kin / vin are not modified; kout / vout
// receive the result and must not overlap them.  V = NoVal: keys only.
template <class K, class V>
inline void radix_sort(hipStream_t s, const K* kin, K* kout, const V* vin, V* vout, int64_t n, unsigned endbit,
                       void* scratch) {
  using U = typename KeyBits<K>::U;
  constexpr bool HAS_V = !std::is_same<V, NoVal>::value;
  static_assert(sizeof(U) == sizeof(K), "keys as unsigned words of their size");
  if (n <= 0) return;
  const int ntiles = (int)((n + RS_TILE - 1) / RS_TILE);
  const int64_t nc = (int64_t)ntiles * RS_BINS;
  char* p = (char*)scratch;
  auto take = [&](size_t bytes) {
    char* q = p;
    p += (bytes + 255) & ~(size_t)255;
    return (void*)q;
  };
  U* kb = (U*)take((size_t)n * sizeof(U));
  V* vb = HAS_V ? (V*)take((size_t)n * sizeof(V)) : nullptr;
  int* counts = (int*)take(((size_t)nc + 1) * sizeof(int));
  int* offs = (int*)take(((size_t)nc + 1) * sizeof(int));
  int* sscr = (int*)take(scan_scratch(nc) * sizeof(int));
  const int passes = (int)((endbit + 7) / 8);
  // destinations alternate so that the last pass writes kout / vout
  for (int ps = 0; ps < passes; ++ps) {
    const bool last = ps == passes - 1;
    const bool to_out = ((passes - 1 - ps) % 2) == 0;
    const void* ksrc = ps == 0 ? (const void*)kin : (to_out ? (const void*)kb : (const void*)kout);
    const V* vsrc = ps == 0 ? vin : (to_out ? vb : vout);
    void* kdst = to_out ? (void*)kout : (void*)kb;
    V* vdst = to_out ? vout : vb;
    const int shift = 8 * ps;
    if (ps == 0)
      hipLaunchKernelGGL((k_rs_hist<K, true>), dim3(ntiles), dim3(RS_THREADS), 0, s, kin, n, shift, counts, ntiles);
    else
      hipLaunchKernelGGL((k_rs_hist<U, false>), dim3(ntiles), dim3(RS_THREADS), 0, s, (const U*)ksrc, n, shift,
                         counts, ntiles);
    exclusive_scan(s, counts, offs, nc, sscr);
    hipLaunchKernelGGL((k_rs_scatter<K, V>), dim3(ntiles), dim3(RS_THREADS), 0, s, ksrc, vsrc, kdst, vdst, n, shift,
                       ps == 0 ? 1 : 0, last ? 1 : 0, (const int*)offs, ntiles);
  }
}

}  // namespace
}  // namespace sortk
}  // namespace lamg
