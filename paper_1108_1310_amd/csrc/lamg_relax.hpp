// The relaxation kernel (multicolour Gauss-Seidel, residual and elimination
// restriction over tiled CSR rows).  Kept in a file of its own: the recorded
// HBM traffic of this kernel is tied to this file's contents and to those of
// the device helpers it inlines (lamg_device.hpp).
#pragma once
#include "lamg_device.hpp"
#include "lamg_internal.hpp"

namespace lamg {

// Relaxation work list of one colour class (or of all rows), as three kinds
// of 512-thread blocks launched together, longest work first:
//   very long rows (> ROW_CHUNK entries): one block per row, its 512-entry
//     chunks spread over the 8 wavefronts;
//   medium rows (65..ROW_CHUNK entries): one wavefront per row, 8 rows per
//     block;
//   stream tiles: up to TILE_ROWS consecutive short rows whose entries fit in
//     TILE_NNZ products staged in LDS, one thread per row for the sums.
// Measured on the Chung-Lu 2^20 FP64 solve (threads / tile entries, ms per
// solve): 512 / 4096 26.2, 512 / 2048 24.8, 512 / 1024 23.7, 512 / 512 24.0,
// 256 / 2048 24.9, 256 / 1024 24.2, 128 / 1024 26.3, 1024 / 1024 30.5,
// 1024 / 4096 30.1; RGG 2^20: 176.0, 167.6, 161.1, 159.9, 168.0, 163.1,
// 164.1, 163.6, 177.3.  Small tiles give more blocks per colour class and
// fewer dependent loads per thread; the long rows want 8 wavefronts.
constexpr int RELAX_THREADS = 512;
constexpr int TILE_ROWS = 512;
constexpr int TILE_NNZ = 1024;
constexpr int LONG_PER_BLOCK = RELAX_THREADS / 64;

// One pass over a set of rows of a colour-ordered level.
//   MODE 0: Gauss-Seidel update x_u <- (b_u + sum_v w_uv x_v) / a_uu (eq. gs)
//   MODE 1: residual r_u <- (b_u + sum_v w_uv x_v) - a_uu x_u
// Stream blocks stage the products w_uv * x_v of up to TILE_NNZ entries of
// consecutive short rows in LDS with coalesced loads, then one thread per row
// sums them left to right.  Long-row blocks give each row a wavefront that
// sums with stride 64 and folds with an xor butterfly.  A GS pass only ever
// covers one colour class, whose rows are pairwise non-adjacent, so the rows
// it writes are never read in the same launch.
// MODE 0: GS update; MODE 1: residual; MODE 2: elimination restriction
// out_u = x_{map(u)} + sum (the gathered vector is the fine residual).
// zthr: the gathered vector is known to hold +0 at every index >= zthr (the
// first sweep after a zero fill: colours at or above the current one are
// untouched), so those entries take the constant +0 instead of a load.  The
// product w * (+0) and its place in the sum are unchanged, so the result is
// bitwise the same; only the gathers are saved.  INT_MAX: gather every entry.
// The per-row operands are loaded as soon as the row is known (relax_pre),
// so that their latency overlaps the gathers; none of them is written in
// the same launch (a GS pass writes only x of its own colour, which it does
// not read for its own rows).
template <class T>
struct RowOps {
  T a, d;  // MODE 0: b_u, a_uu; MODE 1: b_u - a_uu x_u; MODE 2: x_{map(u)}
};
template <class T, int MODE>
__device__ inline RowOps<T> relax_pre(int u, const T* __restrict__ diag, const T* __restrict__ b, const T* x,
                                      const int* __restrict__ map) {
  RowOps<T> o;
  if (MODE == 2) {
    o.a = x[map[u]];
    o.d = T(0);
    return o;
  }
  o.a = b ? b[u] : T(0);
  o.d = diag[u];
  if (MODE == 1) o.d *= x[u];
  return o;
}
template <class T, int MODE>
__device__ inline void relax_store(int u, T s, RowOps<T> o, T* x, T* __restrict__ r) {
  if (MODE == 2) r[u] = o.a + s;
  else if (MODE == 0) x[u] = (o.a + s) / o.d;
  else r[u] = (o.a + s) - o.d;
}

// One 512-entry chunk of a long row, one wavefront: lane j sums the chunk's
// entries j, j+64, ... left to right (all loads issued before the gathers),
// then the butterfly folds the 64 partials.
template <class T>
__device__ inline T chunk_sum(const int* __restrict__ ci, const T* __restrict__ val, const T* x, int p0, int c0,
                              int len, int lane, int zthr) {
  constexpr int UNR = ROW_CHUNK / 64;
  int cj[UNR];
  T wj[UNR], xj[UNR];
#pragma unroll
  for (int q = 0; q < UNR; ++q) {
    const int t = c0 + lane + 64 * q;
    cj[q] = t < len ? ci[p0 + t] : 0;
    wj[q] = t < len ? val[p0 + t] : T(0);
  }
#pragma unroll
  for (int q = 0; q < UNR; ++q) xj[q] = cj[q] < zthr ? x[cj[q]] : T(0);
  T s = 0;
#pragma unroll
  for (int q = 0; q < UNR; ++q)
    if (c0 + lane + 64 * q < len) s += wj[q] * xj[q];
  return dev::wave_fold(s);
}

template <class T, int MODE>
__global__ __launch_bounds__(RELAX_THREADS) void k_relax(
    const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ val,
    const T* __restrict__ diag, const T* __restrict__ b, T* x, T* __restrict__ r,
    const int4* __restrict__ vlong, int nvlong, const int4* __restrict__ med, int nmed, int nmed_blocks,
    const int4* __restrict__ sblk, int nstream, const int* __restrict__ map, int zthr) {
  constexpr int PER = TILE_NNZ / RELAX_THREADS;  // entries per thread in a stream tile
  constexpr int MAXC = 64;                       // chunk sums staged per pass
  __shared__ T prod[TILE_NNZ];
  __shared__ int srp[TILE_ROWS + 1];
  __shared__ T csum[MAXC];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int bid = blockIdx.x;
  if (bid < nvlong) {
    // a very long row: chunks k = wv, wv+4, ... per pass; chunk sums added in order
    const int4 e = vlong[bid];  // (row, first entry, entries)
    const int u = e.x, p0 = e.y, len = e.z;
    const int nch = (len + ROW_CHUNK - 1) / ROW_CHUNK;
    RowOps<T> o{};
    if (threadIdx.x == 0) o = relax_pre<T, MODE>(u, diag, b, x, map);
    T total = 0;
    for (int pass = 0; pass < nch; pass += MAXC) {
      const int lim = min(MAXC, nch - pass);
      for (int k = wv; k < lim; k += LONG_PER_BLOCK) {
        const T sk = chunk_sum<T>(ci, val, x, p0, (pass + k) * ROW_CHUNK, len, lane, zthr);
        if (lane == 0) csum[k] = sk;
      }
      __syncthreads();
      if (threadIdx.x == 0)
        for (int k = 0; k < lim; ++k) total += csum[k];
      __syncthreads();
    }
    if (threadIdx.x == 0) relax_store<T, MODE>(u, total, o, x, r);
    return;
  }
  bid -= nvlong;
  if (bid < nmed_blocks) {
    const int idx = bid * LONG_PER_BLOCK + wv;
    if (idx >= nmed) return;
    const int4 e = med[idx];
    const int u = e.x, p0 = e.y, len = e.z;
    RowOps<T> o{};
    if (lane == 0) o = relax_pre<T, MODE>(u, diag, b, x, map);
    const T sk = chunk_sum<T>(ci, val, x, p0, 0, len, lane, zthr);
    T total = 0;
    total += sk;
    if (lane == 0) relax_store<T, MODE>(u, total, o, x, r);
    return;
  }
  bid -= nmed_blocks;
  const int4 rr = sblk[bid];  // (first row, end row, first entry, entries)
  const int nr = rr.y - rr.x;
  const int base = rr.z, cnt = rr.w;
  // the row pointers go to LDS while the index and weight loads are in
  // flight; then all gathers: PER loads in flight per thread
  for (int i = threadIdx.x; i <= nr; i += RELAX_THREADS) srp[i] = rp[rr.x + i];
  RowOps<T> o{};
  if (threadIdx.x < nr) o = relax_pre<T, MODE>(rr.x + threadIdx.x, diag, b, x, map);
  int cj[PER];
  T wj[PER], xj[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = threadIdx.x + q * RELAX_THREADS;
    cj[q] = j < cnt ? ci[base + j] : 0;
    wj[q] = j < cnt ? val[base + j] : T(0);
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) xj[q] = cj[q] < zthr ? x[cj[q]] : T(0);
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = threadIdx.x + q * RELAX_THREADS;
    if (j < cnt) prod[j] = wj[q] * xj[q];
  }
  __syncthreads();
  if (threadIdx.x < nr) {
    const int j1 = srp[threadIdx.x + 1] - base;
    T s = 0;
    for (int j = srp[threadIdx.x] - base; j < j1; ++j) s += prod[j];
    relax_store<T, MODE>(rr.x + threadIdx.x, s, o, x, r);
  }
}

}  // namespace lamg
