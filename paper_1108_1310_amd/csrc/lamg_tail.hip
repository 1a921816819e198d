// Single-workgroup tail of the cycle (Section 4.2 cycles on the small coarse
// levels).  The coarse levels are visited many times per finest cycle
// (fractional cycle index, eq. cycle_index) but hold few nodes, so one launch
// per colour pass would be dominated by launch latency.  Instead, every entry
// into level tail_lc runs one workgroup (512 threads in FP64, 1024 in FP32)
// that executes a precomputed op program (the same relaxations, transfers,
// recombinations and coarsest solves the multi-launch path performs, in the
// same order), with a workgroup barrier between ops.  Sums keep the fixed order of the other
// kernels: short rows left to right by one thread, long rows (> 64 entries)
// by one wavefront in 512-entry chunks.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lamg_device.hpp"
#include "lamg_internal.hpp"

namespace lamg {

namespace {

// The largest workgroup of the kernels of this file (k_batch launches it):
// it sizes the wavefront-sum scratch sh[..][TAIL_WAVES] and the launch
// bounds.  A launch larger than this would write past that scratch.
constexpr int TAIL_THREADS = 1024;
constexpr int TAIL_WAVES = TAIL_THREADS / 64;
static_assert(TAIL_WAVES * 64 == TAIL_THREADS, "whole wavefronts");
// Launch size (and launch bound) of the single-workgroup tail k_tail, per
// precision.  At 512 threads the FP64 interpreter gets up to 256 VGPRs
// instead of 128 (248 used; private scratch 92 instead of 228 bytes per
// lane), which outweighs the halved thread count; the FP32 one does not
// gain.  Measured on one box, 1024 threads for both / FP64 at 512 / both at
// 512: RGG 2^20 FP64 189.3 / 185.5 / 185.5 ms per solve, FP32 158.5 / 158.2 /
// 167.3 ms, 64^2 grid 5.91 / 5.17 / 5.17 ms, 64^3 anisotropic grid 587 / 556
// / 556 ms, geometric multigrid 1024^2 9.09 / 8.51 / 8.51 ms, 8 columns on
// the 64^3 grid FP64 677 / 648 / 648 ms, FP32 607 / 607 / 628 ms.
template <class T>
constexpr int tail_launch() { return sizeof(T) == 8 ? 512 : 1024; }
static_assert(tail_launch<double>() % 64 == 0 && tail_launch<float>() % 64 == 0, "whole wavefronts");
static_assert(tail_launch<double>() <= TAIL_THREADS && tail_launch<float>() <= TAIL_THREADS, "within the scratch");
// Every stride and wavefront count of the interpreter comes from the
// launch; TAIL_THREADS / TAIL_WAVES only bound it (launch bounds, the size
// of the wavefront-sum scratch).
__device__ __attribute__((always_inline)) inline int tail_nt() { return (int)blockDim.x; }
__device__ __attribute__((always_inline)) inline int tail_nw() { return (int)(blockDim.x >> 6); }

enum TailOp {
  OP_GS = 1,      // a = multicolour sweeps of level l (one staging for all)
  OP_IAGG = 6,    // x_l += P x_{l+1}
  OP_IELIM = 8,   // x_l += exact elimination correction from x_{l+1}
  OP_RECOMB = 9,  // iterate recombination over a = theta sub-cycles
  OP_COARSE = 10, // coarsest solve of level l
  OP_MEAN = 11,   // x_l -= mean(x_l)
  OP_RRAGG = 12,  // fused: residual into src(a), X[sub] = x when a > 0, b_{l+1} = mu^(b) P^T src, x_{l+1} = 0
  OP_RRELIM = 13, // fused: r = residual, b_{l+1} = elimination restriction of r, x_{l+1} = 0
  OP_IGS = 14,    // fused: x_l += P x_{l+1}, then a = multicolour sweeps of level l
};

struct TailParams {
  const TailLevel* L;
  int lc;
  const double* Minv;
  int nL, crelax, csweeps;
  double mu;
  int kc;         // columns of the vector blocks (multi-vector form; 1 otherwise)
  int lds_bytes;  // dynamic LDS of the launch
  int res_bytes;  // of which at most this much holds LDS-resident levels
  int nlev;       // levels lc .. lc + nlev - 1 in the program
  int rnorm;      // norm iterate recombination minimises (0 residual, 1 energy)
};

template <class T> struct TV;
template <> struct TV<double> {
  __device__ static const double* val(const TailLevel& L) { return L.val64; }
  __device__ static const double* diag(const TailLevel& L) { return L.diag64; }
  __device__ static const double* er(const TailLevel& L) { return L.er64; }
  __device__ static double* x(const TailLevel& L) { return L.x64; }
  __device__ static double* b(const TailLevel& L) { return L.b64; }
  __device__ static double* r(const TailLevel& L) { return L.r64; }
  __device__ static double* X(const TailLevel& L, int i) { return L.X64[i]; }
  __device__ static double* R(const TailLevel& L, int i) { return L.R64[i]; }
};
template <> struct TV<float> {
  __device__ static const float* val(const TailLevel& L) { return L.val32; }
  __device__ static const float* diag(const TailLevel& L) { return L.diag32; }
  __device__ static const float* er(const TailLevel& L) { return L.er32; }
  __device__ static float* x(const TailLevel& L) { return L.x32; }
  __device__ static float* b(const TailLevel& L) { return L.b32; }
  __device__ static float* r(const TailLevel& L) { return L.r32; }
  __device__ static float* X(const TailLevel& L, int i) { return L.X32[i]; }
  __device__ static float* R(const TailLevel& L, int i) { return L.R32[i]; }
};

// One column of an n x k row-major block: element i at p[i * k].  With
// MV = false the stride is the compile-time constant 1 (a plain vector).
template <class T, bool MV>
struct Col {
  T* p;
  int k;
  __device__ __attribute__((always_inline)) T& operator[](int i) const {
    if constexpr (MV) return p[i * k];
    else return p[i];
  }
};
template <bool MV>
struct ColOf {
  int j, k;  // column index and stride
  // column j of level L's vector p: strided in global memory, or (for a
  // level whose arrays sit in LDS) this workgroup's contiguous copy
  template <class T>
  __device__ __attribute__((always_inline)) Col<T, MV> v(const TailLevel& L, T* p) const {
    if constexpr (MV) return L.vres ? Col<T, MV>{p, 1} : Col<T, MV>{p + j, k};
    else return Col<T, MV>{p, 1};
  }
};

// Pointer into LDS (address space 3): loads through it are ds_read.
template <class T>
using LP = __attribute__((address_space(3))) T*;

// Sum of a row against vector v, left to right; the index and weight loads of
// 8 entries are issued before their 8 gathers (arrays in global memory or LDS).
template <class T, class VP, class IP, class V>
__device__ __attribute__((always_inline)) inline T row_seq_p(VP val, IP ci, int p0, int len, V v) {
  T s = 0;
  for (int t0 = 0; t0 < len; t0 += 8) {
    int cj[8];
    T wj[8], xj[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int t = t0 + q;
      cj[q] = t < len ? ci[p0 + t] : 0;
      wj[q] = t < len ? val[p0 + t] : T(0);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) xj[q] = v[cj[q]];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (t0 + q < len) s += wj[q] * xj[q];
  }
  return s;
}
template <class T, class V>
__device__ __attribute__((always_inline)) inline T row_seq(const TailLevel& L, int p0, int len, V v) {
  return row_seq_p<T>(TV<T>::val(L), L.ci, p0, len, v);
}
template <class T, class V>
__device__ __attribute__((always_inline)) inline T row_short(const TailLevel& L, int u, V v) {
  const int p0 = L.rp[u];
  return row_seq<T>(L, p0, L.rp[u + 1] - p0, v);
}
template <class T, class V>
__device__ __attribute__((always_inline)) inline T row_long(const TailLevel& L, int u, V v, int lane) {
  const int p0 = L.rp[u], len = L.rp[u + 1] - p0;
  const T* val = TV<T>::val(L);
  return dev::row_sum_wave<T>(len, lane, [&](int t) { return val[p0 + t] * v[L.ci[p0 + t]]; });
}

// One multicolour GS sweep: short rows one per thread, long rows one per
// wavefront, a barrier after each colour class.
template <class T, bool MV>
__device__ __attribute__((always_inline)) inline void tail_gs(const TailLevel& L, ColOf<MV> C) {
  auto x = C.v(L, TV<T>::x(L));
  auto b = C.v(L, TV<T>::b(L));
  const T* dg = TV<T>::diag(L);
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  for (int c = 0; c < L.ncol; ++c) {
    for (int u = L.cptr[c] + tid; u < L.cptr[c + 1]; u += tail_nt())
      if (L.rp[u + 1] - L.rp[u] <= SHORT_ROW) x[u] = (b[u] + row_short<T>(L, u, x)) / dg[u];
    for (int k = L.lptr[c] + wv; k < L.lptr[c + 1]; k += tail_nw()) {
      const int u = L.lrows[k];
      const T s = row_long<T>(L, u, x, lane);
      if (lane == 0) x[u] = (b[u] + s) / dg[u];
    }
    __syncthreads();
  }
}
// The same sweep with the level staged in LDS for its whole duration: x, b,
// diagonal, row pointers and colour bounds.  One bulk load and one write-back
// replace the global round trips of every colour phase.  Same sums in the
// same order.
constexpr int TAIL_LDS = 152 * 1024;  // dynamic LDS of a tail workgroup (of 160 KB per CU)
constexpr int TAIL_RES = 96 * 1024;   // of which at most this much holds resident levels
template <class T>
__host__ __device__ inline size_t tail_vec_bytes(const TailLevel& L) {
  return (size_t)L.n * (3 * sizeof(T) + sizeof(int)) + 2 * sizeof(int) + (size_t)(2 * L.ncol + 2) * sizeof(int);
}
template <class T>
__device__ inline bool tail_fits(const TailLevel& L, int budget) {
  return tail_vec_bytes<T>(L) <= (size_t)budget;
}
// Sweeps over a level staged in LDS: x, b, diagonal, row pointers, colour
// and long-row bounds in LDS; weights and column indices in LDS or global.
template <class T, class VP, class IP>
__device__ __attribute__((always_inline)) inline void lds_sweeps(const TailLevel& L, int sweeps, LP<T> sx, LP<T> sbv,
                                                                 LP<T> sd, LP<int> srp, LP<int> scp, LP<int> slp,
                                                                 VP val, IP ci) {
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int nc = L.ncol;
  for (int sw = 0; sw < sweeps; ++sw)
    for (int c = 0; c < nc; ++c) {
      const int c1 = scp[c + 1];
      for (int u = scp[c] + tid; u < c1; u += tail_nt()) {
        const int p0 = srp[u], len = srp[u + 1] - p0;
        if (len > SHORT_ROW) continue;
        sx[u] = (sbv[u] + row_seq_p<T>(val, ci, p0, len, sx)) / sd[u];
      }
      for (int k = slp[c] + wv; k < slp[c + 1]; k += tail_nw()) {
        const int u = L.lrows[k];
        const int p0 = srp[u], len = srp[u + 1] - p0;
        const T s = dev::row_sum_wave<T>(len, lane, [&](int t) { return val[p0 + t] * sx[ci[p0 + t]]; });
        if (lane == 0) sx[u] = (sbv[u] + s) / sd[u];
      }
      __syncthreads();
    }
}
template <class T, bool MV>
__device__ __attribute__((always_inline)) inline void tail_gs_lds(const TailLevel& L, ColOf<MV> C, char* lds,
                                                                  int budget, int sweeps, const TailLevel* Lq) {
  auto x = C.v(L, TV<T>::x(L));
  auto b = C.v(L, TV<T>::b(L));
  const T* dg = TV<T>::diag(L);
  const int n = L.n, nc = L.ncol;
  LP<T> sx = (LP<T>)lds;
  LP<T> sbv = sx + n;
  LP<T> sd = sbv + n;
  LP<int> srp = (LP<int>)(sd + n);
  LP<int> scp = srp + n + 1;
  LP<int> slp = scp + nc + 1;
  const int tid = threadIdx.x;
  if (Lq) {
    // the aggregation correction x += P x_{l+1} applied while staging
    auto e = C.v(*Lq, TV<T>::x(*Lq));
    for (int i = tid; i < n; i += tail_nt()) sx[i] = x[i] + e[L.agg[i]];
  } else {
    for (int i = tid; i < n; i += tail_nt()) sx[i] = x[i];
  }
  for (int i = tid; i < n; i += tail_nt()) { sbv[i] = b[i]; sd[i] = dg[i]; srp[i] = L.rp[i]; }
  for (int i = tid; i <= nc; i += tail_nt()) { scp[i] = L.cptr[i]; slp[i] = L.lptr[i]; }
  if (tid == 0) srp[n] = L.rp[n];
  __syncthreads();
  // the weights and column indices stay where the level keeps them (global
  // memory, or LDS for a resident level): a variant that also staged them
  // here gave non-converging FP32 cycles in a 512-thread FP32 build (cause not
  // found) and is not used
  lds_sweeps<T>(L, sweeps, sx, sbv, sd, srp, scp, slp, TV<T>::val(L), L.ci);
  for (int i = tid; i < n; i += tail_nt()) x[i] = sx[i];
}

// Sweeps of a small level (n <= R * tail_nt() rows): thread t owns rows
// t, t + tail_nt(), ... for the whole op.  Each row's colour, first RMAX
// weights and column indices, b and diagonal stay in registers and x lives
// in LDS (with the colours' long-row bounds), so a colour phase is one round
// of LDS gathers before the barrier.  The sums run left to right as in every
// other relaxation path; entries past RMAX come from the level's arrays,
// long rows (> 64) from the wavefront path.
template <class T, bool MV, int R>
__device__ __attribute__((always_inline)) inline void tail_gs_small(const TailLevel& L, ColOf<MV> C, char* lds,
                                                                    int sweeps, const TailLevel* Lq) {
  // entries held in registers per row: 16 for one row per thread, 8 for two
  constexpr int RMAX = R == 1 ? 16 : 8;
  auto x = C.v(L, TV<T>::x(L));
  auto b = C.v(L, TV<T>::b(L));
  const T* dg = TV<T>::diag(L);
  const T* val = TV<T>::val(L);
  const int n = L.n, nc = L.ncol;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  LP<T> sx = (LP<T>)lds;
  // the colours' long-row bounds, read every phase, staged beside x (the
  // level's own list may sit in global memory)
  LP<int> slp = (LP<int>)(sx + n);
  for (int c = tid; c <= nc; c += tail_nt()) slp[c] = L.lptr[c];
  int col[R], p0[R], len[R], cj[R][RMAX];
  T bu[R], du[R], wj[R][RMAX];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int u = tid + k * tail_nt();
    col[k] = -1;
    len[k] = 0;
    p0[k] = 0;
    bu[k] = T(0);
    du[k] = T(1);
    if (u < n) {
      if (Lq) {
        // the aggregation correction x += P x_{l+1} applied while staging
        auto e = C.v(*Lq, TV<T>::x(*Lq));
        sx[u] = x[u] + e[L.agg[u]];
      } else {
        sx[u] = x[u];
      }
      bu[k] = b[u];
      du[k] = dg[u];
      p0[k] = L.rp[u];
      len[k] = L.rp[u + 1] - p0[k];
      for (int c = 0; c < nc; ++c)
        if (u >= L.cptr[c] && u < L.cptr[c + 1]) col[k] = c;
      if (len[k] > SHORT_ROW) col[k] = -1;  // long rows: wavefront path below
    }
#pragma unroll
    for (int q = 0; q < RMAX; ++q) {
      const bool in = q < len[k];
      cj[k][q] = in ? L.ci[p0[k] + q] : 0;
      wj[k][q] = in ? val[p0[k] + q] : T(0);
    }
  }
  __syncthreads();
  for (int sw = 0; sw < sweeps; ++sw)
    for (int c = 0; c < nc; ++c) {
#pragma unroll
      for (int k = 0; k < R; ++k) {
        if (col[k] != c) continue;
        T xg[RMAX];
#pragma unroll
        for (int q = 0; q < RMAX; ++q) xg[q] = sx[cj[k][q]];
        T s = 0;
#pragma unroll
        for (int q = 0; q < RMAX; ++q)
          if (q < len[k]) s += wj[k][q] * xg[q];
        for (int t = RMAX; t < len[k]; ++t) s += val[p0[k] + t] * sx[L.ci[p0[k] + t]];
        sx[tid + k * tail_nt()] = (bu[k] + s) / du[k];
      }
      for (int k = slp[c] + wv; k < slp[c + 1]; k += tail_nw()) {
        const int u = L.lrows[k];
        const int q0 = L.rp[u], ln = L.rp[u + 1] - q0;
        const T s = dev::row_sum_wave<T>(ln, lane, [&](int t) { return val[q0 + t] * sx[L.ci[q0 + t]]; });
        if (lane == 0) sx[u] = (b[u] + s) / dg[u];
      }
      __syncthreads();
    }
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int u = tid + k * tail_nt();
    if (u < n) x[u] = sx[u];
  }
}

// Lq (optional): the coarse level of an aggregation whose correction
// x += P x_{l+1} precedes the sweeps; the staged paths add it as they load x.
template <class T, bool MV>
__device__ __attribute__((always_inline)) inline void tail_sweeps(const TailLevel& L, ColOf<MV> C, char* lds,
                                                                  int budget, int sweeps,
                                                                  const TailLevel* Lq = nullptr) {
  const size_t small = (size_t)L.n * sizeof(T) + (size_t)(L.ncol + 1) * sizeof(int);
  if (L.n <= tail_nt() && small <= (size_t)budget) {
    tail_gs_small<T, MV, 1>(L, C, lds, sweeps, Lq);
  } else if (L.n <= 2 * tail_nt() && small <= (size_t)budget) {
    tail_gs_small<T, MV, 2>(L, C, lds, sweeps, Lq);
  } else if (tail_fits<T>(L, budget)) {
    tail_gs_lds<T, MV>(L, C, lds, budget, sweeps, Lq);
  } else {
    if (Lq) {
      auto e = C.v(*Lq, TV<T>::x(*Lq));
      auto x = C.v(L, TV<T>::x(L));
      for (int u = threadIdx.x; u < L.n; u += tail_nt()) x[u] += e[L.agg[u]];
      __syncthreads();
    }
    for (int sw = 0; sw < sweeps; ++sw) tail_gs<T, MV>(L, C);
  }
}

// Residual rows out_u = (b_u + sum_v w_uv x_v) - a_uu x_u of a level, two
// rows per thread per pass with both rows' index and weight loads issued
// before their gathers; x, b, diagonal and row pointers through accessors
// (LDS copies or global memory).  Rows longer than 64 entries: one wavefront
// each in the canonical chunk order.  Optionally also writes the residual to
// an LDS copy rl and the iterate to Xs.
struct NoEpi {
  template <class T>
  __device__ void operator()(int, T, T) const {}
};
template <class T, bool MV, class XA, class BA, class DA, class RA, class EPI = NoEpi>
__device__ __attribute__((always_inline)) inline void res_rows(const TailLevel& L, XA xa, BA ba, DA da, RA rpa,
                                                               const T* val, Col<T, MV> out, LP<T> rl, bool use_rl,
                                                               bool save, Col<T, MV> Xs, EPI epi = EPI()) {
  constexpr int Q = 8;
  const int n = L.n, tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  for (int u0 = tid; u0 < n; u0 += 2 * tail_nt()) {
    const int u[2] = {u0, u0 + tail_nt()};
    int p0[2], len[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      p0[k] = 0;
      len[k] = 0;
      if (u[k] < n) {
        p0[k] = rpa[u[k]];
        len[k] = rpa[u[k] + 1] - p0[k];
      }
    }
    int cj[2][Q];
    T wj[2][Q], xg[2][Q];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const bool in = q < len[k] && len[k] <= SHORT_ROW;
        cj[k][q] = in ? L.ci[p0[k] + q] : 0;
        wj[k][q] = in ? val[p0[k] + q] : T(0);
      }
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int q = 0; q < Q; ++q) xg[k][q] = xa[cj[k][q]];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (u[k] >= n || len[k] > SHORT_ROW) continue;
      T s = 0;
#pragma unroll
      for (int q = 0; q < Q; ++q)
        if (q < len[k]) s += wj[k][q] * xg[k][q];
      for (int t = Q; t < len[k]; ++t) s += val[p0[k] + t] * xa[L.ci[p0[k] + t]];
      const T xu = xa[u[k]];
      const T r = (ba[u[k]] + s) - da[u[k]] * xu;
      out[u[k]] = r;
      if (use_rl) rl[u[k]] = r;
      if (save) Xs[u[k]] = xu;
      epi(u[k], r, xu);
    }
  }
  for (int k = wv; k < L.nlong; k += tail_nw()) {
    const int u = L.lrows[k];
    const int q0 = rpa[u], ln = rpa[u + 1] - q0;
    const T s = dev::row_sum_wave<T>(ln, lane, [&](int t) { return val[q0 + t] * xa[L.ci[q0 + t]]; });
    if (lane == 0) {
      const T xu = xa[u];
      const T r = (ba[u] + s) - da[u] * xu;
      out[u] = r;
      if (use_rl) rl[u] = r;
      if (save) Xs[u] = xu;
    }
  }
}

// The residual of a level into out, its x, b, diagonal and row pointers
// staged in LDS when they fit (and the level does not already sit in LDS).
// Returns whether an LDS copy of the residual was left at *rl.
// epi(u, r_u, x_u): called by the thread that computed short row u, right
// after it (rows longer than 64 entries do not call it).
template <class T, bool MV, class EPI = NoEpi>
__device__ __attribute__((always_inline)) inline bool tail_residual(const TailLevel& L, ColOf<MV> C, char* lds,
                                                                    int budget, Col<T, MV> out, bool save,
                                                                    Col<T, MV> Xs, LP<T>* rl, EPI epi = EPI()) {
  auto x = C.v(L, TV<T>::x(L));
  auto b = C.v(L, TV<T>::b(L));
  const T* dg = TV<T>::diag(L);
  const T* val = TV<T>::val(L);
  const int n = L.n, tid = threadIdx.x;
  if (!L.vres && (size_t)n * (4 * sizeof(T) + 4) + 64 <= (size_t)budget) {
    LP<T> sx = (LP<T>)lds;
    LP<T> sb = sx + n;
    LP<T> sd = sb + n;
    LP<T> sr = sd + n;
    LP<int> srp = (LP<int>)(sr + n);
    for (int i = tid; i < n; i += tail_nt()) { sx[i] = x[i]; sb[i] = b[i]; sd[i] = dg[i]; srp[i] = L.rp[i]; }
    if (tid == 0) srp[n] = L.rp[n];
    __syncthreads();
    res_rows<T, MV>(L, sx, sb, sd, srp, val, out, sr, true, save, Xs, epi);
    *rl = sr;
    return true;
  }
  res_rows<T, MV>(L, x, b, dg, L.rp, val, out, (LP<T>)lds, false, save, Xs, epi);
  return false;
}

// x_r = sum_j M_rj b_j over the rows of the dense coarsest inverse: one
// wavefront per row, lane l summing the entries l, l + 64, ... left to right,
// the butterfly folding the 64 partials.  A wavefront takes four of its rows
// at a time so that their loads are in flight together; each row's sum keeps
// its order.  (FP64 programs only: the FP32 interpreter, at 128 VGPRs, was
// measured slower with it.)
template <class T, class BF, class XO>
__device__ __attribute__((always_inline)) inline void coarse_rows(const double* __restrict__ M, int nL, BF bj,
                                                                  XO x) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = tail_nw();
  int r = wv;
  if constexpr (sizeof(T) == 8)
  for (; r + 3 * nw < nL; r += 4 * nw) {
    const double* m0 = M + (size_t)r * nL;
    const double* m1 = m0 + (size_t)nw * nL;
    const double* m2 = m1 + (size_t)nw * nL;
    const double* m3 = m2 + (size_t)nw * nL;
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int j = lane; j < nL; j += 64) {
      const double v = bj(j);
      s0 += m0[j] * v;
      s1 += m1[j] * v;
      s2 += m2[j] * v;
      s3 += m3[j] * v;
    }
    s0 = dev::wave_fold(s0);
    s1 = dev::wave_fold(s1);
    s2 = dev::wave_fold(s2);
    s3 = dev::wave_fold(s3);
    if (lane == 0) {
      x[r] = (T)s0;
      x[r + nw] = (T)s1;
      x[r + 2 * nw] = (T)s2;
      x[r + 3 * nw] = (T)s3;
    }
  }
  for (; r < nL; r += nw) {
    const double* row = M + (size_t)r * nL;
    double s = 0;
    for (int j = lane; j < nL; j += 64) s += row[j] * bj(j);
    s = dev::wave_fold(s);
    if (lane == 0) x[r] = (T)s;
  }
}

// Fixed-order sum of NV values per thread over the workgroup: a butterfly
// inside each wavefront, then the launch's wavefront sums left to right,
// added by one thread per value (thread i for value i) and read back by all;
// every thread adding all of them cost 16 x NV LDS reads per wavefront.
template <int NV>
__device__ inline void block_sums(double (&v)[NV], double (*sh)[TAIL_WAVES]) {
  static_assert(NV >= 1 && NV <= 6, "the scratch holds six rows");
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const double t = dev::wave_fold(v[i]);
    if (lane == 0) sh[i][wv] = t;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    const int i = threadIdx.x;
    double t = 0;
    for (int w = 0; w < tail_nw(); ++w) t += sh[i][w];
    sh[i][0] = t;  // only this thread reads row i before the barrier
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = sh[i][0];
  __syncthreads();
}

// The op interpreter: runs nops ops of a program with a workgroup barrier
// after each.  lds: the dynamic LDS (staging of sweeps, coarsest right-hand
// side); sh: reduction scratch.  Multi-vector form: column C.j of every block
// (stride P.kc), each column with its own recombination coefficients and mean.
template <class T, bool MV>
__device__ __attribute__((always_inline)) inline void run_ops(const TailParams& P, const TailLevel* Ls,
                                                              const int4* __restrict__ prog, int nops, char* lds,
                                                              int budget, double (*sh)[TAIL_WAVES], ColOf<MV> C) {
  LP<double> sb = (LP<double>)lds;
  const int tid = threadIdx.x;
  const TailParams PP = P;  // one read of the parameters, not one per op
  const int4* pg = prog;
  for (int i = 0; i < nops; ++i) {
    const int4 op = pg[i];
    const TailLevel& L = Ls[op.y - PP.lc];
    switch (op.x) {
      case OP_GS:
        tail_sweeps<T, MV>(L, C, lds, budget, op.z);
        break;
      case OP_IGS:
        tail_sweeps<T, MV>(L, C, lds, budget, op.z, &Ls[op.y + 1 - PP.lc]);
        break;
      case OP_RRAGG: {
        // residual rows (saved iterate alongside), then one thread per
        // aggregate: restricted sum of its members in ascending order, zeroed
        // coarse iterate
        const TailLevel& Lc = Ls[op.y + 1 - PP.lc];
        auto dst = C.v(L, op.z == 0 ? TV<T>::r(L) : TV<T>::R(L, op.z - 1));
        const bool save = op.z != 0;
        auto Xs = C.v(L, save ? TV<T>::X(L, op.z - 1) : TV<T>::x(L));
        LP<T> rl;
        const bool inl = tail_residual<T, MV>(L, C, lds, budget, dst, save, Xs, &rl);
        __syncthreads();
        auto bc = C.v(Lc, TV<T>::b(Lc));
        auto xc = C.v(Lc, TV<T>::x(Lc));
        const T mu = op.w ? (T)PP.mu : T(1);
        for (int U = tid; U < L.nc; U += tail_nt()) {
          T s = 0;
          if (inl)
            for (int j = L.agg_ptr[U]; j < L.agg_ptr[U + 1]; ++j) s += rl[L.members[j]];
          else
            for (int j = L.agg_ptr[U]; j < L.agg_ptr[U + 1]; ++j) s += dst[L.members[j]];
          bc[U] = mu * s;
          xc[U] = T(0);
        }
        break;
      }
      case OP_RRELIM: {
        // residual rows (staged in LDS when they fit), then one thread per
        // coarse node: its fine value plus the eliminated neighbours' terms
        // in stencil order, read from the staged copy; zeroed coarse iterate
        const TailLevel& Lc = Ls[op.y + 1 - PP.lc];
        auto r = C.v(L, TV<T>::r(L));
        LP<T> rl;
        const bool inl = tail_residual<T, MV>(L, C, lds, budget, r, false, r, &rl);
        __syncthreads();
        const T* er = TV<T>::er(L);
        auto bc = C.v(Lc, TV<T>::b(Lc));
        auto xc = C.v(Lc, TV<T>::x(Lc));
        for (int c = tid; c < L.nc; c += tail_nt()) {
          T s = 0;
          if (inl) {
            for (int j = L.er_rp[c]; j < L.er_rp[c + 1]; ++j) s += er[j] * rl[L.er_ci[j]];
            bc[c] = rl[L.cfine[c]] + s;
          } else {
            for (int j = L.er_rp[c]; j < L.er_rp[c + 1]; ++j) s += er[j] * r[L.er_ci[j]];
            bc[c] = r[L.cfine[c]] + s;
          }
          xc[c] = T(0);
        }
        break;
      }
      case OP_IAGG: {
        const TailLevel& Lc = Ls[op.y + 1 - PP.lc];
        auto e = C.v(Lc, TV<T>::x(Lc));
        auto x = C.v(L, TV<T>::x(L));
        for (int u = tid; u < L.n; u += tail_nt()) x[u] += e[L.agg[u]];
        break;
      }
      case OP_IELIM: {
        const TailLevel& Lc = Ls[op.y + 1 - PP.lc];
        auto e = C.v(Lc, TV<T>::x(Lc));
        auto r = C.v(L, TV<T>::r(L));
        const T* val = TV<T>::val(L);
        const T* dg = TV<T>::diag(L);
        auto x = C.v(L, TV<T>::x(L));
        for (int u = tid; u < L.n; u += tail_nt()) {
          const int c = L.cidx[u];
          if (c >= 0) { x[u] += e[c]; continue; }
          T s = r[u];
          for (int t = L.rp[u]; t < L.rp[u + 1]; ++t) s += val[t] * e[L.cidx[L.ci[t]]];
          x[u] += s / dg[u];
        }
        break;
      }
      case OP_RECOMB: {
        const int th = op.z;
        auto r = C.v(L, TV<T>::r(L));
        auto R0 = C.v(L, TV<T>::R(L, 0));
        auto R1 = C.v(L, TV<T>::R(L, 1));
        auto x = C.v(L, TV<T>::x(L));
        auto X0 = C.v(L, TV<T>::X(L, 0));
        auto X1 = C.v(L, TV<T>::X(L, 1));
        const int norm = PP.rnorm;
        double v[6] = {0, 0, 0, 0, 0, 0};
        LP<T> rl;
        if (L.nlong == 0) {
          // every row short: each thread adds its rows' terms as it computes
          // their residuals (its rows in the same order as the separate pass
          // below: tid, tid + threads, ...), no barrier between
          tail_residual<T, MV>(L, C, lds, budget, r, false, r, &rl, [&](int u, T ru, T xu) {
            dev::recomb_terms<T>(norm, th, ru, R0[u], th > 1 ? R1[u] : T(0), norm ? xu : T(0),
                                 norm ? X0[u] : T(0), norm && th > 1 ? X1[u] : T(0), v);
          });
        } else {
          tail_residual<T, MV>(L, C, lds, budget, r, false, r, &rl);
          __syncthreads();
          for (int u = tid; u < L.n; u += tail_nt())
            dev::recomb_terms<T>(norm, th, r[u], R0[u], th > 1 ? R1[u] : T(0), norm ? x[u] : T(0),
                                 norm ? X0[u] : T(0), norm && th > 1 ? X1[u] : T(0), v);
        }
        block_sums<6>(v, sh);
        double a0 = 0, a1 = 0;
        dev::recomb_alpha(norm, th, v, &a0, &a1);
        for (int u = tid; u < L.n; u += tail_nt()) {
          const double xu = (double)x[u];
          double y = xu;
          y += a0 * ((double)X0[u] - xu);
          if (th > 1) y += a1 * ((double)X1[u] - xu);
          x[u] = (T)y;
        }
        break;
      }
      case OP_COARSE: {
        if (PP.crelax) {
          tail_sweeps<T, MV>(L, C, lds, budget, PP.csweeps);
          break;
        }
        // x = M^-1 b: one wavefront per row, coalesced row loads; b staged
        // in LDS unless it already sits there or does not fit
        auto b = C.v(L, TV<T>::b(L));
        auto x = C.v(L, TV<T>::x(L));
        if (L.vres || (size_t)PP.nL * sizeof(double) > (size_t)budget) {
          coarse_rows<T>(PP.Minv, PP.nL, [&](int j) { return (double)b[j]; }, x);
          break;
        }
        for (int j = tid; j < PP.nL; j += tail_nt()) sb[j] = (double)b[j];
        __syncthreads();
        coarse_rows<T>(PP.Minv, PP.nL, [&](int j) { return sb[j]; }, x);
        break;
      }
      case OP_MEAN: {
        auto x = C.v(L, TV<T>::x(L));
        double v[1] = {0};
        for (int u = tid; u < L.n; u += tail_nt()) v[0] += (double)x[u];
        block_sums<1>(v, sh);
        const double mean = v[0] / (double)L.n;
        for (int u = tid; u < L.n; u += tail_nt()) x[u] = (T)((double)x[u] - mean);
        break;
      }
      default:
        break;
    }
    __syncthreads();
  }
}

// The interpreter is inlined into the tail kernels: as a called function it
// kept its arrays and saved registers on a private stack (228 bytes per lane
// in FP64); inlined it uses none (151 VGPRs in FP64 at 512 threads, 125 in
// FP32 at 1024) and the multilevel solves run 1-2.5% faster.  An earlier
// build of this file gave wrong FP32 cycles when inlined; with the level
// descriptors copied into LDS as structs and the wavefront-sum scratch sized
// for the largest launch, every GPU test passes inlined, in both precisions.
// ---------------------------------------------------------- LDS residency
// At the start of a program the level descriptors are copied into LDS and
// the largest suffix of (coarsest) levels whose arrays fit P.res_bytes is
// copied there too: CSR, diagonal, colour and long-row lists, the transfer
// into the next level and all work vectors of the precision T.  Those levels'
// ops then touch no global memory.  Vectors of the levels below the entry
// level are produced inside the program, so only the entry level's x and b are
// loaded, and its x written back at the end.  Every thread computes the same
// plan; one thread rewrites a descriptor after all threads have read it.
__host__ __device__ inline size_t al16(size_t b) { return (b + 15) & ~(size_t)15; }

template <class T>
__host__ __device__ inline size_t res_footprint(const TailLevel& L) {
  const size_t n = L.n, nz = L.nnz, nc = L.nc;
  size_t s = al16((n + 1) * 4) + al16(nz * 4) + al16(nz * sizeof(T)) + al16(n * sizeof(T)) +
             2 * al16((L.ncol + 1) * 4) + al16((size_t)(L.nlong > 0 ? L.nlong : 1) * 4);
  if (L.agg) s += al16(n * 4) + al16((nc + 1) * 4) + al16(n * 4);
  if (L.cidx) {
    const size_t ne = L.nner;
    s += al16(n * 4) + al16(nc * 4) + al16((nc + 1) * 4) + al16(ne * 4) + al16(ne * sizeof(T));
  }
  return s + 7 * al16(n * sizeof(T));
}

// Copies count elements src -> LDS at cur (all threads), returns the copy.
template <class U>
__device__ inline U* lds_put(char*& cur, const U* src, size_t count) {
  U* dst = (U*)cur;
  if (src)
    for (size_t i = threadIdx.x; i < count; i += tail_nt()) dst[i] = src[i];
  cur += al16(count * sizeof(U));
  return dst;
}
template <class U>
__device__ inline U* lds_take(char*& cur, size_t count) {
  U* dst = (U*)cur;
  cur += al16(count * sizeof(U));
  return dst;
}

template <class T> struct TSet;
template <> struct TSet<double> {
  __device__ static void mats(TailLevel& L, const double* v, const double* d, const double* e) {
    L.val64 = v; L.diag64 = d; L.er64 = e;
  }
  __device__ static void vecs(TailLevel& L, double* const (&w)[7]) {
    L.x64 = w[0]; L.b64 = w[1]; L.r64 = w[2]; L.X64[0] = w[3]; L.X64[1] = w[4]; L.R64[0] = w[5]; L.R64[1] = w[6];
  }
};
template <> struct TSet<float> {
  __device__ static void mats(TailLevel& L, const float* v, const float* d, const float* e) {
    L.val32 = v; L.diag32 = d; L.er32 = e;
  }
  __device__ static void vecs(TailLevel& L, float* const (&w)[7]) {
    L.x32 = w[0]; L.b32 = w[1]; L.r32 = w[2]; L.X32[0] = w[3]; L.X32[1] = w[4]; L.R32[0] = w[5]; L.R32[1] = w[6];
  }
};

// The residency plan: the first level of the largest suffix of levels that
// joins LDS.  A level joins only while the LDS left over still stages the
// vectors of every level above the resident ones that relaxes (a level
// followed by an elimination level has no sweeps).  *bytes: their footprint.
template <class T>
__host__ __device__ inline int resident_from(const TailLevel* dl, int nlev, int lds_bytes, int res_bytes,
                                             size_t* bytes) {
  const size_t desc = al16((size_t)nlev * sizeof(TailLevel));
  int rfrom = nlev;
  size_t tot = 0;
  if (desc < (size_t)lds_bytes) {
    const size_t free0 = (size_t)lds_bytes - desc;
    for (int i = nlev - 1; i >= 0; --i) {
      const size_t b = res_footprint<T>(dl[i]);
      size_t stage = 0;
      for (int a = 0; a < i; ++a)
        if (!dl[a].cidx) stage = stage > tail_vec_bytes<T>(dl[a]) + 64 ? stage : tail_vec_bytes<T>(dl[a]) + 64;
      if (tot + b > (size_t)res_bytes || tot + b + stage > free0) break;
      tot += b;
      rfrom = i;
    }
  }
  if (bytes) *bytes = tot;
  return rfrom;
}

template <class T, bool MV>
__device__ __attribute__((always_inline)) inline void run_resident(const TailParams& P, const int4* prog, int nops,
                                                                   char* lds, double (*sh)[TAIL_WAVES]) {
  const int tid = threadIdx.x;
  const ColOf<MV> C{MV ? (int)blockIdx.x : 0, MV ? P.kc : 1};
  const int nlev = P.nlev;
  TailLevel* dl = (TailLevel*)lds;
  // one thread per descriptor, copied as the struct it is (no reinterpreting
  // of its words through another type)
  for (int i = tid; i < nlev; i += tail_nt()) dl[i] = P.L[i];
  __syncthreads();
  char* cur = lds + al16((size_t)nlev * sizeof(TailLevel));
  const int rfrom = resident_from<T>(dl, nlev, P.lds_bytes, P.res_bytes, nullptr);
  T* x0 = nullptr;  // the entry level's x in global memory (written back at the end)
  for (int i = rfrom; i < nlev; ++i) {
    const TailLevel o = dl[i];
    __syncthreads();  // every thread holds the original pointers
    const size_t n = o.n, nz = o.nnz, nc = o.nc;
    TailLevel& L = dl[i];
    const int* rp = lds_put(cur, o.rp, n + 1);
    const int* ci = lds_put(cur, o.ci, nz);
    const T* val = lds_put(cur, TV<T>::val(o), nz);
    const T* dg = lds_put(cur, TV<T>::diag(o), n);
    const int* cp = lds_put(cur, o.cptr, (size_t)o.ncol + 1);
    const int* lp = lds_put(cur, o.lptr, (size_t)o.ncol + 1);
    const int* lr = lds_put(cur, o.lrows, (size_t)(o.nlong > 0 ? o.nlong : 1));
    const int *ag = nullptr, *agp = nullptr, *mem = nullptr, *cx = nullptr, *cf = nullptr, *erp = nullptr,
              *eci = nullptr;
    const T* er = nullptr;
    if (o.agg) {
      ag = lds_put(cur, o.agg, n);
      agp = lds_put(cur, o.agg_ptr, nc + 1);
      mem = lds_put(cur, o.members, n);
    }
    if (o.cidx) {
      cx = lds_put(cur, o.cidx, n);
      cf = lds_put(cur, o.cfine, nc);
      erp = lds_put(cur, o.er_rp, nc + 1);
      eci = lds_put(cur, o.er_ci, (size_t)o.nner);
      er = lds_put(cur, TV<T>::er(o), (size_t)o.nner);
    }
    T* w[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) w[q] = lds_take<T>(cur, n);
    if (i == 0) {
      // the entry level: its right-hand side and iterate come from outside
      x0 = TV<T>::x(o);
      auto gx = C.v(o, TV<T>::x(o));
      auto gb = C.v(o, TV<T>::b(o));
      for (size_t k = tid; k < n; k += tail_nt()) {
        w[0][k] = gx[(int)k];
        w[1][k] = gb[(int)k];
      }
    }
    if (tid == 0) {
      L.rp = rp; L.ci = ci; L.cptr = cp; L.lptr = lp; L.lrows = lr;
      L.agg = ag; L.agg_ptr = agp; L.members = mem;
      L.cidx = cx; L.cfine = cf; L.er_rp = erp; L.er_ci = eci;
      TSet<T>::mats(L, val, dg, er);
      TSet<T>::vecs(L, w);
      L.vres = 1;
    }
  }
  __syncthreads();
  const int budget = P.lds_bytes - (int)(cur - lds);
  run_ops<T, MV>(P, dl, prog, nops, cur, budget, sh, C);
  if (rfrom == 0) {
    // write the entry level's iterate back (the caller interpolates from it)
    const Col<T, MV> gx{MV ? x0 + C.j : x0, C.k};
    const T* sx = TV<T>::x(dl[0]);
    for (int k = tid; k < dl[0].n; k += tail_nt()) gx[k] = sx[k];
    __syncthreads();
  }
}

template <class T, bool MV>
__device__ __attribute__((always_inline)) inline void run_program(const TailParams& P, const int4* prog, int nops,
                                                                  char* lds, double (*sh)[TAIL_WAVES]) {
  run_resident<T, MV>(P, prog, nops, lds, sh);
}
template <class T, bool MV>
__global__ __launch_bounds__(tail_launch<T>()) void k_tail(TailParams P, const int4* __restrict__ prog, int nops) {
  __shared__ double sh[6][TAIL_WAVES];
  extern __shared__ double lds_d[];
  run_program<T, MV>(P, prog, nops, (char*)lds_d, sh);
}

// ------------------------------------------------------ program generation
// Mirrors the host cycle (visit / body) from level lc down, emitting ops.
struct Gen {
  const Hierarchy* H;
  std::vector<int4> prog;
  std::vector<int64_t> count;
  void op(int code, int l, int a = 0, int b = 0) { prog.push_back(make_int4(code, l, a, b)); }
  void visit(int l, int th) {
    const int Lc = (int)H->lv.size() - 1;
    if (l == Lc) { op(OP_COARSE, l); return; }
    for (int i = 0; i < th; ++i) body(l, i);
    if (H->o.ec == LAMG_EC_RECOMBINE && H->lv[l + 1].type == LT_AGG) op(OP_RECOMB, l, th);
  }
  void body(int l, int sub) {
    const int Lc = (int)H->lv.size() - 1;
    if (l == Lc) { op(OP_COARSE, l); return; }
    if (H->lv[l + 1].type == LT_ELIM) {
      op(OP_RRELIM, l);
      visit(l + 1, 1);
      op(OP_IELIM, l);
      return;
    }
    const bool rec = H->o.ec == LAMG_EC_RECOMBINE;
    if (H->o.nu_pre > 0) op(OP_GS, l, H->o.nu_pre);
    const int src = rec ? 1 + sub : 0;
    op(OP_RRAGG, l, src, rec ? 0 : 1);
    const int64_t c = count[l]++;
    const double gl = H->lv[l].gamma_next;
    const int th = (int)(std::ceil((double)(c + 1) * gl) - std::ceil((double)c * gl));
    visit(l + 1, th);
    if (H->o.nu_post > 0) {
      op(OP_IGS, l, H->o.nu_post);
    } else {
      op(OP_IAGG, l);
    }
  }
};

// Replays the host part of the schedule (levels < lc) to find every entry
// into level lc and its theta, in launch order.
void host_walk(const Hierarchy* H, int l, int th, std::vector<int64_t>& count, int lc, Gen& g,
               std::vector<int2>& segs) {
  const int Lc = (int)H->lv.size() - 1;
  if (l == lc) {
    const int off = (int)g.prog.size();
    g.visit(l, th);
    if (lc == 0) g.op(OP_MEAN, 0);
    segs.push_back(make_int2(off, (int)g.prog.size() - off));
    return;
  }
  if (l == Lc) return;
  for (int i = 0; i < th; ++i) {
    if (H->lv[l + 1].type == LT_ELIM) { host_walk(H, l + 1, 1, count, lc, g, segs); continue; }
    const int64_t c = count[l]++;
    const double gl = H->lv[l].gamma_next;
    host_walk(H, l + 1, (int)(std::ceil((double)(c + 1) * gl) - std::ceil((double)c * gl)), count, lc, g, segs);
  }
}

// Device copies of a level's colour bounds and long-row lists (made once).
void level_lists(Hierarchy* H, Level& L) {
  if (L.d_cptr) return;
  int* cp = dnew<int>(H, L.cptr.size());
  int* lp = dnew<int>(H, L.long_ptr.size());
  int* lr = dnew<int>(H, std::max<size_t>(L.long_rows.size(), 1));
  LAMG_HIP(hipMemcpy(cp, L.cptr.data(), L.cptr.size() * sizeof(int), hipMemcpyHostToDevice));
  LAMG_HIP(hipMemcpy(lp, L.long_ptr.data(), L.long_ptr.size() * sizeof(int), hipMemcpyHostToDevice));
  if (!L.long_rows.empty())
    LAMG_HIP(hipMemcpy(lr, L.long_rows.data(), L.long_rows.size() * sizeof(int), hipMemcpyHostToDevice));
  L.d_cptr = cp;
  L.d_lptr = lp;
  L.d_lrows = lr;
}

// Descriptors of levels lc .. nl-1 with the single-vector work vectors.
std::vector<TailLevel> build_desc(Hierarchy* H, int lc) {
  const int nl = (int)H->lv.size();
  std::vector<TailLevel> d(nl - lc);
  for (int l = lc; l < nl; ++l) {
    Level& L = H->lv[l];
    level_lists(H, L);
    TailLevel& t = d[l - lc];
    std::memset(&t, 0, sizeof(t));
    t.n = L.n; t.nnz = L.nnz; t.ncol = L.ncol; t.nc = l + 1 < nl ? H->lv[l + 1].n : 0;
    t.nlong = (int)L.long_rows.size();
    t.nner = l + 1 < nl && H->lv[l + 1].type == LT_ELIM ? (int)H->lv[l + 1].er_tiles.nnz : 0;
    t.rp = L.rp; t.ci = L.ci; t.val64 = L.val; t.diag64 = L.diag; t.val32 = L.val32; t.diag32 = L.diag32;
    t.cptr = L.d_cptr; t.lptr = L.d_lptr; t.lrows = L.d_lrows;
    if (l + 1 < nl) {
      const Level& C = H->lv[l + 1];
      t.agg = C.agg; t.agg_ptr = C.agg_ptr; t.members = C.members;
      t.cidx = C.cidx; t.cfine = C.cfine; t.er_rp = C.er_rp; t.er_ci = C.er_ci; t.er64 = C.er_val; t.er32 = C.er_val32;
    }
    t.x64 = L.v64.x; t.b64 = L.v64.b; t.r64 = L.v64.r;
    t.x32 = L.v32.x; t.b32 = L.v32.b; t.r32 = L.v32.r;
    for (int i = 0; i < 2; ++i) {
      t.X64[i] = L.v64.X[i]; t.R64[i] = L.v64.R[i]; t.X32[i] = L.v32.X[i]; t.R32[i] = L.v32.R[i];
    }
  }
  return d;
}

// The op program of one finest cycle for the levels from lc down: one
// segment per entry into level lc, in launch order.
void build_prog(const Hierarchy* H, int lc, std::vector<int4>& prog, std::vector<int2>& segs) {
  const int nl = (int)H->lv.size();
  Gen g;
  g.H = H;
  g.count.assign(nl, 0);
  std::vector<int64_t> hc(nl, 0);
  segs.clear();
  host_walk(H, 0, 1, hc, lc, g, segs);
  prog.swap(g.prog);
}

// Host-side check, before a program's first launch, of everything its ops
// will touch: every descriptor pointer lies inside a live allocation of the
// hierarchy with room for the extent the ops read or write (n, nnz, colour
// and long-row lists, transfers, both precisions' matrices and work vectors),
// every op's code, level and argument is in range and its level has the
// transfer the op uses, and the LDS residency plan of both precisions fits
// each LDS budget the program may run with.  Returns "" or the first problem.
std::string program_check(const Hierarchy* H, const std::vector<TailLevel>& d, const std::vector<int4>& prog, int lc,
                          const std::vector<int2>& budgets) {
  char buf[200];
  std::vector<std::pair<uintptr_t, size_t>> al(H->owned.size());
  for (size_t i = 0; i < al.size(); ++i) al[i] = {(uintptr_t)H->owned[i], H->owned_bytes[i]};
  std::sort(al.begin(), al.end());
  auto inside = [&](const void* p, size_t bytes) {
    const uintptr_t a = (uintptr_t)p;
    auto it = std::upper_bound(al.begin(), al.end(), std::make_pair(a, ~(size_t)0));
    if (it == al.begin()) return false;
    --it;
    return a >= it->first && a + bytes <= it->first + it->second;
  };
  const int nlev = (int)d.size();
  for (int i = 0; i < nlev; ++i) {
    const TailLevel& t = d[i];
    const size_t n = t.n, nz = t.nnz, nc = t.nc, ne = t.nner;
    if (t.n < 1 || t.nnz < 0 || t.ncol < 1 || t.vres != 0) {
      std::snprintf(buf, sizeof(buf), "level %d: bad sizes", lc + i);
      return buf;
    }
    struct Ext { const void* p; size_t bytes; const char* what; bool need; };
    const Ext ex[] = {
        {t.rp, (n + 1) * 4, "rp", true}, {t.ci, nz * 4, "ci", nz > 0}, {t.val64, nz * 8, "val64", nz > 0},
        {t.val32, nz * 4, "val32", nz > 0}, {t.diag64, n * 8, "diag64", true}, {t.diag32, n * 4, "diag32", true},
        {t.cptr, ((size_t)t.ncol + 1) * 4, "cptr", true}, {t.lptr, ((size_t)t.ncol + 1) * 4, "lptr", true},
        {t.lrows, (size_t)(t.nlong > 0 ? t.nlong : 1) * 4, "lrows", true},
        {t.agg, n * 4, "agg", t.agg != nullptr}, {t.agg_ptr, (nc + 1) * 4, "agg_ptr", t.agg != nullptr},
        {t.members, n * 4, "members", t.agg != nullptr}, {t.cidx, n * 4, "cidx", t.cidx != nullptr},
        {t.cfine, nc * 4, "cfine", t.cidx != nullptr}, {t.er_rp, (nc + 1) * 4, "er_rp", t.cidx != nullptr},
        {t.er_ci, ne * 4, "er_ci", t.cidx != nullptr && ne > 0}, {t.er64, ne * 8, "er64", t.cidx != nullptr && ne > 0},
        {t.er32, ne * 4, "er32", t.cidx != nullptr && ne > 0},
        {t.x64, n * 8, "x64", true}, {t.b64, n * 8, "b64", true}, {t.r64, n * 8, "r64", true},
        {t.X64[0], n * 8, "X64", true}, {t.X64[1], n * 8, "X64", true}, {t.R64[0], n * 8, "R64", true},
        {t.R64[1], n * 8, "R64", true}, {t.x32, n * 4, "x32", true}, {t.b32, n * 4, "b32", true},
        {t.r32, n * 4, "r32", true}, {t.X32[0], n * 4, "X32", true}, {t.X32[1], n * 4, "X32", true},
        {t.R32[0], n * 4, "R32", true}, {t.R32[1], n * 4, "R32", true}};
    for (const Ext& e : ex)
      if (e.need && !inside(e.p, e.bytes)) {
        std::snprintf(buf, sizeof(buf), "level %d: %s (%zu bytes) outside the hierarchy's allocations", lc + i,
                      e.what, e.bytes);
        return buf;
      }
    if ((t.agg != nullptr) + (t.cidx != nullptr) > 1 || (i + 1 < nlev) != (t.agg || t.cidx) ||
        (i + 1 < nlev && (size_t)d[i + 1].n != nc)) {
      std::snprintf(buf, sizeof(buf), "level %d: transfer does not match level %d", lc + i, lc + i + 1);
      return buf;
    }
  }
  for (size_t k = 0; k < prog.size(); ++k) {
    const int4 op = prog[k];
    const int li = op.y - lc;
    bool ok = op.x >= OP_GS && op.x <= OP_IGS && li >= 0 && li < nlev;
    if (ok) {
      const TailLevel& t = d[li];
      switch (op.x) {
        case OP_GS: ok = op.z >= 0; break;
        case OP_RRAGG: ok = t.agg != nullptr && op.z >= 0 && op.z <= 2; break;
        case OP_IAGG: ok = t.agg != nullptr; break;
        case OP_IGS: ok = t.agg != nullptr && op.z >= 1; break;
        case OP_IELIM: case OP_RRELIM: ok = t.cidx != nullptr; break;
        case OP_MEAN: break;
        case OP_RECOMB: ok = op.z >= 1 && op.z <= 2 && t.agg != nullptr; break;
        case OP_COARSE: ok = li == nlev - 1; break;
        default: ok = false;
      }
    }
    if (!ok) {
      std::snprintf(buf, sizeof(buf), "op %zu (%d, %d, %d, %d) out of range", k, op.x, op.y, op.z, op.w);
      return buf;
    }
  }
  if (!H->coarsest_relax && !inside(H->cinv, (size_t)H->nL * H->nL * 8)) return "coarsest inverse outside the allocations";
  for (const int2 b : budgets) {
    const size_t desc = al16((size_t)nlev * sizeof(TailLevel));
    size_t t64 = 0, t32 = 0;
    resident_from<double>(d.data(), nlev, b.x, b.y, &t64);
    resident_from<float>(d.data(), nlev, b.x, b.y, &t32);
    if (desc >= (size_t)b.x || desc + t64 > (size_t)b.x || desc + t32 > (size_t)b.x || t64 > (size_t)b.y ||
        t32 > (size_t)b.y) {
      std::snprintf(buf, sizeof(buf), "LDS plan of %d levels exceeds a budget of %d bytes", nlev, b.x);
      return buf;
    }
  }
  return "";
}

void check_or_throw(const std::string& e) {
  if (e.empty()) return;
  set_error_detail(e.c_str());
  throw DevError{hipErrorInvalidValue};
}

}  // namespace

void tail_prepare(Hierarchy* H) {
  if (H->tail_lc >= 0) return;
  const int nl = (int)H->lv.size();
  const int tmax = H->o.tail_max_n;
  int lc = nl;
  if (tmax > 0)
    for (int l = nl - 1; l >= 0 && H->lv[l].n <= tmax; --l) lc = l;
  if (lc >= nl) { H->tail_lc = lc; return; }
  std::vector<TailLevel> d = build_desc(H, lc);
  TailLevel* dd = dnew<TailLevel>(H, d.size());
  LAMG_HIP(hipMemcpy(dd, d.data(), d.size() * sizeof(TailLevel), hipMemcpyHostToDevice));
  H->tail_levels = dd;
  H->tail_host = d;
  std::vector<int4> prog;
  build_prog(H, lc, prog, H->tail_segs);
  check_or_throw(program_check(H, d, prog, lc, {make_int2(TAIL_LDS, TAIL_RES)}));
  H->tail_prog = dnew<int4>(H, std::max<size_t>(prog.size(), 1));
  LAMG_HIP(hipMemcpy(H->tail_prog, prog.data(), prog.size() * sizeof(int4), hipMemcpyHostToDevice));
  H->tail_lc = lc;  // ready
}

namespace {
template <class T, bool MV>
void launch_tail(Hierarchy* H, const void* levels, int kc) {
  const int2 seg = H->tail_segs[H->tail_cursor++];
  TailParams P;
  P.L = (const TailLevel*)levels;
  P.lc = H->tail_lc;
  P.Minv = H->cinv;
  P.nL = H->nL;
  P.crelax = H->coarsest_relax ? 1 : 0;
  P.csweeps = H->o.coarsest_sweeps;
  P.mu = H->o.mu;
  P.kc = kc;
  // TAIL_LDS covers the coarsest right-hand side too: n_L <= 8192 doubles
  const size_t lds = TAIL_LDS;
  P.lds_bytes = (int)lds;
  P.res_bytes = TAIL_RES;
  P.nlev = (int)H->lv.size() - H->tail_lc;
  P.rnorm = H->o.recomb_norm;
  static bool attr_set = false;
  if (!attr_set) {
    LAMG_HIP(hipFuncSetAttribute((const void*)k_tail<T, MV>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr_set = true;
  }
  const int kid = sizeof(T) == 8 ? 14 : 15;
  if (!MV) prof_begin(H->s, kid);
  if (!MV && prof_on()) prof_count(kid, 0);  // latency-bound: time and launches only
  hipLaunchKernelGGL((k_tail<T, MV>), dim3(MV ? kc : 1), dim3(tail_launch<T>()), lds, H->s, P,
                     (const int4*)(H->tail_prog + seg.x), seg.y);
  if (!MV) prof_end(H->s);
  LAMG_HIP(hipGetLastError());
}
}  // namespace

template <class T>
void tail_run_next(Hierarchy* H) {
  launch_tail<T, false>(H, H->tail_levels, 1);
}
template void tail_run_next<double>(Hierarchy*);
template void tail_run_next<float>(Hierarchy*);

// Descriptors of the tail levels that point at the multi-vector workspace
// (rebuilt whenever the workspace or the single-vector descriptors change).
void tail_prepare_mv(Hierarchy* H) {
  tail_prepare(H);
  MVWork& W = H->mv;
  const int nl = (int)H->lv.size();
  const int lc = H->tail_lc;
  if (lc >= nl || W.tail_src == H->tail_levels) return;
  std::vector<TailLevel> d = H->tail_host;
  for (int l = lc; l < nl; ++l) {
    TailLevel& t = d[l - lc];
    const Vecs<double>& a = W.v64[l];
    const Vecs<float>& f = W.v32[l];
    t.x64 = a.x; t.b64 = a.b; t.r64 = a.r;
    t.x32 = f.x; t.b32 = f.b; t.r32 = f.r;
    for (int i = 0; i < 2; ++i) { t.X64[i] = a.X[i]; t.R64[i] = a.R[i]; t.X32[i] = f.X[i]; t.R32[i] = f.R[i]; }
  }
  void* p = dev_alloc(H->o, d.size() * sizeof(TailLevel));
  W.owned.push_back(p);
  LAMG_HIP(hipMemcpy(p, d.data(), d.size() * sizeof(TailLevel), hipMemcpyHostToDevice));
  W.tail = (TailLevel*)p;
  W.tail_src = H->tail_levels;
}

template <class T>
void tail_run_next_mv(Hierarchy* H) {
  launch_tail<T, true>(H, H->mv.tail, H->mv.k);
}
template void tail_run_next_mv<double>(Hierarchy*);
template void tail_run_next_mv<float>(Hierarchy*);

void invalidate_programs(Hierarchy* H) {
  H->tail_lc = -1;
  // the whole-hierarchy descriptors do not depend on the options; its
  // program does (released here: solves are synchronous, none is in flight)
  if (H->full_prog) {
    dev_free(H->o, H->full_prog);
    const size_t i = std::find(H->owned.begin(), H->owned.end(), (void*)H->full_prog) - H->owned.begin();
    H->owned.erase(H->owned.begin() + i);
    H->owned_bytes.erase(H->owned_bytes.begin() + i);
  }
  H->full_prog = nullptr;
  H->full_nops = 0;
  H->full_prog_host.clear();
  H->full_checked = false;
}

// ============================================== persistent many-graph solve
// One launch solves a batch of independent graphs.  Each workgroup takes the
// next graph from a queue (largest estimated work first) and runs that
// graph's whole solve: mean removal of b, the FP64 outer residual and its
// norm, cycles (the whole-hierarchy op program, the same ops as the
// single-vector cycle) until the graph's tolerance or cycle limit, and the
// scatter of x.  FP64 and FP32-with-FP64-refinement graphs can share a launch.
namespace {

struct BatchGraph {
  TailParams P;       // levels from 0
  const int4* prog;   // one finest cycle, mean removal included
  int nops, n, fp32, warm, max_cycles;
  double tol;
  const int* perm;    // colour order -> input order
  const double* b;    // caller's right-hand side (input order)
  double* x;          // caller's solution (input order)
  double* r64;        // outer residual (colour order)
};
struct BatchOut {
  double rel, r0, rk, removed;
  int cycles, status;
};

// One cycle's op program for a graph of the batch.  Called once per cycle,
// so the call costs nothing; inlining the interpreter into the batch loop
// would spill registers in its hot paths.
template <class T>
__device__ __attribute__((noinline)) void run_cycle(const TailParams& P, const int4* prog, int nops, char* lds,
                                                    double (*sh)[TAIL_WAVES]) {
  run_resident<T, false>(P, prog, nops, lds, sh);
}

// Fixed-order workgroup sum of f(i) over i < n.
template <class F>
__device__ inline double wg_sum(int n, double (*sh)[TAIL_WAVES], F f) {
  double v[1] = {0};
  for (int i = threadIdx.x; i < n; i += tail_nt()) v[0] += f(i);
  block_sums<1>(v, sh);
  return v[0];
}

__device__ __attribute__((always_inline)) inline void solve_graph(const BatchGraph& g, BatchOut* out, char* lds,
                                                                  double (*sh)[TAIL_WAVES], int cap) {
  const int tid = threadIdx.x, n = g.n;
  const TailLevel& L0 = g.P.L[0];
  double* b64 = L0.b64;
  double* x64 = L0.x64;
  double* r64 = g.r64;
  const double mean = wg_sum(n, sh, [&](int i) { return g.b[i]; }) / (double)n;
  for (int i = tid; i < n; i += tail_nt()) {
    b64[i] = g.b[g.perm[i]] - mean;
    x64[i] = g.warm ? g.x[g.perm[i]] : 0.0;
  }
  __syncthreads();
  const double nb = sqrt(wg_sum(n, sh, [&](int i) { return b64[i] * b64[i]; }));
  res_rows<double, false>(L0, x64, b64, L0.diag64, L0.rp, L0.val64, Col<double, false>{r64, 1}, (LP<double>)lds,
                          false, false, Col<double, false>{r64, 1});
  __syncthreads();
  const double r0 = sqrt(wg_sum(n, sh, [&](int i) { return r64[i] * r64[i]; }));
  double rk = r0;
  int it = 0;
  if (nb > 0) {
    const int maxc = g.max_cycles < cap ? g.max_cycles : cap;
    while (rk > g.tol * nb && it < maxc && isfinite(rk)) {
      if (!g.fp32) {
        run_cycle<double>(g.P, g.prog, g.nops, lds, sh);
      } else {
        float* b32 = L0.b32;
        float* x32 = L0.x32;
        const double mr = wg_sum(n, sh, [&](int i) { return r64[i]; }) / (double)n;
        for (int i = tid; i < n; i += tail_nt()) {
          b32[i] = (float)(r64[i] - mr);
          x32[i] = 0.0f;
        }
        __syncthreads();
        run_cycle<float>(g.P, g.prog, g.nops, lds, sh);
        for (int i = tid; i < n; i += tail_nt()) x64[i] += (double)x32[i];
        __syncthreads();
        const double mx = wg_sum(n, sh, [&](int i) { return x64[i]; }) / (double)n;
        for (int i = tid; i < n; i += tail_nt()) x64[i] -= mx;
        __syncthreads();
      }
      res_rows<double, false>(L0, x64, b64, L0.diag64, L0.rp, L0.val64, Col<double, false>{r64, 1}, (LP<double>)lds,
                              false, false, Col<double, false>{r64, 1});
      __syncthreads();
      rk = sqrt(wg_sum(n, sh, [&](int i) { return r64[i] * r64[i]; }));
      ++it;
    }
  }
  for (int i = tid; i < n; i += tail_nt()) g.x[g.perm[i]] = x64[i];
  if (tid == 0) {
    out->rel = nb > 0 ? rk / nb : 0.0;
    out->r0 = r0;
    out->rk = rk;
    out->removed = mean;
    out->cycles = it;
    out->status = !isfinite(rk) ? (int)LAMG_E_BREAKDOWN
                                : (nb > 0 && rk > g.tol * nb ? (int)LAMG_E_NOT_CONVERGED : (int)LAMG_OK);
  }
  __syncthreads();
}

__global__ __launch_bounds__(TAIL_THREADS) void k_batch(const BatchGraph* __restrict__ G, const int* __restrict__ order,
                                                        int count, int* queue, BatchOut* out, int cap) {
  __shared__ double sh[6][TAIL_WAVES];
  __shared__ int slot;
  extern __shared__ double lds_d[];
  for (;;) {
    if (threadIdx.x == 0) slot = atomicAdd(queue, 1);
    __syncthreads();
    const int q = slot;
    __syncthreads();
    if (q >= count) break;  // every workgroup leaves once the queue is drained
    const int gi = order[q];
    solve_graph(G[gi], out + gi, (char*)lds_d, sh, cap);
  }
}

// Launch configuration of the persistent kernel: the LDS staging budget of
// each workgroup, workgroups per compute unit, and the queue order.  Results
// do not depend on it (the same sums in the same order); only time does.
struct BatchConfig {
  int lds, per_cu, lpt;
};
// the LDS budgets (one copy of the graphs' descriptors each); two workgroups
// fit a compute unit's 160 KB only with the smallest
constexpr int kNumBatchLds = 4;
constexpr int kBatchLds[kNumBatchLds] = {128 * 1024, 64 * 1024, 96 * 1024, 152 * 1024};
constexpr BatchConfig kBatchConfigs[] = {
    {128 * 1024, 1, 1}, {64 * 1024, 2, 1}, {64 * 1024, 1, 1}, {128 * 1024, 1, 0}, {96 * 1024, 1, 1},
    {152 * 1024, 1, 1}, {64 * 1024, 2, 0}, {96 * 1024, 1, 0}, {152 * 1024, 1, 0}, {64 * 1024, 1, 0}};
constexpr int kNumBatchConfigs = sizeof(kBatchConfigs) / sizeof(kBatchConfigs[0]);
constexpr int kBatchMaxLds = 152 * 1024;
// tuning runs cap every graph at this many cycles: the ranking of the
// configurations is that of the per-cycle work, at a fraction of a solve
constexpr int kTuneCycles = 2;
int lds_slot(int lds) {
  for (int v = 0; v < kNumBatchLds; ++v)
    if (kBatchLds[v] == lds) return v;
  return 0;
}

struct TunerEntry {
  uint64_t key;
  int best;
};
std::vector<TunerEntry> g_tuned;  // best configuration per batch signature (process lifetime)
int g_batch_forced = -1;          // test hook: force a configuration
bool g_cache_loaded = false;

// Persisted choices: with LAMG_TUNE_CACHE set to a file, every tuned batch
// signature is appended to it as "<key hex> <config>" and a later process
// reads the file before its first tuning (entries with a configuration index
// outside the table are ignored).  The key covers the device (name and
// compute units) and the batch's shape.
void tune_cache_load() {
  if (g_cache_loaded) return;
  g_cache_loaded = true;
  const char* path = std::getenv("LAMG_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  unsigned long long k = 0;
  int c = 0;
  while (std::fscanf(f, "%llx %d", &k, &c) == 2)
    if (c >= 0 && c < kNumBatchConfigs) g_tuned.push_back({(uint64_t)k, c});
  std::fclose(f);
}
void tune_cache_store(uint64_t key, int best) {
  const char* path = std::getenv("LAMG_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%016llx %d\n", (unsigned long long)key, best);
  std::fclose(f);
}

}  // namespace

void batch_prepare(Hierarchy* H) {
  if (H->full_prog) return;
  if (!H->full_levels) {
    std::vector<TailLevel> d = build_desc(H, 0);
    TailLevel* dd = dnew<TailLevel>(H, d.size());
    LAMG_HIP(hipMemcpy(dd, d.data(), d.size() * sizeof(TailLevel), hipMemcpyHostToDevice));
    H->full_levels = dd;
    H->full_host = d;
  }
  std::vector<int4> prog;
  std::vector<int2> segs;
  build_prog(H, 0, prog, segs);
  int4* dp = dnew<int4>(H, std::max<size_t>(prog.size(), 1));
  LAMG_HIP(hipMemcpy(dp, prog.data(), prog.size() * sizeof(int4), hipMemcpyHostToDevice));
  H->full_nops = (int)prog.size();
  H->full_prog = dp;
  H->full_prog_host = prog;
  H->full_checked = false;
}

namespace {
// Device block of one persistent launch: the graphs' descriptors (one copy
// per LDS budget), the two queue orders, the queue counter and the results.
constexpr size_t batch_buffer_bytes(size_t count) {
  return 4 * count * sizeof(BatchGraph) + 2 * count * sizeof(int) + 256 + count * sizeof(BatchOut);
}

// Scratch of the allocation-free entry (lamg_solve_batch_noalloc): the block
// above for up to LAMG_NOALLOC_MAX_GRAPHS graphs, one copy per device for the
// life of the process.  Host code never passes this symbol to a kernel: its
// device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kNoallocBytes = batch_buffer_bytes(LAMG_NOALLOC_MAX_GRAPHS);
static __device__ __align__(256) char scratch[kNoallocBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (looked up on the first call on
// that device, with the device current).
char* noalloc_scratch() {
  int dev = 0;
  LAMG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw DevError{hipErrorInvalidDevice};
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    LAMG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw DevError{hipErrorInvalidSymbol};
    g_scratch_ptr[dev] = (char*)p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" lamg_status lamg_t_batch_config(int32_t config) {
  if (config < -1 || config >= kNumBatchConfigs) return LAMG_E_INVALID_ARG;
  g_batch_forced = config;
  return LAMG_OK;
}

lamg_status solve_graphs(int count, Hierarchy* const* hs, const double* const* B, double* const* X,
                         lamg_info* infos, bool noalloc) {
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = hs[0]->s;
  std::vector<BatchGraph> G(count);
  std::vector<double> work(count);
  uint64_t key = 1469598103934665603ULL;  // FNV-1a over the batch's shape
  bool warm = false;
  for (int i = 0; i < count; ++i) {
    Hierarchy* H = hs[i];
    if (noalloc && (!H->full_prog || !H->full_levels)) return LAMG_E_INVALID_ARG;  // (prepared at setup)
    batch_prepare(H);
    if (!H->full_checked) {
      std::vector<int2> budgets;
      for (int v = 0; v < kNumBatchLds; ++v) budgets.push_back(make_int2(kBatchLds[v], kBatchLds[v] / 2));
      check_or_throw(program_check(H, H->full_host, H->full_prog_host, 0, budgets));
      H->full_checked = true;
    }
    BatchGraph& g = G[i];
    std::memset(&g, 0, sizeof(g));
    g.P.L = (const TailLevel*)H->full_levels;
    g.P.lc = 0;
    g.P.Minv = H->cinv;
    g.P.nL = H->nL;
    g.P.crelax = H->coarsest_relax ? 1 : 0;
    g.P.csweeps = H->o.coarsest_sweeps;
    g.P.mu = H->o.mu;
    g.P.kc = 1;
    g.P.nlev = (int)H->lv.size();
    g.P.rnorm = H->o.recomb_norm;
    g.prog = H->full_prog;
    g.nops = H->full_nops;
    g.n = H->lv[0].n;
    g.fp32 = H->o.precision == LAMG_FP32_REFINE;
    g.warm = H->o.warm_start != 0;
    g.max_cycles = H->o.max_cycles;
    g.tol = H->o.tol;
    g.perm = H->lv[0].perm;
    g.b = B[i];
    g.x = X[i];
    g.r64 = H->r64;
    work[i] = (double)H->bytes_per_cycle;
    warm = warm || g.warm;
    for (uint64_t v : {(uint64_t)g.n, (uint64_t)H->lv[0].nnz, (uint64_t)H->lv.size(), (uint64_t)g.fp32}) {
      key ^= v;
      key *= 1099511628211ULL;
    }
  }
  // largest estimated work first (ties: input order)
  std::vector<int> lpt(count), natural(count);
  for (int i = 0; i < count; ++i) lpt[i] = natural[i] = i;
  std::stable_sort(lpt.begin(), lpt.end(), [&](int a, int b) { return work[a] > work[b]; });
  int dev = 0, ncu = 0;
  LAMG_HIP(hipGetDevice(&dev));
  LAMG_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  {
    hipDeviceProp_t prop;
    LAMG_HIP(hipGetDeviceProperties(&prop, dev));
    for (const char* c = prop.gcnArchName; *c; ++c) {
      key ^= (uint64_t)(unsigned char)*c;
      key *= 1099511628211ULL;
    }
    key ^= (uint64_t)ncu;
    key *= 1099511628211ULL;
  }
  static bool attr = false;
  if (!attr) {
    LAMG_HIP(hipFuncSetAttribute((const void*)k_batch, hipFuncAttributeMaxDynamicSharedMemorySize, kBatchMaxLds));
    attr = true;
  }
  // device copies: graphs (one copy per LDS budget), orders, queue, results;
  // in the call's own block (through the first handle's allocator) or in
  // the static scratch of the allocation-free entry
  const size_t gb = (size_t)count * sizeof(BatchGraph);
  const size_t bytes = batch_buffer_bytes((size_t)count);
  const lamg_options& ao = hs[0]->o;
  char* buf = noalloc ? noalloc_scratch() : (char*)dev_alloc(ao, bytes);
  struct Free {
    const lamg_options& o;
    char* p;
    ~Free() {
      if (p) dev_free(o, p);
    }
  } guard{ao, noalloc ? nullptr : buf};
  static_assert(kNumBatchLds == 4, "batch_buffer_bytes holds one descriptor copy per LDS budget");
  BatchGraph* dG[kNumBatchLds];
  for (int v = 0; v < kNumBatchLds; ++v) dG[v] = (BatchGraph*)(buf + v * gb);
  int* dorder[2] = {(int*)(buf + kNumBatchLds * gb), (int*)(buf + kNumBatchLds * gb) + count};
  int* queue = (int*)(buf + kNumBatchLds * gb + 2 * (size_t)count * sizeof(int));
  BatchOut* dout = (BatchOut*)(buf + kNumBatchLds * gb + 2 * (size_t)count * sizeof(int) + 256);
  for (int v = 0; v < kNumBatchLds; ++v) {
    const int lds = kBatchLds[v];
    for (BatchGraph& g : G) {
      g.P.lds_bytes = lds;
      g.P.res_bytes = lds / 2;
    }
    LAMG_HIP(hipMemcpyAsync(dG[v], G.data(), gb, hipMemcpyHostToDevice, s));
    LAMG_HIP(hipStreamSynchronize(s));
  }
  LAMG_HIP(hipMemcpyAsync(dorder[0], natural.data(), count * sizeof(int), hipMemcpyHostToDevice, s));
  LAMG_HIP(hipMemcpyAsync(dorder[1], lpt.data(), count * sizeof(int), hipMemcpyHostToDevice, s));
  auto launch = [&](int c, int cap) {
    const BatchConfig& cf = kBatchConfigs[c];
    fill<int>(s, queue, 0, 1);
    const int grid = std::max(1, std::min(count, ncu * cf.per_cu));
    hipLaunchKernelGGL(k_batch, dim3(grid), dim3(TAIL_THREADS), cf.lds, s, (const BatchGraph*)dG[lds_slot(cf.lds)],
                       (const int*)dorder[cf.lpt], count, queue, dout, cap);
    LAMG_HIP(hipGetLastError());
  };
  int best = 0;
  if (g_batch_forced >= 0) {
    best = g_batch_forced;
  } else {
    if (!noalloc) tune_cache_load();
    bool found = false;
    for (const TunerEntry& e : g_tuned)
      if (e.key == key) { best = e.best; found = true; }
    if (!found && !warm && !noalloc) {
      // time every configuration on this batch, each graph capped at
      // kTuneCycles cycles (the same ops per cycle as the real solve), and
      // keep the fastest for this batch signature
      hipEvent_t a, b;
      LAMG_HIP(hipEventCreate(&a));
      LAMG_HIP(hipEventCreate(&b));
      float bestms = 0;
      for (int c = 0; c < kNumBatchConfigs; ++c) {
        LAMG_HIP(hipEventRecord(a, s));
        launch(c, kTuneCycles);
        LAMG_HIP(hipEventRecord(b, s));
        LAMG_HIP(hipEventSynchronize(b));
        float ms = 0;
        LAMG_HIP(hipEventElapsedTime(&ms, a, b));
        if (c == 0 || ms < bestms) { bestms = ms; best = c; }
      }
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
      g_tuned.push_back({key, best});
      tune_cache_store(key, best);
    }
  }
  launch(best, 1 << 30);
  std::vector<BatchOut> out(count);
  LAMG_HIP(hipMemcpyAsync(out.data(), dout, count * sizeof(BatchOut), hipMemcpyDeviceToHost, s));
  LAMG_HIP(hipStreamSynchronize(s));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  lamg_status worst = LAMG_OK;
  for (int i = 0; i < count; ++i) {
    const BatchOut& o = out[i];
    if (o.status != LAMG_OK && worst == LAMG_OK) worst = (lamg_status)o.status;
    if (!infos) continue;
    lamg_info& f = infos[i];
    std::memset(&f, 0, sizeof(f));
    f.cycles = o.cycles;
    f.levels = (int)hs[i]->lv.size();
    f.rel_residual = o.rel;
    f.acf = o.cycles > 0 && o.r0 > 0 ? std::pow(o.rk / o.r0, 1.0 / o.cycles) : 0.0;
    f.removed_mean = o.removed;
    f.setup_ms = hs[i]->setup_ms;
    f.solve_ms = ms;
    f.bytes_moved = (int64_t)o.cycles * cycle_bytes(hs[i], hs[i]->o.precision);
  }
  return worst;
}

}  // namespace lamg
