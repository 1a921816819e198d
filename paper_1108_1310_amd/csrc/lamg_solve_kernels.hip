// Solve-phase kernels: multicolour Gauss-Seidel and residual over tiled CSR
// rows, aggregation / elimination transfers, deterministic reductions for
// iterate recombination, mean removal and norms, and the coarsest solve.
#include <algorithm>
#include <climits>
#include <cmath>

#include "lamg_device.hpp"
#include "lamg_internal.hpp"
#include "lamg_relax.hpp"
#include "../../include/lamg_test.h"

namespace lamg {

// ---------------------------------------------------------------- relaxation
// ---------------------------------------------------------- instrumentation
// A span is an event pair around a run of back-to-back launches of one
// kernel (a whole sweep: every colour class of a level).  Kernels of one
// stream run without gaps between them once they are queued, so span time /
// launches is the kernel's average duration; one pair per launch would add
// the event markers' own latency to every launch.  Instrumented cycles are
// launched eagerly from the host, which enqueues a launch more slowly than
// a short colour class runs; a span of several launches therefore starts
// behind a hold (one wavefront sleeping for a bounded wall-clock time, 15 us
// per launch of the span, 40 us for the multi-vector kernels, whose launches
// take the host longer) during which the host queues the span's launches, so
// that the span holds kernel time and not host gaps.
namespace {
__global__ void k_prof_hold(long long ticks) {
  const long long t0 = wall_clock64();
  // bounded twice: by the wall clock and by an iteration cap (~50 ms)
  for (int i = 0; i < (1 << 20) && wall_clock64() - t0 < ticks; ++i) __builtin_amdgcn_s_sleep(2);
}
long long wall_ticks_per_us() {
  static long long t = [] {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
      khz = 100000;  // 100 MHz
    return std::max<long long>(1, khz / 1000);
  }();
  return t;
}
struct Pair {
  hipEvent_t a, b;
  int kid;
  int64_t bytes, launches;
};
struct Prof {
  bool on = false;
  bool open = false;
  Pair cur{};
  std::vector<Pair> pend;  // closed spans whose events are not read yet
  std::vector<hipEvent_t> pool;
  double ms[PROF_KERNELS] = {};
  int64_t bytes[PROF_KERNELS] = {}, launches[PROF_KERNELS] = {};
};
Prof g_prof;
hipEvent_t new_event() {
  Prof& P = g_prof;
  if (!P.pool.empty()) {
    hipEvent_t e = P.pool.back();
    P.pool.pop_back();
    return e;
  }
  hipEvent_t e;
  LAMG_HIP(hipEventCreate(&e));
  return e;
}
}  // namespace
bool prof_on() { return g_prof.on; }
void prof_begin(hipStream_t s, int kernel, int launches) {
  Prof& P = g_prof;
  if (!P.on || P.open) return;
  if (launches > 1) {
    const long long us = kernel >= 4 && kernel <= 7 ? 40 : 15;
    hipLaunchKernelGGL(k_prof_hold, dim3(1), dim3(64), 0, s, (long long)launches * us * wall_ticks_per_us());
    LAMG_HIP(hipGetLastError());
  }
  P.cur = Pair{new_event(), nullptr, kernel, 0, 0};
  LAMG_HIP(hipEventRecord(P.cur.a, s));
  P.open = true;
}
void prof_count(int kernel, int64_t bytes) {
  Prof& P = g_prof;
  if (!P.open || P.cur.kid != kernel) return;
  P.cur.bytes += bytes;
  P.cur.launches += 1;
}
void prof_end(hipStream_t s) {
  Prof& P = g_prof;
  if (!P.open) return;
  P.cur.b = new_event();
  LAMG_HIP(hipEventRecord(P.cur.b, s));
  P.pend.push_back(P.cur);
  P.open = false;
}
// Read every pending span (waiting for it) into the per-kernel totals.
void prof_flush() {
  Prof& P = g_prof;
  for (const Pair& q : P.pend) {
    float t = 0;
    LAMG_HIP(hipEventSynchronize(q.b));
    LAMG_HIP(hipEventElapsedTime(&t, q.a, q.b));
    P.ms[q.kid] += t;
    P.bytes[q.kid] += q.bytes;
    P.launches[q.kid] += q.launches;
    P.pool.push_back(q.a);
    P.pool.push_back(q.b);
  }
  P.pend.clear();
}

template <class T, int MODE>
static void launch_relax(hipStream_t s, const int* rp, const int* ci, const Tiles& t, const T* val, const T* diag,
                         const T* b, T* x, T* r, const int* map = nullptr, int zthr = INT_MAX) {
  const int grid = t.blocks();
  if (grid == 0) return;
  if (MODE == 2) {
    hipLaunchKernelGGL((k_relax<T, MODE>), dim3(grid), dim3(RELAX_THREADS), 0, s, rp, ci, val, diag, b, x, r,
                       (const int4*)t.vlong, t.nvlong, (const int4*)t.med, t.nmed, t.nmed_blocks, (const int4*)t.stream, t.nstream, map,
                       zthr);
    LAMG_HIP(hipGetLastError());
    return;
  }
  const bool prof = prof_on();
  const int kid = MODE + (sizeof(T) == 4 ? 2 : 0);
  // matrix stream (column index + value per entry, row pointer + diagonal per
  // row) and three vector streams per row (b or x read, x read, x or r write)
  const int64_t bytes = t.nnz * (4 + (int64_t)sizeof(T)) + t.rows * (4 + (int64_t)sizeof(T)) +
                        3 * t.rows * (int64_t)sizeof(T);
  if (prof) prof_count(kid, bytes);
  hipLaunchKernelGGL((k_relax<T, MODE>), dim3(grid), dim3(RELAX_THREADS), 0, s, rp, ci, val, diag, b, x, r,
                     (const int4*)t.vlong, t.nvlong, (const int4*)t.med, t.nmed, t.nmed_blocks, (const int4*)t.stream, t.nstream, map,
                       zthr);
  LAMG_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ hubs
// Partial sums of the hub rows once colours < hub_k are final for the sweep:
// p_u = b_u + the row's entries into those colours (its column prefix), one
// wavefront per row, 64 strided partial sums folded by the butterfly.
template <class T>
__global__ __launch_bounds__(256) void k_hub_partial(int nh, int r0, const int* __restrict__ rp,
                                                     const int* __restrict__ ci, const T* __restrict__ val,
                                                     const int* __restrict__ hrp, const T* __restrict__ b,
                                                     const T* __restrict__ x, T* __restrict__ p) {
  const int i = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6), lane = threadIdx.x & 63;
  if (i >= nh) return;
  const int u = r0 + i;
  const int p0 = rp[u];
  const int pe = rp[u + 1] - (hrp[i + 1] - hrp[i]);
  const T bu = b ? b[u] : T(0);
  T s = 0;
  int t = p0 + lane;
  for (; t + 192 < pe; t += 256) {
    const int c0 = ci[t], c1 = ci[t + 64], c2 = ci[t + 128], c3 = ci[t + 192];
    const T w0 = val[t], w1 = val[t + 64], w2 = val[t + 128], w3 = val[t + 192];
    const T x0 = x[c0], x1 = x[c1], x2 = x[c2], x3 = x[c3];
    s += w0 * x0;
    s += w1 * x1;
    s += w2 * x2;
    s += w3 * x3;
  }
  for (; t < pe; t += 64) s += val[t] * x[ci[t]];
  s = dev::wave_fold(s);
  if (lane == 0) p[i] = bu + s;
}

// Sum over the 16 lanes of a DPP row: swap neighbours, swap pairs, mirror of
// 8, mirror of 16.  The two operands of every add are the same pair in every
// lane, so all 16 lanes end with the same value.  The 16 lanes must be all
// active or all inactive.
template <int CTRL>
__device__ inline float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_f(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <class T>
__device__ inline T row16_sum(T s) {
  s += dpp_f<0xB1>(s);   // quad_perm(1, 0, 3, 2)
  s += dpp_f<0x4E>(s);   // quad_perm(2, 3, 0, 1)
  s += dpp_f<0x141>(s);  // row_half_mirror
  s += dpp_f<0x140>(s);  // row_mirror
  return s;
}

// The hub colour phases in one workgroup.  x, p and the diagonal of the hub
// rows stay in LDS for the whole sweep.  The phases are cut into chunks of
// whole rows of one colour with at most HUB_CHUNK hub-to-hub entries (a
// chunk table built at setup; no row is longer, since its columns are
// distinct hub rows).  A chunk stages the products of its entries in LDS,
// then each group of 16 lanes takes rows of the chunk, sums a row's products
// with 16 strided partial sums folded by DPP (row16_sum), and sets
// x_u = (p_u + sum) / a_uu.  Rows of one colour are not adjacent, so a chunk
// never reads what it writes.  The index and weight loads of a chunk do not
// depend on x: they are issued HUB_DEPTH chunks ahead, into HUB_DEPTH
// register sets used in turn.  A chunk is bound by the LDS traffic of its
// one compute unit (x gathers, product writes and reads: 24 bytes per FP64
// entry), not by these loads.
constexpr int HUB_DEPTH = 2;
template <class T>
struct HubSm {
  T *prod, *xs, *ps, *ds;
  int* srp;
  int2* sck;
};
template <class T>
__device__ __forceinline__ void hub_load(const HubSm<T>& m, int k, int nck, const int* __restrict__ hci,
                                         const T* __restrict__ hval, int (&cj)[HUB_PER], T (&wj)[HUB_PER]) {
  int e0 = 0, e1 = 0;
  if (k < nck) {
    const int2 c = m.sck[k];
    e0 = m.srp[c.x];
    e1 = m.srp[c.y];
  }
#pragma unroll
  for (int q = 0; q < HUB_PER; ++q) {
    const int e = e0 + (int)threadIdx.x + q * HUB_THREADS;
    cj[q] = e < e1 ? hci[e] : 0;
    wj[q] = e < e1 ? hval[e] : T(0);
  }
}
template <class T>
__device__ __forceinline__ void hub_chunk(const HubSm<T>& m, int k, int nck, const int* __restrict__ hci,
                                          const T* __restrict__ hval, int (&cj)[HUB_PER], T (&wj)[HUB_PER]) {
  const int t = threadIdx.x, g = t >> 4, gl = t & 15;
  const int2 c = m.sck[k];
  const int e0 = m.srp[c.x], e1 = m.srp[c.y];
#pragma unroll
  for (int q = 0; q < HUB_PER; ++q) {
    const int e = e0 + t + q * HUB_THREADS;
    if (e < e1) m.prod[e - e0] = wj[q] * m.xs[cj[q]];
  }
  hub_load<T>(m, k + HUB_DEPTH, nck, hci, hval, cj, wj);
  __syncthreads();
  for (int u = c.x + g; u < c.y; u += HUB_THREADS / 16) {
    const int a = m.srp[u] - e0, z = m.srp[u + 1] - e0;
    const T pu = m.ps[u], du = m.ds[u];
    T s = 0;
    int e = a + gl;
    for (; e + 48 < z; e += 64) {
      const T v0 = m.prod[e], v1 = m.prod[e + 16], v2 = m.prod[e + 32], v3 = m.prod[e + 48];
      s += v0;
      s += v1;
      s += v2;
      s += v3;
    }
    for (; e < z; e += 16) s += m.prod[e];
    s = row16_sum<T>(s);
    if (gl == 0) m.xs[u] = (pu + s) / du;
  }
  __syncthreads();
}
template <class T>
__global__ __launch_bounds__(HUB_THREADS) void k_hub_sweep(int nh, int nck, const int2* __restrict__ ck,
                                                          const int* __restrict__ hrp, const int* __restrict__ hci,
                                                          const T* __restrict__ hval, const T* __restrict__ p,
                                                          const T* __restrict__ dg, T* __restrict__ xh) {
  extern __shared__ __align__(16) unsigned char hub_smem[];
  constexpr int HT = HUB_THREADS;
  HubSm<T> m;
  m.prod = (T*)hub_smem;       // [HUB_CHUNK]
  m.xs = m.prod + HUB_CHUNK;   // [nh]
  m.ps = m.xs + nh;            // [nh]
  m.ds = m.ps + nh;            // [nh]
  m.srp = (int*)(m.ds + nh);   // [nh + 1]
  const size_t ck_off = ((size_t)HUB_CHUNK * sizeof(T) + 3 * (size_t)nh * sizeof(T) + ((size_t)nh + 1) * 4 + 7) & ~(size_t)7;
  m.sck = (int2*)(hub_smem + ck_off);  // [nck]
  const int t = threadIdx.x;
  for (int i = t; i < nh; i += HT) {
    m.xs[i] = xh[i];
    m.ps[i] = p[i];
    m.ds[i] = dg[i];
  }
  for (int i = t; i <= nh; i += HT) m.srp[i] = hrp[i];
  for (int i = t; i < nck; i += HT) m.sck[i] = ck[i];
  __syncthreads();
  int cja[HUB_PER], cjb[HUB_PER];
  T wja[HUB_PER], wjb[HUB_PER];
  hub_load<T>(m, 0, nck, hci, hval, cja, wja);
  hub_load<T>(m, 1, nck, hci, hval, cjb, wjb);
  for (int k = 0; k < nck; k += HUB_DEPTH) {
    hub_chunk<T>(m, k, nck, hci, hval, cja, wja);
    if (k + 1 < nck) hub_chunk<T>(m, k + 1, nck, hci, hval, cjb, wjb);
  }
  for (int i = t; i < nh; i += HT) xh[i] = m.xs[i];
}

template <class T>
struct HubVals;
template <>
struct HubVals<double> {
  static const double* val(const Level& L) { return L.hub_val; }
  static double* p(const Level& L) { return L.hub_p; }
};
template <>
struct HubVals<float> {
  static const float* val(const Level& L) { return L.hub_val32; }
  static float* p(const Level& L) { return L.hub_p32; }
};

// The colours >= hub_k of one GS sweep: the partial sums, then the phases.
template <class T>
static void hub_sweep(hipStream_t s, const Level& L, const T* val, const T* diag, const T* b, T* x) {
  const int nh = L.hub_n, r0 = L.hub_r0;
  const size_t lds = (((size_t)HUB_CHUNK * sizeof(T) + 3 * (size_t)nh * sizeof(T) + ((size_t)nh + 1) * 4 + 7) &
                      ~(size_t)7) + (size_t)L.hub_nck * sizeof(int2);
  static bool attr_set = false;
  if (!attr_set) {
    LAMG_HIP(hipFuncSetAttribute((const void*)k_hub_sweep<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)(HUB_CHUNK * sizeof(T) + 3 * HUB_MAX_ROWS * sizeof(T) +
                                       (HUB_MAX_ROWS + 2) * sizeof(int) + HUB_MAX_CHUNKS * sizeof(int2))));
    attr_set = true;
  }
  if (nh > HUB_MAX_ROWS || L.hub_nck < 1 || L.hub_nck > HUB_MAX_CHUNKS) throw DevError{hipErrorInvalidValue};
  T* p = HubVals<T>::p(L);
  const bool prof = prof_on();
  const int kid = sizeof(T) == 8 ? 8 : 9;
  const int64_t s_v = sizeof(T);
  if (prof) prof_count(kid, L.hub_low_nnz * (4 + s_v) + (int64_t)nh * (8 + 3 * s_v));
  hipLaunchKernelGGL(k_hub_partial<T>, dim3((unsigned)(((int64_t)nh * 64 + 255) / 256)), dim3(256), 0, s, nh, r0,
                     (const int*)L.rp, (const int*)L.ci, val, (const int*)L.hub_rp, b, (const T*)x, p);
  LAMG_HIP(hipGetLastError());
  if (prof) prof_count(kid, (int64_t)L.hub_nnz * (4 + s_v) + (int64_t)nh * (4 + 4 * s_v));
  hipLaunchKernelGGL(k_hub_sweep<T>, dim3(1), dim3(HUB_THREADS), lds, s, nh, L.hub_nck, (const int2*)L.hub_ck,
                     (const int*)L.hub_rp, (const int*)L.hub_ci, HubVals<T>::val(L), (const T*)p, diag + r0, x + r0);
  LAMG_HIP(hipGetLastError());
}

template <class T>
void gs_colour(hipStream_t s, const Level& L, int c, const T* val, const T* diag, const T* b, T* x, bool from_zero) {
  // from a zero iterate, colours c and above still hold +0: no gathers there
  launch_relax<T, 0>(s, L.rp, L.ci, L.tiles[c], val, diag, b, x, (T*)nullptr, nullptr,
                     from_zero ? L.cptr[c] : INT_MAX);
}
template <class T>
void gs_sweep(hipStream_t s, const Level& L, const T* val, const T* diag, const T* b, T* x, bool from_zero) {
  const int K = L.hub_k >= 0 ? L.hub_k : L.ncol;
  prof_begin(s, sizeof(T) == 4 ? 2 : 0, K);
  for (int c = 0; c < K; ++c) gs_colour<T>(s, L, c, val, diag, b, x, from_zero);
  prof_end(s);
  if (K < L.ncol) {
    prof_begin(s, sizeof(T) == 4 ? 9 : 8);
    hub_sweep<T>(s, L, val, diag, b, x);
    prof_end(s);
  }
}
template <class T>
void residual(hipStream_t s, const Level& L, const T* val, const T* diag, const T* b, const T* x, T* r) {
  prof_begin(s, sizeof(T) == 4 ? 3 : 1);
  launch_relax<T, 1>(s, L.rp, L.ci, L.all, val, diag, b, (T*)x, r);
  prof_end(s);
}
template void gs_colour<double>(hipStream_t, const Level&, int, const double*, const double*, const double*, double*,
                                bool);
template void gs_colour<float>(hipStream_t, const Level&, int, const float*, const float*, const float*, float*, bool);
template void gs_sweep<double>(hipStream_t, const Level&, const double*, const double*, const double*, double*, bool);
template void gs_sweep<float>(hipStream_t, const Level&, const float*, const float*, const float*, float*, bool);
template void residual<double>(hipStream_t, const Level&, const double*, const double*, const double*, const double*, double*);
template void residual<float>(hipStream_t, const Level&, const float*, const float*, const float*, const float*, float*);

// Multi-vector GS on A X = 0 or A X = B for K <= 10 vectors stored n x K
// row-major (test-vector relaxation).  Thread per short row, K running sums.
constexpr int KMAX = 10;
__global__ __launch_bounds__(256) void k_gs_multi_short(const int* __restrict__ rp, const int* __restrict__ ci,
                                                        const double* __restrict__ val, const double* __restrict__ diag,
                                                        const double* __restrict__ B, double* X, int K, int r0, int r1) {
  const int u = r0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= r1) return;
  const int p0 = rp[u], len = rp[u + 1] - p0;
  if (len > SHORT_ROW) return;
  double s[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) s[k] = 0;
  for (int t = 0; t < len; ++t) {
    const double w = val[p0 + t];
    const double* xv = X + (size_t)ci[p0 + t] * K;
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      if (k < K) s[k] += w * xv[k];
  }
  const double d = diag[u];
#pragma unroll
  for (int k = 0; k < KMAX; ++k)
    if (k < K) {
      const double bu = B ? B[(size_t)u * K + k] : 0.0;
      X[(size_t)u * K + k] = (bu + s[k]) / d;
    }
}
__global__ __launch_bounds__(256) void k_gs_multi_long(const int* __restrict__ rp, const int* __restrict__ ci,
                                                       const double* __restrict__ val, const double* __restrict__ diag,
                                                       const double* __restrict__ B, double* X, int K,
                                                       const int* __restrict__ longrows, int nlong) {
  const int idx = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (idx >= nlong) return;
  const int u = longrows[idx];
  const int p0 = rp[u], len = rp[u + 1] - p0;
  for (int k = 0; k < K; ++k) {
    const double s = dev::row_sum_wave<double>(len, lane, [&](int t) { return val[p0 + t] * X[(size_t)ci[p0 + t] * K + k]; });
    if (lane == 0) {
      const double bu = B ? B[(size_t)u * K + k] : 0.0;
      X[(size_t)u * K + k] = (bu + s) / diag[u];
    }
  }
}

void gs_multi_sweep(hipStream_t s, const Level& L, const double* b, double* X, int K) {
  for (int c = 0; c < L.ncol; ++c) {
    const int r0 = L.cptr[c], r1 = L.cptr[c + 1];
    if (r1 > r0)
      hipLaunchKernelGGL(k_gs_multi_short, dim3((r1 - r0 + 255) / 256), dim3(256), 0, s, L.rp, L.ci, L.val, L.diag, b,
                         X, K, r0, r1);
    const Tiles& t = L.tiles[c];
    if (t.nlong)
      hipLaunchKernelGGL(k_gs_multi_long, dim3((t.nlong + 3) / 4), dim3(256), 0, s, L.rp, L.ci, L.val, L.diag, b, X, K,
                         t.longrows, t.nlong);
  }
  LAMG_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- transfers
// Aggregation restriction b^c_U = mu * sum_{u in T_U} r_u (eq. galerkin2),
// members summed in ascending id order.
template <class T>
__global__ void k_restrict_agg(int nc, const int* __restrict__ aptr, const int* __restrict__ mem,
                               const T* __restrict__ r, T* __restrict__ bc, T mu) {
  const int U = blockIdx.x * blockDim.x + threadIdx.x;
  if (U >= nc) return;
  T s = 0;
  for (int j = aptr[U]; j < aptr[U + 1]; ++j) s += r[mem[j]];
  bc[U] = mu * s;
}
// Caliber-1 interpolation x_u += e_{agg(u)} (eq. correction).
template <class T>
__global__ void k_interp_agg(int n, const int* __restrict__ agg, const T* __restrict__ e, T* __restrict__ x) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n) x[u] += e[agg[u]];
}
// Exact elimination correction: e_C = e^c, e_F = (r_F + W_FC e^c) / a_FF.
template <class T>
__global__ void k_interp_elim(int n, const int* __restrict__ cidx, const int* __restrict__ rp, const int* __restrict__ ci,
                              const T* __restrict__ val, const T* __restrict__ diag, const T* __restrict__ r,
                              const T* __restrict__ e, T* __restrict__ x) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const int c = cidx[u];
  if (c >= 0) { x[u] += e[c]; return; }
  T s = r[u];
  for (int t = rp[u]; t < rp[u + 1]; ++t) s += val[t] * e[cidx[ci[t]]];
  x[u] += s / diag[u];
}
template <class T>
__global__ void k_fill(T* p, T v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

static inline dim3 g1(int n, int b = 256) { return dim3((unsigned)std::max(1, (n + b - 1) / b)); }

template <class T>
void restrict_agg(hipStream_t s, const Level& C, int nfine, const T* r, T* bc, T mu) {
  const int kid = sizeof(T) == 8 ? 10 : 11;
  const int64_t sx = sizeof(T);
  prof_begin(s, kid);
  // members' indices and residuals, aggregate pointers and coarse values
  if (prof_on()) prof_count(kid, (int64_t)nfine * (sx + 4) + (int64_t)C.n * (sx + 4));
  hipLaunchKernelGGL(k_restrict_agg<T>, g1(C.n), dim3(256), 0, s, C.n, C.agg_ptr, C.members, r, bc, mu);
  prof_end(s);
}
template <class T>
void interp_agg(hipStream_t s, const Level& C, int nfine, const T* e, T* x) {
  const int kid = sizeof(T) == 8 ? 12 : 13;
  const int64_t sx = sizeof(T);
  prof_begin(s, kid);
  // aggregate index, x read and written per fine node; coarse values
  if (prof_on()) prof_count(kid, (int64_t)nfine * (4 + 2 * sx) + (int64_t)C.n * sx);
  hipLaunchKernelGGL(k_interp_agg<T>, g1(nfine), dim3(256), 0, s, nfine, C.agg, e, x);
  prof_end(s);
}
// Elimination restriction on the precomputed C-side stencil, with the
// relaxation kernel's tiling (hub rows of C nodes have many F neighbours).
template <class T>
void restrict_elim(hipStream_t s, const Level& C, const T* r, T* bc) {
  const T* ev;
  if constexpr (sizeof(T) == 8) ev = (const T*)C.er_val;
  else ev = (const T*)C.er_val32;
  launch_relax<T, 2>(s, C.er_rp, C.er_ci, C.er_tiles, ev, (const T*)nullptr, (const T*)nullptr, (T*)r, bc,
                     C.cfine);
}
template <class T>
void interp_elim(hipStream_t s, const Level& F, const Level& C, const T* val, const T* diag, const T* r, const T* e,
                 T* x) {
  hipLaunchKernelGGL(k_interp_elim<T>, g1(F.n), dim3(256), 0, s, F.n, C.cidx, F.rp, F.ci, val, diag, r, e, x);
}
template <class T>
void fill(hipStream_t s, T* p, T v, int n) {
  if (n > 0) hipLaunchKernelGGL(k_fill<T>, g1(n), dim3(256), 0, s, p, v, n);
}
#define INST(T)                                                                                         \
  template void restrict_agg<T>(hipStream_t, const Level&, int, const T*, T*, T);                      \
  template void interp_agg<T>(hipStream_t, const Level&, int, const T*, T*);                           \
  template void restrict_elim<T>(hipStream_t, const Level&, const T*, T*);                             \
  template void interp_elim<T>(hipStream_t, const Level&, const Level&, const T*, const T*, const T*, const T*, T*); \
  template void fill<T>(hipStream_t, T*, T, int);
INST(double)
INST(float)
template void fill<int>(hipStream_t, int*, int, int);
#undef INST

// ---------------------------------------------------------------- reductions
// Layout of H->red: [0, RED_BLOCKS * 8) block partials (8 slots each);
// [RED_BLOCKS * 8, +16) results.
constexpr int NSLOT = 8;
static inline double* red_part(Hierarchy* H) { return H->red; }
static inline double* red_res(Hierarchy* H) { return H->red + k::RED_BLOCKS * NSLOT; }

template <int NV>
__device__ inline void block_sum_store(double (&v)[NV], double* out) {
  __shared__ double sh[NV][k::RED_THREADS];
#pragma unroll
  for (int i = 0; i < NV; ++i) sh[i][threadIdx.x] = v[i];
  __syncthreads();
  for (int w = k::RED_THREADS / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int i = 0; i < NV; ++i) sh[i][threadIdx.x] += sh[i][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) out[i] = sh[i][0];
}

// Recombination sums of the chosen norm (dev::recomb_terms), six slots.
template <class T>
__global__ __launch_bounds__(k::RED_THREADS) void k_recomb_dots(int n, int th, int norm, const T* __restrict__ r,
                                                                const T* __restrict__ R0, const T* __restrict__ R1,
                                                                const T* __restrict__ x, const T* __restrict__ X0,
                                                                const T* __restrict__ X1, double* part) {
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x)
    dev::recomb_terms<T>(norm, th, r[u], R0[u], th > 1 ? R1[u] : T(0), norm ? x[u] : T(0), norm ? X0[u] : T(0),
                         norm && th > 1 ? X1[u] : T(0), v);
  block_sum_store<6>(v, part + blockIdx.x * NSLOT);
}
// Sum the block partials in a fixed order and solve the th x th normal
// equations of min || r + sum_i alpha_i d_i || (eq. recomb).  A direction is
// dropped when its Gram entry is negligible or the 2x2 system is singular.
// Sum slot `slot` of nblk block partials with a fixed tree (256 threads).
__device__ inline double finish_slot(int nblk, const double* part, int slot) {
  __shared__ double sh[256];
  double v = 0;
  for (int b = threadIdx.x; b < nblk; b += 256) v += part[b * NSLOT + slot];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}
__global__ __launch_bounds__(256) void k_recomb_alpha(int nblk, int th, int norm, const double* part, double* res) {
  __shared__ double tot[6];
  for (int q = 0; q < 6; ++q) {
    const double v = finish_slot(nblk, part, q);
    if (threadIdx.x == 0) tot[q] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double t[6];
  for (int q = 0; q < 6; ++q) t[q] = tot[q];
  dev::recomb_alpha(norm, th, t, &res[0], &res[1]);
}
template <class T>
__global__ void k_recomb_update(int n, int th, const double* __restrict__ res, const T* __restrict__ X0,
                                const T* __restrict__ X1, T* __restrict__ x) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const double a0 = res[0], a1 = res[1];
  const double xu = (double)x[u];
  double y = xu;
  y += a0 * ((double)X0[u] - xu);
  if (th > 1) y += a1 * ((double)X1[u] - xu);
  x[u] = (T)y;
}

static inline int red_grid(int n) {
  return std::max(1, std::min(k::RED_BLOCKS, (n + k::RED_THREADS - 1) / k::RED_THREADS));
}

template <class T>
void recombine(hipStream_t s, Hierarchy* H, const Level& L, Vecs<T>& v, int th) {
  const T* val;
  const T* dg;
  if constexpr (sizeof(T) == 8) { val = (const T*)L.val; dg = (const T*)L.diag; }
  else { val = (const T*)L.val32; dg = (const T*)L.diag32; }
  residual<T>(s, L, val, dg, v.b, v.x, v.r);
  const int nb = red_grid(L.n);
  const int norm = H->o.recomb_norm;
  hipLaunchKernelGGL(k_recomb_dots<T>, dim3(nb), dim3(k::RED_THREADS), 0, s, L.n, th, norm, (const T*)v.r,
                     (const T*)v.R[0], (const T*)v.R[1], (const T*)v.x, (const T*)v.X[0], (const T*)v.X[1],
                     red_part(H));
  hipLaunchKernelGGL(k_recomb_alpha, dim3(1), dim3(256), 0, s, nb, th, norm, red_part(H), red_res(H));
  hipLaunchKernelGGL(k_recomb_update<T>, g1(L.n), dim3(256), 0, s, L.n, th, red_res(H), v.X[0], v.X[1], v.x);
  LAMG_HIP(hipGetLastError());
}
template void recombine<double>(hipStream_t, Hierarchy*, const Level&, Vecs<double>&, int);
template void recombine<float>(hipStream_t, Hierarchy*, const Level&, Vecs<float>&, int);

template <class T>
__global__ __launch_bounds__(k::RED_THREADS) void k_sum(int n, const T* __restrict__ x, double* part) {
  double v[1] = {0};
  for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) v[0] += (double)x[u];
  block_sum_store<1>(v, part + blockIdx.x * NSLOT);
}
template <class T>
__global__ __launch_bounds__(k::RED_THREADS) void k_sumsq(int n, const T* __restrict__ x, double* part) {
  double v[1] = {0};
  for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
    const double t = (double)x[u];
    v[0] += t * t;
  }
  block_sum_store<1>(v, part + blockIdx.x * NSLOT);
}
// res[slot] = (sum of the block partials) / div: a mean divides by n, as its
// definition does (a constant vector then loses its mean exactly).
__global__ __launch_bounds__(256) void k_finish(int nblk, const double* part, double* res, int slot, double div) {
  const double s = finish_slot(nblk, part, 0);
  if (threadIdx.x == 0) res[slot] = s / div;
}
template <class T>
__global__ void k_sub_mean(int n, const double* __restrict__ res, int slot, T* __restrict__ x) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n) x[u] = (T)((double)x[u] - res[slot]);
}

void sum_to_slot(hipStream_t s, Hierarchy* H, const double* x, int n, int slot, double div) {
  const int nb = red_grid(n);
  hipLaunchKernelGGL(k_sum<double>, dim3(nb), dim3(k::RED_THREADS), 0, s, n, x, red_part(H));
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, nb, red_part(H), red_res(H), slot, div);
}

template <class T>
void subtract_mean(hipStream_t s, Hierarchy* H, T* x, int n) {
  const int nb = red_grid(n);
  hipLaunchKernelGGL(k_sum<T>, dim3(nb), dim3(k::RED_THREADS), 0, s, n, x, red_part(H));
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, nb, red_part(H), red_res(H), 4, (double)n);
  hipLaunchKernelGGL(k_sub_mean<T>, g1(n), dim3(256), 0, s, n, red_res(H), 4, x);
  LAMG_HIP(hipGetLastError());
}
template void subtract_mean<double>(hipStream_t, Hierarchy*, double*, int);
template void subtract_mean<float>(hipStream_t, Hierarchy*, float*, int);

// ||r||^2 into the pinned host slot (copied asynchronously; caller syncs).
void norm2_async(hipStream_t s, Hierarchy* H, const double* r, int n, double* dst_host) {
  const int nb = red_grid(n);
  hipLaunchKernelGGL(k_sumsq<double>, dim3(nb), dim3(k::RED_THREADS), 0, s, n, r, red_part(H));
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, nb, red_part(H), red_res(H), 5, 1.0);
  LAMG_HIP(hipMemcpyAsync(dst_host, red_res(H) + 5, sizeof(double), hipMemcpyDeviceToHost, s));
}

// --------------------------------------------------------------- coarsest
// x = M^-1 b with M = A_L + (mean diag / n_L) 1 1^T, whose inverse is formed
// at setup.  One workgroup; b staged in LDS.
template <class T>
__global__ __launch_bounds__(256) void k_dense_solve(int n, const double* __restrict__ Minv, const T* __restrict__ b,
                                                     T* __restrict__ x) {
  extern __shared__ double sb[];
  for (int j = threadIdx.x; j < n; j += blockDim.x) sb[j] = (double)b[j];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double s = 0;
    const double* row = Minv + (size_t)i * n;
    for (int j = 0; j < n; ++j) s += row[j] * sb[j];
    x[i] = (T)s;
  }
}
void coarsest_solve(hipStream_t s, Hierarchy* H, const double* b, double* x) {
  hipLaunchKernelGGL(k_dense_solve<double>, dim3(1), dim3(256), H->nL * sizeof(double), s, H->nL, H->cinv, b, x);
}
void coarsest_solve32(hipStream_t s, Hierarchy* H, const float* b, float* x) {
  hipLaunchKernelGGL(k_dense_solve<float>, dim3(1), dim3(256), H->nL * sizeof(double), s, H->nL, H->cinv, b, x);
}

// Dense augmented matrix, Cholesky factor and inverse (single workgroup).
__global__ void k_dense_build(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                              const double* __restrict__ val, const double* __restrict__ diag, double* M) {
  __shared__ double cfac;
  if (threadIdx.x == 0) {
    double s = 0;
    for (int u = 0; u < n; ++u) s += diag[u];
    double dbar = s / (double)n;
    if (!(dbar > 0)) dbar = 1.0;
    cfac = dbar / (double)n;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n * n; i += blockDim.x) M[i] = cfac;
  __syncthreads();
  for (int u = threadIdx.x; u < n; u += blockDim.x) {
    M[(size_t)u * n + u] += diag[u];
    for (int t = rp[u]; t < rp[u + 1]; ++t) M[(size_t)u * n + ci[t]] -= val[t];
  }
}
__global__ void k_cholesky_inverse(int n, double* M, double* Y, double* Minv) {
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) M[(size_t)j * n + j] = sqrt(M[(size_t)j * n + j]);
    __syncthreads();
    const double djj = M[(size_t)j * n + j];
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) M[(size_t)i * n + j] /= djj;
    __syncthreads();
    const int m = n - j - 1;
    for (int p = threadIdx.x; p < m * m; p += blockDim.x) {
      const int i = j + 1 + p / m, kk = j + 1 + p % m;
      if (kk <= i) M[(size_t)i * n + kk] -= M[(size_t)i * n + j] * M[(size_t)kk * n + j];
    }
    __syncthreads();
  }
  // column t of the inverse: L y = e_t, L^T z = y
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    double* y = Y + (size_t)t * n;
    for (int i = 0; i < n; ++i) {
      double s = (i == t) ? 1.0 : 0.0;
      for (int q = 0; q < i; ++q) s -= M[(size_t)i * n + q] * y[q];
      y[i] = s / M[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = y[i];
      for (int q = i + 1; q < n; ++q) s -= M[(size_t)q * n + i] * y[q];
      y[i] = s / M[(size_t)i * n + i];
    }
    for (int i = 0; i < n; ++i) Minv[(size_t)i * n + t] = y[i];
  }
}

void coarsest_factor(Hierarchy* H, const Level& L) {
  const int n = L.n;
  H->nL = n;
  double* M = dnew<double>(H, (size_t)n * n);
  double* Y = dnew<double>(H, (size_t)n * n);
  H->cinv = dnew<double>(H, (size_t)n * n);
  hipLaunchKernelGGL(k_dense_build, dim3(1), dim3(256), 0, H->s, n, L.rp, L.ci, L.val, L.diag, M);
  hipLaunchKernelGGL(k_cholesky_inverse, dim3(1), dim3(256), 0, H->s, n, M, Y, H->cinv);
  LAMG_HIP(hipGetLastError());
}

}  // namespace lamg

extern "C" {
void lamg_t_prof_enable(int on) {
  lamg::Prof& P = lamg::g_prof;
  try {
    lamg::prof_flush();
  } catch (const lamg::DevError&) {
  }
  P.on = on != 0;
  for (int k = 0; k < lamg::PROF_KERNELS; ++k) { P.ms[k] = 0; P.bytes[k] = 0; P.launches[k] = 0; }
}
lamg_status lamg_t_prof_read(int kernel, double* ms, int64_t* launches, int64_t* bytes) {
  lamg::Prof& P = lamg::g_prof;
  if (kernel < 0 || kernel >= lamg::PROF_KERNELS || !ms || !launches || !bytes) return LAMG_E_INVALID_ARG;
  try {
    lamg::prof_flush();
  } catch (const lamg::DevError&) {
    return LAMG_E_DEVICE;
  }
  *ms = P.ms[kernel];
  *launches = P.launches[kernel];
  *bytes = P.bytes[kernel];
  return LAMG_OK;
}
}
