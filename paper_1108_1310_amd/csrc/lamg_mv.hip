// Multi-vector form of the solve: k right-hand sides share one hierarchy
// (the setup depends on A only, Section 1; many right-hand sides are cheap to
// re-solve).  Every level's work vectors are n_l x k row-major blocks, right-
// hand side index fastest, so a row's k values are one contiguous segment and
// a CSR entry's weight and column index are read once for all k columns.
//
// Each column follows exactly the single-vector cycle (Section 4.2): the same
// relaxations, transfers and visit schedule, with its own recombination
// coefficients (eq. recomb), its own mean and its own convergence test.  Row
// sums keep the canonical order of the single-vector kernels per column:
// short rows (<= 64 entries) left to right, longer rows in 512-entry chunks of
// 64 strided partials folded by an xor butterfly, chunk sums in order.
//
// The outer loop is in correction form for both precisions: R = B - A X in
// FP64, one cycle from zero on the zero-mean R (FP64, or FP32 for the
// refinement variant), X += correction for the columns still iterating.
#include <algorithm>
#include <climits>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "lamg_device.hpp"
#include "lamg_internal.hpp"
#include "../../include/lamg_test.h"

namespace lamg {

namespace {

constexpr int MVT = 256;  // threads per block of the multi-vector kernels

inline dim3 gridn(int64_t n, int b = MVT) {
  return dim3((unsigned)std::max<int64_t>(1, (n + b - 1) / b));
}

// VW consecutive values from a 16-byte aligned address (VW = 1: any address).
template <class T, int VW>
__device__ __attribute__((always_inline)) inline void ldv(const T* p, T (&v)[VW]) {
  if constexpr (VW == 1) {
    v[0] = p[0];
  } else if constexpr (sizeof(T) == 8) {
    const double2 q = *(const double2*)p;
    v[0] = q.x; v[1] = q.y;
  } else {
    const float4 q = *(const float4*)p;
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  }
}
template <class T, int VW>
__device__ __attribute__((always_inline)) inline void stv(T* p, const T (&v)[VW]) {
  if constexpr (VW == 1) {
    p[0] = v[0];
  } else if constexpr (sizeof(T) == 8) {
    *(double2*)p = make_double2(v[0], v[1]);
  } else {
    *(float4*)p = make_float4(v[0], v[1], v[2], v[3]);
  }
}

// MODE 0: GS update x_u <- (b_u + s) / a_uu (eq. gs); MODE 1: residual
// r_u <- (b_u + s) - a_uu x_u; MODE 2: elimination restriction out_u =
// x_{map(u)} + s, where x is the fine residual.  One VW-wide column slice.
template <class T, int MODE, int VW>
__device__ __attribute__((always_inline)) inline void store_mv(int u, size_t o, int k, const T (&s)[VW],
                                                               const T* __restrict__ diag, const T* __restrict__ b,
                                                               T* x, T* __restrict__ r, const int* __restrict__ map) {
  T out[VW];
  if constexpr (MODE == 2) {
    T xv[VW];
    ldv<T, VW>(x + (size_t)map[u] * k + (o - (size_t)u * k), xv);
#pragma unroll
    for (int i = 0; i < VW; ++i) out[i] = xv[i] + s[i];
    stv<T, VW>(r + o, out);
    return;
  }
  T bv[VW];
  if (b) ldv<T, VW>(b + o, bv);
  else
#pragma unroll
    for (int i = 0; i < VW; ++i) bv[i] = T(0);
  const T d = diag[u];
  if constexpr (MODE == 0) {
#pragma unroll
    for (int i = 0; i < VW; ++i) out[i] = (bv[i] + s[i]) / d;
    stv<T, VW>(x + o, out);
  } else {
    T xv[VW];
    ldv<T, VW>(x + o, xv);
#pragma unroll
    for (int i = 0; i < VW; ++i) out[i] = (bv[i] + s[i]) - d * xv[i];
    stv<T, VW>(r + o, out);
  }
}

// Relaxation / residual / elimination restriction over rows [r0, r1) of a
// level for n x k blocks.  Short rows: a group of G = 2^glog lanes per row,
// lane g handling the VW-wide column slices g, g + G, ... (the G lanes of a
// row read one contiguous segment per entry).  Long rows (listed in lrows):
// 2^wlog wavefronts per row, wavefront w taking the column slices w,
// w + 2^wlog, ... one after the other (each slice's sums in the canonical
// chunk order, so the split does not change a bit).  The first nlb blocks
// take the long rows.  zthr: rows >= zthr of x hold +0 (the first
// sweep from a zero iterate), so their slices are taken as +0 without a
// load; the terms and their order are unchanged.
template <class T, int MODE, int VW>
__global__ __launch_bounds__(MVT) void k_relax_mv(const int* __restrict__ rp, const int* __restrict__ ci,
                                                  const T* __restrict__ val, const T* __restrict__ diag,
                                                  const T* __restrict__ b, T* x, T* __restrict__ r,
                                                  const int* __restrict__ map, int k, int glog, int r0, int r1,
                                                  const int* __restrict__ lrows, int nlong, int nlb, int zthr,
                                                  int wlog) {
  const int ncv = k / VW;
  int bid = blockIdx.x;
  if (bid < nlb) {
    const int wv = (int)threadIdx.x >> 6;
    const int idx = bid * ((MVT / 64) >> wlog) + (wv >> wlog);
    if (idx >= nlong) return;
    const int lane = threadIdx.x & 63;
    const int u = lrows[idx];
    const int p0 = rp[u], len = rp[u + 1] - p0;
    for (int cv = wv & ((1 << wlog) - 1); cv < ncv; cv += 1 << wlog) {
      T tot[VW];
#pragma unroll
      for (int i = 0; i < VW; ++i) tot[i] = T(0);
      for (int c0 = 0; c0 < len; c0 += dev::CHUNK) {
        T s[VW];
#pragma unroll
        for (int i = 0; i < VW; ++i) s[i] = T(0);
        for (int q = 0; q < dev::CHUNK / 64; ++q) {
          const int t = c0 + lane + 64 * q;
          if (t < len) {
            const T w = val[p0 + t];
            const int cj = ci[p0 + t];
            T xv[VW];
            if (cj < zthr) ldv<T, VW>(x + (size_t)cj * k + cv * VW, xv);
            else
#pragma unroll
              for (int i = 0; i < VW; ++i) xv[i] = T(0);
#pragma unroll
            for (int i = 0; i < VW; ++i) s[i] += w * xv[i];
          }
        }
#pragma unroll
        for (int i = 0; i < VW; ++i) tot[i] += dev::wave_fold(s[i]);
      }
      if (lane == 0) store_mv<T, MODE, VW>(u, (size_t)u * k + cv * VW, k, tot, diag, b, x, r, map);
    }
    return;
  }
  bid -= nlb;
  const int G = 1 << glog;
  const int row = r0 + bid * (MVT >> glog) + ((int)threadIdx.x >> glog);
  const int g = threadIdx.x & (G - 1);
  if (row >= r1) return;
  const int p0 = rp[row], len = rp[row + 1] - p0;
  if (len > SHORT_ROW) return;
  for (int cv = g; cv < ncv; cv += G) {
    T s[VW];
#pragma unroll
    for (int i = 0; i < VW; ++i) s[i] = T(0);
    int t = 0;
    // four entries' loads in flight, then their sums in column order
    for (; t + 4 <= len; t += 4) {
      int cj[4];
      T wj[4], xv[4][VW];
#pragma unroll
      for (int q = 0; q < 4; ++q) { cj[q] = ci[p0 + t + q]; wj[q] = val[p0 + t + q]; }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (cj[q] < zthr) ldv<T, VW>(x + (size_t)cj[q] * k + cv * VW, xv[q]);
        else
#pragma unroll
          for (int i = 0; i < VW; ++i) xv[q][i] = T(0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < VW; ++i) s[i] += wj[q] * xv[q][i];
    }
    for (; t < len; ++t) {
      const T w = val[p0 + t];
      const int cj = ci[p0 + t];
      T xv[VW];
      if (cj < zthr) ldv<T, VW>(x + (size_t)cj * k + cv * VW, xv);
      else
#pragma unroll
        for (int i = 0; i < VW; ++i) xv[i] = T(0);
#pragma unroll
      for (int i = 0; i < VW; ++i) s[i] += w * xv[i];
    }
    store_mv<T, MODE, VW>(row, (size_t)row * k + cv * VW, k, s, diag, b, x, r, map);
  }
}

// Widest 16-byte slice that divides k.
template <class T>
int mv_width(int k) {
  const int w = 16 / (int)sizeof(T);
  return k % w == 0 ? w : 1;
}

template <class T, int MODE>
void relax_mv(hipStream_t s, const int* rp, const int* ci, const T* val, const T* diag, const T* b, T* x, T* r,
              const int* map, int k, int r0, int r1, const Tiles& t, int zthr = INT_MAX) {
  if (r1 <= r0) return;
  const int vw = mv_width<T>(k);
  const int ncv = k / vw;
  int glog = 0;
  while ((1 << glog) < ncv && glog < 6) ++glog;
  const int rows_per_block = MVT >> glog;
  const int nsb = (r1 - r0 + rows_per_block - 1) / rows_per_block;
  // long rows: up to all the block's wavefronts per row, one per column slice
  int wlog = 0;
  while ((2 << wlog) <= MVT / 64 && (2 << wlog) <= ncv) ++wlog;
  const int rpb = (MVT / 64) >> wlog;
  const int nlb = (t.nlong + rpb - 1) / rpb;
  const int grid = nlb + nsb;
  const bool prof = MODE != 2 && prof_on();
  const int kid = 4 + MODE + (sizeof(T) == 4 ? 2 : 0);
  // matrix stream once for all columns; per row and column: b or x read, x
  // read, x or r write
  const int64_t bytes = t.nnz * (4 + (int64_t)sizeof(T)) + t.rows * (4 + (int64_t)sizeof(T)) +
                        3 * t.rows * (int64_t)k * (int64_t)sizeof(T);
  const int* lr = (const int*)t.longrows;
  if (prof) prof_count(kid, bytes);
  if (vw == 1)
    hipLaunchKernelGGL((k_relax_mv<T, MODE, 1>), dim3(grid), dim3(MVT), 0, s, rp, ci, val, diag, b, x, r, map, k, glog,
                       r0, r1, lr, t.nlong, nlb, zthr, wlog);
  else if constexpr (sizeof(T) == 8)
    hipLaunchKernelGGL((k_relax_mv<T, MODE, 2>), dim3(grid), dim3(MVT), 0, s, rp, ci, val, diag, b, x, r, map, k, glog,
                       r0, r1, lr, t.nlong, nlb, zthr, wlog);
  else
    hipLaunchKernelGGL((k_relax_mv<T, MODE, 4>), dim3(grid), dim3(MVT), 0, s, rp, ci, val, diag, b, x, r, map, k, glog,
                       r0, r1, lr, t.nlong, nlb, zthr, wlog);
  LAMG_HIP(hipGetLastError());
}

template <class T> struct PrecM;
template <> struct PrecM<double> {
  static Vecs<double>& v(Hierarchy* H, int l) { return H->mv.v64[l]; }
  static const double* val(const Level& L) { return L.val; }
  static const double* diag(const Level& L) { return L.diag; }
  static const double* er(const Level& L) { return L.er_val; }
};
template <> struct PrecM<float> {
  static Vecs<float>& v(Hierarchy* H, int l) { return H->mv.v32[l]; }
  static const float* val(const Level& L) { return L.val32; }
  static const float* diag(const Level& L) { return L.diag32; }
  static const float* er(const Level& L) { return L.er_val32; }
};

// from_zero: x is +0 on entry, so colour c gathers only colours < c
template <class T>
void gs_sweep_mv(hipStream_t s, const Level& L, int k, const T* b, T* x, bool from_zero = false) {
  prof_begin(s, sizeof(T) == 4 ? 6 : 4, L.ncol);
  for (int c = 0; c < L.ncol; ++c)
    relax_mv<T, 0>(s, L.rp, L.ci, PrecM<T>::val(L), PrecM<T>::diag(L), b, x, (T*)nullptr, nullptr, k, L.cptr[c],
                   L.cptr[c + 1], L.tiles[c], from_zero ? L.cptr[c] : INT_MAX);
  prof_end(s);
}
template <class T>
void residual_mv(hipStream_t s, const Level& L, int k, const T* b, const T* x, T* r) {
  prof_begin(s, sizeof(T) == 4 ? 7 : 5);
  relax_mv<T, 1>(s, L.rp, L.ci, PrecM<T>::val(L), PrecM<T>::diag(L), b, (T*)x, r, nullptr, k, 0, L.n, L.all);
  prof_end(s);
}

// ---------------------------------------------------------------- transfers
// b^c_U = mu * sum of the members' residuals, members in ascending order.
template <class T>
__global__ void k_restrict_agg_mv(int nc, int k, const int* __restrict__ aptr, const int* __restrict__ mem,
                                  const T* __restrict__ r, T* __restrict__ bc, T mu) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)nc * k) return;
  const int U = (int)(g / k), c = (int)(g % k);
  T s = 0;
  for (int j = aptr[U]; j < aptr[U + 1]; ++j) s += r[(size_t)mem[j] * k + c];
  bc[g] = mu * s;
}
template <class T>
__global__ void k_interp_agg_mv(int n, int k, const int* __restrict__ agg, const T* __restrict__ e, T* __restrict__ x) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)n * k) return;
  const int u = (int)(g / k), c = (int)(g % k);
  x[g] += e[(size_t)agg[u] * k + c];
}
template <class T>
__global__ void k_interp_elim_mv(int n, int k, const int* __restrict__ cidx, const int* __restrict__ rp,
                                 const int* __restrict__ ci, const T* __restrict__ val, const T* __restrict__ diag,
                                 const T* __restrict__ r, const T* __restrict__ e, T* __restrict__ x) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)n * k) return;
  const int u = (int)(g / k), c = (int)(g % k);
  const int cu = cidx[u];
  if (cu >= 0) { x[g] += e[(size_t)cu * k + c]; return; }
  T s = r[g];
  for (int t = rp[u]; t < rp[u + 1]; ++t) s += val[t] * e[(size_t)cidx[ci[t]] * k + c];
  x[g] += s / diag[u];
}
template <class T>
__global__ void k_fill_mv(int64_t n, T* __restrict__ p, T v) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) p[g] = v;
}
template <class T>
__global__ void k_copy_mv(int64_t n, const T* __restrict__ a, T* __restrict__ b) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) b[g] = a[g];
}
template <class T>
void fill_mv(hipStream_t s, T* p, int64_t n) {
  if (n > 0) hipLaunchKernelGGL(k_fill_mv<T>, gridn(n), dim3(MVT), 0, s, n, p, T(0));
}

// ------------------------------------------------------- column reductions
// Thread g < k * rows owns column g % k and rows g / k, g / k + rows, ...; its
// partial goes to part[slot * k * W.rows + g].  A second kernel sums each
// column's partials with a fixed tree.  rows does not depend on k, so a
// column's sums (and with them its whole solve) are bitwise the same whatever
// other columns share the batch.
constexpr int MV_RED_ROWS = 4096;
template <class T>
__global__ __launch_bounds__(MVT) void k_colsum(int n, int k, int rows, const T* __restrict__ x, int squares,
                                                double* __restrict__ part) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= k * rows) return;
  const int c = g % k;
  double v = 0;
  for (int i = g / k; i < n; i += rows) {
    const double t = (double)x[(size_t)i * k + c];
    v += squares ? t * t : t;
  }
  part[g] = v;
}
// Recombination dots per column with d_i = R_i - r: G00, G01, G11, g0, g1, r.r
template <class T>
__global__ __launch_bounds__(MVT) void k_coldots(int n, int k, int rows, int stride, int th, int norm,
                                                 const T* __restrict__ r, const T* __restrict__ R0,
                                                 const T* __restrict__ R1, const T* __restrict__ x,
                                                 const T* __restrict__ X0, const T* __restrict__ X1,
                                                 double* __restrict__ part) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= k * rows) return;
  const int c = g % k;
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int i = g / k; i < n; i += rows) {
    const size_t o = (size_t)i * k + c;
    dev::recomb_terms<T>(norm, th, r[o], R0[o], th > 1 ? R1[o] : T(0), norm ? x[o] : T(0), norm ? X0[o] : T(0),
                         norm && th > 1 ? X1[o] : T(0), v);
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) part[(size_t)q * stride + g] = v[q];
}
// Sum of column c's partials of one slot (block c, 256 threads, fixed tree).
__device__ inline double col_total(int k, int rows, const double* part, int c) {
  __shared__ double sh[MVT];
  double v = 0;
  for (int i = threadIdx.x; i < rows; i += MVT) v += part[(size_t)i * k + c];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = MVT / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double t = sh[0];
  __syncthreads();
  return t;
}
__global__ __launch_bounds__(MVT) void k_colfinish(int k, int rows, const double* __restrict__ part,
                                                   double* __restrict__ out, double div) {
  const int c = blockIdx.x;
  const double t = col_total(k, rows, part, c);
  if (threadIdx.x == 0) out[c] = t / div;  // a mean divides by n, as defined
}
// Per column: the th x th normal equations of min || r + sum_i alpha_i d_i ||
// (eq. recomb), with the drop rules of the single-vector kernel.
__global__ __launch_bounds__(MVT) void k_colalpha(int k, int rows, int stride, int th, int norm,
                                                  const double* __restrict__ part, double* __restrict__ alpha) {
  const int c = blockIdx.x;
  double tot[6];
  for (int q = 0; q < 6; ++q) tot[q] = col_total(k, rows, part + (size_t)q * stride, c);
  if (threadIdx.x != 0) return;
  dev::recomb_alpha(norm, th, tot, &alpha[2 * c], &alpha[2 * c + 1]);
}
template <class T>
__global__ void k_colupdate(int n, int k, int th, const double* __restrict__ alpha, const T* __restrict__ X0,
                            const T* __restrict__ X1, T* __restrict__ x) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)n * k) return;
  const int c = (int)(g % k);
  const double a0 = alpha[2 * c], a1 = alpha[2 * c + 1];
  const double xu = (double)x[g];
  double y = xu;
  y += a0 * ((double)X0[g] - xu);
  if (th > 1) y += a1 * ((double)X1[g] - xu);
  x[g] = (T)y;
}
// x[:, c] -= m[c] for the columns whose mask is set (every column without a mask)
template <class T>
__global__ void k_colsub(int n, int k, const double* __restrict__ m, const int* __restrict__ mask, T* __restrict__ x) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)n * k) return;
  const int c = (int)(g % k);
  if (mask && !mask[c]) return;
  x[g] = (T)((double)x[g] - m[c]);
}

// Result slots of W.res, k values each.
enum { RS_BMEAN = 0, RS_BNORM = 1, RS_RNORM = 2, RS_RMEAN = 3, RS_XMEAN = 4, RS_TMP = 5, RS_ALPHA = 6 };  // ALPHA: 2k

int red_rows(const MVWork& W, int n) { return std::max(1, std::min(W.rows, n)); }

template <class T>
void col_reduce(hipStream_t s, Hierarchy* H, const T* x, int n, int squares, int slot, double div) {
  MVWork& W = H->mv;
  const int rows = red_rows(W, n), k = W.k;
  hipLaunchKernelGGL(k_colsum<T>, gridn((int64_t)k * rows), dim3(MVT), 0, s, n, k, rows, x, squares, W.part);
  hipLaunchKernelGGL(k_colfinish, dim3(k), dim3(MVT), 0, s, k, rows, (const double*)W.part, W.res + slot * k, div);
}
template <class T>
void subtract_mean_mv(hipStream_t s, Hierarchy* H, T* x, int n, const int* mask) {
  const int k = H->mv.k;
  col_reduce<T>(s, H, x, n, 0, RS_TMP, (double)n);
  hipLaunchKernelGGL(k_colsub<T>, gridn((int64_t)n * k), dim3(MVT), 0, s, n, k, (const double*)(H->mv.res + RS_TMP * k),
                     mask, x);
}

template <class T>
void recombine_mv(hipStream_t s, Hierarchy* H, const Level& L, Vecs<T>& v, int th) {
  MVWork& W = H->mv;
  const int k = W.k, n = L.n;
  residual_mv<T>(s, L, k, v.b, v.x, v.r);
  const int rows = red_rows(W, n);
  const int stride = k * W.rows;
  const int norm = H->o.recomb_norm;
  hipLaunchKernelGGL(k_coldots<T>, gridn((int64_t)k * rows), dim3(MVT), 0, s, n, k, rows, stride, th, norm,
                     (const T*)v.r, (const T*)v.R[0], (const T*)v.R[1], (const T*)v.x, (const T*)v.X[0],
                     (const T*)v.X[1], W.part);
  double* alpha = W.res + RS_ALPHA * k;
  hipLaunchKernelGGL(k_colalpha, dim3(k), dim3(MVT), 0, s, k, rows, stride, th, norm, (const double*)W.part, alpha);
  hipLaunchKernelGGL(k_colupdate<T>, gridn((int64_t)n * k), dim3(MVT), 0, s, n, k, th, (const double*)alpha,
                     (const T*)v.X[0], (const T*)v.X[1], v.x);
  LAMG_HIP(hipGetLastError());
}

// ----------------------------------------------------------------- coarsest
// x[:, c] = M^-1 b[:, c], block c; the same left-to-right row sums as the
// single-vector dense solve.
template <class T>
__global__ __launch_bounds__(256) void k_dense_solve_mv(int n, int k, const double* __restrict__ Minv,
                                                        const T* __restrict__ b, T* __restrict__ x) {
  extern __shared__ double sb[];
  const int c = blockIdx.x;
  for (int j = threadIdx.x; j < n; j += blockDim.x) sb[j] = (double)b[(size_t)j * k + c];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double s = 0;
    const double* row = Minv + (size_t)i * n;
    for (int j = 0; j < n; ++j) s += row[j] * sb[j];
    x[(size_t)i * k + c] = (T)s;
  }
}

// -------------------------------------------------------------------- cycle
template <class T>
void visit_mv(Hierarchy* H, int l, int th, std::vector<int64_t>& count);

template <class T>
void body_mv(Hierarchy* H, int l, int sub, std::vector<int64_t>& count) {
  hipStream_t s = H->s;
  const int Lc = (int)H->lv.size() - 1;
  const int k = H->mv.k;
  Level& L = H->lv[l];
  Vecs<T>& v = PrecM<T>::v(H, l);
  if (l == Lc) {
    if (H->coarsest_relax) {
      // x = 0 on entry below the finest level (the caller's fill) and at the
      // finest in correction form
      const bool z = l > 0 || H->top_res_known;
      for (int i = 0; i < H->o.coarsest_sweeps; ++i) gs_sweep_mv<T>(s, L, k, v.b, v.x, z && i == 0);
      return;
    }
    hipLaunchKernelGGL(k_dense_solve_mv<T>, dim3(k), dim3(256), H->nL * sizeof(double), s, H->nL, k,
                       (const double*)H->cinv, (const T*)v.b, v.x);
    return;
  }
  Level& C = H->lv[l + 1];
  Vecs<T>& vc = PrecM<T>::v(H, l + 1);
  const int64_t nk = (int64_t)L.n * k, nck = (int64_t)C.n * k;
  if (C.type == LT_ELIM) {
    const T* r = v.r;
    if (l == 0 && H->top_res_known) r = v.b;  // x = 0 on entry
    else residual_mv<T>(s, L, k, v.b, v.x, v.r);
    relax_mv<T, 2>(s, C.er_rp, C.er_ci, PrecM<T>::er(C), (const T*)nullptr, (const T*)nullptr, const_cast<T*>(r), vc.b, C.cfine, k,
                   0, C.n, C.er_tiles);
    fill_mv<T>(s, vc.x, nck);
    visit_mv<T>(H, l + 1, 1, count);
    hipLaunchKernelGGL(k_interp_elim_mv<T>, gridn(nk), dim3(MVT), 0, s, L.n, k, C.cidx, L.rp, L.ci,
                       PrecM<T>::val(L), PrecM<T>::diag(L), r, (const T*)vc.x, v.x);
    return;
  }
  const bool rec = H->o.ec == LAMG_EC_RECOMBINE;
  const bool z = (l > 0 || H->top_res_known) && sub == 0;
  for (int i = 0; i < H->o.nu_pre; ++i) gs_sweep_mv<T>(s, L, k, v.b, v.x, z && i == 0);
  T* r = rec ? v.R[sub] : v.r;
  residual_mv<T>(s, L, k, v.b, v.x, r);
  if (rec) hipLaunchKernelGGL(k_copy_mv<T>, gridn(nk), dim3(MVT), 0, s, nk, (const T*)v.x, v.X[sub]);
  const T mu = rec ? T(1) : (T)H->o.mu;
  hipLaunchKernelGGL(k_restrict_agg_mv<T>, gridn(nck), dim3(MVT), 0, s, C.n, k, C.agg_ptr, C.members, (const T*)r,
                     vc.b, mu);
  fill_mv<T>(s, vc.x, nck);
  const int64_t c = count[l]++;
  const double gl = L.gamma_next;
  const int th = (int)(std::ceil((double)(c + 1) * gl) - std::ceil((double)c * gl));
  visit_mv<T>(H, l + 1, th, count);
  hipLaunchKernelGGL(k_interp_agg_mv<T>, gridn(nk), dim3(MVT), 0, s, L.n, k, C.agg, (const T*)vc.x, v.x);
  for (int i = 0; i < H->o.nu_post; ++i) gs_sweep_mv<T>(s, L, k, v.b, v.x);
}

template <class T>
void visit_mv(Hierarchy* H, int l, int th, std::vector<int64_t>& count) {
  const int Lc = (int)H->lv.size() - 1;
  if (l == H->tail_lc) { tail_run_next_mv<T>(H); return; }
  if (l == Lc) { body_mv<T>(H, l, 0, count); return; }
  for (int i = 0; i < th; ++i) body_mv<T>(H, l, i, count);
  if (H->o.ec == LAMG_EC_RECOMBINE && H->lv[l + 1].type == LT_AGG)
    recombine_mv<T>(H->s, H, H->lv[l], PrecM<T>::v(H, l), th);
}

template <class T>
void cycle_mv(Hierarchy* H, bool top_res_known = false) {
  tail_prepare_mv(H);
  H->tail_cursor = 0;
  std::vector<int64_t> count(H->lv.size(), 0);
  H->top_res_known = top_res_known;
  try {
    visit_mv<T>(H, 0, 1, count);
  } catch (...) {
    H->top_res_known = false;
    throw;
  }
  H->top_res_known = false;
  if (H->tail_lc != 0) subtract_mean_mv<T>(H->s, H, PrecM<T>::v(H, 0).x, H->lv[0].n, nullptr);
  LAMG_HIP(hipGetLastError());
}

// Captured once per precision and workspace, replayed per cycle (eager when
// instrumented, so each relaxation launch has its own event pair).  The
// solve loop runs the cycle in correction form (x = 0 on entry), so the
// finest residual of the recorded cycle is b itself.
template <class T>
void cycle_graph_mv(Hierarchy* H) {
  if (prof_on()) { cycle_mv<T>(H, true); return; }
  MVWork& W = H->mv;
  const int p = sizeof(T) == 8 ? 0 : 1;
  tail_prepare_mv(H);  // synchronous uploads: before any capture
  if (!W.gexec[p]) {
    if (!H->cs) LAMG_HIP(hipStreamCreateWithFlags(&H->cs, hipStreamNonBlocking));
    hipStream_t user = H->s;
    H->s = H->cs;
    hipGraph_t g = nullptr;
    LAMG_HIP(hipStreamBeginCapture(H->cs, hipStreamCaptureModeThreadLocal));
    try {
      cycle_mv<T>(H, true);
    } catch (...) {
      (void)hipStreamEndCapture(H->cs, &g);
      if (g) (void)hipGraphDestroy(g);
      H->s = user;
      throw;
    }
    LAMG_HIP(hipStreamEndCapture(H->cs, &g));
    H->s = user;
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    LAMG_HIP(e);
    W.gexec[p] = ex;
  }
  LAMG_HIP(hipGraphLaunch(W.gexec[p], H->s));
}

// ------------------------------------------------------------ outer kernels
// out[i, c] = B[perm[i], c] - m[c] (m may be null)
__global__ void k_mv_gather(int n, int k, const int* __restrict__ perm, const double* __restrict__ B,
                            const double* __restrict__ m, double* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)n * k) return;
  const int i = (int)(g / k), c = (int)(g % k);
  out[g] = B[(size_t)perm[i] * k + c] - (m ? m[c] : 0.0);
}
__global__ void k_mv_scatter(int n, int k, const int* __restrict__ perm, const double* __restrict__ a,
                             double* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)n * k) return;
  const int i = (int)(g / k), c = (int)(g % k);
  out[(size_t)perm[i] * k + c] = a[g];
}
// level-0 right-hand side of the inner cycle: R - mean(R), in T
template <class T>
__global__ void k_mv_rhs(int64_t nk, int k, const double* __restrict__ R, const double* __restrict__ m,
                         T* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nk) return;
  out[g] = (T)(R[g] - m[g % k]);
}
template <class T>
__global__ void k_mv_add(int64_t nk, int k, const T* __restrict__ e, const int* __restrict__ mask,
                         double* __restrict__ X) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nk || !mask[g % k]) return;
  X[g] += (double)e[g];
}

}  // namespace

// ---------------------------------------------------------------- workspace
void mv_drop_graphs(Hierarchy* H) {
  for (int p = 0; p < 2; ++p) {
    if (H->mv.gexec[p]) (void)hipGraphExecDestroy(H->mv.gexec[p]);
    H->mv.gexec[p] = nullptr;
  }
}

void mv_release(Hierarchy* H) {
  MVWork& W = H->mv;
  mv_drop_graphs(H);
  for (void* p : W.owned) dev_free(H->o, p);
  if (W.hres) (void)hipHostFree(W.hres);
  if (W.hmask) (void)hipHostFree(W.hmask);
  W = MVWork();
}

namespace {
void mv_alloc(Hierarchy* H, int k) {
  MVWork& W = H->mv;
  if (W.k == k) return;
  if (H->s) LAMG_HIP(hipStreamSynchronize(H->s));
  else LAMG_HIP(hipDeviceSynchronize());
  mv_release(H);
  auto A = [&](size_t bytes) {
    void* p = dev_alloc(H->o, bytes + 16);
    W.owned.push_back(p);
    return p;
  };
  const size_t nl = H->lv.size();
  W.v64.resize(nl);
  W.v32.resize(nl);
  for (size_t l = 0; l < nl; ++l) {
    const size_t nk = (size_t)H->lv[l].n * k;
    Vecs<double>& a = W.v64[l];
    Vecs<float>& f = W.v32[l];
    a.x = (double*)A(nk * 8); a.b = (double*)A(nk * 8); a.r = (double*)A(nk * 8);
    f.x = (float*)A(nk * 4); f.b = (float*)A(nk * 4); f.r = (float*)A(nk * 4);
    for (int i = 0; i < 2; ++i) {
      a.X[i] = (double*)A(nk * 8); a.R[i] = (double*)A(nk * 8);
      f.X[i] = (float*)A(nk * 4); f.R[i] = (float*)A(nk * 4);
    }
  }
  const size_t n0k = (size_t)H->lv[0].n * k;
  W.B = (double*)A(n0k * 8);
  W.X = (double*)A(n0k * 8);
  W.R = (double*)A(n0k * 8);
  W.rows = MV_RED_ROWS;
  W.part = (double*)A((size_t)6 * k * W.rows * 8);
  W.res = (double*)A((size_t)(RS_ALPHA + 2) * k * 8);
  W.mask = (int*)A((size_t)k * 4);
  LAMG_HIP(hipHostMalloc((void**)&W.hres, (size_t)(RS_ALPHA + 2) * k * 8, hipHostMallocDefault));
  LAMG_HIP(hipHostMalloc((void**)&W.hmask, (size_t)k * 4, hipHostMallocDefault));
  W.cycles.assign(k, 0);
  W.rel.assign(k, 0.0);
  W.removed.assign(k, 0.0);
  W.k = k;
}
}  // namespace

lamg_status solve_multi(Hierarchy* H, int k, const double* B, double* X, lamg_info* info) {
  Level& L = H->lv[0];
  const int n = L.n;
  if ((int64_t)n * k > (int64_t)0x7fffffff) return LAMG_E_INVALID_ARG;
  mv_alloc(H, k);
  MVWork& W = H->mv;
  hipStream_t s = H->s;
  const int64_t nk = (int64_t)n * k;
  auto t0 = std::chrono::steady_clock::now();
  double* res = W.res;
  double* hr = W.hres;
  // B <- B - mean(B) per column, in colour order
  col_reduce<double>(s, H, B, n, 0, RS_BMEAN, (double)n);
  hipLaunchKernelGGL(k_mv_gather, gridn(nk), dim3(MVT), 0, s, n, k, L.perm, B, (const double*)(res + RS_BMEAN * k),
                     W.B);
  if (H->o.warm_start)
    hipLaunchKernelGGL(k_mv_gather, gridn(nk), dim3(MVT), 0, s, n, k, L.perm, (const double*)X, (const double*)nullptr,
                       W.X);
  else
    fill_mv<double>(s, W.X, nk);
  col_reduce<double>(s, H, W.B, n, 1, RS_BNORM, 1.0);
  residual_mv<double>(s, L, k, W.B, W.X, W.R);
  col_reduce<double>(s, H, W.R, n, 1, RS_RNORM, 1.0);
  LAMG_HIP(hipMemcpyAsync(hr, res, (size_t)3 * k * sizeof(double), hipMemcpyDeviceToHost, s));
  LAMG_HIP(hipStreamSynchronize(s));
  std::vector<double> nb(k), r0(k), rk(k);
  int active = 0;
  for (int c = 0; c < k; ++c) {
    W.removed[c] = hr[RS_BMEAN * k + c];
    nb[c] = std::sqrt(hr[RS_BNORM * k + c]);
    r0[c] = rk[c] = std::sqrt(hr[RS_RNORM * k + c]);
    W.cycles[c] = 0;
    W.hmask[c] = nb[c] > 0 && std::isfinite(rk[c]) && rk[c] > H->o.tol * nb[c];
    active += W.hmask[c];
  }
  const bool fp32 = H->o.precision == LAMG_FP32_REFINE;
  int it = 0;
  while (active > 0 && it < H->o.max_cycles) {
    LAMG_HIP(hipMemcpyAsync(W.mask, W.hmask, (size_t)k * sizeof(int), hipMemcpyHostToDevice, s));
    col_reduce<double>(s, H, W.R, n, 0, RS_RMEAN, (double)n);
    const double* rm = res + RS_RMEAN * k;
    if (!fp32) {
      Vecs<double>& v = W.v64[0];
      hipLaunchKernelGGL(k_mv_rhs<double>, gridn(nk), dim3(MVT), 0, s, nk, k, (const double*)W.R, rm, v.b);
      fill_mv<double>(s, v.x, nk);
      cycle_graph_mv<double>(H);
      hipLaunchKernelGGL(k_mv_add<double>, gridn(nk), dim3(MVT), 0, s, nk, k, (const double*)v.x,
                         (const int*)W.mask, W.X);
    } else {
      Vecs<float>& v = W.v32[0];
      hipLaunchKernelGGL(k_mv_rhs<float>, gridn(nk), dim3(MVT), 0, s, nk, k, (const double*)W.R, rm, v.b);
      fill_mv<float>(s, v.x, nk);
      cycle_graph_mv<float>(H);
      hipLaunchKernelGGL(k_mv_add<float>, gridn(nk), dim3(MVT), 0, s, nk, k, (const float*)v.x, (const int*)W.mask,
                         W.X);
    }
    subtract_mean_mv<double>(s, H, W.X, n, W.mask);
    residual_mv<double>(s, L, k, W.B, W.X, W.R);
    col_reduce<double>(s, H, W.R, n, 1, RS_RNORM, 1.0);
    LAMG_HIP(hipMemcpyAsync(hr + RS_RNORM * k, res + RS_RNORM * k, (size_t)k * sizeof(double), hipMemcpyDeviceToHost,
                            s));
    LAMG_HIP(hipStreamSynchronize(s));
    ++it;
    active = 0;
    for (int c = 0; c < k; ++c) {
      if (!W.hmask[c]) continue;
      ++W.cycles[c];
      rk[c] = std::sqrt(hr[RS_RNORM * k + c]);
      W.hmask[c] = std::isfinite(rk[c]) && rk[c] > H->o.tol * nb[c];
      active += W.hmask[c];
    }
  }
  hipLaunchKernelGGL(k_mv_scatter, gridn(nk), dim3(MVT), 0, s, n, k, L.perm, (const double*)W.X, X);
  LAMG_HIP(hipStreamSynchronize(s));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  bool bad = false, open = false;
  double worst = 0, worst_acf = 0, big_mean = 0;
  for (int c = 0; c < k; ++c) {
    W.rel[c] = nb[c] > 0 ? rk[c] / nb[c] : 0.0;
    if (!std::isfinite(rk[c])) bad = true;
    else if (nb[c] > 0 && rk[c] > H->o.tol * nb[c]) open = true;
    worst = std::max(worst, W.rel[c]);
    if (W.cycles[c] > 0 && r0[c] > 0) worst_acf = std::max(worst_acf, std::pow(rk[c] / r0[c], 1.0 / W.cycles[c]));
    if (std::fabs(W.removed[c]) > std::fabs(big_mean)) big_mean = W.removed[c];
  }
  if (info) {
    info->cycles = it;
    info->levels = (int)H->lv.size();
    info->rel_residual = worst;
    info->acf = worst_acf;
    info->removed_mean = big_mean;
    info->setup_ms = H->setup_ms;
    info->solve_ms = ms;
    info->bytes_moved = (int64_t)it * cycle_bytes_k(H, H->o.precision, k);
  }
  if (bad) return LAMG_E_BREAKDOWN;
  if (open) return LAMG_E_NOT_CONVERGED;
  return LAMG_OK;
}

// Y = -A X for an n x k block of level 0 in colour order (the residual kernel
// with b = 0).
void mv_neg_apply(Hierarchy* H, int k, const double* Xp, double* Yp) {
  mv_alloc(H, k);
  residual_mv<double>(H->s, H->lv[0], k, nullptr, Xp, Yp);
}

// Xp <- `cycles` cycles of the correction-form outer loop on A x = Bp - mean(Bp)
// from x = 0, every column iterating (colour order, level 0).  The inner
// cycle runs in the handle's precision.  Xp leaves zero-mean.
void mv_precondition(Hierarchy* H, int k, const double* Bp, double* Xp, int cycles) {
  mv_alloc(H, k);
  MVWork& W = H->mv;
  Level& L = H->lv[0];
  hipStream_t s = H->s;
  const int n = L.n;
  const int64_t nk = (int64_t)n * k;
  for (int c = 0; c < k; ++c) W.hmask[c] = 1;
  LAMG_HIP(hipMemcpyAsync(W.mask, W.hmask, (size_t)k * sizeof(int), hipMemcpyHostToDevice, s));
  fill_mv<double>(s, Xp, nk);
  hipLaunchKernelGGL(k_copy_mv<double>, gridn(nk), dim3(MVT), 0, s, nk, Bp, W.R);
  const bool fp32 = H->o.precision == LAMG_FP32_REFINE;
  for (int it = 0; it < cycles; ++it) {
    if (it > 0) residual_mv<double>(s, L, k, Bp, Xp, W.R);
    col_reduce<double>(s, H, W.R, n, 0, RS_RMEAN, (double)n);
    const double* rm = W.res + RS_RMEAN * k;
    if (!fp32) {
      Vecs<double>& v = W.v64[0];
      hipLaunchKernelGGL(k_mv_rhs<double>, gridn(nk), dim3(MVT), 0, s, nk, k, (const double*)W.R, rm, v.b);
      fill_mv<double>(s, v.x, nk);
      cycle_graph_mv<double>(H);
      hipLaunchKernelGGL(k_mv_add<double>, gridn(nk), dim3(MVT), 0, s, nk, k, (const double*)v.x,
                         (const int*)W.mask, Xp);
    } else {
      Vecs<float>& v = W.v32[0];
      hipLaunchKernelGGL(k_mv_rhs<float>, gridn(nk), dim3(MVT), 0, s, nk, k, (const double*)W.R, rm, v.b);
      fill_mv<float>(s, v.x, nk);
      cycle_graph_mv<float>(H);
      hipLaunchKernelGGL(k_mv_add<float>, gridn(nk), dim3(MVT), 0, s, nk, k, (const float*)v.x, (const int*)W.mask,
                         Xp);
    }
    subtract_mean_mv<double>(s, H, Xp, n, W.mask);
  }
  LAMG_HIP(hipGetLastError());
}

// Zero-mean columns of an n x k block of level 0.
void mv_project(Hierarchy* H, int k, double* Xp) {
  mv_alloc(H, k);
  MVWork& W = H->mv;
  for (int c = 0; c < k; ++c) W.hmask[c] = 1;
  LAMG_HIP(hipMemcpyAsync(W.mask, W.hmask, (size_t)k * sizeof(int), hipMemcpyHostToDevice, H->s));
  subtract_mean_mv<double>(H->s, H, Xp, H->lv[0].n, W.mask);
}

}  // namespace lamg

using namespace lamg;

extern "C" {

lamg_status lamg_t_mv_cycle(lamg_handle h, int32_t k, const double* b, double* x) {
  if (!h || k < 1 || !b || !x) return LAMG_E_INVALID_ARG;
  Hierarchy* H = &h->H;
  const int n = H->lv[0].n;
  if ((int64_t)n * k > (int64_t)0x7fffffff) return LAMG_E_INVALID_ARG;
  try {
    mv_alloc(H, k);
    const int64_t nk = (int64_t)n * k;
    hipStream_t s = H->s;
    Vecs<double>& v = H->mv.v64[0];
    LAMG_HIP(hipMemcpyAsync(v.b, b, nk * sizeof(double), hipMemcpyDeviceToDevice, s));
    LAMG_HIP(hipMemcpyAsync(v.x, x, nk * sizeof(double), hipMemcpyDeviceToDevice, s));
    cycle_mv<double>(H);
    LAMG_HIP(hipMemcpyAsync(x, v.x, nk * sizeof(double), hipMemcpyDeviceToDevice, s));
    LAMG_HIP(hipStreamSynchronize(s));
  } catch (const DevError& e) {
    set_last_error("lamg_t_mv_cycle", e.e);
    return LAMG_E_DEVICE;
  }
  return LAMG_OK;
}

lamg_status lamg_t_mv_columns(lamg_handle h, int32_t k, int32_t* cycles, double* rel, double* removed_mean) {
  if (!h || k < 1 || h->H.mv.k != k || !cycles || !rel || !removed_mean) return LAMG_E_INVALID_ARG;
  const MVWork& W = h->H.mv;
  for (int c = 0; c < k; ++c) {
    cycles[c] = W.cycles[c];
    rel[c] = W.rel[c];
    removed_mean[c] = W.removed[c];
  }
  return LAMG_OK;
}

}  // extern "C"
