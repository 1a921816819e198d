// Setup phase on the GPU (Section 4.1): Laplacian assembly, greedy colouring
// by Jones-Plassmann rounds, colour-major renumbering, low-degree elimination
// (Section 3.2), test vectors / affinity / energy-ratio test / hubs / weak
// edges (Sections 3.3-3.4), staged aggregation, and Galerkin coarsening.
// Every integer decision and every value that feeds one is computed in the
// same floating-point order as the CPU reference: short rows left to right,
// long rows as 64 strided partial sums and an xor butterfly, no contraction.
#include <cstring>

#include <algorithm>
#include <cmath>
#include <vector>

#include "lamg_device.hpp"
#include "lamg_internal.hpp"
#include "lamg_relax.hpp"
#include "lamg_sort.hpp"

namespace lamg {

void* dev_alloc(const lamg_options& o, size_t bytes) {
  void* p = nullptr;
  bytes = std::max<size_t>(bytes, 16);
  if (o.alloc) p = o.alloc(bytes, o.alloc_ctx);
  else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
  if (!p) throw DevError{hipErrorOutOfMemory};
  return p;
}
void dev_free(const lamg_options& o, void* p) {
  if (!p) return;
  if (o.dealloc) o.dealloc(p, o.alloc_ctx);
  else (void)hipFree(p);
}

namespace {
thread_local const lamg_options* t_scope_alloc = nullptr;
}  // namespace
AllocScope::AllocScope(const lamg_options* o) : prev(t_scope_alloc) { t_scope_alloc = o; }
AllocScope::~AllocScope() { t_scope_alloc = prev; }

void* dalloc(Hierarchy* H, size_t bytes) {
  void* p = dev_alloc(H->o, bytes);
  H->owned.push_back(p);
  H->owned_bytes.push_back(std::max<size_t>(bytes, 16));
  return p;
}

namespace {

// Temporary device buffers of one setup step, released at scope exit, through
// the allocator of the setup running on this thread.
struct Tmp {
  lamg_options o = t_scope_alloc ? *t_scope_alloc : options_defaults();
  std::vector<void*> ps;
  ~Tmp() { for (void* p : ps) dev_free(o, p); }
  template <class T>
  T* get(size_t count) {
    void* p = dev_alloc(o, count * sizeof(T));
    ps.push_back(p);
    return (T*)p;
  }
};

inline dim3 grid1(int64_t n, int b = 256) { return dim3((unsigned)std::max<int64_t>(1, (n + b - 1) / b)); }

unsigned bits_for(uint64_t maxkey) {
  unsigned b = 1;
  while (b < 64 && (maxkey >> b) != 0) ++b;
  return b;
}

template <class K, class V>
void sort_pairs(hipStream_t s, Tmp& tmp, const K* kin, K* kout, const V* vin, V* vout, int64_t n, unsigned endbit) {
  if (n == 0) return;
  void* t = tmp.get<char>(sortk::sort_scratch_bytes<K, V>(n));
  sortk::radix_sort<K, V>(s, kin, kout, vin, vout, n, endbit, t);
  LAMG_HIP(hipGetLastError());
}
template <class K>
void sort_keys_double(hipStream_t s, Tmp& tmp, const K* kin, K* kout, int64_t n) {
  if (n == 0) return;
  void* t = tmp.get<char>(sortk::sort_scratch_bytes<K, sortk::NoVal>(n));
  sortk::radix_sort<K, sortk::NoVal>(s, kin, kout, nullptr, nullptr, n, (unsigned)(8 * sizeof(K)), t);
  LAMG_HIP(hipGetLastError());
}
// exclusive scan of n ints; out has n+1 entries (out[n] = total)
void excl_scan(hipStream_t s, Tmp& tmp, const int* in, int* out, int64_t n) {
  int* t = tmp.get<int>(sortk::scan_scratch(n));
  sortk::exclusive_scan(s, in, out, n, t);
  LAMG_HIP(hipGetLastError());
}
template <class T>
T to_host(hipStream_t s, const T* p) {
  T v;
  LAMG_HIP(hipMemcpyAsync(&v, p, sizeof(T), hipMemcpyDeviceToHost, s));
  LAMG_HIP(hipStreamSynchronize(s));
  return v;
}
template <class T>
std::vector<T> to_host_vec(hipStream_t s, const T* p, size_t n) {
  std::vector<T> v(n);
  if (n) {
    LAMG_HIP(hipMemcpyAsync(v.data(), p, n * sizeof(T), hipMemcpyDeviceToHost, s));
    LAMG_HIP(hipStreamSynchronize(s));
  }
  return v;
}

// ------------------------------------------------------------- primitives
__global__ void k_iota(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i;
}
__global__ void k_zero_i(int* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}
// mark run heads of a sorted key array
__global__ void k_heads(const uint64_t* __restrict__ key, int64_t n, int* __restrict__ head) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) head[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}
// sum each run of equal keys sequentially in list order
__global__ void k_run_sums(const uint64_t* __restrict__ key, const double* __restrict__ v, int64_t n,
                           const int* __restrict__ head, const int* __restrict__ pos, uint64_t* __restrict__ ukey,
                           double* __restrict__ uval) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !head[i]) return;
  const uint64_t k0 = key[i];
  double s = v[i];
  for (int64_t j = i + 1; j < n && key[j] == k0; ++j) s += v[j];
  ukey[pos[i]] = k0;
  uval[pos[i]] = s;
}
// unique (row, col) keys -> CSR columns; row counts by atomics
__global__ void k_split_keys(const uint64_t* __restrict__ ukey, int64_t nu, uint64_t ncols, int* __restrict__ ci,
                             int* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nu) return;
  const uint64_t k = ukey[i];
  ci[i] = (int)(k % ncols);
  atomicAdd(&cnt[k / ncols], 1);
}

// Row sums in the fixed order (diagonal = sum of the row's weights).
__global__ void k_rowsum_short(int n, const int* __restrict__ rp, const double* __restrict__ val,
                               double* __restrict__ out) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const int p0 = rp[u], len = rp[u + 1] - p0;
  if (len > SHORT_ROW) return;
  out[u] = dev::row_sum_seq<double>(len, [&](int t) { return val[p0 + t]; });
}
__global__ void k_rowsum_long(const int* __restrict__ rows, int nrows, const int* __restrict__ rp,
                              const double* __restrict__ val, double* __restrict__ out) {
  const int idx = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, lane = threadIdx.x & 63;
  if (idx >= nrows) return;
  const int u = rows[idx];
  const int p0 = rp[u], len = rp[u + 1] - p0;
  const double s = dev::row_sum_wave<double>(len, lane, [&](int t) { return val[p0 + t]; });
  if (lane == 0) out[u] = s;
}
__global__ void k_collect_long(int n, const int* __restrict__ rp, int* __restrict__ list, int* __restrict__ cnt) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n && rp[u + 1] - rp[u] > SHORT_ROW) list[atomicAdd(cnt, 1)] = u;
}

// Long rows of a CSR, ascending (the order does not affect any result).
std::vector<int> long_rows_host(const std::vector<int>& rph, int n) {
  std::vector<int> v;
  for (int u = 0; u < n; ++u)
    if (rph[u + 1] - rph[u] > SHORT_ROW) v.push_back(u);
  return v;
}

void row_sums(hipStream_t s, Tmp& tmp, int n, const int* rp, const double* val, double* out) {
  hipLaunchKernelGGL(k_rowsum_short, grid1(n), dim3(256), 0, s, n, rp, val, out);
  std::vector<int> rph = to_host_vec(s, rp, (size_t)n + 1);
  std::vector<int> lr = long_rows_host(rph, n);
  if (!lr.empty()) {
    int* d = tmp.get<int>(lr.size());
    LAMG_HIP(hipMemcpyAsync(d, lr.data(), lr.size() * sizeof(int), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_rowsum_long, grid1((int64_t)lr.size() * 64), dim3(256), 0, s, d, (int)lr.size(), rp, val, out);
  }
  LAMG_HIP(hipGetLastError());
}

// Merge (row, col, value) triples given as keys row*ncols + col: stable sort,
// sum runs in list order, build the CSR and its diagonal.
void merge_triples(Hierarchy* H, Tmp& tmp, Level& C, int nrows, uint64_t* keys, double* vals, int64_t nt) {
  hipStream_t s = H->s;
  uint64_t* ks = tmp.get<uint64_t>(nt);
  double* vs = tmp.get<double>(nt);
  const uint64_t maxkey = (uint64_t)nrows * (uint64_t)nrows;
  sort_pairs(s, tmp, keys, ks, vals, vs, nt, bits_for(maxkey));
  int* head = tmp.get<int>(nt + 1);
  int* pos = tmp.get<int>(nt + 1);
  hipLaunchKernelGGL(k_heads, grid1(nt), dim3(256), 0, s, ks, nt, head);
  excl_scan(s, tmp, head, pos, nt);
  const int nu = nt ? to_host(s, pos + nt) : 0;
  uint64_t* uk = tmp.get<uint64_t>(nu);
  C.n = nrows;
  C.nnz = nu;
  C.val = dnew<double>(H, nu);
  hipLaunchKernelGGL(k_run_sums, grid1(nt), dim3(256), 0, s, ks, vs, nt, head, pos, uk, C.val);
  C.ci = dnew<int>(H, nu);
  int* cnt = tmp.get<int>((size_t)nrows + 1);
  hipLaunchKernelGGL(k_zero_i, grid1(nrows + 1), dim3(256), 0, s, cnt, (int64_t)nrows + 1);
  hipLaunchKernelGGL(k_split_keys, grid1(nu), dim3(256), 0, s, uk, (int64_t)nu, (uint64_t)nrows, C.ci, cnt);
  C.rp = dnew<int>(H, (size_t)nrows + 1);
  excl_scan(s, tmp, cnt, C.rp, nrows);
  C.diag = dnew<double>(H, nrows);
  row_sums(s, tmp, nrows, C.rp, C.val, C.diag);
}

// ------------------------------------------------------------ finest level
__global__ void k_validate(int64_t m, int64_t n, const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                           const double* __restrict__ w, int allow_negative, int* flags) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const int a = eu[e], b = ev[e];
  if (a < 0 || a >= n || b < 0 || b >= n || a == b) atomicOr(&flags[0], 1);
  const double x = w[e];
  if (!isfinite(x) || (allow_negative ? x == 0 : !(x > 0))) atomicOr(&flags[0], 2);
}
__global__ void k_count_negative(int64_t m, const double* __restrict__ v, int* cnt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < m && v[e] < 0) atomicAdd(cnt, 1);
}
__global__ void k_abs(int64_t m, const double* __restrict__ v, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < m) out[e] = fabs(v[e]);
}
__global__ void k_edge_keys(int64_t m, int64_t n, const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                            uint64_t* __restrict__ key) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const uint64_t a = (uint64_t)min(eu[e], ev[e]), b = (uint64_t)max(eu[e], ev[e]);
  key[e] = a * (uint64_t)n + b;
}
__global__ void k_directed(int64_t nu, uint64_t n, const uint64_t* __restrict__ ukey, const double* __restrict__ uw,
                           uint64_t* __restrict__ dkey, double* __restrict__ dval) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nu) return;
  const uint64_t a = ukey[i] / n, b = ukey[i] % n;
  dkey[2 * i] = a * n + b;
  dkey[2 * i + 1] = b * n + a;
  dval[2 * i] = uw[i];
  dval[2 * i + 1] = uw[i];
}
// connected components by min-label hooking and pointer jumping
__global__ void k_hook(int n, const int* __restrict__ rp, const int* __restrict__ ci, int* lab, int* changed) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  int best = lab[u];
  for (int t = rp[u]; t < rp[u + 1]; ++t) best = min(best, lab[ci[t]]);
  if (best < lab[u]) {
    atomicMin(&lab[lab[u]], best);
    atomicMin(&lab[u], best);
    *changed = 1;
  }
}
__global__ void k_jump(int n, int* lab) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  int l = lab[u];
  while (lab[l] != l) l = lab[l];
  lab[u] = l;
}
__global__ void k_count_nonzero(int n, const int* lab, int* cnt) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n && lab[u] != 0) atomicAdd(cnt, 1);
}

}  // namespace

lamg_status build_finest(Hierarchy* H, int64_t n, int64_t m, const int32_t* eu, const int32_t* ev, const double* w) {
  hipStream_t s = H->s;
  Tmp tmp;
  int* flags = tmp.get<int>(4);
  LAMG_HIP(hipMemsetAsync(flags, 0, 4 * sizeof(int), s));
  if (m > 0)
    hipLaunchKernelGGL(k_validate, grid1(m), dim3(256), 0, s, m, n, eu, ev, w, H->o.allow_negative_weights, flags);
  const int f = to_host(s, flags);
  if (f & 1) return LAMG_E_INVALID_ARG;
  if (f & 2) return LAMG_E_BAD_WEIGHT;
  Level L;
  L.type = LT_FINEST;
  if (m > 0) {
    uint64_t* key = tmp.get<uint64_t>(m);
    uint64_t* ks = tmp.get<uint64_t>(m);
    double* ws = tmp.get<double>(m);
    hipLaunchKernelGGL(k_edge_keys, grid1(m), dim3(256), 0, s, m, n, eu, ev, key);
    sort_pairs(s, tmp, (const uint64_t*)key, ks, w, ws, m, bits_for((uint64_t)n * (uint64_t)n));
    int* head = tmp.get<int>(m + 1);
    int* pos = tmp.get<int>(m + 1);
    hipLaunchKernelGGL(k_heads, grid1(m), dim3(256), 0, s, ks, m, head);
    excl_scan(s, tmp, head, pos, m);
    const int nu = to_host(s, pos + m);
    uint64_t* uk = tmp.get<uint64_t>(nu);
    double* uw = tmp.get<double>(nu);
    hipLaunchKernelGGL(k_run_sums, grid1(m), dim3(256), 0, s, ks, ws, m, head, pos, uk, uw);
    uint64_t* dk = tmp.get<uint64_t>(2 * (size_t)nu);
    double* dv = tmp.get<double>(2 * (size_t)nu);
    hipLaunchKernelGGL(k_directed, grid1(nu), dim3(256), 0, s, (int64_t)nu, (uint64_t)n, uk, uw, dk, dv);
    merge_triples(H, tmp, L, (int)n, dk, dv, 2 * (int64_t)nu);
  } else {
    L.n = (int)n;
    L.nnz = 0;
    L.rp = dnew<int>(H, n + 1);
    hipLaunchKernelGGL(k_zero_i, grid1(n + 1), dim3(256), 0, s, L.rp, n + 1);
    L.ci = dnew<int>(H, 1);
    L.val = dnew<double>(H, 1);
    L.diag = dnew<double>(H, n);
    LAMG_HIP(hipMemsetAsync(L.diag, 0, n * sizeof(double), s));
  }
  // connectivity (Section 1: the graph must be connected)
  int* lab = tmp.get<int>(n);
  int* chg = tmp.get<int>(2);
  hipLaunchKernelGGL(k_iota, grid1(n), dim3(256), 0, s, lab, (int)n);
  for (int it = 0; it < 100000; ++it) {
    LAMG_HIP(hipMemsetAsync(chg, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_hook, grid1(n), dim3(256), 0, s, (int)n, L.rp, L.ci, lab, chg);
    hipLaunchKernelGGL(k_jump, grid1(n), dim3(256), 0, s, (int)n, lab);
    if (!to_host(s, chg)) break;
  }
  LAMG_HIP(hipMemsetAsync(chg, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_count_nonzero, grid1(n), dim3(256), 0, s, (int)n, lab, chg);
  if (to_host(s, chg) != 0) return LAMG_E_NOT_CONNECTED;
  H->lv.push_back(L);
  return LAMG_OK;
}

// ---------------------------------------------------------------- colouring
namespace {
__global__ void k_prio_hash(int n, uint64_t seed, uint64_t level, uint64_t* h) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n) h[u] = dev::hash5(seed, STREAM_COLOUR, level, 0, (uint64_t)u);
}
__device__ inline bool higher(int a, int b, const int* deg, const uint64_t* h) {
  const int da = deg[a], db = deg[b];
  if (da != db) return da > db;
  const uint64_t ha = h[a], hb = h[b];
  if (ha != hb) return ha < hb;
  return a < b;
}
__global__ void k_degrees(int n, const int* __restrict__ rp, int* __restrict__ deg) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n) deg[u] = rp[u + 1] - rp[u];
}
// Greedy first fit in priority order as a topological sweep: pending[u]
// counts u's higher-priority neighbours not yet coloured.  A round colours the
// ready frontier (pending 0; pairwise non-adjacent, since of two neighbours
// the lower one waits for the higher), and each frontier node decrements its
// lower-priority neighbours; those reaching 0 form the next frontier.  A
// node's colour is the smallest one its higher-priority neighbours do not
// use, exactly as in the sequential rule.  The sweep takes as many rounds as
// the longest chain of decreasing priority; on power-law graphs most rounds
// hold a few hubs, so a node of more than COL_HEAVY entries gets a whole
// block and the others a wavefront each.
constexpr int COL_HEAVY = 64;
constexpr int COL_BLOCK = 1024;

// frontier lists of one round: heavy and light nodes, with their counts at
// cnt[2 * (r % 3)] and cnt[2 * (r % 3) + 1]
struct Frontier {
  int* heavy;
  int* light;
};

__device__ inline void col_append(int w, const int* __restrict__ rp, Frontier G, int* __restrict__ gcnt) {
  if (rp[w + 1] - rp[w] > COL_HEAVY) G.heavy[atomicAdd(&gcnt[0], 1)] = w;
  else G.light[atomicAdd(&gcnt[1], 1)] = w;
}

__device__ inline uint64_t wave_or(uint64_t m) {
  unsigned lo = (unsigned)m, hi = (unsigned)(m >> 32);
  for (int o = 32; o > 0; o >>= 1) {
    lo |= __shfl_xor(lo, o, 64);
    hi |= __shfl_xor(hi, o, 64);
  }
  return ((uint64_t)hi << 32) | lo;
}

__global__ void __launch_bounds__(256) k_pending(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                 const int* __restrict__ deg, const uint64_t* __restrict__ h,
                                                 int* __restrict__ pending, Frontier F, int* __restrict__ cnt) {
  const int lane = threadIdx.x & 63;
  const int u = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (u >= n) return;
  int c = 0;
  for (int t = rp[u] + lane; t < rp[u + 1]; t += 64) c += higher(ci[t], u, deg, h) ? 1 : 0;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if (lane == 0) {
    pending[u] = c;
    if (c == 0) col_append(u, rp, F, cnt);
  }
}

// One pass over u's row by `width` threads (lane k of them): the colours of
// higher neighbours in [base, base + 64) as a bit mask; on the first pass
// also the decrements of the lower neighbours.
__device__ inline uint64_t col_pass(int u, int p0, int p1, int k, int width, int base, bool first,
                                    const int* __restrict__ rp, const int* __restrict__ ci,
                                    const int* __restrict__ deg, const uint64_t* __restrict__ h,
                                    const int* __restrict__ col, int* __restrict__ pending, Frontier G,
                                    int* __restrict__ gcnt) {
  uint64_t mask = 0;
  for (int t = p0 + k; t < p1; t += width) {
    const int v = ci[t];
    if (higher(v, u, deg, h)) {
      const int cv = col[v];
      if (cv >= base && cv < base + 64) mask |= 1ULL << (cv - base);
    } else if (first && atomicSub(&pending[v], 1) == 1) {
      col_append(v, rp, G, gcnt);
    }
  }
  return mask;
}

// Round r: blocks take the heavy frontier nodes one each, then every
// wavefront takes light nodes one each.  The counters of the round after
// next are cleared here: the previous round, which read them, has finished.
__global__ void __launch_bounds__(COL_BLOCK) k_frontier(Frontier F, Frontier G, int* cnt, int r,
                                                        int* __restrict__ pending, const int* __restrict__ rp,
                                                        const int* __restrict__ ci, const int* __restrict__ deg,
                                                        const uint64_t* __restrict__ h, int* __restrict__ col) {
  __shared__ uint64_t red[COL_BLOCK / 64];
  __shared__ int chosen;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (blockIdx.x == 0 && threadIdx.x < 2) cnt[2 * ((r + 2) % 3) + threadIdx.x] = 0;
  const int nh = cnt[2 * (r % 3)], nl = cnt[2 * (r % 3) + 1];
  int* gcnt = cnt + 2 * ((r + 1) % 3);
  for (int i = blockIdx.x; i < nh; i += gridDim.x) {
    const int u = F.heavy[i];
    const int p0 = rp[u], p1 = rp[u + 1];
    int c = -1;
    for (int base = 0; c < 0; base += 64) {
      uint64_t m = wave_or(col_pass(u, p0, p1, threadIdx.x, COL_BLOCK, base, base == 0, rp, ci, deg, h, col,
                                    pending, G, gcnt));
      if (lane == 0) red[wid] = m;
      __syncthreads();
      if (threadIdx.x == 0) {
        uint64_t all = 0;
        for (int w = 0; w < COL_BLOCK / 64; ++w) all |= red[w];
        chosen = all != ~0ULL ? base + __builtin_ctzll(~all) : -1;
      }
      __syncthreads();
      c = chosen;
      __syncthreads();
    }
    if (threadIdx.x == 0) col[u] = c;
  }
  const int gw = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int nw = (int)((gridDim.x * blockDim.x) >> 6);
  for (int i = gw; i < nl; i += nw) {
    const int u = F.light[i];
    const int p0 = rp[u], p1 = rp[u + 1];
    int c = -1;
    for (int base = 0; c < 0; base += 64) {
      const uint64_t m = wave_or(col_pass(u, p0, p1, lane, 64, base, base == 0, rp, ci, deg, h, col, pending, G,
                                          gcnt));
      if (m != ~0ULL) c = base + __builtin_ctzll(~m);
    }
    if (lane == 0) col[u] = c;
  }
}

__global__ void k_max_i(int n, const int* __restrict__ a, int* __restrict__ out) {
  int m = -1;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) m = max(m, a[i]);
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}
// red-black colour of node i + side j of a side x side grid
__global__ void k_red_black(int n, int side, int* __restrict__ col) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n) col[u] = ((u % side) + (u / side)) & 1;
}
__global__ void k_inverse(int n, const int* __restrict__ perm, int* __restrict__ inv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) inv[perm[i]] = i;
}
// Histogram of labels: per-block LDS counters for labels < 1024, global
// atomics for the rest.
__global__ void k_count_colours(int n, const int* __restrict__ col, int* __restrict__ cnt) {
  __shared__ int lc[1024];
  for (int i = threadIdx.x; i < 1024; i += blockDim.x) lc[i] = 0;
  __syncthreads();
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n) {
    const int c = col[u];
    if (c < 1024) atomicAdd(&lc[c], 1);
    else atomicAdd(&cnt[c], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 1024; i += blockDim.x)
    if (lc[i]) atomicAdd(&cnt[i], lc[i]);
}
__global__ void k_perm_deg(int n, const int* __restrict__ perm, const int* __restrict__ rp, int* __restrict__ deg,
                           const double* __restrict__ dold, double* __restrict__ dnew_) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int o = perm[i];
  deg[i] = rp[o + 1] - rp[o];
  dnew_[i] = dold[o];
}
__global__ void k_perm_keys(int n, const int* __restrict__ rp, const int* __restrict__ ci, const int* __restrict__ inv,
                            uint64_t* __restrict__ key) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const uint64_t nu = (uint64_t)inv[u];
  for (int t = rp[u]; t < rp[u + 1]; ++t) key[t] = nu * (uint64_t)n + (uint64_t)inv[ci[t]];
}
__global__ void k_key_cols(int64_t nnz, uint64_t n, const uint64_t* __restrict__ key, int* __restrict__ ci) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nnz) ci[i] = (int)(key[i] % n);
}
}  // namespace

// Colour the level, renumber it into (colour, previous id) order, and build
// its relaxation tiles.  Returns the inverse permutation (old -> new) in
// `inv_dev` owned by the caller's temporaries.
// Greedy first-fit colouring in priority order by Jones-Plassmann rounds;
// returns the number of colours.
int colour_greedy(hipStream_t s, int n, const int* rp, const int* ci, uint64_t seed, int level, int* col) {
  Tmp tmp;
  int* deg = tmp.get<int>(n);
  uint64_t* h = tmp.get<uint64_t>(n);
  int* ctr = tmp.get<int>(2);
  hipLaunchKernelGGL(k_degrees, grid1(n), dim3(256), 0, s, n, rp, deg);
  hipLaunchKernelGGL(k_prio_hash, grid1(n), dim3(256), 0, s, n, seed, (uint64_t)level, h);
  LAMG_HIP(hipMemsetAsync(col, 0xff, (size_t)n * sizeof(int), s));
  LAMG_HIP(hipMemsetAsync(ctr, 0xff, 2 * sizeof(int), s));
  Frontier fr[2] = {{tmp.get<int>(n), tmp.get<int>(n)}, {tmp.get<int>(n), tmp.get<int>(n)}};
  int* cnt = tmp.get<int>(6);
  int* pending = tmp.get<int>(n);
  LAMG_HIP(hipMemsetAsync(cnt, 0, 6 * sizeof(int), s));
  hipLaunchKernelGGL(k_pending, dim3((unsigned)(((int64_t)n + 3) / 4)), dim3(256), 0, s, n, rp, ci, deg, h, pending,
                     fr[0], cnt);
  // rounds until every node is coloured; the host checks every 16 rounds
  // (rounds past the last are empty)
  const int grid = std::max(1, std::min(256, (n + 15) / 16));
  int r = 0;
  for (;;) {
    for (int k = 0; k < 16; ++k, ++r)
      hipLaunchKernelGGL(k_frontier, dim3(grid), dim3(COL_BLOCK), 0, s, fr[r & 1], fr[(r + 1) & 1], cnt, r, pending,
                         rp, ci, deg, h, col);
    LAMG_HIP(hipGetLastError());
    const int c0 = to_host(s, cnt + 2 * (r % 3)), c1 = to_host(s, cnt + 2 * (r % 3) + 1);
    if (c0 == 0 && c1 == 0) break;
    if (r > n + 16) throw DevError{hipErrorUnknown};
  }
  hipLaunchKernelGGL(k_max_i, dim3(std::max(1, std::min(1024, (n + 255) / 256))), dim3(256), 0, s, n, (const int*)col,
                     ctr + 1);
  return to_host(s, ctr + 1) + 1;
}

// rb_side > 0: the level is an rb_side x rb_side grid in natural order and
// takes the red-black colouring (i + j) mod 2 instead of the greedy one.
static int* colour_order_impl(Hierarchy* H, Tmp& tmp, Level& L, int level, int rb_side = 0) {
  hipStream_t s = H->s;
  const int n = L.n;
  int* col = tmp.get<int>(n);
  int ncol = 0;
  if (rb_side > 0) {
    hipLaunchKernelGGL(k_red_black, grid1(n), dim3(256), 0, s, n, rb_side, col);
    ncol = n > 1 ? 2 : 1;
  } else {
    ncol = colour_greedy(s, n, L.rp, L.ci, (uint64_t)H->o.seed, level, col);
  }
  // permutation: stable sort of ids by colour
  int* ids = tmp.get<int>(n);
  int* cs = tmp.get<int>(n);
  int* perm = dnew<int>(H, n);
  hipLaunchKernelGGL(k_iota, grid1(n), dim3(256), 0, s, ids, n);
  sort_pairs(s, tmp, (const unsigned*)col, (unsigned*)cs, (const int*)ids, perm, n, bits_for((uint64_t)ncol));
  int* cc = tmp.get<int>(ncol + 1);
  int* cptr = tmp.get<int>(ncol + 1);
  hipLaunchKernelGGL(k_zero_i, grid1(ncol + 1), dim3(256), 0, s, cc, (int64_t)ncol + 1);
  hipLaunchKernelGGL(k_count_colours, grid1(n), dim3(256), 0, s, n, col, cc);
  excl_scan(s, tmp, cc, cptr, ncol);
  L.ncol = ncol;
  L.cptr = to_host_vec(s, cptr, (size_t)ncol + 1);
  int* inv = tmp.get<int>(n);
  hipLaunchKernelGGL(k_inverse, grid1(n), dim3(256), 0, s, n, perm, inv);
  // permuted CSR: rows by perm, columns renamed and re-sorted
  int* ndeg = tmp.get<int>(n + 1);
  double* ndiag = dnew<double>(H, n);
  hipLaunchKernelGGL(k_perm_deg, grid1(n), dim3(256), 0, s, n, perm, L.rp, ndeg, L.diag, ndiag);
  int* nrp = dnew<int>(H, (size_t)n + 1);
  excl_scan(s, tmp, ndeg, nrp, n);
  if (L.nnz > 0) {
    uint64_t* key = tmp.get<uint64_t>(L.nnz);
    uint64_t* ks = tmp.get<uint64_t>(L.nnz);
    double* nval = dnew<double>(H, L.nnz);
    int* nci = dnew<int>(H, L.nnz);
    hipLaunchKernelGGL(k_perm_keys, grid1(n), dim3(256), 0, s, n, L.rp, L.ci, inv, key);
    sort_pairs(s, tmp, (const uint64_t*)key, ks, (const double*)L.val, nval, L.nnz,
               bits_for((uint64_t)n * (uint64_t)n));
    hipLaunchKernelGGL(k_key_cols, grid1(L.nnz), dim3(256), 0, s, (int64_t)L.nnz, (uint64_t)n, ks, nci);
    L.ci = nci;
    L.val = nval;
  }
  L.rp = nrp;
  L.diag = ndiag;
  L.perm = perm;
  build_tiles(H, L);
  LAMG_HIP(hipGetLastError());
  return inv;
}

// Relaxation tiles per colour: consecutive short rows packed into stream
// tiles (<= TILE_ROWS rows, <= TILE_NNZ entries); medium and very long rows
// listed apart, longest first, so that their blocks are dispatched first.
static void upload_tiles(Hierarchy* H, Tiles& t, const std::vector<int2>& blocks, std::vector<int> vl,
                         std::vector<int> md, const std::vector<int>& rph) {
  hipStream_t s = H->s;
  auto longer = [&](int a, int b) {
    const int da = rph[a + 1] - rph[a], db = rph[b + 1] - rph[b];
    return da != db ? da > db : a < b;
  };
  std::sort(vl.begin(), vl.end(), longer);
  std::sort(md.begin(), md.end(), longer);
  std::vector<int> all(vl);
  all.insert(all.end(), md.begin(), md.end());
  t.nstream = (int)blocks.size();
  t.nvlong = (int)vl.size();
  t.nmed = (int)md.size();
  t.nmed_blocks = (t.nmed + LONG_PER_BLOCK - 1) / LONG_PER_BLOCK;
  t.nlong = (int)all.size();
  // work-list entries carry the row extents, so a block starts its entry
  // loads without first reading the row pointers
  std::vector<int4> sb(blocks.size()), v4(vl.size()), m4(md.size());
  for (size_t i = 0; i < blocks.size(); ++i)
    sb[i] = make_int4(blocks[i].x, blocks[i].y, rph[blocks[i].x], rph[blocks[i].y] - rph[blocks[i].x]);
  for (size_t i = 0; i < vl.size(); ++i) v4[i] = make_int4(vl[i], rph[vl[i]], rph[vl[i] + 1] - rph[vl[i]], 0);
  for (size_t i = 0; i < md.size(); ++i) m4[i] = make_int4(md[i], rph[md[i]], rph[md[i] + 1] - rph[md[i]], 0);
  t.stream = dnew<int4>(H, sb.size());
  t.vlong = dnew<int4>(H, v4.size());
  t.med = dnew<int4>(H, m4.size());
  t.longrows = dnew<int>(H, all.size());
  if (!sb.empty()) LAMG_HIP(hipMemcpyAsync(t.stream, sb.data(), sb.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  if (!v4.empty()) LAMG_HIP(hipMemcpyAsync(t.vlong, v4.data(), v4.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  if (!m4.empty()) LAMG_HIP(hipMemcpyAsync(t.med, m4.data(), m4.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  if (!all.empty()) LAMG_HIP(hipMemcpyAsync(t.longrows, all.data(), all.size() * sizeof(int), hipMemcpyHostToDevice, s));
  LAMG_HIP(hipStreamSynchronize(s));
}

void build_tiles(Hierarchy* H, Level& L) {
  hipStream_t s = H->s;
  std::vector<int> rph = to_host_vec(s, L.rp, (size_t)L.n + 1);
  L.tiles.assign(L.ncol, Tiles());
  L.long_ptr.assign(1, 0);
  L.long_rows.clear();
  std::vector<int2> all_s;
  std::vector<int> all_v, all_m;
  for (int c = 0; c < L.ncol; ++c) {
    std::vector<int2> blocks;
    std::vector<int> vl, md;
    int a = L.cptr[c];
    const int e = L.cptr[c + 1];
    while (a < e) {
      const int d0 = rph[a + 1] - rph[a];
      if (d0 > SHORT_ROW) { (d0 > ROW_CHUNK ? vl : md).push_back(a); ++a; continue; }
      int b = a, nz = 0;
      while (b < e && b - a < TILE_ROWS) {
        const int d = rph[b + 1] - rph[b];
        if (d > SHORT_ROW || nz + d > TILE_NNZ) break;
        nz += d;
        ++b;
      }
      blocks.push_back(make_int2(a, b));
      a = b;
    }
    Tiles& t = L.tiles[c];
    t.rows = e - L.cptr[c];
    t.nnz = rph[e] - rph[L.cptr[c]];
    upload_tiles(H, t, blocks, vl, md, rph);
    L.long_rows.insert(L.long_rows.end(), vl.begin(), vl.end());
    L.long_rows.insert(L.long_rows.end(), md.begin(), md.end());
    L.long_ptr.push_back((int)L.long_rows.size());
    all_s.insert(all_s.end(), blocks.begin(), blocks.end());
    all_v.insert(all_v.end(), vl.begin(), vl.end());
    all_m.insert(all_m.end(), md.begin(), md.end());
  }
  L.all.rows = L.n;
  L.all.nnz = rph[L.n];
  upload_tiles(H, L.all, all_s, all_v, all_m, rph);
}

void colour_and_order(Hierarchy* H, Level& L, int level, std::vector<int>*) {
  Tmp tmp;
  colour_order_impl(H, tmp, L, level);
}

// -------------------------------------------------------------- elimination
namespace {
// Section 3.2: in (colour, id) order, a node of degree <= maxdeg with no
// neighbour in F joins F.  Nodes of one colour are pairwise non-adjacent, so
// each colour class decides at once and later classes see its result.
__global__ void k_elim_colour(int r0, int r1, const int* __restrict__ rp, const int* __restrict__ ci, int maxdeg,
                              int* inF, int* cnt) {
  const int u = r0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= r1) return;
  const int p0 = rp[u], p1 = rp[u + 1];
  if (p1 - p0 > maxdeg) return;
  for (int t = p0; t < p1; ++t)
    if (inF[ci[t]]) return;
  inF[u] = 1;
  atomicAdd(cnt, 1);
}
__global__ void k_not(int n, const int* __restrict__ a, int* __restrict__ b) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n) b[u] = 1 - a[u];
}
// emission counts: C rows -> number of C neighbours; F rows -> deg (deg - 1)
__global__ void k_schur_counts(int n, const int* __restrict__ rp, const int* __restrict__ ci, const int* __restrict__ inF,
                               int* __restrict__ ccnt, int* __restrict__ fcnt) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const int d = rp[u + 1] - rp[u];
  if (inF[u]) { ccnt[u] = 0; fcnt[u] = d * (d - 1); return; }
  int c = 0;
  for (int t = rp[u]; t < rp[u + 1]; ++t) c += inF[ci[t]] ? 0 : 1;
  ccnt[u] = c;
  fcnt[u] = 0;
}
// w^c_ij = w_ij + sum_f w_fi w_fj / a_ff (eq. elim), emitted C-C edges first,
// then each F node's ordered neighbour pairs.
__global__ void k_schur_emit(int n, uint64_t nc, const int* __restrict__ rp, const int* __restrict__ ci,
                             const double* __restrict__ val, const double* __restrict__ diag, const int* __restrict__ inF,
                             const int* __restrict__ crank, const int* __restrict__ coff, const int* __restrict__ foff,
                             int ctot, uint64_t* __restrict__ key, double* __restrict__ v) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const int p0 = rp[u], p1 = rp[u + 1];
  if (!inF[u]) {
    int o = coff[u];
    const uint64_t cu = (uint64_t)crank[u];
    for (int t = p0; t < p1; ++t)
      if (!inF[ci[t]]) { key[o] = cu * nc + (uint64_t)crank[ci[t]]; v[o] = val[t]; ++o; }
    return;
  }
  int o = ctot + foff[u];
  const double d = diag[u];
  for (int a = p0; a < p1; ++a)
    for (int b = p0; b < p1; ++b) {
      if (a == b) continue;
      key[o] = (uint64_t)crank[ci[a]] * nc + (uint64_t)crank[ci[b]];
      v[o] = (val[a] * val[b]) / d;
      ++o;
    }
}
// C-side restriction stencil: for coarse node c (fine node cfine[c]) the F
// neighbours f in column order with coefficient w_cf / a_ff.
__global__ void k_er_counts(int nc, const int* __restrict__ cfine, const int* __restrict__ cidx,
                            const int* __restrict__ rp, const int* __restrict__ ci, int* __restrict__ cnt) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const int u = cfine[c];
  int k = 0;
  for (int t = rp[u]; t < rp[u + 1]; ++t) k += cidx[ci[t]] < 0;
  cnt[c] = k;
}
__global__ void k_er_fill(int nc, const int* __restrict__ cfine, const int* __restrict__ cidx,
                          const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ val,
                          const double* __restrict__ diag, const int* __restrict__ erp, int* __restrict__ eci,
                          double* __restrict__ ev, float* __restrict__ ev32) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const int u = cfine[c];
  int o = erp[c];
  for (int t = rp[u]; t < rp[u + 1]; ++t) {
    const int f = ci[t];
    if (cidx[f] >= 0) continue;
    eci[o] = f;
    ev[o] = val[t] / diag[f];
    ev32[o] = (float)val[t] / (float)diag[f];
    ++o;
  }
}
__global__ void k_elim_maps(int n, const int* __restrict__ inF, const int* __restrict__ crank,
                            const int* __restrict__ cinv, int* __restrict__ cidx, int* __restrict__ cfine) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  if (inF[u]) { cidx[u] = -1; return; }
  const int c = cinv[crank[u]];
  cidx[u] = c;
  cfine[c] = u;
}
}  // namespace

void build_elim_restriction(Hierarchy* H, const Level& F, Level& C) {
  hipStream_t s = H->s;
  Tmp tmp;
  const int nc = C.n;
  int* cnt = tmp.get<int>(nc + 1);
  hipLaunchKernelGGL(k_er_counts, grid1(nc), dim3(256), 0, s, nc, C.cfine, C.cidx, F.rp, F.ci, cnt);
  C.er_rp = dnew<int>(H, (size_t)nc + 1);
  excl_scan(s, tmp, cnt, C.er_rp, nc);
  const int ne = to_host(s, C.er_rp + nc);
  C.er_ci = dnew<int>(H, std::max(ne, 1));
  C.er_val = dnew<double>(H, std::max(ne, 1));
  C.er_val32 = dnew<float>(H, std::max(ne, 1));
  hipLaunchKernelGGL(k_er_fill, grid1(nc), dim3(256), 0, s, nc, C.cfine, C.cidx, F.rp, F.ci, F.val, F.diag, C.er_rp,
                     C.er_ci, C.er_val, C.er_val32);
  // tiles over the stencil rows (a single class: rows are independent)
  Level R;
  R.n = nc;
  R.rp = C.er_rp;
  R.ci = C.er_ci;
  R.ncol = 1;
  R.cptr = {0, nc};
  build_tiles(H, R);
  C.er_tiles = R.all;
}

bool try_eliminate(Hierarchy* H, int l) {
  hipStream_t s = H->s;
  Tmp tmp;
  const Level& F = H->lv[l];
  const int n = F.n;
  int* inF = tmp.get<int>(n);
  int* cnt = tmp.get<int>(1);
  LAMG_HIP(hipMemsetAsync(inF, 0, (size_t)n * sizeof(int), s));
  LAMG_HIP(hipMemsetAsync(cnt, 0, sizeof(int), s));
  for (int c = 0; c < F.ncol; ++c) {
    const int r0 = F.cptr[c], r1 = F.cptr[c + 1];
    if (r1 > r0)
      hipLaunchKernelGGL(k_elim_colour, grid1(r1 - r0), dim3(256), 0, s, r0, r1, F.rp, F.ci, H->o.elim_max_degree, inF,
                         cnt);
  }
  const int nF = to_host(s, cnt);
  if (nF == 0 || (double)nF < H->o.elim_stop_frac * (double)n) return false;
  int* isC = tmp.get<int>(n + 1);
  int* crank = tmp.get<int>(n + 1);
  hipLaunchKernelGGL(k_not, grid1(n), dim3(256), 0, s, n, inF, isC);
  excl_scan(s, tmp, isC, crank, n);
  const int nc = n - nF;
  int* ccnt = tmp.get<int>(n + 1);
  int* fcnt = tmp.get<int>(n + 1);
  int* coff = tmp.get<int>(n + 1);
  int* foff = tmp.get<int>(n + 1);
  hipLaunchKernelGGL(k_schur_counts, grid1(n), dim3(256), 0, s, n, F.rp, F.ci, inF, ccnt, fcnt);
  excl_scan(s, tmp, ccnt, coff, n);
  excl_scan(s, tmp, fcnt, foff, n);
  const int ctot = to_host(s, coff + n), ftot = to_host(s, foff + n);
  const int64_t nt = (int64_t)ctot + ftot;
  uint64_t* key = tmp.get<uint64_t>(nt);
  double* v = tmp.get<double>(nt);
  hipLaunchKernelGGL(k_schur_emit, grid1(n), dim3(256), 0, s, n, (uint64_t)nc, F.rp, F.ci, F.val, F.diag, inF, crank,
                     coff, foff, ctot, key, v);
  Level C;
  C.type = LT_ELIM;
  C.nF = nF;
  merge_triples(H, tmp, C, nc, key, v, nt);
  int* cinv = colour_order_impl(H, tmp, C, l + 1);
  C.cidx = dnew<int>(H, n);
  C.cfine = dnew<int>(H, nc);
  hipLaunchKernelGGL(k_elim_maps, grid1(n), dim3(256), 0, s, n, inF, crank, cinv, C.cidx, C.cfine);
  build_elim_restriction(H, F, C);
  LAMG_HIP(hipStreamSynchronize(s));
  H->lv.push_back(C);
  return true;
}

// -------------------------------------------------------------- aggregation
namespace {
__global__ void k_tv_init(int n, int K, uint64_t seed, uint64_t level, double* X) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * K) return;
  const int u = (int)(i / K), k = (int)(i % K);
  X[i] = dev::unit_pm1(dev::hash5(seed, STREAM_TV, level, (uint64_t)k, (uint64_t)u));
}
// Node quantities: |X_u|^2, y*_k = (sum_v w_uv x_v)/a_uu, Emin_k =
// 1/2 sum_v w_uv (x_v - y*_k)^2 (minimum of the local energy, Section 3.4.4),
// sum_v w_uv, sum_v w_uv |E_v| (hub test), max_v w_uv (weak edges).
struct NodeOut {
  double *nrm, *ystar, *emin, *sw, *swd, *maxw;
};
__global__ void k_node_short(int n, int K, const int* __restrict__ rp, const int* __restrict__ ci,
                             const double* __restrict__ val, const double* __restrict__ diag, const int* __restrict__ deg,
                             const double* __restrict__ X, NodeOut o) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const int p0 = rp[u], len = rp[u + 1] - p0;
  double s = 0;
  for (int k = 0; k < K; ++k) s += X[(size_t)u * K + k] * X[(size_t)u * K + k];
  o.nrm[u] = s;
  double mw = 0;
  for (int t = p0; t < p0 + len; ++t) mw = fmax(mw, val[t]);
  o.maxw[u] = mw;
  if (len > SHORT_ROW) return;
  for (int k = 0; k < K; ++k) {
    const double B = dev::row_sum_seq<double>(len, [&](int t) { return val[p0 + t] * X[(size_t)ci[p0 + t] * K + k]; });
    const double y = B / diag[u];
    const double S2 = dev::row_sum_seq<double>(len, [&](int t) {
      const double d = X[(size_t)ci[p0 + t] * K + k] - y;
      return val[p0 + t] * (d * d);
    });
    o.ystar[(size_t)u * K + k] = y;
    o.emin[(size_t)u * K + k] = 0.5 * S2;
  }
  o.sw[u] = dev::row_sum_seq<double>(len, [&](int t) { return val[p0 + t]; });
  o.swd[u] = dev::row_sum_seq<double>(len, [&](int t) { return val[p0 + t] * (double)deg[ci[p0 + t]]; });
}
__global__ void k_node_long(const int* __restrict__ rows, int nrows, int K, const int* __restrict__ rp,
                            const int* __restrict__ ci, const double* __restrict__ val, const double* __restrict__ diag,
                            const int* __restrict__ deg, const double* __restrict__ X, NodeOut o) {
  const int idx = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, lane = threadIdx.x & 63;
  if (idx >= nrows) return;
  const int u = rows[idx];
  const int p0 = rp[u], len = rp[u + 1] - p0;
  for (int k = 0; k < K; ++k) {
    const double B = dev::row_sum_wave<double>(len, lane, [&](int t) { return val[p0 + t] * X[(size_t)ci[p0 + t] * K + k]; });
    const double y = B / diag[u];
    const double S2 = dev::row_sum_wave<double>(len, lane, [&](int t) {
      const double d = X[(size_t)ci[p0 + t] * K + k] - y;
      return val[p0 + t] * (d * d);
    });
    if (lane == 0) {
      o.ystar[(size_t)u * K + k] = y;
      o.emin[(size_t)u * K + k] = 0.5 * S2;
    }
  }
  const double sw = dev::row_sum_wave<double>(len, lane, [&](int t) { return val[p0 + t]; });
  const double swd = dev::row_sum_wave<double>(len, lane, [&](int t) { return val[p0 + t] * (double)deg[ci[p0 + t]]; });
  if (lane == 0) { o.sw[u] = sw; o.swd[u] = swd; }
}
// Per directed edge: affinity c_us (eq. cuv), energy-ratio admissibility
// (eq. qut, ratio >= 1 form: a_uu (x_s - y*)^2 <= 2 (q_max - 1) Emin for all
// test vectors), weak flag (w < ratio * max neighbouring weight).
__global__ void k_edges(int n, int K, const int* __restrict__ rp, const int* __restrict__ ci,
                        const double* __restrict__ val, const double* __restrict__ diag, const double* __restrict__ X,
                        NodeOut o, double qfac, double wratio, double* __restrict__ aff, uint8_t* __restrict__ ok,
                        uint8_t* __restrict__ weak) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const double nu = o.nrm[u], du = diag[u], mu = o.maxw[u];
  for (int t = rp[u]; t < rp[u + 1]; ++t) {
    const int s = ci[t];
    double p = 0;
    for (int k = 0; k < K; ++k) p += X[(size_t)u * K + k] * X[(size_t)s * K + k];
    double c = 1.0;
    const double ns = o.nrm[s];
    if (nu > 0 && ns > 0) {
      c = 1.0 - (p * p) / (nu * ns);
      if (c < 0) c = 0;
    }
    aff[t] = c;
    bool good = true;
    for (int k = 0; k < K && good; ++k) {
      const double d = X[(size_t)s * K + k] - o.ystar[(size_t)u * K + k];
      good = (du * (d * d)) <= (qfac * o.emin[(size_t)u * K + k]);
    }
    ok[t] = good ? 1 : 0;
    weak[t] = (val[t] < wratio * fmax(mu, o.maxw[s])) ? 1 : 0;
  }
}
// Node energies e_uk = sum_v w_uv (x_uk - x_vk)^2 of K vectors (fixed row order).
__global__ void k_energy_short(int n, int K, const int* __restrict__ rp, const int* __restrict__ ci,
                               const double* __restrict__ val, const double* __restrict__ X, double* __restrict__ e) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const int p0 = rp[u], len = rp[u + 1] - p0;
  if (len > SHORT_ROW) return;
  for (int k = 0; k < K; ++k)
    e[(size_t)u * K + k] = dev::row_sum_seq<double>(len, [&](int t) {
      const double d = X[(size_t)u * K + k] - X[(size_t)ci[p0 + t] * K + k];
      return val[p0 + t] * (d * d);
    });
}
__global__ void k_energy_long(const int* __restrict__ rows, int nrows, int K, const int* __restrict__ rp,
                              const int* __restrict__ ci, const double* __restrict__ val, const double* __restrict__ X,
                              double* __restrict__ e) {
  const int idx = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, lane = threadIdx.x & 63;
  if (idx >= nrows) return;
  const int u = rows[idx];
  const int p0 = rp[u], len = rp[u + 1] - p0;
  for (int k = 0; k < K; ++k) {
    const double s = dev::row_sum_wave<double>(len, lane, [&](int t) {
      const double d = X[(size_t)u * K + k] - X[(size_t)ci[p0 + t] * K + k];
      return val[p0 + t] * (d * d);
    });
    if (lane == 0) e[(size_t)u * K + k] = s;
  }
}
// column sums of an n x K array, one block per column, fixed tree order
__global__ __launch_bounds__(256) void k_colsum(int n, int K, const double* __restrict__ e, double* __restrict__ out) {
  __shared__ double sh[256];
  const int k = blockIdx.x;
  double v = 0;
  for (int u = threadIdx.x; u < n; u += 256) v += e[(size_t)u * K + k];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = sh[0];
}
// Initial states: hubs (Section 3.4.1 footnote) are seeds; nodes whose every
// edge is weak go to the dummy aggregate; others are undecided.
__global__ void k_init_state(int n, const int* __restrict__ rp, const int* __restrict__ deg, NodeOut o,
                             double hubf, const uint8_t* __restrict__ weak, int* __restrict__ st,
                             uint8_t* __restrict__ hub, int* __restrict__ seedof) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  seedof[u] = -1;
  if ((double)deg[u] * o.sw[u] >= hubf * o.swd[u]) { hub[u] = 1; st[u] = ST_SEED; return; }
  hub[u] = 0;
  bool allweak = rp[u + 1] > rp[u];
  for (int t = rp[u]; t < rp[u + 1]; ++t)
    if (!weak[t]) { allweak = false; break; }
  st[u] = allweak ? ST_DUMMY : ST_UNDECIDED;
}
__device__ inline bool candidate(int t, const int* ci, const int* st, const uint8_t* weak, const uint8_t* ok,
                                 const double* aff, double delta) {
  const int ss = st[ci[t]];
  return (ss == ST_SEED || ss == ST_UNDECIDED) && !weak[t] && ok[t] && aff[t] <= delta;
}
// best candidate affinity of each undecided node (2.0 when none)
__global__ void k_best(int n, const int* __restrict__ rp, const int* __restrict__ ci, const int* __restrict__ st,
                       const uint8_t* __restrict__ weak, const uint8_t* __restrict__ ok, const double* __restrict__ aff,
                       double* __restrict__ best, int* cnt) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  double b = 2.0;
  if (st[u] == ST_UNDECIDED)
    for (int t = rp[u]; t < rp[u + 1]; ++t)
      if (candidate(t, ci, st, weak, ok, aff, 1.0)) b = fmin(b, aff[t]);
  best[u] = b;
  if (b <= 1.0) atomicAdd(cnt, 1);
}
// One colour class of an aggregation stage (Section 3.4.2): each undecided
// node joins its non-associate neighbour of smallest affinity (ties: smallest
// id) among admissible non-weak candidates within the stage threshold.
__global__ void k_agg_colour(int r0, int r1, const int* __restrict__ rp, const int* __restrict__ ci, int* st,
                             int* __restrict__ seedof, const uint8_t* __restrict__ weak, const uint8_t* __restrict__ ok,
                             const double* __restrict__ aff, double delta) {
  const int u = r0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= r1) return;
  if (st[u] != ST_UNDECIDED) return;
  int bt = -1;
  for (int t = rp[u]; t < rp[u + 1]; ++t) {
    const int ss = __hip_atomic_load(&st[ci[t]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((ss == ST_SEED || ss == ST_UNDECIDED) && !weak[t] && ok[t] && aff[t] <= delta)
      if (bt < 0 || aff[t] < aff[bt]) bt = t;
  }
  if (bt < 0) return;
  const int sd = ci[bt];
  st[u] = ST_ASSOC;
  seedof[u] = sd;
  __hip_atomic_store(&st[sd], (int)ST_SEED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__global__ void k_count_states(int n, const int* __restrict__ st, int* cnt) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const int x = st[u];
  if (x == ST_SEED || x == ST_UNDECIDED) atomicAdd(&cnt[0], 1);
  else if (x == ST_DUMMY) { atomicAdd(&cnt[1], 1); atomicMin(&cnt[2], u); }
}
__global__ void k_finalise(int n, int* __restrict__ st, int dmin, int* __restrict__ rep) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  if (st[u] == ST_UNDECIDED) st[u] = ST_SEED;
  rep[u] = (st[u] == ST_SEED || u == dmin) ? 1 : 0;
}
__global__ void k_number(int n, const int* __restrict__ st, const int* __restrict__ seedof, const int* __restrict__ id,
                         int dmin, int* __restrict__ agg) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const int x = st[u];
  agg[u] = x == ST_SEED ? id[u] : (x == ST_ASSOC ? id[seedof[u]] : id[dmin]);
}
// Galerkin P^T A P (eq. galerkin): inter-aggregate fine edges, listed by fine
// row and column order.
__global__ void k_gal_counts(int n, const int* __restrict__ rp, const int* __restrict__ ci, const int* __restrict__ agg,
                             int* __restrict__ cnt) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  int c = 0;
  const int a = agg[u];
  for (int t = rp[u]; t < rp[u + 1]; ++t) c += agg[ci[t]] != a;
  cnt[u] = c;
}
__global__ void k_gal_emit(int n, uint64_t nc, const int* __restrict__ rp, const int* __restrict__ ci,
                           const double* __restrict__ val, const int* __restrict__ agg, const int* __restrict__ off,
                           uint64_t* __restrict__ key, double* __restrict__ v) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const int a = agg[u];
  int o = off[u];
  for (int t = rp[u]; t < rp[u + 1]; ++t) {
    const int b = agg[ci[t]];
    if (b == a) continue;
    key[o] = (uint64_t)a * nc + (uint64_t)b;
    v[o] = val[t];
    ++o;
  }
}
__global__ void k_map(int n, const int* __restrict__ a, const int* __restrict__ inv, int* __restrict__ out) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n) out[u] = inv[a[u]];
}
__global__ void k_copy_u8(int64_t n, const int* __restrict__ a, uint8_t* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (uint8_t)a[i];
}
}  // namespace

// Energies x_k^T A x_k (up to a factor 2) of the K test vectors.
static std::vector<double> tv_energies(Hierarchy* H, Tmp& tmp, const Level& F, int K) {
  hipStream_t s = H->s;
  double* e = tmp.get<double>((size_t)F.n * K);
  double* out = tmp.get<double>(K);
  hipLaunchKernelGGL(k_energy_short, grid1(F.n), dim3(256), 0, s, F.n, K, F.rp, F.ci, F.val, F.tv, e);
  if (F.all.nlong)
    hipLaunchKernelGGL(k_energy_long, grid1((int64_t)F.all.nlong * 64), dim3(256), 0, s, F.all.longrows, F.all.nlong,
                       K, F.rp, F.ci, F.val, F.tv, e);
  hipLaunchKernelGGL(k_colsum, dim3(K), dim3(256), 0, s, F.n, K, e, out);
  LAMG_HIP(hipGetLastError());
  return to_host_vec(s, out, (size_t)K);
}

static int galerkin_level(Hierarchy* H, Tmp& tmp, int l, const int* aggn, int nc, int rb_side);

int aggregate(Hierarchy* H, int l, int agg_index) {
  hipStream_t s = H->s;
  Tmp tmp;
  Level& F = H->lv[l];
  const int n = F.n;
  const int K = std::min(H->o.tv_k_max, H->o.tv_k_min + 2 * agg_index);
  F.K = K;
  // test vectors: U[-1,1) then tv_sweeps GS sweeps on A x = 0 (Section 3.3.1)
  F.tv = dnew<double>(H, (size_t)n * K);
  hipLaunchKernelGGL(k_tv_init, grid1((int64_t)n * K), dim3(256), 0, s, n, K, (uint64_t)H->o.seed, (uint64_t)l, F.tv);
  for (int sw = 0; sw + 1 < H->o.tv_sweeps; ++sw) gs_multi_sweep(s, F, nullptr, F.tv, K);
  // Section 4.1: stop coarsening when relaxation converges rapidly, judged by
  // the energy reduction of the last test-vector sweep.
  {
    const std::vector<double> E0 = tv_energies(H, tmp, F, K);
    if (H->o.tv_sweeps > 0) gs_multi_sweep(s, F, nullptr, F.tv, K);
    const std::vector<double> E1 = tv_energies(H, tmp, F, K);
    double rate = 0;
    for (int k = 0; k < K; ++k) rate = std::max(rate, E0[k] > 0 ? E1[k] / E0[k] : 0.0);
    F.rate = rate;
    if (H->o.tv_sweeps > 0 && rate <= H->o.relax_fast_ratio) return 2;
  }
  int* deg = tmp.get<int>(n);
  hipLaunchKernelGGL(k_degrees, grid1(n), dim3(256), 0, s, n, F.rp, deg);
  NodeOut o;
  o.nrm = tmp.get<double>(n);
  o.ystar = tmp.get<double>((size_t)n * K);
  o.emin = tmp.get<double>((size_t)n * K);
  o.sw = tmp.get<double>(n);
  o.swd = tmp.get<double>(n);
  o.maxw = tmp.get<double>(n);
  // Section 5.2: on a level with a negative weight the hub, affinity and
  // energy tests use |w| (the Laplacian of the absolute weights, diagonal in
  // the fixed row order); other levels use their own matrix
  const double* tval = F.val;
  const double* tdiag = F.diag;
  if (H->o.allow_negative_weights && F.nnz > 0) {
    int* nneg = tmp.get<int>(1);
    LAMG_HIP(hipMemsetAsync(nneg, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_count_negative, grid1(F.nnz), dim3(256), 0, s, (int64_t)F.nnz, (const double*)F.val, nneg);
    if (to_host(s, nneg) > 0) {
      double* av = tmp.get<double>(F.nnz);
      double* ad = tmp.get<double>(n);
      hipLaunchKernelGGL(k_abs, grid1(F.nnz), dim3(256), 0, s, (int64_t)F.nnz, (const double*)F.val, av);
      row_sums(s, tmp, n, F.rp, av, ad);
      tval = av;
      tdiag = ad;
    }
  }
  hipLaunchKernelGGL(k_node_short, grid1(n), dim3(256), 0, s, n, K, F.rp, F.ci, tval, tdiag, deg, F.tv, o);
  if (F.all.nlong)
    hipLaunchKernelGGL(k_node_long, grid1((int64_t)F.all.nlong * 64), dim3(256), 0, s, F.all.longrows, F.all.nlong, K,
                       F.rp, F.ci, tval, tdiag, deg, F.tv, o);
  const int64_t E2 = F.nnz;
  F.aff = dnew<double>(H, E2);
  F.ok = dnew<uint8_t>(H, E2);
  F.weak = dnew<uint8_t>(H, E2);
  F.hub = dnew<uint8_t>(H, n);
  F.state = dnew<int>(H, n);
  const double qfac = 2.0 * (H->o.q_max - 1.0);
  hipLaunchKernelGGL(k_edges, grid1(n), dim3(256), 0, s, n, K, F.rp, F.ci, tval, tdiag, F.tv, o, qfac,
                     H->o.weak_edge_ratio, F.aff, F.ok, F.weak);
  int* st = F.state;
  int* seedof = tmp.get<int>(n);
  hipLaunchKernelGGL(k_init_state, grid1(n), dim3(256), 0, s, n, F.rp, deg, o, H->o.hub_factor, F.weak, st, F.hub,
                     seedof);
  // stage-1 threshold: quantile of the best candidate affinities
  double* best = tmp.get<double>(n);
  double* bsorted = tmp.get<double>(n);
  int* cnt = tmp.get<int>(4);
  LAMG_HIP(hipMemsetAsync(cnt, 0, 4 * sizeof(int), s));
  hipLaunchKernelGGL(k_best, grid1(n), dim3(256), 0, s, n, F.rp, F.ci, st, F.weak, F.ok, F.aff, best, cnt);
  sort_keys_double(s, tmp, (const double*)best, bsorted, n);
  const int nbest = to_host(s, cnt);
  double delta1 = 1.0;
  if (nbest > 0) {
    const size_t idx = (size_t)((double)(nbest - 1) * H->o.stage1_quantile);
    delta1 = to_host(s, bsorted + idx);
  }
  F.delta1 = delta1;
  const double amax = 0.7 / H->o.gamma;
  int dmin = -1;
  auto run_stage = [&](double delta) {
    for (int c = 0; c < F.ncol; ++c) {
      const int r0 = F.cptr[c], r1 = F.cptr[c + 1];
      if (r1 > r0)
        hipLaunchKernelGGL(k_agg_colour, grid1(r1 - r0), dim3(256), 0, s, r0, r1, F.rp, F.ci, st, seedof, F.weak, F.ok,
                           F.aff, delta);
    }
    int h0[3] = {0, 0, 0x7fffffff};
    LAMG_HIP(hipMemcpyAsync(cnt, h0, 3 * sizeof(int), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_count_states, grid1(n), dim3(256), 0, s, n, st, cnt);
    int h1[3];
    LAMG_HIP(hipMemcpyAsync(h1, cnt, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
    LAMG_HIP(hipStreamSynchronize(s));
    dmin = h1[1] > 0 ? h1[2] : -1;
    return (double)(h1[0] + (h1[1] > 0 ? 1 : 0)) / (double)n;
  };
  F.alpha1 = run_stage(delta1);
  F.stage = 1;
  F.alpha2 = -1;
  if (F.alpha1 > amax) {
    int* st1 = tmp.get<int>(n);
    int* so1 = tmp.get<int>(n);
    LAMG_HIP(hipMemcpyAsync(st1, st, (size_t)n * sizeof(int), hipMemcpyDeviceToDevice, s));
    LAMG_HIP(hipMemcpyAsync(so1, seedof, (size_t)n * sizeof(int), hipMemcpyDeviceToDevice, s));
    const int dmin1 = dmin;
    F.alpha2 = run_stage(1.0);
    if (std::fabs(F.alpha1 - amax) <= std::fabs(F.alpha2 - amax)) {
      LAMG_HIP(hipMemcpyAsync(st, st1, (size_t)n * sizeof(int), hipMemcpyDeviceToDevice, s));
      LAMG_HIP(hipMemcpyAsync(seedof, so1, (size_t)n * sizeof(int), hipMemcpyDeviceToDevice, s));
      dmin = dmin1;
      F.stage = 1;
    } else {
      F.stage = 2;
    }
  }
  int* rep = tmp.get<int>(n + 1);
  int* id = tmp.get<int>(n + 1);
  hipLaunchKernelGGL(k_finalise, grid1(n), dim3(256), 0, s, n, st, dmin, rep);
  excl_scan(s, tmp, rep, id, n);
  const int nc = to_host(s, id + n);
  if (nc >= n) return 0;  // no coarsening possible
  int* aggn = tmp.get<int>(n);
  hipLaunchKernelGGL(k_number, grid1(n), dim3(256), 0, s, n, st, seedof, id, dmin, aggn);
  return galerkin_level(H, tmp, l, aggn, nc, 0);
}

// The coarse level of aggregation aggn (fine node in level l's order ->
// aggregate 0..nc-1): Galerkin operator, colouring and order (red-black of
// an rb_side grid if rb_side > 0), transfer maps.  Returns 1.
static int galerkin_level(Hierarchy* H, Tmp& tmp, int l, const int* aggn, int nc, int rb_side) {
  hipStream_t s = H->s;
  const Level& F = H->lv[l];
  const int n = F.n;
  // Galerkin coarse operator
  int* gcnt = tmp.get<int>(n + 1);
  int* goff = tmp.get<int>(n + 1);
  hipLaunchKernelGGL(k_gal_counts, grid1(n), dim3(256), 0, s, n, F.rp, F.ci, aggn, gcnt);
  excl_scan(s, tmp, gcnt, goff, n);
  const int nt = to_host(s, goff + n);
  uint64_t* key = tmp.get<uint64_t>(nt);
  double* v = tmp.get<double>(nt);
  hipLaunchKernelGGL(k_gal_emit, grid1(n), dim3(256), 0, s, n, (uint64_t)nc, F.rp, F.ci, F.val, aggn, goff, key, v);
  Level C;
  C.type = LT_AGG;
  merge_triples(H, tmp, C, nc, key, v, nt);
  int* cinv = colour_order_impl(H, tmp, C, l + 1, rb_side);
  C.agg = dnew<int>(H, n);
  hipLaunchKernelGGL(k_map, grid1(n), dim3(256), 0, s, n, aggn, cinv, C.agg);
  // P^T as CSR: members of each aggregate in ascending fine id
  int* ids = tmp.get<int>(n);
  int* ks = tmp.get<int>(n);
  C.members = dnew<int>(H, n);
  hipLaunchKernelGGL(k_iota, grid1(n), dim3(256), 0, s, ids, n);
  sort_pairs(s, tmp, (const unsigned*)C.agg, (unsigned*)ks, (const int*)ids, C.members, n, bits_for((uint64_t)nc));
  int* acnt = tmp.get<int>(nc + 1);
  hipLaunchKernelGGL(k_zero_i, grid1(nc + 1), dim3(256), 0, s, acnt, (int64_t)nc + 1);
  hipLaunchKernelGGL(k_count_colours, grid1(n), dim3(256), 0, s, n, C.agg, acnt);
  C.agg_ptr = dnew<int>(H, (size_t)nc + 1);
  excl_scan(s, tmp, acnt, C.agg_ptr, nc);
  LAMG_HIP(hipStreamSynchronize(s));
  H->lv.push_back(C);
  return 1;
}

// ------------------------------------------------ lean geometric multigrid
// Section 5.3: the periodic Poisson problem on a side x side grid (unit
// weights, node (i, j) = i + side j), coarsened 1:2 in each dimension at
// every level: fine node (i, j) joins aggregate (i / 2, j / 2), numbered
// i / 2 + (side / 2)(j / 2), and every level is coloured red-black.
namespace {
__global__ void k_lgm_edges(int side, int32_t* __restrict__ eu, int32_t* __restrict__ ev, double* __restrict__ w) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)side * side;
  if (k >= 2 * n) return;
  const int u = (int)(k >> 1), i = u % side, j = u / side;
  eu[k] = u;
  ev[k] = (k & 1) ? i + side * ((j + 1) % side) : (i + 1) % side + side * j;  // up : right
  w[k] = 1.0;
}
__global__ void k_lgm_agg(int n, int side, const int* __restrict__ perm, int* __restrict__ agg) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const int v = perm[u];
  agg[u] = (v % side) / 2 + (side / 2) * ((v / side) / 2);
}
}  // namespace

lamg_status build_lgm_finest(Hierarchy* H, int side) {
  Tmp tmp;
  const int64_t n = (int64_t)side * side, m = 2 * n;
  int32_t* eu = tmp.get<int32_t>(m);
  int32_t* ev = tmp.get<int32_t>(m);
  double* w = tmp.get<double>(m);
  hipLaunchKernelGGL(k_lgm_edges, grid1(m), dim3(256), 0, H->s, side, eu, ev, w);
  LAMG_HIP(hipGetLastError());
  const lamg_status st = build_finest(H, n, m, eu, ev, w);
  if (st != LAMG_OK) return st;
  colour_order_impl(H, tmp, H->lv[0], 0, side);
  return LAMG_OK;
}

void lgm_coarsen(Hierarchy* H, int l, int side) {
  Tmp tmp;
  const int n = H->lv[l].n;
  int* agg = tmp.get<int>(n);
  hipLaunchKernelGGL(k_lgm_agg, grid1(n), dim3(256), 0, H->s, n, side, (const int*)H->lv[l].perm, agg);
  LAMG_HIP(hipGetLastError());
  galerkin_level(H, tmp, l, agg, (side / 2) * (side / 2), side / 2);
}

// Cycle indices (Section 4.2, eq. cycle_index with gamma^l >= 1), FP32 level
// copies, work vectors and the coarsest factor.
namespace {
__global__ void k_to_f32(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}
// Hub rows [r0, r0 + nh): entries into the hub rows themselves.  Columns are
// sorted within a row and hub ids are the largest, so they are each row's
// suffix; the count is found by bisection.
__global__ void k_hub_count(int nh, int r0, const int* __restrict__ rp, const int* __restrict__ ci,
                            int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nh) return;
  const int end = rp[r0 + i + 1];
  int lo = rp[r0 + i], hi = end;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (ci[mid] < r0) lo = mid + 1;
    else hi = mid;
  }
  cnt[i] = end - lo;
}
// One wavefront per hub row copies its suffix with local column ids.
__global__ void k_hub_fill(int nh, int r0, const int* __restrict__ rp, const int* __restrict__ ci,
                           const double* __restrict__ val, const float* __restrict__ val32,
                           const int* __restrict__ hrp, int* __restrict__ hci, double* __restrict__ hv,
                           float* __restrict__ hv32) {
  const int i = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6), lane = threadIdx.x & 63;
  if (i >= nh) return;
  const int dst = hrp[i], len = hrp[i + 1] - dst;
  const int src = rp[r0 + i + 1] - len;
  for (int j = lane; j < len; j += 64) {
    hci[dst + j] = ci[src + j] - r0;
    hv[dst + j] = val[src + j];
    hv32[dst + j] = val32[src + j];
  }
}
}  // namespace

// Chunks of whole rows of one colour, at most HUB_CHUNK hub-to-hub entries
// each, over the hub colours [K, nc); hr: hub row pointers (local rows from
// the first hub row).  Returns the chunk count; appends the chunks if out.
static int hub_chunks(const Level& L, int K, int r0, const std::vector<int>& hr, std::vector<int2>* out) {
  int count = 0;
  for (int c = K; c < L.ncol; ++c) {
    const int a = L.cptr[c] - r0, z = L.cptr[c + 1] - r0;
    int first = a;
    for (int u = a; u < z; ++u)
      if (hr[u + 1] - hr[first] > HUB_CHUNK) {
        if (out) out->push_back(make_int2(first, u));
        ++count;
        first = u;
      }
    if (out) out->push_back(make_int2(first, z));
    ++count;
  }
  return count;
}

void build_hub(Hierarchy* H, Level& L) {
  L.hub_k = -1;
  const int n = L.n, nc = L.ncol;
  if (n <= HUB_MAX_ROWS || nc < HUB_MIN_COLOURS || (int)L.cptr.size() != nc + 1) return;
  // K0: the smallest K >= 1 whose colours >= K hold at most HUB_MAX_ROWS rows
  int K0 = nc;
  for (int c = nc - 1; c >= 1; --c) {
    if (n - L.cptr[c] > HUB_MAX_ROWS) break;
    K0 = c;
  }
  if (nc - K0 < HUB_MIN_COLOURS) return;
  hipStream_t s = H->s;
  Tmp tmp;
  // hub-to-hub columns of the rows >= cptr[K0] (a later split keeps a suffix
  // of each row), to price every admissible split on the host
  auto count_fill = [&](int r0, int nh, int* hrp, int** hci_out, int* hnnz_out) {
    int* cnt = tmp.get<int>(nh + 1);
    hipLaunchKernelGGL(k_hub_count, grid1(nh), dim3(256), 0, s, nh, r0, (const int*)L.rp, (const int*)L.ci, cnt);
    excl_scan(s, tmp, cnt, hrp, nh);
    *hnnz_out = to_host(s, hrp + nh);
    *hci_out = tmp.get<int>(std::max(*hnnz_out, 1));
  };
  int K = K0;
  {
    const int r0 = L.cptr[K0], nh = n - r0;
    int* hrp0 = tmp.get<int>(nh + 1);
    int* hci0 = nullptr;
    int hnnz0 = 0;
    count_fill(r0, nh, hrp0, &hci0, &hnnz0);
    double* hv0 = tmp.get<double>(std::max(hnnz0, 1));
    float* hv32_0 = tmp.get<float>(std::max(hnnz0, 1));
    hipLaunchKernelGGL(k_hub_fill, dim3((unsigned)(((int64_t)nh * 64 + 255) / 256)), dim3(256), 0, s, nh, r0,
                       (const int*)L.rp, (const int*)L.ci, (const double*)L.val, (const float*)L.val32,
                       (const int*)hrp0, hci0, hv0, hv32_0);
    std::vector<int> hr0(nh + 1), hc0(std::max(hnnz0, 1));
    LAMG_HIP(hipMemcpyAsync(hr0.data(), hrp0, (size_t)(nh + 1) * sizeof(int), hipMemcpyDeviceToHost, s));
    LAMG_HIP(hipMemcpyAsync(hc0.data(), hci0, (size_t)std::max(hnnz0, 1) * sizeof(int), hipMemcpyDeviceToHost, s));
    LAMG_HIP(hipStreamSynchronize(s));
    // cost of split K2: its extra launched colours plus the chunks of the
    // hub sweep (hub rows' columns are sorted: the entries into colours
    // >= K2 are each row's suffix)
    int64_t best = -1;
    std::vector<int> hr2;
    for (int K2 = K0; nc - K2 >= HUB_MIN_COLOURS; ++K2) {
      const int d = L.cptr[K2] - r0, nh2 = nh - d;
      hr2.assign(nh2 + 1, 0);
      for (int u = 0; u < nh2; ++u) {
        const int* b0 = hc0.data() + hr0[d + u];
        const int* b1 = hc0.data() + hr0[d + u + 1];
        hr2[u + 1] = hr2[u] + (int)(b1 - std::lower_bound(b0, b1, d));
      }
      const int64_t cost = (int64_t)(K2 - K0) * HUB_COST_LAUNCH +
                           (int64_t)hub_chunks(L, K2, L.cptr[K2], hr2, nullptr) * HUB_COST_CHUNK;
      if (best < 0 || cost < best) {
        best = cost;
        K = K2;
      }
    }
  }
  const int r0 = L.cptr[K], nh = n - r0;
  int* hrp = dnew<int>(H, (size_t)nh + 1);
  int* cnt = tmp.get<int>(nh + 1);
  hipLaunchKernelGGL(k_hub_count, grid1(nh), dim3(256), 0, s, nh, r0, (const int*)L.rp, (const int*)L.ci, cnt);
  excl_scan(s, tmp, cnt, hrp, nh);
  const int hnnz = to_host(s, hrp + nh);
  int* hci = dnew<int>(H, std::max(hnnz, 1));
  double* hv = dnew<double>(H, std::max(hnnz, 1));
  float* hv32 = dnew<float>(H, std::max(hnnz, 1));
  hipLaunchKernelGGL(k_hub_fill, dim3((unsigned)(((int64_t)nh * 64 + 255) / 256)), dim3(256), 0, s, nh, r0,
                     (const int*)L.rp, (const int*)L.ci, (const double*)L.val, (const float*)L.val32, (const int*)hrp,
                     hci, hv, hv32);
  std::vector<int> hr(nh + 1);
  LAMG_HIP(hipMemcpyAsync(hr.data(), hrp, (size_t)(nh + 1) * sizeof(int), hipMemcpyDeviceToHost, s));
  LAMG_HIP(hipStreamSynchronize(s));
  std::vector<int2> ck;
  hub_chunks(L, K, r0, hr, &ck);
  if ((int)ck.size() > HUB_MAX_CHUNKS) return;  // (the device arrays stay with the handle, unused)
  L.hub_ck = dnew<int2>(H, ck.size());
  LAMG_HIP(hipMemcpyAsync(L.hub_ck, ck.data(), ck.size() * sizeof(int2), hipMemcpyHostToDevice, s));
  L.hub_nck = (int)ck.size();
  const int low0 = to_host(s, L.rp + r0);
  L.hub_low_nnz = (int64_t)L.nnz - low0 - hnnz;
  L.hub_p = dnew<double>(H, nh);
  L.hub_p32 = dnew<float>(H, nh);
  L.hub_rp = hrp;
  L.hub_ci = hci;
  L.hub_val = hv;
  L.hub_val32 = hv32;
  L.hub_r0 = r0;
  L.hub_n = nh;
  L.hub_nnz = hnnz;
  LAMG_HIP(hipStreamSynchronize(s));  // ck leaves scope
  L.hub_k = K;
}

void finish_levels(Hierarchy* H) {
  hipStream_t s = H->s;
  const double E1 = (double)H->lv[0].nnz;
  for (size_t l = 0; l + 1 < H->lv.size(); ++l) {
    Level& F = H->lv[l];
    const Level& C = H->lv[l + 1];
    if (C.type == LT_ELIM) { F.gamma_next = 1.0; continue; }
    if (H->gamma_every_level) { F.gamma_next = H->o.gamma; continue; }
    const double El = (double)F.nnz, Ec = (double)C.nnz;
    if (El > 0.1 * E1) F.gamma_next = H->o.gamma;
    else if (Ec <= 0) F.gamma_next = 1.0;
    else F.gamma_next = std::max(1.0, std::min(2.0, 0.7 * El / Ec));
  }
  for (Level& L : H->lv) {
    L.val32 = dnew<float>(H, std::max(L.nnz, 1));
    L.diag32 = dnew<float>(H, L.n);
    if (L.nnz) hipLaunchKernelGGL(k_to_f32, grid1(L.nnz), dim3(256), 0, s, (int64_t)L.nnz, L.val, L.val32);
    hipLaunchKernelGGL(k_to_f32, grid1(L.n), dim3(256), 0, s, (int64_t)L.n, L.diag, L.diag32);
    auto mk64 = [&](Vecs<double>& v) {
      v.x = dnew<double>(H, L.n); v.b = dnew<double>(H, L.n); v.r = dnew<double>(H, L.n);
      for (int i = 0; i < 2; ++i) { v.X[i] = dnew<double>(H, L.n); v.R[i] = dnew<double>(H, L.n); }
    };
    auto mk32 = [&](Vecs<float>& v) {
      v.x = dnew<float>(H, L.n); v.b = dnew<float>(H, L.n); v.r = dnew<float>(H, L.n);
      for (int i = 0; i < 2; ++i) { v.X[i] = dnew<float>(H, L.n); v.R[i] = dnew<float>(H, L.n); }
    };
    mk64(L.v64);
    mk32(L.v32);
    build_hub(H, L);
  }
  if (H->lv.back().n > H->o.dense_max) H->coarsest_relax = true;
  if (!H->coarsest_relax) coarsest_factor(H, H->lv.back());
  else H->nL = H->lv.back().n;
  H->red = dnew<double>(H, k::RED_BLOCKS * 8 + 16);
  LAMG_HIP(hipHostMalloc((void**)&H->hred, 64 * sizeof(double), hipHostMallocDefault));
  LAMG_HIP(hipStreamSynchronize(s));
}

}  // namespace lamg
