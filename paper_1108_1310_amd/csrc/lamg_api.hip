// Cycle driver (Section 4.2), FP64 and FP32-with-FP64-refinement solve loops,
// batched solves and the C ABI.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "lamg_device.hpp"
#include "lamg_internal.hpp"

namespace lamg {

namespace {
template <class T> struct Prec;
template <> struct Prec<double> {
  static Vecs<double>& v(Level& L) { return L.v64; }
  static const double* val(const Level& L) { return L.val; }
  static const double* diag(const Level& L) { return L.diag; }
};
template <> struct Prec<float> {
  static Vecs<float>& v(Level& L) { return L.v32; }
  static const float* val(const Level& L) { return L.val32; }
  static const float* diag(const Level& L) { return L.diag32; }
};

inline dim3 grid1(int64_t n, int b = 256) { return dim3((unsigned)std::max<int64_t>(1, (n + b - 1) / b)); }

template <class T>
__global__ void k_copy(int n, const T* __restrict__ a, T* __restrict__ b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}
// b_perm[i] = b[perm[i]] - mean, mean taken from the reduction slot
__global__ void k_gather_sub(int n, const int* __restrict__ perm, const double* __restrict__ b,
                             const double* __restrict__ res, int slot, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = b[perm[i]] - (res ? res[slot] : 0.0);
}
__global__ void k_scatter(int n, const int* __restrict__ perm, const double* __restrict__ a, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[perm[i]] = a[i];
}
__global__ void k_sub_to_f32(int n, const double* __restrict__ r, const double* __restrict__ res, int slot,
                             float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)(r[i] - res[slot]);
}
__global__ void k_add_f32(int n, const float* __restrict__ e, double* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += (double)e[i];
}
// mean of a device vector into reduction slot `slot` (device side only)
void mean_to_slot(hipStream_t s, Hierarchy* H, const double* x, int n, int slot) {
  sum_to_slot(s, H, x, n, slot, (double)n);
}
double* res_slots(Hierarchy* H) { return H->red + k::RED_BLOCKS * 8; }

// ------------------------------------------------------------------- cycle
template <class T>
void visit(Hierarchy* H, int l, int th, std::vector<int64_t>& count);

template <class T>
void body(Hierarchy* H, int l, int sub, std::vector<int64_t>& count) {
  hipStream_t s = H->s;
  const int Lc = (int)H->lv.size() - 1;
  Level& L = H->lv[l];
  Vecs<T>& v = Prec<T>::v(L);
  if (l == Lc) {
    if (H->coarsest_relax) {  // relaxation converges rapidly on this level
      // below the finest level a visit starts from the zero fill of its caller
      for (int i = 0; i < H->o.coarsest_sweeps; ++i)
        gs_sweep<T>(s, L, Prec<T>::val(L), Prec<T>::diag(L), v.b, v.x, l > 0 && i == 0);
      return;
    }
    if constexpr (sizeof(T) == 8) coarsest_solve(s, H, (const double*)v.b, (double*)v.x);
    else coarsest_solve32(s, H, (const float*)v.b, (float*)v.x);
    return;
  }
  Level& C = H->lv[l + 1];
  Vecs<T>& vc = Prec<T>::v(C);
  const T* val = Prec<T>::val(L);
  const T* dg = Prec<T>::diag(L);
  if (C.type == LT_ELIM) {
    const T* r = v.r;
    if (l == 0 && H->top_res_known) r = sizeof(T) == 8 ? (const T*)H->r64 : v.b;
    else residual<T>(s, L, val, dg, v.b, v.x, v.r);
    restrict_elim<T>(s, C, r, vc.b);
    fill<T>(s, vc.x, T(0), C.n);
    visit<T>(H, l + 1, 1, count);
    interp_elim<T>(s, L, C, val, dg, r, vc.x, v.x);
    return;
  }
  const bool rec = H->o.ec == LAMG_EC_RECOMBINE;
  for (int i = 0; i < H->o.nu_pre; ++i) gs_sweep<T>(s, L, val, dg, v.b, v.x, l > 0 && sub == 0 && i == 0);
  T* r = rec ? v.R[sub] : v.r;
  residual<T>(s, L, val, dg, v.b, v.x, r);
  if (rec) hipLaunchKernelGGL(k_copy<T>, grid1(L.n), dim3(256), 0, s, L.n, (const T*)v.x, v.X[sub]);
  const T mu = rec ? T(1) : (T)H->o.mu;
  restrict_agg<T>(s, C, L.n, r, vc.b, mu);
  fill<T>(s, vc.x, T(0), C.n);
  const int64_t c = count[l]++;
  const double gl = L.gamma_next;
  const int th = (int)(std::ceil((double)(c + 1) * gl) - std::ceil((double)c * gl));
  visit<T>(H, l + 1, th, count);
  interp_agg<T>(s, C, L.n, vc.x, v.x);
  for (int i = 0; i < H->o.nu_post; ++i) gs_sweep<T>(s, L, val, dg, v.b, v.x);
}

template <class T>
void visit(Hierarchy* H, int l, int th, std::vector<int64_t>& count) {
  const int Lc = (int)H->lv.size() - 1;
  if (l == H->tail_lc) { tail_run_next<T>(H); return; }  // this entry's program segment
  if (l == Lc) { body<T>(H, l, 0, count); return; }
  for (int i = 0; i < th; ++i) body<T>(H, l, i, count);
  if (H->o.ec == LAMG_EC_RECOMBINE && H->lv[l + 1].type == LT_AGG)
    recombine<T>(H->s, H, H->lv[l], Prec<T>::v(H->lv[l]), th);
}
}  // namespace

template <class T>
void cycle(Hierarchy* H, bool top_res_known) {
  tail_prepare(H);
  H->tail_cursor = 0;
  std::vector<int64_t> count(H->lv.size(), 0);
  H->top_res_known = top_res_known;
  try {
    visit<T>(H, 0, 1, count);
  } catch (...) {
    H->top_res_known = false;
    throw;
  }
  H->top_res_known = false;
  Level& L = H->lv[0];
  if (H->tail_lc != 0) subtract_mean<T>(H->s, H, Prec<T>::v(L).x, L.n);  // else in the tail program
  LAMG_HIP(hipGetLastError());
}
template void cycle<double>(Hierarchy*, bool);
template void cycle<float>(Hierarchy*, bool);

// The kernel sequence of a cycle depends only on the hierarchy and the solve
// options, so it is captured once into a graph and replayed.  The replays
// serve the single-vector solve loop, which enters every cycle with the
// finest residual known (FP64: r64 from the stopping test; FP32: x = 0, so
// the residual is b), so the recorded cycle does not recompute it.  Capture runs on
// the hierarchy's private stream; replays go to the caller's stream.  With
// instrumentation on, the cycle is launched eagerly instead.
template <class T>
void cycle_graph(Hierarchy* H, int inst) {
  if (prof_on()) { cycle<T>(H, true); return; }
  const int p = sizeof(T) == 8 ? 0 : 1;
  tail_prepare(H);  // uploads with synchronous copies: before any capture
  if (!H->gexec[p][inst]) {
    if (!H->cs) LAMG_HIP(hipStreamCreateWithFlags(&H->cs, hipStreamNonBlocking));
    hipStream_t user = H->s;
    H->s = H->cs;
    hipGraph_t g = nullptr;
    LAMG_HIP(hipStreamBeginCapture(H->cs, hipStreamCaptureModeThreadLocal));
    try {
      cycle<T>(H, true);
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
    H->gexec[p][inst] = ex;
  }
  LAMG_HIP(hipGraphLaunch(H->gexec[p][inst], H->s));
}
template void cycle_graph<double>(Hierarchy*, int);
template void cycle_graph<float>(Hierarchy*, int);

void drop_graphs(Hierarchy* H) {
  for (int p = 0; p < 2; ++p)
    for (int i = 0; i < 2; ++i) {
      if (H->gexec[p][i]) (void)hipGraphExecDestroy(H->gexec[p][i]);
      H->gexec[p][i] = nullptr;
    }
}

namespace {
thread_local char g_last_error[512] = "";
thread_local char g_error_detail[256] = "";
}
void set_error_detail(const char* msg) { std::snprintf(g_error_detail, sizeof(g_error_detail), "%s", msg); }
void set_last_error(const char* where, hipError_t e) {
  std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%d)%s%s", where, hipGetErrorString(e), (int)e,
                g_error_detail[0] ? ": " : "", g_error_detail);
  g_error_detail[0] = 0;
}
void set_last_error_msg(const char* msg) { std::snprintf(g_last_error, sizeof(g_last_error), "%s", msg); }

// Algorithmic bytes of one cycle on k right-hand sides: the matrix streams of
// every pass once, its vector streams k times.
int64_t cycle_bytes_k(const Hierarchy* H, int prec, int k) {
  const int64_t sv = prec == LAMG_FP64 ? 8 : 4, sx = sv * k;
  const size_t nl = H->lv.size();
  std::vector<int64_t> bodies(nl, 0), ctr(nl, 0), visits(nl, 0);
  std::vector<int> ths;
  // replay the schedule
  std::vector<std::pair<int, int>> stack;
  struct F { static void run(const Hierarchy* H, int l, int th, std::vector<int64_t>& b, std::vector<int64_t>& c,
                             std::vector<int64_t>& vis, std::vector<int64_t>& recth) {
    const int Lc = (int)H->lv.size() - 1;
    vis[l] += 1;
    if (l == Lc) { b[l] += 1; return; }
    for (int i = 0; i < th; ++i) {
      b[l] += 1;
      if (H->lv[l + 1].type == LT_ELIM) { run(H, l + 1, 1, b, c, vis, recth); continue; }
      const int64_t k = c[l]++;
      const double g = H->lv[l].gamma_next;
      run(H, l + 1, (int)(std::ceil((double)(k + 1) * g) - std::ceil((double)k * g)), b, c, vis, recth);
    }
    if (H->lv[l + 1].type == LT_AGG) recth[l] += th;
  } };
  std::vector<int64_t> recth(nl, 0);
  F::run(H, 0, 1, bodies, ctr, visits, recth);
  int64_t tot = 0;
  for (size_t l = 0; l < nl; ++l) {
    const Level& L = H->lv[l];
    const int64_t n = L.n;
    const int64_t M = (int64_t)L.nnz * (4 + sv) + n * (4 + sv);
    if (l + 1 == nl) {
      if (H->coarsest_relax) tot += bodies[l] * H->o.coarsest_sweeps * (M + 3 * n * sx);
      else tot += bodies[l] * ((int64_t)H->nL * H->nL * 8 + 2 * n * sx);
      continue;
    }
    const Level& C = H->lv[l + 1];
    int64_t body;
    if (C.type == LT_ELIM) {
      body = (M + 3 * n * sx)                               // residual
             + (M + 2 * n * sx)                             // restriction (rows of C nodes)
             + (M + 3 * n * sx);                            // exact correction
    } else {
      const int sweeps = H->o.nu_pre + H->o.nu_post;
      body = sweeps * (M + 3 * n * sx) + (M + 3 * n * sx)   // relaxation, residual
             + n * (sx + 4) + (int64_t)C.n * (sx + 4)         // restriction
             + n * (4 + 2 * sx) + (int64_t)C.n * sx;          // interpolation
      if (H->o.ec == LAMG_EC_RECOMBINE) body += 2 * n * sx;   // saved iterate
    }
    tot += bodies[l] * body;
    if (H->o.ec == LAMG_EC_RECOMBINE && C.type == LT_AGG) {
      // per visit: final residual, Gram (residuals: th+1 vectors; energy
      // norm: iterates too, 2 (th+1)), update (th+2 vectors)
      const int64_t th = visits[l] ? (recth[l] + visits[l] - 1) / visits[l] : 1;
      const int64_t gram = (H->o.recomb_norm == LAMG_RECOMB_ENERGY ? 2 : 1) * (th + 1);
      tot += visits[l] * ((M + 3 * n * sx) + gram * n * sx + (th + 2) * n * sx);
    }
  }
  tot += 2 * (int64_t)H->lv[0].n * sx;  // mean removal
  return tot;
}
int64_t cycle_bytes(const Hierarchy* H, int prec) { return cycle_bytes_k(H, prec, 1); }

}  // namespace lamg

// ====================================================================== C ABI
using namespace lamg;


extern "C" {

void lamg_options_default(lamg_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(lamg_options);
  o->gamma = 1.5;
  o->nu_pre = 1;
  o->nu_post = 2;
  o->tv_k_min = 4;
  o->tv_k_max = 10;
  o->tv_sweeps = 3;
  o->q_max = 2.5;
  o->mu = 4.0 / 3.0;
  o->hub_factor = 8.0;
  o->elim_max_degree = 4;
  o->coarsest_max_n = 150;
  o->weak_edge_ratio = 1e-3;
  o->elim_stop_frac = 0.05;
  o->stage1_quantile = 1.0;
  o->relax_fast_ratio = 0.1;
  o->coarsest_sweeps = 3;
  o->dense_max = 8192;
  // measured 2048 / 3072 / 4096 (ms per solve; FP64, FP32): RGG 2^20 153.1 /
  // 152.5 / 158.8, 138.4 / 135.6 / 136.7; 64^3 grid 461 / 470 / 469, 432 / 428 /
  // 427; geometric multigrid 1024^2 6.75 / 6.78 / 7.64, 6.48 / 6.49 / 7.28;
  // 64^2 grid at 3072 / 4096: 4.89 / 5.07, 4.98 / 5.10
  o->tail_max_n = 3072;
  o->ec = LAMG_EC_RECOMBINE;
  o->precision = LAMG_FP64;
  o->tol = 1e-8;
  o->max_cycles = 100;
  o->warm_start = 0;
  o->seed = 0;
  o->stream = nullptr;
  o->alloc = nullptr;
  o->dealloc = nullptr;
  o->alloc_ctx = nullptr;
  o->allow_negative_weights = 0;
  o->recomb_norm = LAMG_RECOMB_RESIDUAL;
}

const char* lamg_last_error(void) { return g_last_error; }

const char* lamg_status_str(lamg_status s) {
  switch (s) {
    case LAMG_OK: return "ok";
    case LAMG_E_INVALID_ARG: return "invalid argument";
    case LAMG_E_BAD_WEIGHT: return "edge weight not finite and positive";
    case LAMG_E_NOT_CONNECTED: return "graph is not connected";
    case LAMG_E_NOT_CONVERGED: return "tolerance not reached within max_cycles";
    case LAMG_E_BREAKDOWN: return "non-finite residual";
    case LAMG_E_OUT_OF_MEMORY: return "out of device memory";
    case LAMG_E_DEVICE: return "HIP runtime error";
  }
  return "unknown status";
}

static bool opts_ok(const lamg_options& o) {
  return o.gamma >= 1.0 && o.gamma <= 2.0 && o.nu_pre >= 0 && o.nu_post >= 0 && o.tv_k_min >= 1 &&
         o.tv_k_max >= o.tv_k_min && o.tv_k_max <= 10 && o.tv_sweeps >= 0 && o.q_max > 1.0 && o.coarsest_max_n >= 2 &&
         o.elim_max_degree >= 0 && o.stage1_quantile >= 0.0 && o.stage1_quantile <= 1.0 && o.tol >= 0 &&
         o.max_cycles >= 0 && o.coarsest_sweeps >= 1 && o.dense_max >= 1 && o.dense_max <= 8192 && o.tail_max_n >= 0 &&
         (o.alloc == nullptr) == (o.dealloc == nullptr) &&
         (o.allow_negative_weights == 0 || o.allow_negative_weights == 1) &&
         (o.recomb_norm == LAMG_RECOMB_RESIDUAL || o.recomb_norm == LAMG_RECOMB_ENERGY);
}

}  // extern "C"

namespace {
// LAMG_LOG verbosity (0 silent, 1 one line per setup / solve, 2 also the level
// table and every cycle's residual), read once.
int log_level() {
  static const int v = [] {
    const char* e = std::getenv("LAMG_LOG");
    return e ? std::atoi(e) : 0;
  }();
  return v;
}
// A roctx range for the lifetime of the object.
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};
struct LevelRange {
  explicit LevelRange(int l) {
    char b[32];
    std::snprintf(b, sizeof(b), "lamg_level %d", l);
    roctxRangePushA(b);
  }
  ~LevelRange() { roctxRangePop(); }
  LevelRange(const LevelRange&) = delete;
  LevelRange& operator=(const LevelRange&) = delete;
};

// Bodies per finest-level cycle at every level: the recursion of visit and
// body above (an elimination level is visited once per body of its finer
// level; an aggregation level th times, th from the fractional cycle index).
void count_bodies(const Hierarchy* H, int l, int th, std::vector<int64_t>& count, std::vector<double>& bodies) {
  const int Lc = (int)H->lv.size() - 1;
  const int reps = l == Lc ? 1 : th;
  for (int i = 0; i < reps; ++i) {
    bodies[l] += 1;
    if (l == Lc) return;
    if (H->lv[l + 1].type == LT_ELIM) {
      count_bodies(H, l + 1, 1, count, bodies);
      continue;
    }
    const int64_t c = count[l]++;
    const double gl = H->lv[l].gamma_next;
    count_bodies(H, l + 1, (int)(std::ceil((double)(c + 1) * gl) - std::ceil((double)c * gl)), count, bodies);
  }
}
std::vector<double> bodies_per_cycle(const Hierarchy* H) {
  std::vector<int64_t> count(H->lv.size(), 0);
  std::vector<double> bodies(H->lv.size(), 0.0);
  count_bodies(H, 0, 1, count, bodies);
  return bodies;
}
int tail_first_level(const Hierarchy* H) {
  const int nl = (int)H->lv.size();
  int lc = nl;
  if (H->o.tail_max_n > 0)
    for (int l = nl - 1; l >= 0 && H->lv[l].n <= H->o.tail_max_n; --l) lc = l;
  return lc;
}
void log_setup(const Hierarchy* H) {
  if (log_level() < 1) return;
  std::fprintf(stderr, "[lamg] setup: n %d, m %lld, %d levels, %.2f ms\n", H->n, (long long)H->m, (int)H->lv.size(),
               H->setup_ms);
  if (log_level() < 2) return;
  const std::vector<double> bod = bodies_per_cycle(H);
  const int tl = tail_first_level(H);
  static const char* kind[] = {"finest", "elim", "agg"};
  for (size_t l = 0; l < H->lv.size(); ++l) {
    const Level& L = H->lv[l];
    std::fprintf(stderr, "[lamg]   level %2zu %-6s n %9d nnz %10d colours %3d hub %3d gamma %.4f bodies %6.0f%s\n", l,
                 kind[L.type], L.n, L.nnz, L.ncol, L.hub_k >= 0 ? L.ncol - L.hub_k : 0, L.gamma_next, bod[l],
                 (int)l >= tl ? " tail" : "");
  }
}
}  // namespace

// Setup frame shared by the entry points: options, handle, allocator scope,
// the level construction `levels` (returns a status), finishing and errors.
template <class Levels>
static lamg_status run_setup(int64_t n, int64_t m, const lamg_options* o, lamg_handle* out, Levels levels,
                             bool gamma_every_level = false, int ec = -1, double mu = 0) {
  lamg_options opt;
  lamg_options_default(&opt);
  if (o) {
    if (o->struct_size != sizeof(lamg_options)) return LAMG_E_INVALID_ARG;
    opt = *o;
  }
  if (ec >= 0) {
    opt.ec = (lamg_energy_correction)ec;
    opt.mu = mu;
  }
  if (!opts_ok(opt)) return LAMG_E_INVALID_ARG;
  lamg_hierarchy* h = new lamg_hierarchy;
  Hierarchy* H = &h->H;
  H->o = opt;
  H->s = (hipStream_t)opt.stream;
  H->gamma_every_level = gamma_every_level;
  AllocScope scope(&H->o);  // setup temporaries through the same allocator
  Range range("lamg_setup");
  H->n = (int)n;
  H->m = m;
  auto t0 = std::chrono::steady_clock::now();
  try {
    lamg_status st = levels(H);
    if (st != LAMG_OK) { lamg_free(h); return st; }
    finish_levels(H);
    H->bsave = H->lv[0].v64.b;
    H->x64 = H->lv[0].v64.x;
    H->r64 = dnew<double>(H, n);
    H->colb = dnew<double>(H, n);
    H->colx = dnew<double>(H, n);
    H->bytes_per_cycle = cycle_bytes(H, LAMG_FP64);
    if (H->lv[0].n <= BATCH_MAX_N) batch_prepare(H);  // the persistent many-graph program
    LAMG_HIP(hipStreamSynchronize(H->s));
  } catch (const DevError& e) {
    set_last_error("lamg_setup", e.e);
    lamg_free(h);
    return e.e == hipErrorOutOfMemory ? LAMG_E_OUT_OF_MEMORY : LAMG_E_DEVICE;
  }
  H->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  log_setup(H);
  *out = h;
  return LAMG_OK;
}

extern "C" {

lamg_status lamg_setup(int64_t n, int64_t m, const int32_t* eu, const int32_t* ev, const double* w,
                       const lamg_options* o, lamg_handle* out) {
  if (!out) return LAMG_E_INVALID_ARG;
  *out = nullptr;
  if (n < 1 || m < 0 || n > (int64_t)0x7fffffff / 2 || m > (int64_t)0x3fffffff) return LAMG_E_INVALID_ARG;
  if (m > 0 && (!eu || !ev || !w)) return LAMG_E_INVALID_ARG;
  return run_setup(n, m, o, out, [&](Hierarchy* H) {
    lamg_status st = build_finest(H, n, m, eu, ev, w);
    if (st != LAMG_OK) return st;
    colour_and_order(H, H->lv[0], 0, nullptr);
    int nagg = 0;
    while (H->lv.back().n >= H->o.coarsest_max_n && (int)H->lv.size() < 60) {
      const int l = (int)H->lv.size() - 1;
      LevelRange lr(l + 1);
      if (try_eliminate(H, l)) continue;
      const int r = aggregate(H, l, nagg);
      if (r == 2) { H->coarsest_relax = true; break; }
      if (r == 0) break;
      ++nagg;
    }
    return (lamg_status)LAMG_OK;
  });
}

lamg_status lamg_setup_lgm(int32_t side, const lamg_options* o, lamg_handle* out) {
  if (!out) return LAMG_E_INVALID_ARG;
  *out = nullptr;
  if (side < 4 || side > LAMG_LGM_MAX_SIDE || (side & (side - 1))) return LAMG_E_INVALID_ARG;
  const int64_t n = (int64_t)side * side;
  return run_setup(n, 2 * n, o, out, [&](Hierarchy* H) {
    lamg_status st = build_lgm_finest(H, side);
    if (st != LAMG_OK) return st;
    int sd = side;
    while (H->lv.back().n >= H->o.coarsest_max_n && sd >= 4 && (int)H->lv.size() < 60) {
      LevelRange lr((int)H->lv.size());
      lgm_coarsen(H, (int)H->lv.size() - 1, sd);
      sd /= 2;
    }
    return (lamg_status)LAMG_OK;
  }, true, LAMG_EC_FLAT_MU, 2.0);
}

lamg_status lamg_set_solve_options(lamg_handle h, const lamg_options* o) {
  if (!h || !o || o->struct_size != sizeof(lamg_options)) return LAMG_E_INVALID_ARG;
  if (o->tol < 0 || o->max_cycles < 0 || (o->precision != LAMG_FP64 && o->precision != LAMG_FP32_REFINE) ||
      (o->ec != LAMG_EC_RECOMBINE && o->ec != LAMG_EC_FLAT_MU) ||
      (o->recomb_norm != LAMG_RECOMB_RESIDUAL && o->recomb_norm != LAMG_RECOMB_ENERGY))
    return LAMG_E_INVALID_ARG;
  Hierarchy* H = &h->H;
  // the captured cycles and the tail program depend on these options
  if (o->nu_pre < 0 || o->nu_post < 0) return LAMG_E_INVALID_ARG;
  // captured cycles hold the options as kernel arguments; op programs hold ec, mu and nu
  const bool regraph = o->recomb_norm != H->o.recomb_norm;
  const bool reprogram =
      o->ec != H->o.ec || o->mu != H->o.mu || o->nu_pre != H->o.nu_pre || o->nu_post != H->o.nu_post;
  if (regraph && !reprogram) {
    drop_graphs(H);
    mv_drop_graphs(H);
  }
  if (reprogram) {
    drop_graphs(H);
    mv_drop_graphs(H);
    invalidate_programs(H);
  }
  H->o.precision = o->precision;
  H->o.ec = o->ec;
  H->o.mu = o->mu;
  H->o.tol = o->tol;
  H->o.max_cycles = o->max_cycles;
  H->o.warm_start = o->warm_start;
  H->o.stream = o->stream;
  H->o.nu_pre = o->nu_pre;
  H->o.nu_post = o->nu_post;
  H->o.recomb_norm = o->recomb_norm;
  H->s = (hipStream_t)o->stream;
  if (reprogram && H->lv[0].n <= BATCH_MAX_N) {
    try {
      batch_prepare(H);  // ready for the allocation-free batch entry
    } catch (const DevError& e) {
      set_last_error("lamg_set_solve_options", e.e);
      return e.e == hipErrorOutOfMemory ? LAMG_E_OUT_OF_MEMORY : LAMG_E_DEVICE;
    }
  }
  return LAMG_OK;
}

// One solve on a hierarchy; b and x are device vectors in input node order.
static lamg_status solve_one(Hierarchy* H, const double* b, double* x, lamg_info* info) {
  hipStream_t s = H->s;
  Level& L = H->lv[0];
  const int n = L.n;
  auto t0 = std::chrono::steady_clock::now();
  double* rs = res_slots(H);
  // b <- b - mean(b), in colour order
  mean_to_slot(s, H, b, n, 6);
  hipLaunchKernelGGL(k_gather_sub, grid1(n), dim3(256), 0, s, n, L.perm, b, rs, 6, H->bsave);
  double* hr = H->hred;
  LAMG_HIP(hipMemcpyAsync(hr + 6, rs + 6, sizeof(double), hipMemcpyDeviceToHost, s));
  if (H->o.warm_start) hipLaunchKernelGGL(k_gather_sub, grid1(n), dim3(256), 0, s, n, L.perm, x, nullptr, 0, H->x64);
  else fill<double>(s, H->x64, 0.0, n);
  norm2_async(s, H, H->bsave, n, hr + 0);
  residual<double>(s, L, L.val, L.diag, H->bsave, H->x64, H->r64);
  norm2_async(s, H, H->r64, n, hr + 1);
  LAMG_HIP(hipStreamSynchronize(s));
  const double removed = hr[6];
  const double nb = std::sqrt(hr[0]);
  const double r0 = std::sqrt(hr[1]);
  double rk = r0;
  int it = 0;
  const bool fp32 = H->o.precision == LAMG_FP32_REFINE;
  if (nb > 0) {
    Vecs<float>& v32 = L.v32;
    while (rk > H->o.tol * nb && it < H->o.max_cycles && std::isfinite(rk)) {
      const int inst = 0;
      if (!fp32) {
        cycle_graph<double>(H, inst);  // level-1 vectors alias bsave / x64
      } else {
        // inner FP32 cycle on the projected FP64 residual
        mean_to_slot(s, H, H->r64, n, 7);
        hipLaunchKernelGGL(k_sub_to_f32, grid1(n), dim3(256), 0, s, n, (const double*)H->r64, rs, 7, v32.b);
        fill<float>(s, v32.x, 0.0f, n);
        cycle_graph<float>(H, inst);
        hipLaunchKernelGGL(k_add_f32, grid1(n), dim3(256), 0, s, n, (const float*)v32.x, H->x64);
        subtract_mean<double>(s, H, H->x64, n);
      }
      residual<double>(s, L, L.val, L.diag, H->bsave, H->x64, H->r64);
      norm2_async(s, H, H->r64, n, hr + 2);
      LAMG_HIP(hipStreamSynchronize(s));
      rk = std::sqrt(hr[2]);
      ++it;
      if (log_level() >= 2) std::fprintf(stderr, "[lamg]   cycle %3d  rel. residual %.3e\n", it, rk / nb);
    }
  }
  hipLaunchKernelGGL(k_scatter, grid1(n), dim3(256), 0, s, n, L.perm, (const double*)H->x64, x);
  LAMG_HIP(hipStreamSynchronize(s));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) {
    info->cycles = it;
    info->levels = (int)H->lv.size();
    info->rel_residual = nb > 0 ? rk / nb : 0.0;
    info->acf = it > 0 && r0 > 0 ? std::pow(rk / r0, 1.0 / it) : 0.0;
    info->removed_mean = removed;
    info->setup_ms = H->setup_ms;
    info->solve_ms = ms;
    info->bytes_moved = (int64_t)it * cycle_bytes(H, H->o.precision);
  }
  if (log_level() >= 1)
    std::fprintf(stderr, "[lamg] solve: %s, %d cycles, rel. residual %.3e, %.3f ms\n", fp32 ? "fp32+refine" : "fp64", it,
                 nb > 0 ? rk / nb : 0.0, ms);
  if (!std::isfinite(rk)) return LAMG_E_BREAKDOWN;
  if (nb > 0 && rk > H->o.tol * nb) return LAMG_E_NOT_CONVERGED;
  return LAMG_OK;
}

lamg_status lamg_solve(lamg_handle h, const double* b, double* x, lamg_info* info) {
  if (!h || !b || !x) return LAMG_E_INVALID_ARG;
  Range range("lamg_solve");
  try {
    return solve_one(&h->H, b, x, info);
  } catch (const DevError& e) {
    set_last_error("lamg_solve", e.e);
    return e.e == hipErrorOutOfMemory ? LAMG_E_OUT_OF_MEMORY : LAMG_E_DEVICE;
  }
}

lamg_status lamg_solve_batch(int32_t count, const lamg_handle* hs, const int32_t* nrhs, const double* const* B,
                             double* const* X, lamg_info* infos) {
  if (count < 0 || (count > 0 && (!hs || !nrhs || !B || !X))) return LAMG_E_INVALID_ARG;
  lamg_status worst = LAMG_OK;
  for (int i = 0; i < count; ++i) {
    if (!hs[i] || nrhs[i] < 1 || !B[i] || !X[i]) return LAMG_E_INVALID_ARG;
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return LAMG_E_INVALID_ARG;  // one handle, one solve at a time
  }
  Range range("lamg_solve_batch");
  try {
    std::vector<int> many;  // single right-hand sides of small graphs: one persistent launch
    for (int i = 0; i < count; ++i) {
      Hierarchy* H = &hs[i]->H;
      lamg_info acc{};
      lamg_status st = LAMG_OK;
      if (nrhs[i] > 1) st = solve_multi(H, nrhs[i], B[i], X[i], &acc);
      else if (count > 1 && H->lv[0].n <= BATCH_MAX_N) { many.push_back(i); continue; }
      else st = solve_one(H, B[i], X[i], &acc);
      if (st == LAMG_E_INVALID_ARG) return st;
      if (st != LAMG_OK && worst == LAMG_OK) worst = st;
      if (infos) infos[i] = acc;
    }
    if (!many.empty()) {
      std::vector<Hierarchy*> H(many.size());
      std::vector<const double*> b(many.size());
      std::vector<double*> x(many.size());
      std::vector<lamg_info> inf(many.size());
      for (size_t j = 0; j < many.size(); ++j) {
        H[j] = &hs[many[j]]->H;
        b[j] = B[many[j]];
        x[j] = X[many[j]];
      }
      const lamg_status st = solve_graphs((int)many.size(), H.data(), b.data(), x.data(), inf.data());
      if (st != LAMG_OK && worst == LAMG_OK) worst = st;
      if (infos)
        for (size_t j = 0; j < many.size(); ++j) infos[many[j]] = inf[j];
    }
  } catch (const DevError& e) {
    set_last_error("lamg_solve_batch", e.e);
    return e.e == hipErrorOutOfMemory ? LAMG_E_OUT_OF_MEMORY : LAMG_E_DEVICE;
  }
  return worst;
}

lamg_status lamg_solve_batch_noalloc(int32_t count, const lamg_handle* hs, const double* const* B,
                                     double* const* X, lamg_info* infos) {
  char msg[200];
  if (count < 0 || (count > 0 && (!hs || !B || !X))) return LAMG_E_INVALID_ARG;
  if (count > LAMG_NOALLOC_MAX_GRAPHS) {
    std::snprintf(msg, sizeof(msg), "lamg_solve_batch_noalloc: %d graphs exceed the static scratch of %d graphs",
                  (int)count, (int)LAMG_NOALLOC_MAX_GRAPHS);
    set_last_error_msg(msg);
    return LAMG_E_INVALID_ARG;
  }
  if (count == 0) return LAMG_OK;
  std::vector<Hierarchy*> H(count);
  for (int i = 0; i < count; ++i) {
    if (!hs[i] || !B[i] || !X[i]) return LAMG_E_INVALID_ARG;
    H[i] = &hs[i]->H;
    if (H[i]->lv[0].n > BATCH_MAX_N) {
      std::snprintf(msg, sizeof(msg), "lamg_solve_batch_noalloc: graph %d has %d nodes (at most %d)", i,
                    H[i]->lv[0].n, BATCH_MAX_N);
      set_last_error_msg(msg);
      return LAMG_E_INVALID_ARG;
    }
  }
  std::vector<Hierarchy*> sorted(H);
  std::sort(sorted.begin(), sorted.end());
  if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) return LAMG_E_INVALID_ARG;
  Range range("lamg_solve_batch_noalloc");
  try {
    return solve_graphs(count, H.data(), B, X, infos, true);
  } catch (const DevError& e) {
    set_last_error("lamg_solve_batch_noalloc", e.e);
    return e.e == hipErrorOutOfMemory ? LAMG_E_OUT_OF_MEMORY : LAMG_E_DEVICE;
  }
}

namespace {
__global__ void k_edge_grad(int64_t m, const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                            const double* __restrict__ x, const double* __restrict__ lam, double* __restrict__ g) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const int u = eu[e], v = ev[e];
  g[e] = -(lam[u] - lam[v]) * (x[u] - x[v]);
}
}  // namespace

lamg_status lamg_edge_gradient(int64_t m, const int32_t* eu, const int32_t* ev, const double* x, const double* lam,
                               double* grad_w, void* stream) {
  if (m < 0 || (m > 0 && (!eu || !ev || !x || !lam || !grad_w))) return LAMG_E_INVALID_ARG;
  if (m == 0) return LAMG_OK;
  try {
    hipLaunchKernelGGL(k_edge_grad, grid1(m), dim3(256), 0, (hipStream_t)stream, m, eu, ev, x, lam, grad_w);
    LAMG_HIP(hipGetLastError());
    LAMG_HIP(hipStreamSynchronize((hipStream_t)stream));
  } catch (const DevError& e) {
    set_last_error("lamg_edge_gradient", e.e);
    return LAMG_E_DEVICE;
  }
  return LAMG_OK;
}

lamg_status lamg_level_info(lamg_handle h, int32_t l, lamg_level_stats* out) {
  if (!h || !out || l < 0 || l >= (int32_t)h->H.lv.size()) return LAMG_E_INVALID_ARG;
  const Hierarchy* H = &h->H;
  const Level& L = H->lv[l];
  const std::vector<double> bod = bodies_per_cycle(H);
  std::memset(out, 0, sizeof(*out));
  out->nnz = L.nnz;
  out->n = L.n;
  out->kind = L.type;
  out->colours = L.ncol;
  out->hub_colours = L.hub_k >= 0 ? L.ncol - L.hub_k : 0;
  out->in_tail = l >= tail_first_level(H) ? 1 : 0;
  out->gamma = l + 1 < (int32_t)H->lv.size() ? L.gamma_next : 1.0;
  out->visits = bod[l];
  return LAMG_OK;
}

void lamg_free(lamg_handle h) {
  if (!h) return;
  Hierarchy* H = &h->H;
  if (H->s) (void)hipStreamSynchronize(H->s);
  else (void)hipDeviceSynchronize();
  drop_graphs(H);
  mv_release(H);
  if (H->cs) (void)hipStreamDestroy(H->cs);
  for (void* p : H->owned) dev_free(H->o, p);
  if (H->hred) (void)hipHostFree(H->hred);
  delete h;
}

}  // extern "C"
