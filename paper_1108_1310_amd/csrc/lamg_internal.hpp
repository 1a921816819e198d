// Internal declarations of the LAMG HIP library (gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../include/lamg.h"

namespace lamg {

// ----------------------------------------------------------------- checks
struct DevError {
  hipError_t e;
};
#define LAMG_HIP(call)                                   \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) throw ::lamg::DevError{e_};    \
  } while (0)

enum LevelType { LT_FINEST = 0, LT_ELIM = 1, LT_AGG = 2 };
enum NodeState { ST_UNDECIDED = 0, ST_SEED = 1, ST_ASSOC = 2, ST_DUMMY = 3 };

// Streams of the counter hash: colouring priorities and test-vector draws.
constexpr uint64_t STREAM_COLOUR = 7, STREAM_TV = 3;

// Rows longer than this are reduced with 64 strided partial sums and an xor
// butterfly; shorter rows are summed sequentially in column order.
constexpr int SHORT_ROW = 64;

// Chunk length of the wavefront sum of a long row (the fixed summation order).
constexpr int ROW_CHUNK = 512;

// Hub sweep of a relaxed level.  On power-law levels the last colour classes
// hold few rows (the hubs) with long rows, and a GS sweep spends most of its
// time in their dependent phases.  From colour hub_k on, once colours
// < hub_k are final for the sweep, every hub row's sum over those colours is
// one launch (k_hub_partial), and the remaining colour phases run in one
// workgroup with the hubs' x in LDS and only the hub-to-hub entries left to
// gather (k_hub_sweep).  Taken when the hub rows are at most HUB_MAX_ROWS,
// at least HUB_MIN_COLOURS colours are hub colours, and the chunk table has
// at most HUB_MAX_CHUNKS entries; the split point follows the cost model
// below.
constexpr int HUB_MAX_ROWS = 4096;
constexpr int HUB_MIN_COLOURS = 8;
constexpr int HUB_THREADS = 1024;
constexpr int HUB_PER = 4;                          // entries per thread per chunk
constexpr int HUB_CHUNK = HUB_THREADS * HUB_PER;    // products staged per chunk
static_assert(HUB_CHUNK >= HUB_MAX_ROWS, "a hub row's hub-to-hub entries fit one chunk");
constexpr int HUB_MAX_CHUNKS = 1024;
// The split point: from the first colour whose classes onwards hold at most
// HUB_MAX_ROWS rows, the later start that minimises the sweep's modelled
// time, in tenths of a microsecond as measured on MI355X (FP64): a launch of
// a small colour class about 10 us, a hub-sweep chunk about 1.8 us.  A later
// start launches more colours but leaves fewer hub-to-hub entries.
constexpr int HUB_COST_LAUNCH = 100;
constexpr int HUB_COST_CHUNK = 18;

struct Tiles {
  int64_t rows = 0, nnz = 0;  // rows and entries covered (algorithmic bytes per launch)
  int nstream = 0;
  int4* stream = nullptr;     // [nstream] stream tiles: (first row, end row, first entry, entries)
  int nvlong = 0;
  int4* vlong = nullptr;      // very long rows, longest first: (row, first entry, entries, 0)
  int nmed = 0, nmed_blocks = 0;
  int4* med = nullptr;        // medium rows, longest first: (row, first entry, entries, 0)
  int* longrows = nullptr;    // every row longer than SHORT_ROW (device; setup kernels)
  int nlong = 0;
  int blocks() const { return nvlong + nmed_blocks + nstream; }
};

template <class T>
struct Vecs {
  T *x = nullptr, *b = nullptr, *r = nullptr;
  T *X[2] = {nullptr, nullptr}, *R[2] = {nullptr, nullptr};
};

struct Level {
  int n = 0, nnz = 0, type = LT_FINEST, ncol = 0;
  std::vector<int> cptr;            // host copy, colour class boundaries
  int *rp = nullptr, *ci = nullptr; // CSR of off-diagonal weights (positive)
  double *val = nullptr, *diag = nullptr;
  float *val32 = nullptr, *diag32 = nullptr;
  int* perm = nullptr;              // node order: perm[new] = natural id
  std::vector<Tiles> tiles;         // per colour
  Tiles all;                        // every row (residual)
  std::vector<int> long_ptr, long_rows;  // host: rows > SHORT_ROW grouped by colour
  int *d_cptr = nullptr, *d_lptr = nullptr, *d_lrows = nullptr;  // device copies (op programs)
  // transfer from the previous level into this one
  int* agg = nullptr;               // AGG: fine node -> this level's node
  int *agg_ptr = nullptr, *members = nullptr;  // P^T as CSR (aggregate members ascending)
  int* cidx = nullptr;              // ELIM: fine node -> this level's node or -1
  int* cfine = nullptr;             // ELIM: this level's node -> fine node
  // ELIM restriction P^T r = r_C + R r_F as a CSR over this level's nodes:
  // columns are fine F nodes, values w_cf / a_ff (FP64 and FP32)
  int *er_rp = nullptr, *er_ci = nullptr;
  double* er_val = nullptr;
  float* er_val32 = nullptr;
  Tiles er_tiles;
  int nF = 0;
  double gamma_next = 1.0;          // cycle index for visits from this level to the next
  // aggregation diagnostics (this level as the fine side), kept for parity tests
  int K = 0, stage = 0;
  double delta1 = 1, alpha1 = 0, alpha2 = -1, rate = -1;
  double* tv = nullptr;
  double* aff = nullptr;
  uint8_t *ok = nullptr, *weak = nullptr, *hub = nullptr;
  int* state = nullptr;
  Vecs<double> v64;
  Vecs<float> v32;
  // hub sweep (hub_k < 0: not taken): hub rows [hub_r0, n) in colours
  // [hub_k, ncol); their hub-to-hub entries as a CSR with local column ids
  int hub_k = -1, hub_r0 = 0, hub_n = 0, hub_nnz = 0;
  int64_t hub_low_nnz = 0;                  // entries of hub rows into colours < hub_k
  int *hub_rp = nullptr, *hub_ci = nullptr; // [hub_n + 1], [hub_nnz]
  int2* hub_ck = nullptr;                   // [hub_nck] chunks: (first row, end row), local ids
  int hub_nck = 0;
  double *hub_val = nullptr, *hub_p = nullptr;
  float *hub_val32 = nullptr, *hub_p32 = nullptr;
};

// Device descriptor of one level for the single-workgroup tail program.
struct TailLevel {
  int n, nnz, ncol, nc;  // nc: nodes of level l+1 (0 for the coarsest)
  int nlong;             // rows longer than 64 entries
  int nner;              // entries of the elimination stencil into level l+1
  int vres;              // set on the device: this level's arrays sit in LDS
  int pad_;
  const int *rp, *ci;
  const double *val64, *diag64;
  const float *val32, *diag32;
  const int *cptr, *lptr, *lrows;
  const int *agg, *agg_ptr, *members;                 // into level l+1 (aggregation)
  const int *cidx, *cfine, *er_rp, *er_ci;            // into level l+1 (elimination)
  const double* er64;
  const float* er32;
  double *x64, *b64, *r64, *X64[2], *R64[2];
  float *x32, *b32, *r32, *X32[2], *R32[2];
};

// Multi-vector workspace: every level's work vectors as n_l x k row-major
// blocks (right-hand side index fastest), the FP64 outer vectors of level 0,
// per-column reduction scratch and convergence mask, and the captured
// multi-vector cycles.  Reallocated when k changes.
struct MVWork {
  int k = 0;
  std::vector<Vecs<double>> v64;
  std::vector<Vecs<float>> v32;
  double *B = nullptr, *X = nullptr, *R = nullptr;  // level 0, colour order
  int rows = 0;                // rows per pass of the column reductions
  double* part = nullptr;      // column reduction partials [6][k * rows]
  double* res = nullptr;       // per-column results [8][k]
  double* hres = nullptr;      // pinned host mirror of res
  int* mask = nullptr;         // per-column: 1 while the column still iterates
  int* hmask = nullptr;        // pinned host mirror
  TailLevel* tail = nullptr;   // tail descriptors pointing at this workspace
  const void* tail_src = nullptr;  // the single-vector descriptors they were built from
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  std::vector<void*> owned;    // device allocations of this workspace
  std::vector<int> cycles;     // last solve, per column
  std::vector<double> rel, removed;
};

inline lamg_options options_defaults() {
  lamg_options o;
  lamg_options_default(&o);
  return o;
}

struct Hierarchy {
  lamg_options o = options_defaults();
  hipStream_t s = nullptr;
  int n = 0;
  int64_t m = 0;
  std::vector<Level> lv;
  double* cinv = nullptr;  // dense inverse of the augmented coarsest matrix (n_L x n_L)
  bool coarsest_relax = false;  // coarsest level solved by relaxation sweeps
  int nL = 0;
  double* red = nullptr;   // reduction scratch (partials + results)
  double* hred = nullptr;  // pinned host mirror of reduction results
  double* bsave = nullptr; // level-1 rhs (FP64, colour order)
  double* x64 = nullptr;   // level-1 iterate (FP64, colour order)
  double* r64 = nullptr;   // level-1 outer residual
  double *colb = nullptr, *colx = nullptr;  // column staging of multi-RHS solves
  std::vector<void*> owned;  // every device allocation, freed with the handle
  std::vector<size_t> owned_bytes;  // their sizes (same order)
  // captured cycles: [precision][2 alternating instances]
  hipStream_t cs = nullptr;  // capture stream
  hipGraphExec_t gexec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  double setup_ms = 0;
  int64_t bytes_per_cycle = 0;
  // single-workgroup tail: levels >= tail_lc run from an op program
  int tail_lc = -1;               // -1: not prepared; == lv.size(): no tail
  void* tail_levels = nullptr;    // device array of level descriptors
  int4* tail_prog = nullptr;      // device op program of one finest cycle
  std::vector<int2> tail_segs;    // (offset, length) per entry into the tail
  int tail_cursor = 0;
  // set while a cycle is recorded whose finest residual is already known:
  // FP64, in r64 (the stopping test's); FP32, equal to b (x starts at 0)
  bool top_res_known = false;
  bool gamma_every_level = false;  // cycle index o.gamma at every level (geometric)
  std::vector<TailLevel> tail_host;  // host copy of the descriptors
  MVWork mv;
  // whole-hierarchy op program (every level, from level 0) for the
  // persistent many-graph solve
  void* full_levels = nullptr;
  int4* full_prog = nullptr;
  int full_nops = 0;
  std::vector<TailLevel> full_host;  // host copies of the descriptors and program
  std::vector<int4> full_prog_host;
  bool full_checked = false;         // validated against the allocations (program_check)
};

// -------------------------------------------------------- instrumentation
// When enabled, every relaxation / residual launch is bracketed by HIP events
// on its stream and its algorithmic bytes are accumulated per kernel:
// 0 GS FP64, 1 residual FP64, 2 GS FP32, 3 residual FP32, 4..7 the same
// four for the multi-vector kernels, 8 / 9 the hub sweep (FP64 / FP32: the
// partial-sum launch and the single-workgroup sweep of each GS sweep),
// 10 / 11 aggregation restriction, 12 / 13 aggregation interpolation,
// 14 / 15 the single-workgroup tail launches (FP64 / FP32).
constexpr int PROF_KERNELS = 16;
// Spans: prof_begin records the opening event of a run of launches of one
// kernel, prof_count adds each launch (and its algorithmic bytes) of that
// kernel to the open span, prof_end records the closing event.
void prof_begin(hipStream_t s, int kernel, int launches = 1);
void prof_count(int kernel, int64_t bytes);
void prof_end(hipStream_t s);
bool prof_on();
// Instrumented cycles run eagerly (not from captured graphs) so that every
// launch has its own timed event pair; prof_flush reads the pending pairs.
void prof_flush();
// Message of the last device error on this thread (lamg_last_error).
void set_last_error(const char* where, hipError_t e);
void set_last_error_msg(const char* msg);
// Detail appended to the next set_last_error on this thread (and cleared).
void set_error_detail(const char* msg);

// ------------------------------------------------------------- allocation
// Device memory through the options' allocator (hipMalloc / hipFree when
// none is set); dev_alloc throws DevError{hipErrorOutOfMemory} on failure.
void* dev_alloc(const lamg_options& o, size_t bytes);
void dev_free(const lamg_options& o, void* p);
// The allocator of the setup running on this thread (for its temporaries).
struct AllocScope {
  const lamg_options* prev;
  explicit AllocScope(const lamg_options* o);
  ~AllocScope();
};
void* dalloc(Hierarchy* H, size_t bytes);
template <class T>
T* dnew(Hierarchy* H, size_t count) { return (T*)dalloc(H, count * sizeof(T) + 16); }

// ----------------------------------------------------------- kernel entry
// (declared here, defined in the .hip sources)
namespace k {
// reductions: fixed grid and tree, results deterministic run to run
constexpr int RED_BLOCKS = 512, RED_THREADS = 256;
}

void build_tiles(Hierarchy* H, Level& L);
// Relaxation and residual (FP64 / FP32), k vectors row-major for the multi-vector form.
template <class T>
void gs_colour(hipStream_t s, const Level& L, int c, const T* val, const T* diag, const T* b, T* x,
               bool from_zero = false);
template <class T>
void gs_sweep(hipStream_t s, const Level& L, const T* val, const T* diag, const T* b, T* x, bool from_zero = false);
template <class T>
void residual(hipStream_t s, const Level& L, const T* val, const T* diag, const T* b, const T* x, T* r);
void gs_multi_sweep(hipStream_t s, const Level& L, const double* b, double* X, int K);

// transfers
template <class T>
void restrict_agg(hipStream_t s, const Level& C, int nfine, const T* r, T* bc, T mu);
template <class T>
void interp_agg(hipStream_t s, const Level& C, int nfine, const T* e, T* x);
template <class T>
void restrict_elim(hipStream_t s, const Level& C, const T* r, T* bc);
void build_elim_restriction(Hierarchy* H, const Level& F, Level& C);
template <class T>
void interp_elim(hipStream_t s, const Level& F, const Level& C, const T* val, const T* diag, const T* r, const T* e, T* x);
template <class T>
void fill(hipStream_t s, T* p, T v, int n);

// recombination / mean / norms (partials in H->red)
template <class T>
void recombine(hipStream_t s, Hierarchy* H, const Level& L, Vecs<T>& v, int th);
template <class T>
void subtract_mean(hipStream_t s, Hierarchy* H, T* x, int n);
void norm2_async(hipStream_t s, Hierarchy* H, const double* r, int n, double* dst_host);
// sum of x times scale into result slot `slot` (device side)
void sum_to_slot(hipStream_t s, Hierarchy* H, const double* x, int n, int slot, double div);
void coarsest_solve(hipStream_t s, Hierarchy* H, const double* b, double* x);
void coarsest_solve32(hipStream_t s, Hierarchy* H, const float* b, float* x);
void coarsest_factor(Hierarchy* H, const Level& L);

// setup
lamg_status build_finest(Hierarchy* H, int64_t n, int64_t m, const int32_t* eu, const int32_t* ev, const double* w);
void colour_and_order(Hierarchy* H, Level& L, int level, std::vector<int>* inv_host_unused);
int colour_greedy(hipStream_t s, int n, const int* rp, const int* ci, uint64_t seed, int level, int* col);
bool try_eliminate(Hierarchy* H, int l);
// 1: coarse level added; 0: no coarsening possible; 2: relaxation is fast
int aggregate(Hierarchy* H, int l, int agg_index);
void finish_levels(Hierarchy* H);
void build_hub(Hierarchy* H, Level& L);
// lean geometric multigrid (Section 5.3): the periodic side x side grid as
// the finest level, red-black ordered; one 2 x 2 coarsening of level l
lamg_status build_lgm_finest(Hierarchy* H, int side);
void lgm_coarsen(Hierarchy* H, int l, int side);

// solve
int64_t cycle_bytes(const Hierarchy* H, int prec);
int64_t cycle_bytes_k(const Hierarchy* H, int prec, int k);
template <class T>
void cycle(Hierarchy* H, bool top_res_known = false);
// Replay one captured cycle (capturing it on first use); `inst` alternates.
template <class T>
void cycle_graph(Hierarchy* H, int inst);
void drop_graphs(Hierarchy* H);
// Tail: prepare the descriptors and the op program (idempotent), and run the
// next program segment (one entry into level tail_lc) on the stream.
void tail_prepare(Hierarchy* H);
template <class T>
void tail_run_next(Hierarchy* H);
// Drop the op programs (they depend on nu, ec and mu).
void invalidate_programs(Hierarchy* H);
// Graphs up to this size join the persistent launch of a many-graph batch;
// larger ones are solved one after another with the multi-launch cycle.
constexpr int BATCH_MAX_N = 1 << 18;
// Persistent many-graph solve: every graph's whole solve in one workgroup.
// noalloc: the launch's buffers come from the library's static device
// scratch (at most LAMG_NOALLOC_MAX_GRAPHS graphs, every hierarchy already
// prepared, no tuning) instead of the first handle's allocator.
lamg_status solve_graphs(int count, Hierarchy* const* hs, const double* const* B, double* const* X,
                         lamg_info* infos, bool noalloc = false);
// The whole-hierarchy descriptors and op program of the persistent solve
// (idempotent; made at setup for graphs of at most BATCH_MAX_N nodes and again
// after a change of the options the program depends on).
void batch_prepare(Hierarchy* H);
// Multi-vector tail: one workgroup per column of the workspace blocks.
void tail_prepare_mv(Hierarchy* H);
template <class T>
void tail_run_next_mv(Hierarchy* H);

// multi-vector cycle and solve
void mv_release(Hierarchy* H);
void mv_drop_graphs(Hierarchy* H);
lamg_status solve_multi(Hierarchy* H, int k, const double* B, double* X, lamg_info* info);
void mv_neg_apply(Hierarchy* H, int k, const double* Xp, double* Yp);
void mv_precondition(Hierarchy* H, int k, const double* Bp, double* Xp, int cycles);
void mv_project(Hierarchy* H, int k, double* Xp);

}  // namespace lamg

// The opaque handle of the C ABI.
struct lamg_hierarchy {
  lamg::Hierarchy H;
};
