/* lamg.h -- C ABI of the MI355X Lean Algebraic Multigrid (LAMG) library.
 *
 * Solves the graph-Laplacian system A x = b, 1^T x = 0 for a zero-sum b
 * (Livne & Brandt, Section 1, eq. linsys), where A is the Laplacian of a
 * connected undirected graph with positive edge weights (Section 1, eq. lap).
 * Setup (Section 4.1) builds a multilevel hierarchy that depends on A only;
 * each solve (Section 4.2) runs multigrid cycles until
 * ||b - A x||_2 <= tol ||b||_2.
 *
 * Pointers marked DEVICE must be device memory of the current HIP device
 * (for example torch tensors); HOST pointers are ordinary host memory.
 * All work is enqueued on options.stream (NULL = the null stream); every call
 * returns only after its work on that stream is complete.
 * No function throws or aborts across this interface; errors are returned as
 * lamg_status codes.  A handle may be used by one stream at a time; distinct
 * handles are independent.
 */
#ifndef LAMG_H
#define LAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lamg_hierarchy* lamg_handle;

typedef enum {
  LAMG_OK = 0,
  LAMG_E_INVALID_ARG = 1,   /* n < 1, m < 0, an index out of range, a self-loop, NULL pointer */
  LAMG_E_BAD_WEIGHT = 2,    /* a weight that is not finite and > 0 */
  LAMG_E_NOT_CONNECTED = 3, /* the graph has more than one connected component (Section 1) */
  LAMG_E_NOT_CONVERGED = 4, /* tol not reached in max_cycles; x holds the last iterate */
  LAMG_E_BREAKDOWN = 5,     /* a non-finite residual (NaN/Inf in b, or overflow) */
  LAMG_E_OUT_OF_MEMORY = 6,
  LAMG_E_DEVICE = 7         /* a HIP runtime error */
} lamg_status;

typedef enum { LAMG_FP64 = 0, LAMG_FP32_REFINE = 1 } lamg_precision;
/* Energy correction (Section 3.4.4-3.4.5): iterate recombination (eq. recomb)
 * or a flat factor mu on the restricted residual (eq. galerkin2). */
typedef enum { LAMG_EC_RECOMBINE = 0, LAMG_EC_FLAT_MU = 1 } lamg_energy_correction;
/* The norm iterate recombination minimises over its combinations: the
 * residual 2-norm as eq. recomb prints it (default), or the energy norm of the
 * error (y - x*)^T A (y - x*), computable as 1/2 y^T A y - b^T y.  The energy
 * norm converges on smooth right-hand sides where the printed norm can stall
 * (random geometric graphs, anisotropic grids) but is unreliable close to the
 * rounding floor of large graphs (tolerances near 1e-10); the flat energy
 * correction (LAMG_EC_FLAT_MU) converges in both regimes. */
typedef enum { LAMG_RECOMB_RESIDUAL = 0, LAMG_RECOMB_ENERGY = 1 } lamg_recomb_norm;

typedef struct lamg_options {
  uint32_t struct_size;     /* sizeof(lamg_options); set by lamg_options_default */
  double gamma;             /* cycle index at fine levels, 1.5 (Section 4.1) */
  int nu_pre, nu_post;      /* relaxation sweeps per level visit, 1 and 2 (eq. cycle_index) */
  int tv_k_min, tv_k_max;   /* test vectors: 4 at the first aggregation, up to 10 (Section 4.1) */
  int tv_sweeps;            /* relaxation sweeps per test vector, 3 (Section 4.1) */
  double q_max;             /* energy-ratio threshold, 2.5 (Section 3.4.4) */
  double mu;                /* flat energy correction factor, 4/3 (eq. optimal_mu) */
  double hub_factor;        /* hub degree factor, 8 (Section 3.4.1 footnote) */
  int elim_max_degree;      /* low-degree elimination bound, 4 (Section 3.2) */
  int coarsest_max_n;       /* stop coarsening below this many nodes, 150 (Section 4.1) */
  double weak_edge_ratio;   /* edge weak if w < ratio * max neighbouring weight, 1e-3 */
  double elim_stop_frac;    /* stop eliminating when |F| < frac * n, 0.05 */
  double stage1_quantile;   /* stage-1 affinity threshold quantile, 1.0 */
  double relax_fast_ratio;  /* stop coarsening when the last test-vector sweep
                               leaves at most this fraction of the energy, 0.1
                               (Section 4.1: "until relaxation converges rapidly") */
  int coarsest_sweeps;      /* GS sweeps solving such a coarsest level, 3 */
  int dense_max;            /* largest coarsest level solved densely, 8192 */
  int tail_max_n;           /* coarse levels with at most this many nodes (and all
                               coarser ones) run inside one workgroup per entry, 3072;
                               0 = every level launches its own kernels */
  lamg_energy_correction ec;
  lamg_precision precision;
  double tol;               /* relative residual target, 1e-8 */
  int max_cycles;           /* 100 */
  int warm_start;           /* 1: x holds the initial guess on entry */
  uint64_t seed;            /* colouring priorities and test vectors */
  void* stream;             /* hipStream_t */
  /* Device memory of the hierarchy, its workspaces and the setup's
   * temporaries (e.g. a framework's caching allocator): alloc(bytes, ctx)
   * returns a device pointer aligned to at least 256 bytes, or NULL (the call
   * then fails with LAMG_E_OUT_OF_MEMORY); dealloc(ptr, ctx) releases one.
   * Called on the calling thread, never concurrently for one handle; memory
   * of a handle is released by lamg_free, temporaries before the call
   * returns.  Both NULL: hipMalloc / hipFree.  Set both or neither; fixed at
   * setup (lamg_set_solve_options ignores them). */
  void* (*alloc)(size_t bytes, void* ctx);
  void (*dealloc)(void* ptr, void* ctx);
  void* alloc_ctx;
  /* 1: accept negative (non-zero, finite) edge weights, Section 5.2; the
   * caller vouches that the Laplacian is positive semi-definite.  The hub,
   * affinity and energy-ratio tests of a level with a negative weight then
   * use |w|.  0 (default): weights must be > 0 (LAMG_E_BAD_WEIGHT). */
  int allow_negative_weights;
  /* lamg_recomb_norm of iterate recombination (solve phase; changeable by
   * lamg_set_solve_options), LAMG_RECOMB_RESIDUAL by default. */
  int recomb_norm;
} lamg_options;

typedef struct lamg_info {
  int32_t cycles;           /* cycles run (FP32 refinement: inner FP32 cycles) */
  int32_t levels;
  double rel_residual;      /* final ||b - A x|| / ||b|| in FP64 */
  double acf;               /* (r_p / r_0)^(1/p), Section 5.1 */
  double removed_mean;      /* mean of the input b, removed before solving */
  double setup_ms, solve_ms;
  int64_t bytes_moved;      /* algorithmic bytes of the solve (matrix + vector streams) */
} lamg_info;

/* Fill o with the paper's defaults (Sections 3-4). */
void lamg_options_default(lamg_options* o);

/* Build the hierarchy of the Laplacian of the graph given as a COO edge list.
 *   n       number of nodes, >= 1
 *   m       number of edge entries, >= 0
 *   eu, ev  DEVICE int32[m] endpoints in [0, n), eu[e] != ev[e]; entries of the
 *           same unordered pair are summed (Section 5.1 preprocessing)
 *   w       DEVICE double[m] weights, finite and > 0 (finite and non-zero with
 *           o->allow_negative_weights; else LAMG_E_BAD_WEIGHT)
 *   o       HOST options (NULL = defaults)
 *   out     HOST; receives the handle, or NULL on error.
 * The inputs are copied; the caller may free them on return.  The handle owns
 * all hierarchy memory until lamg_free. */
lamg_status lamg_setup(int64_t n, int64_t m, const int32_t* eu, const int32_t* ev, const double* w,
                       const lamg_options* o, lamg_handle* out);

/* Lean geometric multigrid (Section 5.3): the hierarchy of the periodic
 * Poisson problem on a side x side grid (unit weights; node (i, j) has id
 * i + side j, so b and x of lamg_solve are in that order).  Every level is
 * the Galerkin operator of 1:2 coarsening in each dimension (aggregate
 * (i/2, j/2) of the finer grid, first-order transfers) and is relaxed by
 * Gauss-Seidel in red-black order; the cycle index is o->gamma at every
 * level and the correction is the flat energy correction with mu = 2
 * (eq. galerkin2), which this call sets in place of o->ec and o->mu (they
 * stay changeable by lamg_set_solve_options).  Coarsening stops below
 * o->coarsest_max_n nodes.
 *   side  a power of two, 4 <= side <= LAMG_LGM_MAX_SIDE, else
 *         LAMG_E_INVALID_ARG
 *   o, out as for lamg_setup. */
#define LAMG_LGM_MAX_SIDE 16384
lamg_status lamg_setup_lgm(int32_t side, const lamg_options* o, lamg_handle* out);

/* Solve A x = b - mean(b) (Section 4.2 cycles, mean removed each cycle).
 *   b     DEVICE double[n]; not modified
 *   x     DEVICE double[n]; the zero-mean solution (warm_start: initial guess on entry)
 *   info  HOST, may be NULL
 * LAMG_E_NOT_CONVERGED still writes the last iterate and fills info. */
lamg_status lamg_solve(lamg_handle h, const double* b, double* x, lamg_info* info);

/* Batched solves (re-solving for many b is cheap once the setup is done,
 * Section 1).  For each i < count: handle hs[i] solves nrhs[i] right-hand
 * sides stored DEVICE B[i] (n_i x nrhs[i], row-major, RHS index fastest) into
 * DEVICE X[i] of the same shape.  A handle may appear only once.
 *   nrhs[i] == 1, count == 1 (or n_i > 2^18): the single-vector solve of
 *     lamg_solve.
 *   nrhs[i] == 1, count > 1, n_i <= 2^18: all such entries are solved in ONE
 *     persistent launch on hs[0]'s stream: each workgroup takes the next graph
 *     from a queue (largest estimated work first) and runs its whole solve
 *     (the same cycle as lamg_solve, each graph with its own precision, tol,
 *     max_cycles and warm start).  The launch configuration is autotuned: the
 *     first batch of a given shape is solved once per candidate configuration
 *     and the fastest is kept for the process (no tuning when a warm start is
 *     requested); results do not depend on the configuration.
 *   nrhs[i] == k > 1: the multi-vector cycle.  Every level works on n_l x k
 *     blocks; each column has its own recombination coefficients, mean and
 *     convergence test, and stops updating once it meets tol (its mask is
 *     cleared).  The outer loop is R = B - A X in FP64, one cycle from zero on
 *     R - mean(R) (FP64, or FP32 under LAMG_FP32_REFINE), X += correction.  The
 *     handle keeps an n_l x k workspace (reallocated when k changes; requires
 *     n * k < 2^31).
 * infos: HOST[count], may be NULL; for k > 1 it reports the worst column
 * (largest residual, cycles = cycles of the batch).  Statuses as lamg_solve;
 * the first failing entry's status is returned.  All handles must live on the
 * current device. */
lamg_status lamg_solve_batch(int32_t count, const lamg_handle* hs, const int32_t* nrhs,
                             const double* const* B, double* const* X, lamg_info* infos);

/* Allocation-free form of the many-graph persistent solve of lamg_solve_batch
 * (nrhs[i] == 1 for every entry), for callers that cannot allocate device
 * memory during the call: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  The launch's own buffers (the graphs'
 * descriptors, the queue orders and counter, the per-graph results) live in a
 * static device array of the library, one copy per GPU held until the
 * process ends, of LAMG_NOALLOC_MAX_GRAPHS graphs at most (about 2.4 MB);
 * the call allocates no device or pinned host memory and does not autotune
 * (it launches the configuration lamg_solve_batch tuned for the same batch
 * shape, else the first one; results do not depend on it).
 *   count  0 <= count <= LAMG_NOALLOC_MAX_GRAPHS, else LAMG_E_INVALID_ARG
 *          with the reason in lamg_last_error()
 *   hs     HOST[count] distinct handles of graphs with at most 2^18 nodes
 *          (their whole-hierarchy program is made by lamg_setup and by
 *          lamg_set_solve_options); else LAMG_E_INVALID_ARG
 *   B, X   HOST[count] arrays of DEVICE double[n_i]: right-hand sides and
 *          solutions in input node order, as in lamg_solve
 *   infos  HOST[count], may be NULL.
 * Solutions, statuses and infos equal those of lamg_solve_batch on the same
 * handles and right-hand sides.  Every call on one GPU shares that GPU's
 * scratch (the queue counter is cleared by a kernel before each launch), so
 * calls that overlap on one GPU, from several threads or streams, race and
 * must be serialised by the caller. */
#define LAMG_NOALLOC_MAX_GRAPHS 4096
lamg_status lamg_solve_batch_noalloc(int32_t count, const lamg_handle* hs, const double* const* B,
                                     double* const* X, lamg_info* infos);

/* Adjoint edge gradient of a solve x = A^+ b (spec differentiable form):
 * for a loss L with dL/dx = g, the caller solves A lam = g (lamg_solve on the
 * same hierarchy, since A is symmetric) and this kernel forms
 *   grad_w[e] = -(lam[eu[e]] - lam[ev[e]]) (x[eu[e]] - x[ev[e]])
 * for every input edge e.  eu, ev DEVICE int32[m] (indices are not checked
 * here: pass the arrays given to lamg_setup); x, lam DEVICE double[n];
 * grad_w DEVICE double[m] out.  stream: hipStream_t (NULL = null stream). */
lamg_status lamg_edge_gradient(int64_t m, const int32_t* eu, const int32_t* ev, const double* x,
                               const double* lam, double* grad_w, void* stream);

/* Lowest eigenpairs (Section 6.4, the eigensolver: the LAMG solver inside a
 * block Rayleigh-quotient iteration, the alternative that section names to
 * FAS).  Computes the k smallest eigenvalues of A on the zero-sum subspace
 * (the non-zero part of the spectrum of a connected graph's Laplacian) and
 * their eigenvectors by LOBPCG preconditioned with `cycles` LAMG cycles of
 * this hierarchy (its solve options: precision, energy correction).
 *   X      DEVICE double[n * k] row-major (eigenvector index fastest), in:
 *          the initial block (e.g. seeded random; projected to zero-sum
 *          here; its columns must be linearly independent after that),
 *          out: orthonormal eigenvectors in ascending eigenvalue order.
 *   evals  HOST double[k] out, ascending.
 *   tol    stop when ||A x_j - lambda_j x_j||_2 <= tol * lambda_j for all j.
 *   max_iter  LOBPCG iterations at most; cycles >= 1 per preconditioner call.
 *   iters  HOST int32 out (nullable): iterations taken.
 *   resid  HOST double[k] out (nullable): ||A x_j - lambda_j x_j|| / lambda_j
 *          of the returned vectors.
 * 1 <= k <= 8 and 4k <= n, else LAMG_E_INVALID_ARG.  LAMG_E_NOT_CONVERGED
 * still writes the last iterate; LAMG_E_BREAKDOWN when the search space
 * loses rank or a Ritz value or residual is not finite: then X, evals and
 * resid are left untouched and iters holds the iterations run.  Runs on the hierarchy's stream and returns after it.
 * Internally the iterated block has kb = k + min(k, 4) columns (at most n/4);
 * only the first k are tested and returned.  For the call it allocates, through
 * the hierarchy's allocator: eleven n x kb FP64 blocks, about 19 MB of Gram
 * partial sums and the multi-vector cycle workspace for kb columns (the last
 * one is kept by the handle).  It also allocates a few KB of pinned host
 * memory. */
lamg_status lamg_eigs(lamg_handle h, int32_t k, double* X, double* evals, double tol, int32_t max_iter,
                      int32_t cycles, int32_t* iters, double* resid);

/* Change solve-phase options of an existing hierarchy (precision, ec, mu,
 * nu_pre, nu_post, recomb_norm, tol, max_cycles, warm_start, stream);
 * setup-phase fields are ignored. */
lamg_status lamg_set_solve_options(lamg_handle h, const lamg_options* o);

/* Statistics of one level of a hierarchy (Sections 3-4). */
typedef struct lamg_level_stats {
  int64_t nnz;          /* stored off-diagonal entries (each edge twice) */
  int32_t n;            /* nodes */
  int32_t kind;         /* 0 finest, 1 elimination (Section 3.2), 2 aggregation (Section 3.4) */
  int32_t colours;      /* colour classes of the Gauss-Seidel order */
  int32_t hub_colours;  /* of these, the last ones swept by the single-workgroup hub kernel (0: none) */
  int32_t in_tail;      /* 1: relaxed inside the single-workgroup coarse-level kernel */
  int32_t reserved;     /* 0 */
  double gamma;         /* cycle index of the visits from this level to the next (eq. cycle_index; 1 if none) */
  double visits;        /* bodies run at this level per finest-level cycle (the coarsest: its solves) */
} lamg_level_stats;

/* Fill *out for level l in [0, levels) of h (0 = finest).  Host-side only: no
 * device work.  LAMG_E_INVALID_ARG for a NULL argument or l out of range.
 *
 * Diagnostics: with the environment variable LAMG_LOG=1 (read once per
 * process) every setup and solve prints one summary line to stderr; with
 * LAMG_LOG=2 also the level table of each setup and the residual of every
 * cycle.  Setups, solves, batches and eigensolves are marked as roctx ranges
 * ("lamg_setup", "lamg_solve", ...; each level's construction as "lamg_level
 * l"), which rocprofv3 --marker-trace records. */
lamg_status lamg_level_info(lamg_handle h, int32_t l, lamg_level_stats* out);

/* Release a hierarchy; NULL is a no-op. */
void lamg_free(lamg_handle h);

/* Static description of a status code. */
const char* lamg_status_str(lamg_status s);

/* Text of the HIP error behind the last LAMG_E_DEVICE / LAMG_E_OUT_OF_MEMORY
 * returned on the calling thread (and the reason of a size refused by
 * lamg_solve_batch_noalloc; "" if none); valid until the next call. */
const char* lamg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LAMG_H */
