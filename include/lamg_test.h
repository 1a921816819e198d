/* lamg_test.h -- inspection and per-kernel entry points of the LAMG library,
 * used by the parity tests.  Not part of the solver contract of lamg.h.
 *
 * Level l = 0 is the finest level.  Every level is stored in colour-major
 * node order (colour class, then the previous node id), its CSR holds the
 * positive off-diagonal weights w_uv with columns ascending, and the
 * diagonal a_uu is the row sum of the weights (Section 1, eq. lap).
 * Arrays marked HOST are written by copying from the device; DEVICE pointers
 * are read/written on the GPU.  Functions return a lamg_status.
 */
#ifndef LAMG_TEST_H
#define LAMG_TEST_H

#include "lamg.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Number of levels of a hierarchy (>= 1). */
int lamg_t_num_levels(lamg_handle h);

/* 1 when the coarsest level is solved by relaxation sweeps, 0 when densely. */
int lamg_t_coarsest_relax(lamg_handle h);

/* dims[8] HOST: n, nnz (directed off-diagonal entries), type (0 finest,
 * 1 produced by elimination, 2 produced by aggregation), colours, |F| of the
 * elimination that produced it, test vectors K used when aggregating it,
 * aggregation stage kept (1 or 2), number of rows longer than 64. */
lamg_status lamg_t_level_dims(lamg_handle h, int l, int64_t* dims);

/* Cycle index used for visits from level l to level l+1 (eq. cycle_index). */
double lamg_t_level_gamma(lamg_handle h, int l);

/* HOST copies of level l: row_ptr[n+1], col[nnz], val[nnz], diag[n],
 * colour_ptr[ncol+1], perm[n] (node order: perm[new] = id before ordering).
 * Any pointer may be NULL. */
lamg_status lamg_t_level_export(lamg_handle h, int l, int32_t* row_ptr, int32_t* col, double* val, double* diag,
                                int32_t* colour_ptr, int32_t* perm);

/* HOST int32[n_{l-1}]: for l produced by aggregation the aggregate of each
 * fine node; for elimination the coarse node of each fine node, -1 for F. */
lamg_status lamg_t_transfer_export(lamg_handle h, int l, int32_t* out);

/* Aggregation quantities of level l as the fine side (Sections 3.3-3.4):
 * tv[n*K] relaxed test vectors, aff[nnz] affinities (eq. cuv), ok[nnz]
 * energy-ratio admissibility (eq. qut), weak[nnz], hub[n], state[n] (0
 * undecided, 1 seed, 2 associate, 3 dummy), scal[5] = delta_1, alpha_1,
 * alpha_2, stage, energy ratio of the last test-vector sweep.  HOST arrays;
 * any may be NULL. */
lamg_status lamg_t_agg_export(lamg_handle h, int l, double* tv, double* aff, uint8_t* ok, uint8_t* weak,
                              uint8_t* hub, int32_t* state, double* scal);

/* One FP64 cycle (Section 4.2) on the finest level in colour-major order:
 * DEVICE b_perm[n] (zero-sum) and x_perm[n] (updated in place). */
lamg_status lamg_t_cycle(lamg_handle h, const double* b_perm, double* x_perm);

/* One FP64 multi-vector cycle (Section 4.2, every column with its own
 * recombination coefficients and mean) on the finest level in colour-major
 * order: DEVICE b_perm[n x k] and x_perm[n x k] row-major (right-hand side
 * index fastest; x updated in place).  Allocates the k-column workspace on
 * first use. */
lamg_status lamg_t_mv_cycle(lamg_handle h, int32_t k, const double* b_perm, double* x_perm);

/* Per-column results of the last multi-vector solve on h with k columns
 * (HOST outputs [k]): cycles the column iterated, final relative residual,
 * removed mean of its right-hand side.  LAMG_E_INVALID_ARG if the last
 * multi-vector solve had another k. */
lamg_status lamg_t_mv_columns(lamg_handle h, int32_t k, int32_t* cycles, double* rel, double* removed_mean);

/* Launch configuration of the persistent many-graph solve (lamg_solve_batch
 * with count > 1): config in [0, LAMG_T_BATCH_CONFIGS) forces that
 * configuration (LDS staging budget 64 / 96 / 128 / 152 KB, 1 or 2 workgroups
 * per compute unit, largest-work-first or input queue order); -1 restores the
 * autotuner, which times every configuration on the first batch of each shape
 * (every graph capped at two cycles) and keeps the fastest, also in the file
 * named by the environment variable LAMG_TUNE_CACHE when set (read before
 * the first tuning of a process, appended after each).  Process-wide; not
 * thread-safe.  LAMG_E_INVALID_ARG outside [-1, LAMG_T_BATCH_CONFIGS). */
#define LAMG_T_BATCH_CONFIGS 10
lamg_status lamg_t_batch_config(int32_t config);

/* Coarsest-level solve x = (A_L + (mean diag / n_L) 1 1^T)^-1 b, DEVICE [n_L]
 * (dense coarsest levels only). */
lamg_status lamg_t_coarsest_solve(lamg_handle h, const double* b, double* x);

/* Standalone kernels on a DEVICE CSR whose nodes are already in colour-major
 * order with colour classes HOST cptr[ncol+1]:
 *   lamg_t_gs:       `sweeps` multicolour Gauss-Seidel sweeps (eq. gs), b may be NULL (b = 0);
 *   lamg_t_gs32:     the same in FP32;
 *   lamg_t_residual: r = b - A x. */
lamg_status lamg_t_gs(int32_t n, const int32_t* rp, const int32_t* ci, const double* val, const double* diag,
                      int32_t ncol, const int32_t* cptr, const double* b, double* x, int32_t sweeps, void* stream);
lamg_status lamg_t_gs32(int32_t n, const int32_t* rp, const int32_t* ci, const float* val, const float* diag,
                        int32_t ncol, const int32_t* cptr, const float* b, float* x, int32_t sweeps, void* stream);
lamg_status lamg_t_residual(int32_t n, const int32_t* rp, const int32_t* ci, const double* val, const double* diag,
                            const double* b, const double* x, double* r, void* stream);

/* Greedy colouring (first fit in priority order: degree desc, hash(seed,
 * level, id) asc, id asc) on a DEVICE CSR, computed as a topological sweep
 * over the priority order; DEVICE colour[n] out. */
lamg_status lamg_t_colour(int32_t n, const int32_t* rp, const int32_t* ci, uint64_t seed, int32_t level,
                          int32_t* colour, void* stream);

/* The setup's stable LSD radix sort (8-bit digits, keys compared on bits
 * [0, endbit), 1 <= endbit <= key bits) and exclusive scan, on DEVICE arrays
 * of n elements (out arrays must not overlap the inputs).  Pairs of 64-bit
 * keys and doubles (sparse assembly), of 32-bit keys and ints (renumbering,
 * aggregate lists), double keys alone (ascending, -0 before +0: the stage-1
 * quantile); scan: out[0] = 0, out[i+1] = in[0] + ... + in[i] (n + 1 outputs).
 * Run on the null stream and return after it; temporaries from hipMalloc. */
lamg_status lamg_t_sort_pairs64(int64_t n, const uint64_t* keys, const double* vals, uint64_t* keys_out,
                                double* vals_out, int32_t endbit);
lamg_status lamg_t_sort_pairs32(int64_t n, const uint32_t* keys, const int32_t* vals, uint32_t* keys_out,
                                int32_t* vals_out, int32_t endbit);
lamg_status lamg_t_sort_f64(int64_t n, const double* keys, double* keys_out);
lamg_status lamg_t_excl_scan(int64_t n, const int32_t* in, int32_t* out);

/* Hub sweep of level l (Section 3.1.1, eq. gs, multicolour order): out[4] =
 * first hub colour (-1: the level's sweeps do not take the hub path), first
 * hub row, hub rows, hub-to-hub entries.  HOST out. */
lamg_status lamg_t_hub_info(lamg_handle h, int32_t l, int64_t* out);

/* `sweeps` GS sweeps of the solve on level l of a hierarchy, hub path where
 * taken: DEVICE b (may be NULL: b = 0) and x of n_l entries in the level's
 * colour order, FP64 (precision 0, the level's FP64 matrix) or FP32
 * (precision 1, its FP32 copy). */
lamg_status lamg_t_level_gs(lamg_handle h, int32_t l, int32_t precision, int32_t sweeps, const void* b, void* x);
/* The same from a zero iterate as the cycle runs it below the finest level:
 * x is zero-filled here and the first sweep skips the gathers of colours not
 * yet relaxed (they hold +0); the result must equal lamg_t_level_gs on a
 * zero x bit for bit. */
lamg_status lamg_t_level_gs_zero(lamg_handle h, int32_t l, int32_t precision, int32_t sweeps, const void* b, void* x);

/* Instrumentation of the relaxation kernel (Section 3.1.1, eq. gs) and of the
 * residual kernel.  lamg_t_prof_enable(1) clears the counters and brackets
 * every later launch with HIP events on the launch's stream; kernel ids:
 * 0 GS FP64, 1 residual FP64, 2 GS FP32, 3 residual FP32, 4..7 the same
 * four for the multi-vector kernels, 8 / 9 the hub sweep (FP64 / FP32; its
 * colours are not in 0 / 2), 10 / 11 the aggregation restriction, 12 / 13 the
 * aggregation interpolation, 14 / 15 the single-workgroup tail launches
 * (single-vector cycles; no bytes counted: latency-bound).  lamg_t_prof_read waits for the recorded events and returns the summed kernel time (ms), the
 * number of launches and their algorithmic bytes (HOST outputs). */
void lamg_t_prof_enable(int on);
lamg_status lamg_t_prof_read(int kernel, double* ms, int64_t* launches, int64_t* bytes);

#ifdef __cplusplus
}
#endif
#endif /* LAMG_TEST_H */
