/*
 * stiles.h -- C ABI of the MI355X (gfx950) sparse tile Cholesky library for
 * symmetric positive-definite block-arrowhead matrices with variable
 * bandwidth (sTiles, arXiv 2501.02483).
 *
 * The paper splits sparse Cholesky into reordering, symbolic factorization
 * and numerical factorization (Section II, the three-step list).  Here:
 *   stiles_analyze / stiles_analyze_profile   -- steps 1 and 2, on the host;
 *   stiles_factorize                          -- step 3, on the GPU;
 *   stiles_solve, stiles_logdet               -- uses of the factor.
 * A symbolic object is built once per sparsity pattern and reused for many
 * numerical factorizations with new values (Section III-A: preprocessing is
 * paid once when many factorizations share a structure; Appendix A).
 *
 * Conventions shared by every entry point:
 *  - Sizes and indices are int64_t, 0-based.  Matrices are symmetric and
 *    given by their lower triangle, diagonal included.
 *  - "arrow" is the number of trailing dense rows/columns of the
 *    block-arrowhead matrix (Section I); the n = N - arrow leading rows form
 *    the band part.  The arrow rows always stay last (partial permutation,
 *    Section III-A).
 *  - Pointers named d_* are device pointers on the current HIP device; all
 *    other pointers are host pointers.  The library never allocates device
 *    memory: the caller owns every device buffer (workspaces, values,
 *    right-hand sides, outputs) and must keep it alive while work that uses
 *    it is in flight on the stream.
 *  - Argument errors are reported synchronously by the return value;
 *    stiles_last_error_arg() then gives the 1-based position of the
 *    offending argument.  Device work is asynchronous on the given stream.
 *  - A numerical failure (a pivot that is not positive, i.e. the matrix is
 *    not SPD) is detected on the device and reported by stiles_factor_info
 *    with the LAPACK potrf convention (1-based index, in the permuted order,
 *    of the first column whose pivot failed).
 */
#ifndef STILES_H
#define STILES_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t stiles_status;
#define STILES_OK 0
#define STILES_EINVAL (-1)   /* bad argument; see stiles_last_error_arg()          */
#define STILES_ENOTSUP (-2)  /* valid request the library does not support          */
#define STILES_ENOMEM (-3)   /* caller-provided workspace too small                 */
#define STILES_EDEVICE (-4)  /* a HIP call failed                                   */
#define STILES_ESTATE (-5)   /* object in the wrong state (e.g. factor failed)      */
#define STILES_ETIMEOUT (-6) /* a wait of the persistent executor passed its deadline
                                (stiles_factor_set_wait_limit): the launch was
                                abandoned and the factor is marked failed          */

/* Orderings (Section III-A).  AUTO tries partial RCM on the band part (the
 * arrow rows are left in place) and keeps it only if it reduces the number
 * of stored tiles (a method that brings no improvement is not used).
 * ADAPTABLE_ND does the same, then cuts the band part into nd_parts
 * partitions (0: the count with the shortest estimated dependency chain)
 * separated by blocks of rows as wide as the local bandwidth; the separators
 * move to the end of the band part and join the arrow, the partitions are
 * factored concurrently, the last one in reverse row order.  It is used only
 * if a feasible cut exists (else the ordering falls back as AUTO).  AMD
 * (approximate minimum degree on the band part, the arrow rows staying last;
 * for irregular patterns) is kept only if L then has fewer tiles than in the
 * input order; it keeps no band shape, so it is not combined with the
 * partitions.  For row-profile input only NONE, AUTO (= NONE) and
 * ADAPTABLE_ND are supported. */
#define STILES_ORDER_AUTO 0
#define STILES_ORDER_NONE 1
#define STILES_ORDER_PARTIAL_RCM 2
#define STILES_ORDER_ADAPTABLE_ND 3
#define STILES_ORDER_AMD 4

/* Precisions of the numerical factorization. */
#define STILES_FP64 0     /* every step in FP64                                     */
#define STILES_MIXED32 1  /* band/arrow tile updates in FP32 on MFMA (under adaptable
                             ND also the separator rows' partial sums); POTRF, TRSM,
                             the arrow-corner accumulation, logdet and refinement
                             FP64                                                   */
#define STILES_MIXED32_FULL 2 /* as STILES_MIXED32, and the arrow-corner accumulation
                             (the partial products summed into the corner tiles) also
                             in FP32: the placement the FP64 corner avoids, kept to
                             measure what that choice buys                          */

typedef struct stiles_symbolic stiles_symbolic; /* opaque, host memory, immutable  */
typedef struct stiles_factor stiles_factor;     /* opaque host handle bound to a
                                                   caller-owned device workspace   */

typedef struct stiles_opts {
  int32_t tile;           /* tile size T: 32 or 64 (0 = 64)                          */
  int32_t ordering;       /* STILES_ORDER_*                                          */
  int32_t tree_min_ratio; /* arrow-corner tree reduction is used when the number of
                             accumulations is >= tree_min_ratio x the number of
                             partial workers (Section IV-A recommends 2); <= 0
                             disables the tree (sequential accumulation chain)       */
  int32_t chunk;          /* tile products per accumulation task, at most 32
                             (0: 12 at T=64, 16 at T=32)                              */
  double refine_tol;      /* mixed mode: a right-hand side stops refining once its
                             backward error is <= refine_tol (0 = 2^-52 (w + a), w the
                             largest band half-width before reordering, a the arrow
                             width), or when a step no longer halves it (the better
                             of the last two iterates is kept), or at the step limit */
  int32_t refine_max_iter;/* mixed mode: at most this many refinement steps per
                             right-hand side (0 = 30)                                */
  int32_t nd_parts;       /* ADAPTABLE_ND: number of partitions, 2..64 (0 = choose:
                             the shortest-chain count and two smaller ones are
                             analyzed, and the least estimated factorization time
                             -- chain steps against executed flops -- wins)       */
  int32_t sched_workers;  /* ticket order of the task DAGs: the start order of a list
                             schedule (longest remaining path first) on this many
                             workgroups (0 = 512, a full MI355X launch), used for a DAG
                             whose critical path is at least half its work per
                             workgroup and for batches; otherwise, and with -1, the
                             order by earliest start with unlimited workgroups.  Only
                             the speed depends on it: every order gives bitwise the
                             same results                                            */
  int32_t ublock;         /* 2 x 2 blocked tile updates (two tile rows of two adjacent
                             band tile columns share their operand tiles): columns per
                             block task, 1..15; 0 or -1 (default): no blocks, every
                             update is a single-tile chain (measured faster on the
                             default workloads)                                      */
} stiles_opts;

typedef struct stiles_symbolic_info {
  int64_t N, n, arrow;    /* order, band part, arrow width of P A P^T (with adaptable
                             ND the separators count as arrow rows)                  */
  int32_t tile;           /* tile size T                                             */
  int32_t ordering_used;  /* STILES_ORDER_NONE, _PARTIAL_RCM, _ADAPTABLE_ND (the
                             last possibly on top of partial RCM) or _AMD            */
  int64_t tile_rows;      /* band tile rows + arrow tile rows                        */
  int64_t band_tile_rows;
  int64_t tiles;          /* stored T x T tiles of the factor                       */
  int64_t nnz_L;          /* entries inside the envelope of P A P^T (lower; the
                             layout of stiles_factor_extract)                        */
  double flops_alg;       /* sum_j (eta_j + 1)^2, eta_j = sub-diagonal count of col j
                             over the envelope before adaptable ND (the same work
                             for every partition count; ND's extra fill is in
                             flops_exec)                                             */
  double flops_exec;      /* flops the tile kernels execute (padded tiles)           */
  int64_t factor_tasks;   /* tasks in the factorization DAG                          */
  int64_t solve_tasks;    /* tasks in the solve DAG                                  */
  int64_t corner_accumulations; /* tile products summed into the arrow-corner tile(s)
                                   from band columns (about one per band tile row)   */
  int32_t tree_used;      /* 1 if the arrow corner is reduced by a tree              */
  int32_t nd_parts;       /* partitions of the adaptable ND ordering (1 if none)     */
  int64_t nnz_L_alg;      /* entries inside the envelope before adaptable ND: nnz(L)
                             of the method, the basis of flops_alg; the algorithmic
                             work of a solve is 4 nnz_L_alg flops per right-hand side
                             (two sweeps, a multiply and an add per entry).  Equals
                             nnz_L when adaptable ND is not used                     */
  int64_t update_blocks;  /* 2 x 2 update blocks of the factorization DAG (ublock)   */
  int64_t nd_chain;       /* adaptable ND: estimated chain of the plan in tile steps
                             (longest partition, separator levels, arrow); 0 if none */
} stiles_symbolic_info;

typedef struct stiles_solve_report {
  int32_t iterations;     /* largest number of refinement steps any right-hand side
                             took (0 in FP64 mode)                                   */
  int32_t converged;      /* 1 if every right-hand side met the stopping test        */
  double backward_error;  /* max over right-hand sides of ||b-Ax||/(||A|| ||x||+||b||),
                             inf-norms, of the returned x; mixed mode only (else -1) */
  double* backward_errors;/* optional (set by the caller, may be NULL): host array of
                             nrhs doubles that receives the backward error of each
                             right-hand side's returned x (-1 in FP64 mode)          */
  int32_t* rhs_iterations;/* optional host array of nrhs: refinement steps applied to
                             each right-hand side (0 in FP64 mode)                   */
} stiles_solve_report;

/* Fill *opts with the defaults (tile 64, AUTO ordering, tree ratio 2). */
void stiles_default_opts(stiles_opts* opts);

/* Human-readable name of a status code (static string). */
const char* stiles_status_string(stiles_status s);

/* 1-based index of the argument rejected by the last call that returned
 * STILES_EINVAL on this thread (0 if none). */
int32_t stiles_last_error_arg(void);

/*
 * Reordering + symbolic factorization from a lower-triangle CSC pattern
 * (the paper's CTSF reads CSC input, Section III-B).
 *   N        order of A (N >= 1);  arrow  trailing dense rows (0 <= arrow <= N)
 *   colptr   N+1 entries, colptr[0] = 0, non-decreasing
 *   rowind   colptr[N] row indices; in each column strictly increasing, all
 *            >= the column index (lower triangle) and < N; each column must
 *            hold its diagonal entry
 *   opts     may be NULL (defaults)
 *   out      receives a new symbolic object (free with stiles_symbolic_destroy)
 * Values passed later to stiles_factorize are in this CSC order.
 * Errors: EINVAL (argument index in stiles_last_error_arg), ENOTSUP (tile).
 */
stiles_status stiles_analyze(int64_t N, int64_t arrow, const int64_t* colptr, const int64_t* rowind,
                             const stiles_opts* opts, stiles_symbolic** out);

/*
 * Same, for a band-plus-arrow envelope given by its profile: band row i
 * (0 <= i < n_band) has nonzeros in columns first_col[i]..i
 * (0 <= first_col[i] <= i), the arrow rows are dense.  Values passed to
 * stiles_factorize are in row-profile order: row 0, row 1, ..., row N-1,
 * each from its first column to its diagonal (arrow row n_band + r holds
 * n_band + r + 1 entries).  Orderings: NONE and AUTO keep the input order
 * (the band is already in envelope order, so partial RCM is not tried);
 * ADAPTABLE_ND cuts the band into partitions as described above (the values
 * stay in the input's row-profile order; the permutation is applied on the
 * device).  PARTIAL_RCM and AMD are rejected (ENOTSUP, argument 4).
 */
stiles_status stiles_analyze_profile(int64_t n_band, int64_t arrow, const int64_t* first_col,
                                     const stiles_opts* opts, stiles_symbolic** out);

stiles_status stiles_symbolic_query(const stiles_symbolic* sym, stiles_symbolic_info* info);

/* perm[i] = original index of permuted row i (N entries, host). */
stiles_status stiles_symbolic_perm(const stiles_symbolic* sym, int64_t* perm);

void stiles_symbolic_destroy(stiles_symbolic* sym);

/*
 * Read-only view of the plan inside a symbolic object, for tests and tools
 * (e.g. a host emulation of the task DAG).  `which`:
 *   0 factorization tasks (int32, 8 per task: type|flags, tile, a, b, c,
 *     successor begin, successor end, predecessor count), in schedule order
 *   1 factorization successor lists (int32)   2 factorization tile pairs (int32, 2 per pair)
 *   3 solve tasks   4 solve successor lists   5 solve pairs (tile, vector block)
 *   6 tile-row pointers (int32, tile_rows + 1)  7 tile columns (int32, tiles)
 *   8 first permuted row of each tile row (int64)  9 real rows per tile row (int32)
 *   10 number of tree partial slots (int32, 1 element)
 *   11 selected-inversion tasks  12 their successor lists  13 their operand
 *     lists (int32; built on first use)
 *   14 merged factorization + solve tasks  15 their successor lists  16 their
 *     pairs (the factorization pairs, then the solve pairs; built on first use)
 *   17 per tile (int32): 1 if an entry of A (P A P^T) falls in it or it is a
 *     diagonal tile, 0 if it holds fill only
 * With out == NULL, *count receives the number of elements; otherwise *count
 * is the capacity of out (elements) and receives the number copied.
 * EINVAL: unknown `which` (argument 2) or capacity too small (argument 4).
 */
stiles_status stiles_symbolic_export(const stiles_symbolic* sym, int32_t which, void* out, int64_t* count);

/*
 * Device workspace bytes for one resident factor of `sym` in the given
 * precision, able to solve with up to nrhs_max right-hand sides at once.
 * The workspace holds the tile store of L (CTSF), the inverse diagonal tiles,
 * the partial sums of the arrow-corner tree, the task tables of the
 * factorization and solve DAGs and their progress counters.
 */
stiles_status stiles_workspace_size(const stiles_symbolic* sym, int32_t precision, int64_t nrhs_max,
                                    size_t* bytes);

/*
 * Bind a factor handle to a caller-owned device workspace (>= the size above,
 * 256-byte aligned) and upload the static task tables into it (asynchronous on
 * `stream`; the symbolic object must outlive the handle).  One workspace holds
 * one factor; calls that use the same workspace must be ordered on one stream.
 */
stiles_status stiles_workspace_init(const stiles_symbolic* sym, int32_t precision, int64_t nrhs_max,
                                    void* d_ws, size_t ws_bytes, hipStream_t stream,
                                    stiles_factor** out);

/*
 * Numerical factorization PAP^T = L L^T (Algorithm 1, left-looking, over the
 * nonzero tiles only; arrow-corner accumulations by a reduction tree,
 * Algorithm 3).  d_values: FP64 values in the order fixed at analysis (CSC or
 * row profile); read by the first kernel, may be reused once the stream has
 * passed this call.  Asynchronous; failures surface in stiles_factor_info.
 */
stiles_status stiles_factorize(stiles_factor* f, const double* d_values, hipStream_t stream);

/*
 * Many independent factorizations in one persistent launch (Appendix A:
 * concurrent factorizations).  factors[i] must use distinct workspaces and
 * share one tile size.  stiles_batch_create builds one ticket order for the
 * union of the matrices' task graphs (a list schedule on the launch's
 * workgroups, longest remaining path first; with opts.sched_workers = -1
 * the per-matrix schedules merged by start estimate) and uploads it, with
 * copies of the task tables whose waits are single-stage (no pivot chain
 * bounds a batch), into d_batch_ws (>= stiles_batch_workspace_size bytes,
 * 256-byte aligned, caller-owned, kept alive with the batch); it
 * synchronizes the stream once.
 * stiles_batch_factorize then scatters every matrix's values (one launch over
 * all tiles when every matrix was analyzed from a row profile) and runs all
 * factorizations in one launch (asynchronous); it may be called again with
 * new values.  d_values is a host array of `count` device pointers; when it
 * differs from the previous call's, the call waits for the stream once to
 * upload it.  Each result is bitwise identical to a single stiles_factorize
 * of the same matrix with the same symbolic object (the accumulation order of
 * every tile is fixed by the plan, not by the schedule).
 * stiles_batch_logdet writes the log-determinant of every matrix of the batch
 * to d_out[0..count) (device, FP64; NaN for a matrix whose factorization
 * failed) in two launches; each value is bitwise identical to stiles_logdet
 * of that factor.  STILES_ESTATE if a factor is not factorized.
 * stiles_factorize_batch = create + factorize + destroy.
 */
/*
 * Out-of-core (streamed) factorization of a band-plus-arrow envelope given
 * by its profile (as stiles_analyze_profile, natural order), for a factor
 * larger than the device memory one wants to commit (the paper leaves
 * matrices beyond device memory to future work, Sections IV-B and VI).
 * The band rows are processed in consecutive segments of seg_rows rows:
 * each segment is factored in core as an arrowhead matrix whose band part is
 * the segment's rows followed by the next segment's rows that couple back
 * into it (with their own profiles) and whose arrow is the true arrow; the
 * trailing factor of that matrix (those coupling rows and the arrow) gives
 * the segment's Schur complement (L_c L_c^T, on the device), which seeds the
 * next segment.  Only one segment is resident at a time; the assembly of a
 * segment's values and the scatter of its factor use up to 16 host threads,
 * and the next segment's symbolic analysis runs on one more meanwhile.
 *   h_values  host, FP64, the matrix in row-profile order (as for
 *             stiles_factorize with a row-profile analysis)
 *   seg_rows  band rows per segment; at least the band's reach (every row
 *             coupling back across a segment boundary must lie in the next
 *             segment), else EINVAL (argument 5)
 *   tile      0, 32 or 64
 *   h_L       host, receives L in the same row-profile layout
 *   logdet    receives log det A (NaN if not SPD); info: 0, or the 1-based
 *             row of the first non-positive pivot
 *   peak_device_bytes  optional: the largest device footprint of a segment
 * This entry point allocates device memory itself (hipMalloc/hipFree, freed
 * before it returns) and synchronizes the stream once per segment.
 */
stiles_status stiles_factorize_ooc(int64_t n_band, int64_t arrow, const int64_t* first_col, const double* h_values,
                                   int64_t seg_rows, int32_t tile, double* h_L, double* logdet, int64_t* info,
                                   size_t* peak_device_bytes, hipStream_t stream);

typedef struct stiles_batch stiles_batch;
stiles_status stiles_batch_workspace_size(int32_t count, stiles_factor* const* factors, size_t* bytes);
stiles_status stiles_batch_create(int32_t count, stiles_factor* const* factors, void* d_batch_ws,
                                  size_t batch_ws_bytes, hipStream_t stream, stiles_batch** out);
stiles_status stiles_batch_factorize(stiles_batch* batch, const double* const* d_values, hipStream_t stream);
stiles_status stiles_batch_logdet(stiles_batch* batch, double* d_out, hipStream_t stream);
void stiles_batch_destroy(stiles_batch* batch);
stiles_status stiles_factorize_batch(int32_t count, stiles_factor* const* factors,
                                     const double* const* d_values, void* d_batch_ws,
                                     size_t batch_ws_bytes, hipStream_t stream);

/* Waits for the stream, then sets *info to 0 (success) or the 1-based
 * permuted column of the first non-positive pivot.  Returns STILES_ETIMEOUT
 * (and *info = -1) when a launch of this factor since its last scatter was
 * abandoned at the executor's wait deadline (see below); the factor then
 * counts as failed until it is factorized again. */
stiles_status stiles_factor_info(stiles_factor* f, hipStream_t stream, int64_t* info);

/* Deadline of every wait of the persistent executor for a task's
 * predecessors (Algorithm 2's progress check), in seconds; 0 restores the
 * default of 10 s; at most 3600 (EINVAL otherwise, argument 2).  A correct
 * plan never waits that long; a wait that does sets an abort flag of the
 * launch, after which every workgroup skips its remaining tasks and exits
 * normally: the launch returns instead of hanging the device, the factor's
 * results are NaN, and stiles_factor_info returns STILES_ETIMEOUT.  It
 * applies to the factorization, solve, merged, batch (the first factor's
 * limit) and selected-inversion launches of this factor. */
stiles_status stiles_factor_set_wait_limit(stiles_factor* f, double seconds);

/*
 * Solve A X = B in place.  d_B: N x nrhs column-major, leading dimension
 * ldb >= N, original (unpermuted) ordering.  1 <= nrhs <= nrhs_max of the
 * workspace.  FP64 mode: one forward and one backward sweep over the tiles.
 * Mixed mode: the same, followed by FP64 iterative refinement against the
 * resident original A, each right-hand side until its own stopping test
 * holds (stiles_opts.refine_tol); the stream is synchronized once per step to
 * test convergence.  report may be NULL; its optional per-right-hand-side
 * arrays are filled when set.  If the factorization failed, the
 * result is NaN (and ESTATE is returned when the failure is already known).
 */
stiles_status stiles_solve(stiles_factor* f, int64_t nrhs, double* d_B, int64_t ldb, hipStream_t stream,
                           stiles_solve_report* report);

/*
 * Factorization and solve in one persistent launch: stiles_factorize(f,
 * d_values) followed by stiles_solve(f, nrhs, d_B, ldb), with the two task
 * graphs merged, so that tile rows whose factor is final are solved while
 * the rest of the matrix is still being factored (the forward sweep of the
 * adaptable-ND partitions overlaps the factorization of the separators).
 * Results are bitwise those of the two separate calls (the same tasks in the
 * same accumulation order).  In mixed precision the launch's solve is the
 * first iterate of the FP64 refinement, which then runs as in stiles_solve
 * (the call waits for it; use stiles_solve for the per-RHS report).
 * d_B: N x nrhs column-major (ldb >= N), original ordering, overwritten by X;
 * right-hand sides beyond the first 16 are solved by ordinary solve sweeps
 * (refined in mixed mode) after the launch.  If the factorization fails, X
 * is NaN and stiles_factor_info reports the column.  The timing hook's
 * factorization event pair brackets the merged launch.
 */
stiles_status stiles_factorize_solve(stiles_factor* f, const double* d_values, int64_t nrhs, double* d_B, int64_t ldb,
                                     hipStream_t stream);

/* logdet A = 2 sum log L_ii, written to *d_out (one FP64 on the device).
 * Deterministic fixed-shape reduction.  NaN if the factorization failed. */
stiles_status stiles_logdet(stiles_factor* f, double* d_out, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * log-determinant as stiles_logdet, bitwise, with the per-tile-row partial
 * sums kept in a fixed device array of the library instead of the factor's
 * workspace.  The array holds STILES_STATIC_LOGDET_MAX_ROWS tile rows
 * (512 KiB per GPU the library runs on, held until the process ends); a
 * factor with more tile rows (stiles_symbolic_info.tile_rows) is rejected
 * with STILES_ENOTSUP before anything is launched.  The call allocates
 * nothing; its address is looked up once per device (with that device
 * current).  Every call on one GPU shares the array: calls that overlap on
 * one GPU (different streams, or host threads) race and must be serialized
 * by the caller.  d_out, the factor's state and the failure value (NaN) as
 * for stiles_logdet. */
#define STILES_STATIC_LOGDET_MAX_ROWS 65536
stiles_status stiles_logdet_static(stiles_factor* f, double* d_out, hipStream_t stream);

/* Copy the factor L out of the tile store into d_L, in row-profile order of
 * the permuted envelope: row i of P A P^T holds columns f_i..i, f_i being the
 * first column of row i in P A P^T (for stiles_analyze_profile input with the
 * natural ordering this is exactly the value layout of d_values).  d_L holds
 * nnz_L doubles (stiles_symbolic_info); envelope entries outside the stored
 * tiles (structural zeros of L under adaptable ND) are written as zero.  For
 * tests and for callers that want L itself. */
stiles_status stiles_factor_extract(stiles_factor* f, double* d_L, hipStream_t stream);

/* Profiling hook: when enabled, the library records a pair of HIP events on
 * the stream around every executor launch of this factor (which = 0: the
 * factorization DAG kernel; which = 1: the solve DAG kernel).
 * stiles_factor_kernel_ms waits for the last recorded pair and returns its
 * elapsed time in milliseconds (ESTATE if timing is off or nothing recorded).
 * For a batch, the factorization pair of the batch's first factor brackets
 * the one batched executor launch. */
stiles_status stiles_factor_set_timing(stiles_factor* f, int32_t enable);
stiles_status stiles_factor_kernel_ms(stiles_factor* f, int32_t which, float* ms);

/* Profiling hook: per-task trace.  When d_factor_trace (d_solve_trace) is not
 * NULL, every task of the factorization (solve) DAG writes four uint64 at
 * index 4*task: the device wall clock (100 MHz) when a workgroup took its
 * ticket, when its predecessors were complete, when it finished, and
 * (workgroup << 32 | task type << 24 | ticket mod 2^24).  Buffers hold 32 bytes per task
 * (stiles_symbolic_info: factor_tasks, solve_tasks); NULL switches it off. */
stiles_status stiles_factor_set_trace(stiles_factor* f, void* d_factor_trace, void* d_solve_trace,
                                      hipStream_t stream);

/* The same per-task trace for the merged launch of stiles_factorize_solve
 * (32 bytes per task of that DAG: stiles_symbolic_export kind 14 holds 8
 * words per task); NULL switches it off. */
stiles_status stiles_factor_set_merged_trace(stiles_factor* f, void* d_trace, hipStream_t stream);

/* Upper bound on the workgroups a factorization launch uses (0 = fill the
 * GPU).  Lets several factorizations on different streams share the GPU.
 * A batch launch takes the cap of its first factor. */
stiles_status stiles_factor_set_max_workgroups(stiles_factor* f, int32_t max_wg);

/* Releases the host handle (the caller frees the workspace). */
void stiles_factor_release(stiles_factor* f);

/*
 * Selected inversion: the entries of Sigma = A^{-1} on the stored tiles of
 * the factor, in particular its diagonal (inverses of block-arrowhead
 * matrices are one of the tasks Section I lists for this class; INLA needs
 * the diagonal, the posterior marginal variances).  Computed from a resident
 * FP64 factor by the block form of the Takahashi recursion, tile column by
 * tile column in reverse elimination order, as one persistent launch over a
 * task DAG of tile products on the FP64 matrix cores.  In mixed precision
 * it inverts the computed factor (no refinement).
 *
 * stiles_selinv_workspace_size: device bytes for Sigma (one T x T tile per
 *   stored tile of L), two per-tile partial stores of the same size, and the
 *   task tables.  The task plan is built on first use and kept in `sym`.
 * stiles_selinv_create: binds the factor f (which must outlive the handle) to
 *   a caller-owned workspace (>= that size, 256-byte aligned) and uploads the
 *   task tables (synchronizes the stream once).
 * stiles_selinv_compute: computes Sigma from f's current factor (asynchronous;
 *   ESTATE if f is not factorized or its factorization is known to have
 *   failed).  Refactorizing f makes Sigma stale until the next compute.
 * stiles_selinv_diag: d_diag[i] = (A^{-1})_ii, i in the original ordering
 *   (N doubles, device; NaN if the factorization failed).
 * stiles_selinv_extract: the selected entries in the layout of
 *   stiles_factor_extract (nnz_L doubles, row-profile order of the permuted
 *   envelope; zero outside the stored tiles).
 * stiles_selinv_query: task count, algorithmic flops sum_j 2 eta_j (eta_j + 1)
 *   over the envelope before adaptable ND, and executed tile-product flops
 *   (each pointer may be NULL).
 * stiles_selinv_set_timing / stiles_selinv_kernel_ms: a pair of HIP events
 *   around each compute launch, as for the factor.
 * stiles_selinv_set_trace: per-task trace of the compute launch in the format
 *   of stiles_factor_set_trace (32 bytes per task; NULL switches it off).
 * Calls that share a handle must be ordered on one stream.
 */
typedef struct stiles_selinv stiles_selinv;
stiles_status stiles_selinv_query(const stiles_symbolic* sym, int64_t* tasks, double* flops_alg, double* flops_exec);
stiles_status stiles_selinv_workspace_size(const stiles_symbolic* sym, size_t* bytes);
stiles_status stiles_selinv_create(stiles_factor* f, void* d_ws, size_t ws_bytes, hipStream_t stream,
                                   stiles_selinv** out);
stiles_status stiles_selinv_compute(stiles_selinv* si, hipStream_t stream);
stiles_status stiles_selinv_diag(stiles_selinv* si, double* d_diag, hipStream_t stream);
stiles_status stiles_selinv_extract(stiles_selinv* si, double* d_out, hipStream_t stream);
stiles_status stiles_selinv_set_timing(stiles_selinv* si, int32_t enable);
stiles_status stiles_selinv_kernel_ms(stiles_selinv* si, float* ms);
stiles_status stiles_selinv_set_trace(stiles_selinv* si, void* d_trace, hipStream_t stream);
void stiles_selinv_destroy(stiles_selinv* si);

#ifdef __cplusplus
}
#endif

#endif /* STILES_H */
