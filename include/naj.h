/*
 * naj.h -- C ABI of the MI355X (gfx950) solver for consistent symmetric
 * positive semidefinite systems Q x = b by the Nesterov-accelerated,
 * adaptively restarted Jacobi-type method of Liang, Pang, Toh and Yang,
 * "Nesterov's accelerated Jacobi-type methods for large-scale symmetric
 * positive semidefinite linear systems" (arXiv 2407.03272).
 *
 * The method (Algorithm 3, Section 3): with a diagonal J such that J - Q is
 * positive semidefinite (default: eq. (J-diag), J_kk = Q_kk + sum_{j!=k}|Q_kj|),
 *     x^t     = y^t + J^{-1} (b - Q y^t)
 *     restart when t > K_re + K_l and <Q y^t - b, x^t - x^{t-1}> >= 0:
 *             K_re = t, K_{l+1} = 2 K_l, alpha_{t+1} = 1, y^{t+1} = x^{t-1}, x^t = x^{t-1}
 *     else    alpha_{t+1} = (1 + sqrt(1 + 4 alpha_t^2)) / 2,
 *             y^{t+1} = x^t + (alpha_t - 1)/alpha_{t+1} (x^t - x^{t-1})
 * starting from x^0 = y^1, alpha_1 = 1, K_re = 0, K_0 >= 2 (Algorithms 1 and 2).
 *
 * Conventions for every entry point:
 *  - Matrix and vector arguments are DEVICE pointers on the current HIP
 *    device unless a comment says "host".  Matrices are CSR: int32 row
 *    pointers [n+1] (rowptr[0] = 0, non-decreasing, rowptr[n] = nnz), int32
 *    column indices [nnz] in [0, n), float64 values [nnz].  Symmetry and
 *    positive semidefiniteness are the caller's contract (Section 1).
 *  - Multi-RHS vectors are row-interleaved: element (i, j) of an n x k block
 *    is at [i * k + j].
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  All
 *    device work is ordered on it.
 *  - Return values: NAJ_OK (0) or NAJ_NOT_CONVERGED (1) mean the outputs are
 *    valid; negative values are errors, with a message in naj_last_error().
 *    No C++ exception crosses this boundary.  Inputs found invalid before
 *    any device work (NAJ_EINVAL) leave every output untouched.
 *  - Objects are not thread-safe: calls on one system/batch/server must not
 *    overlap.  Different objects may be used from different threads.
 */
#ifndef NAJ_H
#define NAJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum naj_status {
    NAJ_OK = 0,
    NAJ_NOT_CONVERGED = 1,   /* max_iter reached; x holds the last iterate x^t           */
    NAJ_EINVAL = -1,         /* invalid argument (bad CSR, tol <= 0, k0 < 2, D <= 0, ...) */
    NAJ_ENOMEM = -2,         /* device allocation failed                                  */
    NAJ_EDEVICE = -3,        /* HIP runtime error or device-side timeout                  */
    NAJ_EBREAKDOWN = -4,     /* a reduction became NaN/Inf (x holds the last finite x^{t-1}) */
    NAJ_ECANCELLED = -5,     /* naj_cancel stopped the solve; x holds the iterate it had   */
    NAJ_EBUSY = -6           /* server: no slot or memory for the request now             */
} naj_status;

enum { NAJ_FP64 = 0, NAJ_MIXED = 1 };
enum { NAJ_STOP_RELRES = 0, NAJ_STOP_OBJECTIVE = 1 };

/* Solver options.  Fill with naj_opts_default() and override fields. */
typedef struct naj_opts {
    double  tol;            /* stop when ||b - Q x^t||_2 / ||b||_2 <= tol (> 0); default 1e-8          */
    int32_t max_iter;       /* iteration cap (per inner solve in mixed mode); default 20000            */
    int32_t restart;        /* IsRestart of Algorithm 3 (0 = Algorithm 1 with S = J - Q); default 1    */
    int32_t k0;             /* K_0 >= 2 of Algorithm 2; default 2                                      */
    int32_t confirm_gap;    /* iterations between residual confirmations (>= 1); default 8             */
    int32_t precision;      /* NAJ_FP64 or NAJ_MIXED; default NAJ_FP64                                 */
    double  inner_tol;      /* mixed: inner stop ||Q y - r|| / ||r|| <= inner_tol; default 1e-4        */
    int32_t max_refine;     /* mixed: maximum float64 refinement steps; default 50                     */
    int32_t inner_stall;    /* mixed: once an inner monitor has fallen to <= 1/2, the inner solve also */
                            /* stops when the monitor has not fallen below 0.9 x its best value for    */
                            /* this many iterations (the float32 rounding floor); >= 1; default 200    */
    int32_t stop;           /* NAJ_STOP_RELRES (default), or NAJ_STOP_OBJECTIVE: the paper's criterion */
                            /* of Section 4, |f(x^t) - f*| / (1 + |f*|) <= tol with f(x) = <x,Qx>/2 -   */
                            /* <b,x> (eq. (eq-qp)) and f* = fstar; float64 single solves only.  The    */
                            /* gap at y^t (free with each pass) is the monitor and f(x^t) is confirmed */
                            /* with one extra product; f(x^t) <= f(y^t), so a monitor <= tol implies   */
                            /* the criterion at x^t                                                    */
    int32_t pad_;           /* reserved, 0                                                             */
    double  fstar;          /* f* for NAJ_STOP_OBJECTIVE; default 0                                    */
} naj_opts;

/* Per-right-hand-side result of a solve (host struct). */
typedef struct naj_result {
    int32_t status;         /* naj_status of this right-hand side                                     */
    int32_t iterations;     /* FP64: t at which x^t was accepted (0 = x^0 accepted); mixed: inner total */
    int32_t restarts;       /* number of restarts (FP64) / inner restarts summed (mixed)               */
    int32_t confirmations;  /* residual confirmations (FP64) / float64 residual passes (mixed)        */
    double  relres;         /* ||b - Q x||_2 / ||b||_2 of the returned x as computed on the device     */
                            /* (also with the objective stop)                                          */
    int32_t hist_len;       /* entries written to hist                                                 */
    int32_t nrestart_log;   /* entries written to the restart log                                      */
    double  kernel_ms;      /* device time of the solve kernel(s), from HIP events on `stream`         */
    int32_t passes;         /* matrix passes of the solve kernel(s): iterations + confirmations (+ refinement residuals) */
    int32_t grid;           /* workgroups per launch of the solve driver (mixed solves: their own grid) */
    double  objgap;         /* NAJ_STOP_OBJECTIVE: |f(x) - f*| / (1 + |f*|) of the returned x, else NaN  */
} naj_result;

typedef struct naj_system naj_system;

/* Fill `o` with the defaults listed in naj_opts. */
void naj_opts_default(naj_opts *o);

/* Thread-local message describing the last error of this thread ("" if none). */
const char *naj_last_error(void);

/* Library version string, e.g. "naj 0.1 gfx950". */
const char *naj_version(void);

/*
 * Create a system from a device CSR matrix (Section 3 setup: the diagonal J
 * and the row-parallel layout of Q; the paper's "J construction" phase).
 *   n, nnz          : dimensions, 1 <= n < 2^31, 0 <= nnz < 2^31
 *   rowptr, colidx,
 *   vals            : device CSR as in the conventions above; copied, so the
 *                     caller may free them once `stream` has passed this call
 *   D               : optional device float64[n] diagonal used in place of J
 *                     (Remark 1: any invertible diagonal with D - Q PSD);
 *                     NULL = J of eq. (J-diag).  Entries must be > 0.
 *   stream          : stream for the setup work; the call returns after it
 *   out             : receives the new system; owned by the caller, release
 *                     with naj_destroy_system
 * Errors: NAJ_EINVAL (sizes, non-monotone rowptr, colidx out of range, D <= 0),
 * NAJ_ENOMEM, NAJ_EDEVICE.
 */
naj_status naj_create_system(int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *colidx,
                             const double *vals, const double *D, void *stream, naj_system **out);

/*
 * Create a system whose J is the block-diagonal matrix of eq. (J-blkdiag)
 * (Section 3): the rows are cut into blocks of `block` consecutive rows (the
 * last block keeps the rows that remain) and
 *     J^{i,i} = Q^{i,i} + sum_{j != i} ||Q^{i,j}||_2 I,
 * with a zero diagonal entry replaced by 1.  The setup computes every block
 * norm and the inverse of every block on the device; each iteration then
 * applies x = y - J^{-1}(Q y - b) block by block.  Same arguments and
 * ownership as naj_create_system, without D.
 *   block           : 1, 2, 4 or 8 (1 gives eq. (J-diag) computed block-wise)
 * The system always uses the sliced layout in caller row order and the
 * two-iterate momentum form.  It serves naj_solve (float64 and mixed; the
 * float32 inner solve applies fl32 of the float64 inverse blocks), naj_step
 * and naj_residual; batches and servers reject it.
 * Errors: as naj_create_system; NAJ_EINVAL also for another block size or a
 * block that is not positive definite (Q not positive semidefinite).
 */
naj_status naj_create_system_blockj(int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *colidx,
                                    const double *vals, int32_t block, void *stream, naj_system **out);

/*
 * The inverse blocks of a block-J system: device float64 out[n * block],
 * out[r * block + k] = entry (r - i*block, k) of (J^{i,i})^{-1} for the block
 * i holding row r.  NAJ_EINVAL for a system with a diagonal J.
 */
naj_status naj_block_inverse(naj_system *sys, double *out, void *stream);

/* Release a system and all device memory it owns.  NULL is ignored. */
void naj_destroy_system(naj_system *sys);

/*
 * Query a system (host outputs, any may be NULL):
 *   n, nnz          : dimensions
 *   device_bytes    : device memory the system owns (matrix layouts, J,
 *                     workspace), for admission control
 *   layout          : 0 = sliced rows of 64 (one row per lane), 1 = CSR row groups
 *   stored_entries  : matrix entries stored in the layout, padding included
 */
naj_status naj_system_info(const naj_system *sys, int64_t *n, int64_t *nnz, int64_t *device_bytes,
                           int32_t *layout, int64_t *stored_entries);

/*
 * Bytes per stored matrix value read by the float64 passes of the single-solve drivers: 4 when every
 * value converts to float32 and back unchanged (checked when the system is created, e.g. a graph
 * Laplacian with integer weights or a stencil), else 8.  With 4, those passes read the float32 copy of
 * the values that mixed precision keeps anyway and widen each value to float64 where it is used, so
 * they compute exactly what they compute from the 8-byte values (every result is the same bit for
 * bit) on half the value bytes; J of eq. (J-diag), the absolute row sum, comes from the same values.
 * NAJ_VALUES32=0 in the environment at creation keeps 8 bytes.  A block-J system (eq. (J-blkdiag))
 * reads its inverse blocks in float64 either way.
 *   bytes : host, 4 or 8
 * Errors: NAJ_EINVAL for a NULL argument.
 */
naj_status naj_system_value_bytes(const naj_system *sys, int32_t *bytes);

/*
 * Slices of the sliced layout (layout 0) stored in the column-offset form.  When all 64 rows of a
 * slice store their entries at columns row + S[0] < row + S[1] < ... of one increasing offset list
 * S common to the slice (a stencil pattern; at most 15 offsets, every row + S[k] inside [0, n)),
 * the slice keeps S once and the single-solve passes form its column indices instead of loading
 * them (4 bytes less per stored entry).  A row lacking an offset stores an explicit zero there,
 * which leaves every sum, and so every result, unchanged.  The form is taken where S is no longer
 * than the slice's longest row (so no more entries are stored); NAJ_OFFSETS=0 in the environment at
 * creation disables it.  The long rows of layout 1 (one wavefront per row) whose columns, in stored
 * order, are one run c0, c0 + 1, ... (dense rows) likewise form their column indices from c0;
 * NAJ_LONG_RUNS=0 disables that.
 *   offset_slices : slices in the column-offset form (0 with layout 1)
 *   nslices       : slices of the layout
 *   offset_nnz    : the caller's nonzeros whose column index the passes form instead of reading: those
 *                   held in the column-offset slices and in the dense-run long rows
 * Any output may be NULL.  Errors: NAJ_EINVAL for a NULL system.
 */
naj_status naj_system_offset_slices(const naj_system *sys, int64_t *offset_slices, int64_t *nslices,
                                    int64_t *offset_nnz);

/*
 * Solve Q x = b for one right-hand side (Algorithm 3; with NAJ_MIXED the same
 * algorithm runs in float32 inside float64 iterative refinement).
 *   b               : device float64[n]
 *   x0              : device float64[n] starting point x^0, or NULL for 0
 *   opts            : host options, NULL = defaults
 *   x               : device float64[n] output (may alias x0, not b)
 *   res             : host result, required
 *   hist            : host float64[hist_cap] or NULL.  FP64: hist[t-1] =
 *                     ||Q y^t - b|| / ||b|| (the monitor at y^t) for each
 *                     iteration t.  Mixed: the float64 relative residual of
 *                     each refinement step.
 *   restart_log     : host int32[log_cap] or NULL: the iterations t at which
 *                     a restart fired (FP64 only), in order
 *   trace           : host float64[2 * trace_cap] or NULL: for FP64, per
 *                     iteration t the restart inner product
 *                     s_t = <Q y^t - b, x^t - x^{t-1}> at [2(t-1)] and
 *                     sum_i |(Q y^t - b)_i (x^t - x^{t-1})_i| at [2(t-1)+1]
 *   stream          : the call returns after the stream has finished the solve
 * Several right-hand sides of one system: a batch of that one system (naj_batch_create with
 * nsys = 1 and nrhs = k, row-interleaved b and x) runs them together, each with its own
 * restart schedule and stop.
 * Errors: NAJ_EINVAL (bad options), NAJ_ENOMEM, NAJ_EDEVICE, NAJ_EBREAKDOWN, NAJ_ECANCELLED
 * (naj_cancel; x, res->iterations and res->relres then describe the iterate the solve held).
 */
naj_status naj_solve(naj_system *sys, const double *b, const double *x0, const naj_opts *opts, double *x,
                     naj_result *res, double *hist, int32_t hist_cap, int32_t *restart_log, int32_t log_cap,
                     double *trace, int32_t trace_cap, void *stream);

/*
 * naj_solve without any device allocation, for callers that cannot allocate: code that
 * must not call hipMalloc/hipFree (tight serving loops, harnesses that forbid allocation
 * after setup).  Same solve, kernels and results as naj_solve (bit-identical x,
 * iterations, restarts, relres) for the same system and options.
 *   b, x0, opts, x, res, restart_log, log_cap, stream : as naj_solve
 * No residual history or trace is recorded (res->hist_len = 0).
 * Scratch: the solve's control block, barrier words, arrival counters and
 * per-workgroup partial sums live in one static device array of 303,104 bytes
 * (partial sums for at most 4096 workgroups) that each device holds for the life of
 * the process; the iterates live in the system (allocated by naj_create_system).
 * Every call on a device shares that device's array and overwrites it, so calls that
 * overlap on one device (from several host threads or on several streams) race:
 * serialize them.  The call returns after `stream` has finished the solve.
 * Errors: as naj_solve; NAJ_EINVAL also when the system's drivers use more than 4096
 * workgroups, for a system owned by a server, and for NAJ_MIXED on a system whose
 * float32 work vectors do not exist yet (the first mixed naj_solve on a system
 * allocates them; this call never does).
 */
naj_status naj_solve_noalloc(naj_system *sys, const double *b, const double *x0, const naj_opts *opts, double *x,
                             naj_result *res, int32_t *restart_log, int32_t log_cap, void *stream);

/*
 * Ask the solve running on `sys` (naj_solve or naj_solve_noalloc, called from another host
 * thread) to stop.  This is the one call that may overlap another call on the same system.
 * The solve's scalar control reads the request at a pass boundary, once every 64 passes (a
 * read of host memory kept off the other passes), ends the solve after that pass's decision
 * and returns NAJ_ECANCELLED with x = the float64 iterate it held (x^t as after the iteration
 * cap; in mixed precision the refinement's current x), res->iterations and res->relres of
 * that x.  A request that arrives while no solve runs is dropped when the next solve starts.
 * Errors: NAJ_EINVAL for a NULL system or one owned by a server.
 */
naj_status naj_cancel(naj_system *sys);

/*
 * Attainable HBM rate of this GPU, for the measurement beside the published peak: a streaming
 * kernel over `bytes` bytes (16 KB blocks taken by the workgroups in turn, four 16-byte accesses in
 * flight per thread; non-temporal loads, and stores when copying; 3 workgroups of 256 threads per CU),
 * launched once untimed and then `reps` times between HIP events on `stream`.
 *   mode  : 0 reads src (dst must hold 16 bytes), 1 copies src to dst, 2 writes dst
 *   src, dst : device buffers of `bytes` bytes (16-byte aligned; src unused in mode 2)
 *   ms    : host, mean milliseconds per launch.  Bytes moved per launch: `bytes` (modes 0, 2) or
 *           2 * `bytes` (mode 1).
 * The call returns after the timed launches have finished.  Errors: NAJ_EINVAL, NAJ_EDEVICE.
 */
naj_status naj_bandwidth_probe(int32_t mode, const void *src, void *dst, int64_t bytes, int32_t reps,
                               double *ms, void *stream);

/*
 * Stand-alone kernels of the hot path, for measurement and tests.
 *
 * naj_step: one fused pass of Algorithm 3's row update (Section 3 display):
 *   x = y - J^{-1} (Q y - b) with y = p + beta (p - r) (r unused when beta == 0),
 *   and the reductions s = <Q y - b, x - p>, gg = ||Q y - b||^2,
 *   sabs = sum |(Q y - b)_i (x - p)_i| written to host red[3].
 *   p, r, b, x are device float64[n]; x must not alias p, r or b.
 */
naj_status naj_step(naj_system *sys, const double *p, const double *r, double beta, const double *b,
                    double *x, double *red, void *stream);

/* naj_residual: out = b - Q x (device float64[n], out may be NULL) and host *rr = ||b - Q x||^2. */
naj_status naj_residual(naj_system *sys, const double *x, const double *b, double *out, double *rr,
                        void *stream);

/* naj_diagonal: the diagonal J in use (eq. (J-diag) or the caller's D), device float64[n] out.
 * NAJ_EINVAL for a block-J system (see naj_block_inverse). */
naj_status naj_diagonal(naj_system *sys, double *out, void *stream);

/*
 * Batches (many systems, up to NAJ_MAX_RHS right-hand sides each, advanced together).
 * Every (system, right-hand side) pair runs its own Algorithm 3 (or the mixed
 * refinement), with its own restart schedule and stopping decision; they share
 * the passes over the matrices.  An instance's result does not depend on which
 * other systems are in the batch (the work split and summation order of a
 * system depend only on the system and its tile size).
 */
#define NAJ_MAX_RHS 8
typedef struct naj_batch naj_batch;

/*
 * Create a batch over existing systems (not copied; they must outlive the batch).
 *   nsys            : number of systems, >= 1
 *   systems         : host array of nsys system handles (same device)
 *   nrhs            : host array, right-hand sides per system, 1..NAJ_MAX_RHS
 *   opts            : options shared by every instance (NULL = defaults)
 * Passes are recorded once as a HIP graph of several launches and replayed.
 * Errors: NAJ_EINVAL, NAJ_ENOMEM, NAJ_EDEVICE.
 */
naj_status naj_batch_create(int32_t nsys, naj_system *const *systems, const int32_t *nrhs, const naj_opts *opts,
                            void *stream, naj_batch **out);

/*
 * Solve every instance of the batch.
 *   b[i], x0[i], x[i]: device float64 arrays of system i, row-interleaved n_i x nrhs_i;
 *                     x0 (the host array) or any x0[i] may be NULL (zero start); x[i] may not alias b[i]
 *   res             : host array of sum(nrhs) results, system-major then right-hand side
 * Returns the worst status over the instances (NAJ_NOT_CONVERGED if any did not converge).
 */
naj_status naj_batch_solve(naj_batch *batch, const double *const *b, const double *const *x0, double *const *x,
                           naj_result *res, void *stream);

/* Batch figures (host outputs, any may be NULL): tiles per pass, workgroups per pass, device bytes owned. */
naj_status naj_batch_info(const naj_batch *batch, int32_t *ntiles, int32_t *grid, int64_t *device_bytes);

/* Release a batch (the systems stay). NULL is ignored. */
void naj_batch_destroy(naj_batch *batch);

/*
 * Autotuner for batch work items: times item sizes of 1..16 slices on copies of `sys`
 * batched together (about 1 M rows in flight, at most 64 copies: a moderately loaded GPU)
 * with `nrhs` right-hand sides for `passes` iterations (mixed precision: one inner solve of
 * that many iterations), and records the fastest in a process-wide table keyed by the
 * system's features (layout, log2 n, nonzeros per row, nrhs, precision); batches created
 * afterwards use it.  *best_tile (host, may be NULL) receives the choice.
 */
naj_status naj_autotune_tiles(naj_system *sys, int32_t nrhs, const naj_opts *opts, int32_t passes, void *stream,
                              int32_t *best_tile);

/* Save / load the tile table (text, one "layout log2n nnz_per_row nrhs precision tile" line per entry). */
naj_status naj_tune_save(const char *path);
naj_status naj_tune_load(const char *path);

/*
 * Serving loop (continuous batching).  A server owns a device memory budget and a
 * fixed number of slots.  Each admitted request (one system, 1..NAJ_MAX_RHS
 * right-hand sides, its own tolerance) occupies a slot and draws its matrix,
 * vectors and work items from the budget; the server advances every occupied slot
 * together, one pass of Algorithm 3 (or of the mixed refinement) per slot at a time,
 * and a request admitted while others run joins at the next chunk of passes.  A
 * request's result is bit-identical to the same request served alone (its work split
 * and summation order depend only on its system).  Options other than the tolerance
 * (precision, max_iter, restart, k0, inner_tol, max_refine, inner_stall, confirm_gap)
 * are the server's.  One host thread drives a server; calls on one server must not
 * overlap.
 */
typedef struct naj_server naj_server;

/*
 * Create a server.
 *   mem_budget      : bytes of device memory for all requests (one allocation)
 *   max_slots       : requests served at once, 1..65536
 *   max_rhs         : most right-hand sides of one request, 1..NAJ_MAX_RHS (kernels are sized for it)
 *   opts            : server options (NULL = defaults; its tol is the default request tolerance)
 *   stream          : stream the passes run on (admission uses a stream of its own)
 * Errors: NAJ_EINVAL, NAJ_ENOMEM (budget not allocatable), NAJ_EDEVICE.
 */
naj_status naj_server_create(int64_t mem_budget, int32_t max_slots, int32_t max_rhs, const naj_opts *opts,
                             void *stream, naj_server **out);

/*
 * Admit a request: build its system (as naj_create_system, inside the budget) and
 * queue its right-hand sides.  Device inputs rowptr/colidx/vals/D and b (row-interleaved
 * n x nrhs) / x0 (may be NULL) are copied before the call returns; x (device, n x nrhs,
 * caller-owned) receives the answer when naj_server_result is called.  tol <= 0 takes the
 * server's.  *ticket identifies the request.
 * Returns NAJ_EBUSY when no slot or not enough budget is free now (nothing was kept:
 * try again after a result has been taken), NAJ_ENOMEM when the request can never fit
 * the budget, NAJ_EINVAL for bad arguments or input.
 */
naj_status naj_server_admit(naj_server *sv, int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *colidx,
                            const double *vals, const double *D, int32_t nrhs, const double *b, const double *x0,
                            double tol, double *x, int64_t *ticket);

/*
 * Advance the server: replay `chunks` chunks of passes over every occupied slot (0 =
 * run none, only collect what has finished), and return in done[0..*ndone) (host, at
 * most cap entries) the tickets of requests found finished since the last call.  A
 * request is found one chunk after the chunk it finished in (the host reads the flags
 * of the previous chunk while the next one runs).
 */
naj_status naj_server_step(naj_server *sv, int32_t chunks, int64_t *done, int32_t cap, int32_t *ndone);

/*
 * Take the result of a finished request: its answer is written to the x given at
 * admission, res (host, nrhs entries) receives the per-right-hand-side results, and the
 * request's slot and memory are released.  NAJ_EBUSY: not finished yet; NAJ_EINVAL:
 * unknown ticket.  Returns the worst status of the request's right-hand sides.
 */
naj_status naj_server_result(naj_server *sv, int64_t ticket, naj_result *res);

/* Server figures (host outputs, any may be NULL): budget bytes in use / total, slots in use / total. */
naj_status naj_server_info(const naj_server *sv, int64_t *bytes_used, int64_t *bytes_total, int32_t *slots_used,
                           int32_t *slots_total);

/* Release a server and every request still in it. NULL is ignored. */
void naj_server_destroy(naj_server *sv);

#ifdef __cplusplus
}
#endif

#endif /* NAJ_H */
