/*
 * dpt.h -- C ABI of the MI355X (gfx950) dynamical-perturbation-theory library.
 *
 * Method: Kenmoe, Smerlak, Zadorin, "Dynamical perturbation theory for
 * eigenvalue problems", arXiv:2002.12872.
 *
 * Problem (Sec. II.B): M = D + lambda * Delta with D = diag(theta), theta simple
 * (pairwise distinct).  The library iterates the bundled map of eq. (dyn),
 *
 *     F(A) = I + lambda * theta-gap (.) (A Delta' - diag(A Delta') A),
 *     gap[n][m] = 1 / (theta_n - theta_m) for m != n, 0 on the diagonal,
 *
 * from A = I (or a caller-given start), where row n of A is the candidate
 * eigenvector z_n in the chart z_n[n] = 1 (Sec. II.A/B).  Eigenvalues are read
 * from the current iterate as E_n = theta_n + lambda * (Delta z_n)[n]
 * (Sec. II.B; the factor lambda follows Supplement B).
 *
 * Layout conventions used throughout this header:
 *   - dense Delta:   delta[m * n + l] = Delta[m][l]  (row-major, n*n entries)
 *   - CSR Delta:     row m holds columns indices[indptr[m] .. indptr[m+1])
 *                    with values delta[...]; indices sorted ascending within a
 *                    row, no duplicates; indptr has n+1 entries, indptr[0] = 0
 *   - eigenvectors:  Z[k * n + m] = component m of eigenvector k, Z[k*n + k] = 1
 *                    (row k = z_k; byte-identical to a column-major matrix whose
 *                    column k is eigenvector k)
 *
 * Memory and ownership:
 *   - DPT_MEM_HOST inputs are copied during the call; the caller may free them
 *     when the call returns.
 *   - DPT_MEM_DEVICE inputs (HIP device pointers, e.g. a torch tensor's
 *     data_ptr()) are borrowed: they must stay valid and unchanged for the life of
 *     the handle; the library never frees or writes them.  (A dense Delta whose
 *     order needs padding, whose dtype differs from the state's or whose address
 *     is not 16-byte aligned is copied instead.)
 *   - Output buffers are always caller-owned.  Each handle owns its internal
 *     device state; dpt_destroy releases it.
 *   - All device work is ordered on problem.stream (a hipStream_t; NULL means the
 *     default stream).  Calls that return host-visible results synchronise that
 *     stream before returning.
 *   - A handle is used by one host thread at a time; distinct handles are
 *     independent.
 *
 * Errors: no exception or abort crosses this interface.  Negative return codes
 * are errors and leave the handle state unchanged; positive codes are
 * numerical outcomes whose results are valid and can be read.
 */
#ifndef DPT_H
#define DPT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ----------------------------------------------------- */
#define DPT_OK 0              /* converged: delta_k < tol in the final phase            */
#define DPT_NOT_CONVERGED 1   /* iteration cap reached (cycles and chaos end here)        */
#define DPT_STALLED 2         /* the final phase stopped improving above tol              */
#define DPT_DIVERGED 3        /* non-finite iterate, or max |Z - I| above options.blowup */
#define DPT_EAGAIN 4          /* serving: result not ready yet                            */
#define DPT_EINVAL (-1)       /* invalid argument                                         */
#define DPT_ENOMEM (-2)       /* device or host allocation failed                         */
#define DPT_EDEVICE (-3)      /* HIP runtime error or no usable gfx950 device             */
#define DPT_ESTATE (-4)       /* call not valid in the handle's current state             */

/* ---- precision forms -------------------------------------------------- */
#define DPT_FP64 0       /* every product and update in FP64                           */
#define DPT_FP32 1       /* FP32 products and updates (gaps from FP64 theta)           */
#define DPT_BF16_FP32 2  /* BF16 products (FP32 accumulate) until stall, then FP32     */
#define DPT_FP8_FP32 3   /* experiment: block-scaled FP8 (OCP E4M3, E8M0 scale per 32   *
                          * values) products until stall, then FP32; dense problems    *
                          * with N >= 1024 only (DPT_EINVAL otherwise)                 */
#define DPT_BF16_X3 4    /* experiment: BF16 products until stall, then FP32-grade      *
                          * sweeps whose product is formed on BF16 matrix cores from   *
                          * split operands x = h + l (h = bf16(x), l = bf16(x - h)):   *
                          * W_h D_h^T + W_l D_h^T + W_h D_l^T with FP32 accumulation;  *
                          * dense problems with N >= 1024 only (DPT_EINVAL otherwise)  */

/* ---- storage ---------------------------------------------------------- */
#define DPT_DENSE 0
#define DPT_CSR 1
#define DPT_MEM_HOST 0
#define DPT_MEM_DEVICE 1
#define DPT_DTYPE_F64 0
#define DPT_DTYPE_F32 1

typedef struct dpt_ctx *dpt_handle;

/* The eigenproblem (Sec. II.B: theta, Delta, lambda). */
typedef struct dpt_problem {
    int64_t n;               /* matrix order, >= 1                                       */
    const double *theta;     /* n unperturbed eigenvalues, pairwise distinct (mem kind)  */
    const void *delta;       /* dense: n*n values; CSR: nnz values (dtype, mem kind)     */
    const int64_t *indptr;   /* CSR only: n+1 row offsets (mem kind)                     */
    const int32_t *indices;  /* CSR only: nnz column indices (mem kind)                  */
    int64_t nnz;             /* CSR only                                                 */
    double lambda;           /* perturbation strength, finite                            */
    void *stream;            /* hipStream_t or NULL                                      */
    int32_t format;          /* DPT_DENSE or DPT_CSR                                     */
    int32_t dtype;           /* DPT_DTYPE_F64 or DPT_DTYPE_F32 (values of delta)         */
    int32_t mem;             /* DPT_MEM_HOST or DPT_MEM_DEVICE (all input arrays)        */
    int32_t reserved;        /* must be 0                                                */
} dpt_problem;

/* Stopping and precision control.  The paper prescribes no stopping rule; the
 * one used here: delta_k = max_{n,m} |Z_k[n][m] - Z_{k-1}[n][m]| after the k-th
 * application of F, convergence when delta_k < tol. */
typedef struct dpt_options {
    double tol;             /* > 0; threshold on delta_k for the final phase              */
    double fp64_final_tol;  /* > 0: after FP32 convergence run FP64 sweeps to this; 0 off */
    double stall_ratio;     /* stall when delta_k >= stall_ratio * min_{j<k} delta_j ...  */
    double blowup;          /* DIVERGED when max |Z - I| exceeds this (> 0)               */
    double ramp_alpha;      /* 0: autonomous map.  In (0, 1): coupling ramp of Supplement *
                             * E, lambda_k = lambda (1 - alpha^k) for the k-th application *
                             * while alpha^k >= 2^-53 (alpha^k by repeated multiplication), *
                             * lambda afterwards; stopping tests wait for the ramp's end   */
    int32_t max_iter;       /* >= 0; cap on applications of F over all phases              */
    int32_t precision;      /* DPT_FP64, DPT_FP32, DPT_BF16_FP32, DPT_FP8_FP32, DPT_BF16_X3 */
    int32_t stall_patience; /* ... for this many consecutive checks (>= 1), or delta_k = 0 */
    int32_t check_every;    /* read delta back every this many steps (>= 1)                */
    int32_t stop_rule;      /* DPT_STOP_DELTA (default) or DPT_STOP_ESTIMATE               */
    int32_t reserved;       /* must be 0                                                  */
} dpt_options;

/* Stopping rules.  DPT_STOP_DELTA: converged when delta_k < tol.
 * DPT_STOP_ESTIMATE: converged when the a-posteriori bound of a contraction,
 * rho * delta_k / (1 - rho), is below tol, with rho the larger of the last two
 * step ratios delta_j / delta_{j-1} measured inside one precision phase (the
 * ratios of the BF16 phase carry over to the first FP32 sweep, whose own delta
 * measures the correction of the BF16 bias).  Without two ratios below 0.5 it
 * falls back to delta_k < tol. */
#define DPT_STOP_DELTA 0
#define DPT_STOP_ESTIMATE 1
/* DPT_STOP_ROW: per-row retirement (Sec. II.B: row n evolves under its own map
 * F_n).  In the final phase (FP32 sweeps of DPT_FP32 / DPT_BF16_FP32, the FP64
 * steps of DPT_FP64) each row is frozen after the first step on which its own
 * delta_k(n) = max_m |Z_k[n][m] - Z_{k-1}[n][m]| is below tol, and later products
 * run on the remaining rows only (row list padded to the product tile); the
 * solve ends with DPT_OK when no row is left.  The phases before the final one
 * follow the delta rule.  Dense problems with those precisions,
 * fp64_final_tol = 0 and check_every = 1 only (DPT_EINVAL otherwise); see
 * dpt_row_status. */
#define DPT_STOP_ROW 2

typedef struct dpt_result {
    double last_delta;      /* delta_k of the last application of F (NaN if none)          */
    double *delta_history;  /* caller-owned array of history_cap entries, or NULL         */
    int32_t history_cap;
    int32_t status;         /* DPT_OK / NOT_CONVERGED / STALLED / DIVERGED                */
    int32_t iters;          /* applications of F made by this call                         */
    int32_t iters_bf16;     /* steps of the reduced-precision phase (BF16, or FP8)        */
    int32_t iters_fp32;     /* FP32-grade sweeps (FP32, or split BF16 for DPT_BF16_X3)  */
    int32_t iters_fp64;
} dpt_result;

/* Fill *o with defaults: tol 1e-6, max_iter 200, DPT_FP32, fp64_final_tol 0,
 * stall_ratio 0.5, stall_patience 2, check_every 1, blowup 1e6, DPT_STOP_DELTA,
 * ramp_alpha 0. */
void dpt_options_default(dpt_options *o);

/* Host-only argument check (no device call): pointer/size/enum sanity and, for
 * host-memory inputs, distinct finite theta and a well-formed CSR.  Returns
 * DPT_OK or DPT_EINVAL.  `o` may be NULL. */
int dpt_validate(const dpt_problem *p, const dpt_options *o);

/* Create a handle for the dense or CSR problem p.  Stages Delta on the device
 * (precision copies, transpose when Delta is not symmetric), validates theta.
 * z0 == NULL starts from A^(0) = I (Sec. II.B); otherwise z0 holds an n*n start
 * in the eigenvector layout above, same dtype and memory kind as the problem
 * (its diagonal is taken as 1: the chart z_k[k] = 1).  This warm start is the
 * paper's refinement of approximate eigenvectors (Sec. II.H, last paragraph),
 * and resumes an interrupted iteration: continuing from the exported iterate of
 * k steps reproduces the uninterrupted iteration (bitwise in FP32 and FP64
 * phases, dense and CSR).  A CSR Delta in device
 * memory is structure-checked on the device (same rules as dpt_validate) and
 * borrowed: row pointers and indices always, values when their dtype is the
 * state's (FP64 for DPT_FP64, else FP32).
 * Returns DPT_OK, or DPT_EINVAL (bad argument, duplicate theta, malformed CSR),
 * DPT_ENOMEM, DPT_EDEVICE; *h is set only on success. */
int dpt_init(dpt_handle *h, const dpt_problem *p, const dpt_options *o, const void *z0);

/* Apply F exactly nsteps (>= 0) times in the handle's current precision phase,
 * with no stopping test (eq. dyn).  *last_delta (may be NULL) receives delta of
 * the last step (NaN when nsteps == 0).  Returns DPT_OK or an error. */
int dpt_step(dpt_handle h, int nsteps, double *last_delta);

/* Iterate until the stopping rule ends the solve (options of dpt_init).
 * DPT_BF16_FP32: BF16 steps until delta_k < tol or a stall, then FP32 sweeps
 * until delta_k < tol (at least one), then FP64 sweeps when fp64_final_tol > 0.
 * The stopping rule sees every step's delta in order (with check_every = 1);
 * dense problems of padded order 64 run several steps per launch and the state
 * ends on the step the rule stops at (later speculative steps are discarded),
 * bitwise as with one launch per step.
 * Returns the status (also in r->status when r != NULL) or an error. */
int dpt_solve(dpt_handle h, dpt_result *r);

/* Per-row retirement record of a handle solved with DPT_STOP_ROW: retired_at
 * (host, n entries, or NULL) receives for each row the number of applications
 * of F after which it was frozen (0: still running); *rows_multiplied (or NULL)
 * the number of rows the products have run on so far, summed over the product
 * steps (ld per step without retirement; ld = padded order). */
int dpt_row_status(dpt_handle h, int32_t *retired_at, int64_t *rows_multiplied);

/* E_k = theta_k + lambda (Delta z_k)[k] for all k from the current iterate
 * (FP64 accumulation).  E: n doubles in memory kind `mem`. */
int dpt_eigenvalues(dpt_handle h, double *E, int mem);

/* Current iterate in the eigenvector layout above, as DPT_DTYPE_F32/F64 in
 * memory kind `mem` (n*n entries). */
int dpt_eigenvectors(dpt_handle h, void *Z, int dtype, int mem);

/* Acceptance check, not part of the method: for the eigenvectors rows[0..nrows)
 * of the current iterate, res[i] = || M z - E z ||_2 with M = diag(theta) +
 * lambda Delta evaluated in FP64 on the device (the eigen-equation, Sec. II.A).
 * rows and res are host arrays. */
int dpt_residuals(dpt_handle h, int64_t nrows, const int64_t *rows, double *res);

/* Dominant-eigenvector mode (Sec. II.H): iterate only the single-line map
 * F_index of eq. (single_line_dyn) on one vector from e_index.  index < 0
 * selects argmax theta.  Uses o->tol, o->max_iter, o->blowup and o->precision
 * (DPT_FP64 -> FP64, otherwise FP32).  eigvec: n values of p->dtype in p->mem
 * (eigvec[index] = 1).  *eigval receives theta_index + lambda (Delta z)[index].
 * Only theta_index has to be simple here (the map divides by theta_index -
 * theta_m alone); other theta values may coincide.  The first iteration, from
 * e_index, is evaluated in closed form (it reads column index of Delta only,
 * with the same arithmetic as the general iteration).  A CSR Delta in device
 * memory is checked on the device and borrowed for the call.  Returns the
 * numerical status, or DPT_EINVAL (bad arguments, non-finite theta, theta_index
 * repeated, malformed CSR), DPT_ENOMEM, DPT_EDEVICE. */
int dpt_dominant(const dpt_problem *p, const dpt_options *o, int64_t index, double *eigval,
                 void *eigvec, dpt_result *r);

/* Dominant-eigenvector mode that allocates no device memory, for callers that
 * cannot call hipMalloc (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same iteration, kernels and results as
 * dpt_dominant (bitwise), with every work buffer (the two iterates, the scalar
 * (Delta z)[index], per-iteration statistics, the stop flag, the theta and CSR
 * checks) in one fixed array per GPU of 64 MiB + 68 KiB, held by each GPU the
 * library runs on until the process ends.  Requirements beyond dpt_dominant's: p->mem ==
 * DPT_MEM_DEVICE; p->dtype is DPT_DTYPE_F64 for o->precision == DPT_FP64 and
 * DPT_DTYPE_F32 otherwise (no conversion copy); eigvec is device memory of n
 * values of that dtype.  Limits: o->max_iter <= 4096 and n <= 8388608 (FP32) or
 * 4194304 (FP64); beyond them DPT_EINVAL.  Host-side results (eigval, r) as in
 * dpt_dominant; the call synchronises p->stream.  All calls on one GPU share
 * that GPU's array and leave their contents in it: calls that overlap on one
 * GPU (from several host threads or streams) race and must be serialised by
 * the caller.  Returns the numerical status, DPT_EINVAL or DPT_EDEVICE. */
int dpt_dominant_noalloc(const dpt_problem *p, const dpt_options *o, int64_t index, double *eigval,
                         void *eigvec, dpt_result *r);

/* Homotopy continuation (Sec. III, Discussion): for a coupling outside the
 * iteration's convergence domain, lambda is split into `stages` equal parts.
 * Stage q diagonalises D + (q lambda / stages) Delta by a full FP64 D-PT solve
 * written in the eigenbasis of the previous stage, where the problem is the
 * diagonal matrix of the previous eigenvalues perturbed by (lambda / stages)
 * B^-1 Delta B (B: the previous eigenvectors as columns).  The basis and its
 * inverse are updated with FP64 matrix-core products: symmetric Delta keeps
 * orthonormal eigenvector rows (B^-1 = B^T); otherwise the left eigenvectors come
 * from the same iteration on the transposed stage perturbation.  With
 * stages = 1 this is dpt_solve in FP64.  Dense problems; o->precision must be
 * DPT_FP64 and every stage uses o's tol, max_iter and stopping rule, with a
 * stall ratio of at least 0.9 (stages can contract slowly near the rounding
 * floor) and without the ramp.  Outputs in p->mem memory: E (n eigenvalues, continued from
 * theta by index) and Z (n*n, z_dtype, eigenvector layout above, Z[k*n+k] = 1).
 * r->iters sums the D-PT iterations of all stage solves.  Returns the worst
 * stage status (the continuation stops at the first stage that does not reach
 * DPT_OK; outputs then hold the last completed stage), DPT_EINVAL, DPT_ENOMEM
 * or DPT_EDEVICE. */
int dpt_homotopy(const dpt_problem *p, const dpt_options *o, int32_t stages, double *E, void *Z, int z_dtype,
                 dpt_result *r);

/* Rayleigh-Schroedinger series, the comparator of Sec. II.D-F (recursion eq.
 * ARS-alpha, Supplement B), in FP64 on the GPU:
 *   a^(0) = I,  a^(l) = gap (.) (a^(l-1) Delta' - sum_{s<l} diag(a^(s) Delta') a^(l-1-s)),
 * one FP64 matrix-core product a^(l-1) Delta' per order.  Outputs: eps (host,
 * order*n doubles) with eps[(l-1)*n + k] = eps_k^(l) = (a^(l-1) Delta')_kk, the
 * order-l eigenvalue coefficient (E_RS = theta + sum_l lambda^l eps^(l));
 * coef_max (host, order doubles or NULL) = max |a^(l)|; Z (or NULL; n*n values
 * of z_dtype in p->mem memory) = the partial sum sum_{l=0}^{order} lambda^l a^(l)
 * in the eigenvector layout above.  Dense problems; 1 <= order <= 4096; memory
 * order+1 coefficient matrices.  Returns DPT_OK, DPT_EINVAL, DPT_ENOMEM or
 * DPT_EDEVICE. */
int dpt_rs_series(const dpt_problem *p, int32_t order, double *eps, double *coef_max, void *Z, int z_dtype);

/* Measurement probe, not part of the method: rate of random gathers of 512-byte
 * rows from a panel of panel_rows rows (the access pattern of the CSR product's
 * state gathers), `gathers` runs per pass (rounded up to the probe's grid),
 * averaged over reps passes after one warm-up, on the default stream.
 * *ms_per_pass and *gbs (gathered bytes / time) receive the result.  Returns
 * DPT_OK, DPT_EINVAL or DPT_EDEVICE. */
int dpt_probe_gather(int64_t panel_rows, int64_t gathers, int reps, double *ms_per_pass, double *gbs);

/* ---- kernel timing --------------------------------------------------------
 * Device time of the library's kernels, measured with HIP events recorded on
 * the handle's stream around each launch (accumulated per kernel class).
 * Timing adds two event records per launch; it is off by default. */
#define DPT_PROF_FIRST 0      /* first iterate F(I), no product                  */
#define DPT_PROF_PREPASS 1    /* diagonal pre-pass d_n = (Delta z_n)[n]           */
#define DPT_PROF_GEMM_BF16 2  /* fused BF16 MFMA product + update                */
#define DPT_PROF_GEMM_FP32 3  /* fused FP32 MFMA product + update                */
#define DPT_PROF_GEMM_FP64 4  /* fused FP64 MFMA product + update                */
#define DPT_PROF_SPMM 5       /* fused CSR product + update                       */
#define DPT_PROF_GEMM_FP8 6   /* fused block-scaled FP8 MFMA product + update     */
#define DPT_PROF_GEMM_X3 7    /* fused split-BF16 MFMA product + update (sweeps)  */
#define DPT_PROF_KINDS 8

typedef struct dpt_profile {
    double ms[DPT_PROF_KINDS];        /* summed device milliseconds per class      */
    int64_t launches[DPT_PROF_KINDS]; /* number of timed launches per class        */
} dpt_profile;

/* on != 0 starts timing (and clears the totals); on == 0 stops it. */
int dpt_profile_enable(dpt_handle h, int on);

/* Synchronise the stream and copy the totals into *out. */
int dpt_profile_read(dpt_handle h, dpt_profile *out);

/* ---- serving: continuous batching of many small dense problems ----------
 * A server owns a device memory arena of budget_bytes and a worker thread.
 * Submitted problems wait in FIFO order and are admitted while the arena and
 * the slot table have room; every engine step advances all admitted problems
 * by one application of F with one persistent grouped launch per precision
 * phase and tile shape (replayed as a HIP graph when use_graph != 0 and
 * every list in the graph has work; only the lists with work are launched
 * otherwise); each problem follows
 * its own stopping rule and is retired individually (freeing its memory for
 * the next admissions).  Results do not depend on which other problems share
 * a step: every problem is computed with tiles chosen from its own padded
 * order and phase (a shape per padded-order class, fixed when the server
 * opens) and with its own statistics.  Besides the worker, a server keeps four
 * host threads that stage large host submissions with the submitting thread.
 * dpt_serve_submit, dpt_serve_poll and dpt_serve_stats_read may be called from
 * several threads at once; dpt_serve_close must not overlap any other call on
 * the same server. */
typedef struct dpt_server_ctx *dpt_server;

typedef struct dpt_serve_config {
    int64_t budget_bytes;   /* device arena for in-flight problems (> 0)              */
    int32_t max_slots;      /* concurrent problems, 1 .. 1024                         */
    int32_t use_graph;      /* 1: replay the grouped step as a HIP graph in steps     *
                             * where every (phase, shape) list has work               */
    int32_t grid_blocks;    /* persistent grid of the grouped kernels; 0 = 1024       */
    int32_t autotune;       /* 1: time the fused-step tile shapes (64x64, 128x64,     *
                             * 128x128) per phase and padded-order class at open, on  *
                             * a full batch and on a lone problem, and keep the one   *
                             * fastest alone among those within 3 % of the fastest on *
                             * the full batch; 0: 128x128 above padded order 512;     *
                             * -1, -2, -3: shape 64x64, 128x64 or 128x128 for every   *
                             * class (orders that are not multiples of 128: 64x64)    */
    void *stream;           /* hipStream_t for all of the server's device work (the   *
                             * caller keeps ownership and enqueues nothing on it      *
                             * while the server is open), or NULL: an own stream      */
} dpt_serve_config;

/* Seconds since dpt_serve_open on a monotonic clock. */
typedef struct dpt_serve_times {
    double submit_s, admit_s, first_step_s, finish_s;
} dpt_serve_times;

typedef struct dpt_serve_stats {
    int64_t submitted, completed, steps;   /* problems and engine steps so far      */
    int64_t peak_active, peak_bytes;       /* largest concurrent set and arena use  */
    int64_t active, pending;               /* current counts                        */
    double busy_s;                         /* wall time spent inside engine steps   */
    int32_t tile_shape[2][4];              /* fused-step tile per phase (BF16, FP32) *
                                            * and padded-order class (ld <= 256,     *
                                            * <= 512, <= 1024, larger): 0 = 64x64,   *
                                            * 1 = 128x64, 2 = 128x128 (orders that   *
                                            * are not multiples of 128 use 64x64)    */
    int64_t graph_steps;                   /* engine steps replayed as the HIP graph *
                                            * (every (phase, shape) list had work)   */
} dpt_serve_stats;

/* Start a server on the current device (on cfg->stream, or a stream of its own,
 * with the device arena of cfg->budget_bytes and a 256 MiB pinned host staging
 * ring for submitted matrices).  Returns DPT_OK, DPT_EINVAL, DPT_ENOMEM (arena or ring
 * allocation) or DPT_EDEVICE. */
int dpt_serve_open(dpt_server *srv, const dpt_serve_config *cfg);

/* Queue a dense problem.  DPT_MEM_HOST: theta and Delta are copied before the
 * call returns (Delta as FP32), into the staging ring when they take at most
 * half of it: the call waits while the ring is full of not yet uploaded
 * problems.  DPT_MEM_DEVICE: theta is read back and checked during the call;
 * theta and Delta (FP32 or FP64) are read on the server's stream when the
 * problem is admitted, so they must be complete when the call is made and stay
 * allocated and unchanged until the ticket's result has been polled; the
 * transpose of Delta is always stored (its symmetry is not tested).
 * o->precision must be DPT_FP32 or DPT_BF16_FP32 (o may be NULL: defaults).
 * want_eigenvectors != 0 keeps Z for dpt_serve_poll.  Returns DPT_OK and a
 * ticket, DPT_EINVAL (bad problem, duplicate theta), DPT_ENOMEM (the problem
 * alone exceeds the arena) or DPT_ESTATE (the server is closing or failed). */
int dpt_serve_submit(dpt_server srv, const dpt_problem *p, const dpt_options *o, int want_eigenvectors,
                     int64_t *ticket);

/* Wait up to wait_ms (0: do not wait, < 0: until done) for a ticket.  Returns
 * DPT_EAGAIN while it is pending; otherwise its numerical status, with r, E (n
 * doubles), Z (n*n values of z_dtype, only if requested at submit) and t filled
 * when non-NULL.  A completed ticket is released by the call that returns its
 * status (a later poll returns DPT_EINVAL). */
int dpt_serve_poll(dpt_server srv, int64_t ticket, int wait_ms, dpt_result *r, double *E, void *Z, int z_dtype,
                   dpt_serve_times *t);

int dpt_serve_stats_read(dpt_server srv, dpt_serve_stats *out);

/* Finish every queued problem, stop the worker and release the server. */
void dpt_serve_close(dpt_server srv);

/* Release the handle (NULL is accepted). */
void dpt_destroy(dpt_handle h);

/* Static description of a return code. */
const char *dpt_status_str(int code);

#ifdef __cplusplus
}
#endif

#endif /* DPT_H */
