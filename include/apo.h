/*
 * apo.h -- C ABI of libapo.so, the gfx950 (MI355X) implementation of the
 * Artificial Protozoa Optimizer (APO) population step.
 *
 * The calls follow Algorithm 1 of "cuAPO: A CUDA-based Parallelization of
 * Artificial Protozoa Optimizer": its input (np, ps, dim, pf_max and the
 * iteration budget) is apo_create's argument list, one pass of its loop
 * body (sort, pf, Dr, the per-protozoan update of Eqs. (1)-(13), bound
 * clamp, evaluation, greedy selection) is apo_step, and its output
 * (f(X_gbest), X_gbest) is apo_best.
 *
 * Conventions shared by every call:
 *   - Plain C types only.  "host" pointers are ordinary CPU memory, "device"
 *     pointers are HIP device memory of the current device.
 *   - Return value: APO_OK (0) or a negative apo_status.  No call throws.
 *   - Host input arrays are copied during the call; the caller keeps
 *     ownership and may free them on return.  Host output arrays are
 *     written by the call and owned by the caller.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - After APO_E_DEVICE a handle is poisoned: every call except
 *     apo_destroy returns APO_E_DEVICE.
 *   - Population layout seen through the ABI: X is [pop][dim] row-major in
 *     protozoan-id order (ids are fixed at creation and never move).
 */
#ifndef APO_H
#define APO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct apo apo_t;   /* opaque handle, owned by the caller until apo_destroy */

typedef enum {
    APO_OK = 0,
    APO_E_INVAL = -1,        /* an argument is out of range or inconsistent      */
    APO_E_NOMEM = -2,        /* host or device allocation failed                 */
    APO_E_DEVICE = -3,       /* a HIP call failed; the handle is poisoned        */
    APO_E_DONE = -4,         /* the iteration budget is spent; state unchanged   */
    APO_E_STATE = -5,        /* the handle cannot serve this call (e.g. no trace)*/
    APO_E_UNSUPPORTED = -6   /* valid arguments outside the sizes built for      */
} apo_status;

typedef enum {
    APO_FP64 = 0,            /* positions and fitness in binary64 */
    APO_FP32 = 1,            /* positions and fitness in binary32 */
    APO_BF16 = 2             /* rotated objectives only: binary32 state; z = M (x - o)
                                estimated on the matrix cores with BF16 operands and
                                binary32 accumulation, every candidate the estimate
                                cannot settle under a rigorous bound (and every
                                acceptance) re-scored in binary32, so the run equals
                                the binary32 form's; apo_best re-scores the elite in
                                binary64 */
} apo_precision;

typedef enum {
    APO_SPHERE = 0,          /* sum z^2 (Eq. (14))                                   */
    APO_RASTRIGIN = 1,       /* sum (z^2 - 10 cos(2 pi z) + 10)                      */
    APO_ROSENBROCK = 2,      /* textbook Rosenbrock on z + 1 (minimum at x = o)      */
    APO_ACKLEY = 3,          /* textbook Ackley                                      */
    APO_KAPUR = 4,           /* minus Kapur entropy of a 256-bin histogram, dim thresholds */
    APO_OTSU = 5             /* minus Otsu between-class variance, dim thresholds    */
} apo_obj_kind;

/* Objective.  For the first four kinds z = M (x - o): shift o is host
 * [dim] (NULL: o = 0), rot M is host [dim*dim] row-major (NULL: M = I),
 * so z_i = sum_j M[i][j] (x_j - o_j).  For APO_KAPUR / APO_OTSU, hist is a
 * host [256] grey-level histogram (not all zero), each coordinate is a
 * threshold rounded half-to-even to a grey level and the bounds must lie
 * in [0, 255]; shift and rot must be NULL. */
typedef struct {
    int32_t kind;             /* apo_obj_kind */
    const double *shift;      /* host [dim] or NULL            (copied) */
    const double *rot;        /* host [dim*dim] or NULL        (copied) */
    const uint64_t *hist;     /* host [256] for KAPUR / OTSU   (copied) */
} apo_objective;

enum {
    APO_FLAG_TRACE = 1u,      /* keep every candidate of the last step for apo_get_trace */
    APO_FLAG_PDR_PLUS = 2u    /* Eq. (13) with the opposite sign before the cosine (a
                                 variant of the printed formula: the worst ranks of Dr,
                                 not the best, are the likeliest to go dormant)       */
};

typedef struct {
    int32_t max_iter;         /* iter_max (T) >= 1: Eqs. (4), (9), (12) use t/T    */
    int32_t precision;        /* apo_precision                                    */
    apo_objective objective;
    uint32_t run_id;          /* fourth Philox counter word (independent runs)    */
    uint32_t flags;           /* APO_FLAG_*                                       */
    void *stream;             /* hipStream_t the library launches on, or NULL for a
                                 stream the library creates and owns; an external
                                 stream must outlive the handle                   */
    void *workspace;          /* device buffer of >= apo_workspace_bytes bytes the
                                 library uses for all its device state, or NULL to
                                 let the library allocate it; an external buffer
                                 must outlive the handle                          */
    size_t workspace_bytes;   /* size of workspace when it is not NULL            */
} apo_options;

/* Device bytes apo_create needs for these sizes and options (0 if the
 * arguments are invalid).  The layout does not depend on np.  Nothing is
 * allocated. */
size_t apo_workspace_bytes(int32_t dim, int32_t pop, const apo_options *opt);

/* Create an optimiser (Algorithm 1, input and initialisation).
 *   dim     D >= 1 coordinates per protozoan
 *   lb, ub  host [dim] bounds X_min < X_max, finite (copied)
 *   pop     population size ps >= 2
 *   np      neighbour pairs in Eqs. (6) and (8), 1 <= np <= 8
 *   pf_max  maximum fraction in Eq. (11), 0 <= pf_max <= 1
 *   seed    Philox key of every random draw
 *   opt     options (required)
 *   out     receives the handle
 * Draws the initial population uniformly in the bounds and evaluates it
 * (ps function evaluations).  Asynchronous on the handle's stream.
 * Errors: APO_E_INVAL (bad argument), APO_E_UNSUPPORTED (sizes the kernels
 * are not built for: pop > 65536; elementwise objectives above dim 1024;
 * rotated objectives above dim 256 in APO_FP64 and above 1024 in APO_FP32
 * and APO_BF16 (above 512 the product runs in the GEMM form, separable
 * objectives only: no Rosenbrock); Kapur / Otsu above 512 thresholds),
 * APO_E_NOMEM, APO_E_DEVICE. */
int apo_create(int32_t dim, const double *lb, const double *ub, int32_t pop, int32_t np,
               double pf_max, uint64_t seed, const apo_options *opt, apo_t **out);

/* One iteration t -> t + 1 of Algorithm 1's loop body: sort by fitness,
 * draw pf and Dr, build every candidate (dormancy Eq. (1), reproduction
 * Eqs. (2)-(3), autotroph Eqs. (4)-(7), heterotroph Eqs. (8)-(10)) from the
 * population as it stood at the start of the iteration, clamp to the
 * bounds, evaluate, and keep a candidate only if its fitness is strictly
 * lower.  Asynchronous.  APO_E_DONE once t == max_iter. */
int apo_step(apo_t *h);

/* Up to iters more iterations (clipped to max_iter - t): Algorithm 1's loop
 * body, as apo_step, repeated.  Returns the number executed (>= 0) or a
 * status.  The sort and step kernels of each iteration are replayed from HIP
 * graphs, captured on the first call (apo_run(h, 0) captures them and
 * executes nothing, so a later timed call does not include the capture).
 * A run whose whole population fits one workgroup of the step (elementwise
 * objectives with pop x lanes <= 256, pop <= 256, e.g. pop 32 at dim 10; or
 * a rotated or thresholding run that one wide tile holds, e.g. Otsu at pop
 * 100, dim 1) instead runs all its iterations in one single-workgroup launch
 * (the persistent form: sort and step separated by workgroup barriers; the
 * elementwise form keeps the run's state in LDS for the launch); the results
 * are the same bit for bit. */
int apo_run(apo_t *h, int32_t iters);

/* The best protozoan (lowest fitness; NaN never wins; lowest id on ties):
 * x_out host [dim], f_out host scalar, fes_out host scalar = function
 * evaluations so far = pop * (t + 1).  Any output may be NULL.
 * Synchronises the handle's stream. */
int apo_best(apo_t *h, double *x_out, double *f_out, int64_t *fes_out);

/* Completed iterations t and function evaluations (either may be NULL). */
int apo_info(const apo_t *h, int32_t *iter, int64_t *fes);

/* Release every resource of the handle (external stream and workspace are
 * left alone).  NULL is accepted. */
int apo_destroy(apo_t *h);

/* Checkpoint: copy out X host [pop][dim], F host [pop] and t.  Any output
 * may be NULL.  Synchronises. */
int apo_get_state(apo_t *h, double *X, double *F, int32_t *iter);

/* Resume / inject: replace X (host [pop][dim], rounded to the handle's
 * precision), F (host [pop], same) and t (0 <= t <= max_iter).  Values are
 * taken as given (F is not recomputed).  Synchronises. */
int apo_set_state(apo_t *h, const double *X, const double *F, int32_t iter);

/* Record of the last apo_step (handles created with APO_FLAG_TRACE only,
 * else APO_E_STATE): Y host [pop][dim] clamped candidates by id, Fy host
 * [pop] their fitness, op host [pop] operation by id (0 dormancy,
 * 1 reproduction, 2 autotroph, 3 heterotroph), perm host [pop] id of each
 * rank (rank 0 best).  Any output may be NULL.  Synchronises. */
int apo_get_trace(apo_t *h, double *Y, double *Fy, int32_t *op, int32_t *perm);

/* Per-kernel timing of n more iterations (n >= 1, clipped like apo_run),
 * measured with HIP events that each launch records itself at the kernel's
 * start and end (kernel execution alone, launch gaps excluded):
 * avg_us[0] rank sort, avg_us[1] step (update + evaluation + selection).
 * Returns the number of iterations executed or a status. */
int apo_time_kernels(apo_t *h, int32_t n, double *avg_us);

/* 256-bin grey-level histogram of an 8-bit image (the input of the Kapur and
 * Otsu objectives; Section 5.2 reduces the image to a threshold criterion):
 *   d_img      device [n] bytes (any alignment)
 *   n          pixels, n < 2^32
 *   host_hist  host [256] uint64 counts (overwritten): count of grey level g
 *   stream     hipStream_t the kernels run on, or NULL (null stream)
 * Allocates a device scratch buffer of about 514 KB for the call (partial
 * counts), runs the histogram kernel and copies the counts to the host;
 * synchronises the stream before returning.  Counts are exact.  Errors:
 * APO_E_INVAL (NULL host_hist, NULL d_img with n > 0, n >= 2^32),
 * APO_E_NOMEM, APO_E_DEVICE. */
int apo_histogram_u8(const uint8_t *d_img, uint64_t n, uint64_t *host_hist, void *stream);

/* The histogram of apo_histogram_u8 for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  It calls no allocating routine: its scratch (partial
 * counts; about 514 KB) is a file-scope device array of
 * the library, one copy per device, held until the process ends; its device
 * address is looked up on the first call on each device.
 *   d_img   device [n] bytes (any alignment)
 *   n       pixels; at most 2^32 - 1 (the scratch holds 32-bit partial
 *           counts): larger n returns APO_E_UNSUPPORTED
 *   d_hist  device [256] uint64 counts, 8-byte aligned (overwritten by the
 *           kernels): count of grey level g
 *   stream  hipStream_t the kernels run on, or NULL (null stream)
 * Stream-ordered and asynchronous (two kernel launches, no memset node, no
 * synchronisation), so it may be captured into a HIP graph.  Every call on a
 * device shares that device's scratch: calls that overlap on one device
 * (concurrent streams, or host threads) race and give wrong counts; calls
 * ordered on one stream do not.  Counts equal apo_histogram_u8's.  Errors:
 * APO_E_INVAL (NULL or misaligned d_hist, NULL d_img with n > 0),
 * APO_E_UNSUPPORTED (n >= 2^32), APO_E_DEVICE (launch failure). */
int apo_histogram_u8_noalloc(const uint8_t *d_img, uint64_t n, uint64_t *d_hist, void *stream);

/* Stage times of a handle whose step runs in the GEMM form (rotated
 * objectives above 512 dimensions in binary32, and every APO_BF16 handle):
 * n more iterations (clipped like apo_run), HIP events recorded by each
 * launch at the kernel's start and end, average microseconds per iteration
 * into us[6]: [0] candidates, [1] product (BF16 estimate, or binary32), [2]
 * BF16 classification, [3] binary32 re-score product, [4] selection, [5]
 * sort ([2] and [3] are 0 in binary32).  Returns n, or APO_E_STATE for a handle
 * of another form. */
int apo_time_gemm_stages(apo_t *h, int32_t iters, double *us);

/* BF16 form: candidates re-scored in binary32 so far and candidates whose
 * fitness was estimated (pop per iteration); both 0 for other handles. */
int apo_precision_stats(apo_t *h, int64_t *rescored, int64_t *estimated);

/* Static description of a status code. */
const char *apo_strerror(int status);

/* ------------------------------------------------------------------------
 * Batches of independent runs.  Many runs of Algorithm 1, each with its own
 * dimension, population, objective, seed and budget, advance together:
 * every iteration is one sort launch per precision and one step launch per
 * kernel shape covering all runs (workgroups are mapped to (run, block)
 * through a device table), replayed from captured graphs.  Each run
 * computes exactly what a standalone handle with the same arguments
 * computes (same kernels, same draws, same arithmetic).
 * ------------------------------------------------------------------------ */
typedef struct apo_batch apo_batch_t;   /* opaque, owned by the caller until apo_batch_destroy */

typedef struct {
    int32_t dim;
    const double *lb, *ub;   /* host [dim], copied                                   */
    int32_t pop;
    int32_t np;
    double pf_max;
    uint64_t seed;
    apo_options opt;         /* max_iter, precision, objective, run_id, flags; its
                                stream and workspace must be NULL / 0 (the batch
                                supplies both)                                      */
} apo_run_desc;

typedef struct {
    void *stream;            /* hipStream_t, or NULL = library-owned stream          */
    void *workspace;         /* device buffer of apo_batch_workspace_bytes, or NULL  */
    size_t workspace_bytes;
} apo_batch_options;

/* Device bytes a batch of these runs needs (0 if any description is
 * invalid): every run's own workspace plus the launch tables. */
size_t apo_batch_workspace_bytes(int32_t n, const apo_run_desc *runs);

/* Creates n >= 1 runs and their initial populations.  Errors: those of
 * apo_create for the first failing run (nothing is left allocated),
 * APO_E_INVAL for n < 1, a run description with a stream or workspace, or
 * a workspace that is too small. */
int apo_batch_create(int32_t n, const apo_run_desc *runs, const apo_batch_options *opt,
                     apo_batch_t **out);

/* Advances every run by min(iters, the smallest remaining budget)
 * iterations, asynchronously on the batch stream.  Returns that count
 * (>= 0) or a status; APO_E_STATE if the runs are not all at the same
 * iteration (after apo_set_state on a member). */
int apo_batch_run(apo_batch_t *b, int32_t iters);

/* View of run i (0 <= i < n) as a handle owned by the batch: apo_best,
 * apo_info, apo_get_state, apo_set_state and apo_get_trace work on it;
 * apo_step, apo_run, apo_time_kernels and apo_destroy return APO_E_STATE. */
int apo_batch_member(apo_batch_t *b, int32_t i, apo_t **run);

/* Launch-schedule autotuner: times `iters` iterations (clipped to the
 * smallest remaining budget; at least 1) under each candidate schedule --
 * step launches in sequence or on parallel graph branches, workgroups in
 * run order or interleaved across runs -- restoring the runs' state after
 * every trial, and keeps the fastest.  Results do not depend on the
 * schedule.  Allocates a temporary device copy of the runs' state.
 * *schedule (may be NULL) receives the chosen schedule (0..3), *us (may be
 * NULL) four timings in microseconds per iteration.
 * Known issue: on an MI355X the process has ended once with a host
 * segmentation fault inside the trials (no GPU fault reported); the cause is
 * not found (the host code passes an AddressSanitizer harness), so callers
 * that cannot risk it keep the default schedule and do not call this. */
int apo_batch_tune(apo_batch_t *b, int32_t iters, int32_t *schedule, double *us);

/* Releases the batch, its members and (if library-allocated) its stream
 * and workspace after the batch stream drains. */
int apo_batch_destroy(apo_batch_t *b);

#ifdef __cplusplus
}
#endif

#endif /* APO_H */
