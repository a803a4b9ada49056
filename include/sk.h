/*
 * sk.h - C ABI of libsk: Sinkhorn diagonal scaling as a preprocessing step for
 * the optimal assignment problem, on AMD Instinct MI355X (gfx950).
 *
 * Method: Sharify, Gaubert, Grigori, "Solution of the optimal assignment
 * problem by diagonal scaling algorithms" (arXiv:1104.3830).
 *   - X(p) = D_r A^(p) D_c is the bistochastic matrix of maximal relative
 *     entropy for the Hadamard power A^(p) = (a_ij^p) (eq. pentropyopt,
 *     Theorem prop-borweinlewisnussbaum); as p grows it tends to the optimal
 *     permutation(s) (Theorem thm:prop-converge1).
 *   - It is computed by Sinkhorn iteration u = I(A^(p) v), v = I(A^(p)T u)
 *     (eqs. dad1-dad3) in log coordinates (Section 4.1.2), with a
 *     continuation in p, stopping when the column-stochastic iterate has
 *     max_i |r_i - 1| < eps (Section 4.2).
 *   - Entries with x_ij(p) < t are deleted (eq. matrixred); the reduced sparse
 *     instance is solved exactly; the certificate of Proposition prop:aoc
 *     bounds the loss (eq. optratio).
 *
 * Conventions (all entry points):
 *   - The input is the log-weight matrix W = log A as int16, row-major, pitch
 *     n. Valid weights lie in [-16384, 16383]; SK_SENTINEL (INT16_MIN) stands
 *     for a_ij = 0. Weights and the deformation parameter p are integers, so
 *     p*w_ij is exact.
 *   - Every buffer is owned by the caller. "device" pointers are HIP device
 *     memory on the context's device; "host" pointers are ordinary host memory.
 *   - Entry points return a status code; no exception crosses the ABI. The
 *     text of the last error of a context is available from sk_last_error.
 *   - A context is used by one host thread at a time, except sk_submit /
 *     sk_poll, which may be called from any thread.
 */
#ifndef SK_H
#define SK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SK_SENTINEL (-32768)
#define SK_MAX_LADDER 32

typedef struct sk_ctx sk_ctx;

typedef enum {
    SK_OK = 0,
    SK_EINVAL = 1,       /* bad argument (size, pointer, parameter) */
    SK_ENOMEM = 2,       /* arena or output capacity too small */
    SK_ENOCONV = 3,      /* a stage hit its iteration cap; results are still usable */
    SK_EINFEASIBLE = 4,  /* the (reduced) matrix has no perfect matching */
    SK_EAGAIN = 5,       /* served request not finished yet / queue full */
    SK_EDEVICE = 6,      /* HIP runtime error */
    SK_ENOSUPPORT = 7    /* a row or column of A has no positive entry */
} sk_status;

/* How the sweeps read the matrix. */
typedef enum {
    SK_W_I16 = 0,   /* recompute exp(p w_ij + f_i + g_j) from int16 W in every sweep */
    SK_K_BF16 = 1,  /* sweep a stored K_ij = exp(p w_ij + f_i + g_j), bfloat16 */
    SK_K_F32 = 2    /* sweep a stored K, float32 */
} sk_storage;

/* Parameters of a scaling run (Algorithm alg:alg1 with a fixed p ladder).
 *   p_ladder/n_p : integer deformation parameters, applied in order; the
 *                  scalings are carried from one p to the next with
 *                  p^-1 log u and p^-1 log v held fixed (warm start).
 *   tol          : a stage stops at the first iterate with max_i |r_i - 1| < tol
 *                  (0 = run exactly max_iters_per_stage iterations).
 *   max_iters_per_stage : iteration cap per stage (>= 1).
 *   check_every  : the host reads the device's convergence flag every
 *                  check_every iterations; the device itself stops at the
 *                  exact iteration, so this only bounds wasted launches.
 *   threshold    : t of eq. matrixred, used by sk_prune (0 < t <= 1).
 *   storage      : see sk_storage.
 *   opt_ratio    : required gamma of eq. optratio; >= 1 makes sk_solve stop at
 *                  the first p that reaches it, < 1 evaluates the last p only.
 *   warm_start   : 0 = cold start (v = 1 for the first p); 1 = start from the
 *                  potentials passed in (their p is p_ladder[0]).
 *   fused        : 0 = a row-sweep launch and a column-sweep launch per
 *                  iteration (each reads the matrix); 1 = one single-pass
 *                  launch per iteration that forms the row sums and the new
 *                  column sums from one read of the matrix (single instance,
 *                  n % 8 == 0 for int16 W). Both give the same iterates up to
 *                  FP32 summation order.
 *   deform_a     : 0 = continuation over the ladder (stages at fixed p).
 *                  > 0 = the deformed Sinkhorn iteration (Section 3.2,
 *                  schedule p_m = a log(m + 1) of Theorem
 *                  logconvergencepositive): one stage in which iteration m
 *                  (from 1) runs at p_m = deform_a * ln(m + 1) kept in
 *                  [p_ladder[0], p_ladder[n_p - 1]], with u and v carried
 *                  unscaled from one p to the next; it stops at the first
 *                  iterate computed at the last p whose residual is below
 *                  tol, or at max_iters_per_stage. int16 W (storage 0)
 *                  rounds p_m to an integer (its exact exponents need an
 *                  integer p); real-valued weights (sk_scale_real) run p_m
 *                  unrounded.
 *   method       : SK_SINKHORN (0) = Sinkhorn iteration; SK_NEWTON (1) =
 *                  Newton iteration (Section 5.2, the Knight-Ruiz method):
 *                  at each p, x o (S x) = 1 for S = [[0, X], [X^T, 0]] with
 *                  conjugate-gradient inner solves, until max_i |1 - (x o S
 *                  x)_i| <= tol; max_iters_per_stage then bounds the products
 *                  with S per stage (reported as iterations). One int16
 *                  instance, not fused, not deformed.
 *   prescale     : real-valued entry points only (0 elsewhere). 1 = p acts on
 *                  the prescaled matrix of Section 4.1.1 (the one Algorithm
 *                  alg:alg1 scales): with w_min, w_max the smallest and
 *                  largest finite log-weights, p on A' = A^(m)/c equals
 *                  p / (w_max - w_min) on A when w_max - w_min > 1 (max/min
 *                  > e), else p (A' = A / min(A)); gamma (eq. optratio) is
 *                  then the prescaled matrix's. 0 = p acts on A. */
typedef struct {
    int32_t p_ladder[SK_MAX_LADDER];
    int32_t n_p;
    double tol;
    int64_t max_iters_per_stage;
    int32_t check_every;
    double threshold;
    int32_t storage;
    double opt_ratio;
    int32_t warm_start;
    int32_t fused;
    double deform_a;
    int32_t method;
    int32_t prescale;
} sk_params;

enum { SK_SINKHORN = 0, SK_NEWTON = 1 };

/* Per-run report. Residuals are max_i |r_i - 1| (rows) and max_j |c_j - 1|
 * (columns) of the returned iterate. "Balanced matrix" is the matrix the
 * sweeps actually scale: exp(p w + log u + log v) for SK_W_I16, the stored K
 * times its scalings for SK_K_BF16 / SK_K_F32. */
typedef struct {
    double residual_fp32;      /* as measured by the sweeps (FP32) */
    double residual_fp64;      /* FP64 recheck of the balanced matrix, rows */
    double col_residual_fp64;  /* FP64 recheck of the balanced matrix, columns */
    double residual_exact_fp64;     /* FP64 rows of exp(p w + log u + log v) from W */
    double col_residual_exact_fp64; /* same, columns */
    double ub;                 /* right-hand side of Proposition prop:aoc */
    int64_t iters_total;
    int64_t iters_stage[SK_MAX_LADDER];
    int32_t p_final;
    int32_t stages_capped;     /* stages that hit max_iters_per_stage */
    int64_t nnz_kept;          /* set by sk_prune */
    int32_t absorbs;           /* K recomputations (stored-K storages) */
    double seconds;
    /* set by sk_solve (NaN / 0 elsewhere): */
    double log_gamma;          /* log of the ratio gamma of eq. optratio: ub - w(B) */
    double threshold_used;     /* threshold t of the returned reduced matrix B */
    int32_t stages_evaluated;  /* stages whose B and gamma were formed */
    int32_t optimal_proved;    /* 1 if ub - w(B) < 1: with integer weights no
                                  permutation of A weighs more than w(B) */
    double p_scale;            /* the stage's p is p_final * p_scale (1 unless
                                  the real-valued path prescales) */
} sk_report;

/* Potentials (scalings) of one instance, in device memory, 16*n bytes laid
 * out as four arrays of n: F int32, phi float32, G int32, gam float32, with
 * log u_i = F_i + phi_i and log v_j = G_j + gam_j (natural logarithms), so
 * x_ij = exp(p w_ij + log u_i + log v_j). */
size_t sk_potentials_bytes(int32_t n);

/* Reduced instance in CSR form: row_ptr int64[n+1], col int32[nnz],
 * w int16[nnz] (the original log-weights of the kept entries); columns in
 * increasing order within a row. `nnz` is the capacity on input to sk_prune
 * and the count on output. */
typedef struct {
    int32_t n;
    int64_t nnz;
    int64_t *row_ptr;
    int32_t *col;
    int16_t *w;
} sk_csr;

/* Device memory a context needs to scale one instance of size n with the
 * given storage (the arena passed to sk_create must be at least this). When
 * n is not a multiple of 8 this includes the library's copy of W at a row
 * pitch of n rounded up to 8 (so that every size takes 16-byte loads).
 * 0 for n outside [1, 65536]. */
size_t sk_arena_bytes(int32_t n, int32_t storage);

/* Creates a context on `device`, launching on `hip_stream` (a hipStream_t;
 * NULL = the null stream), sub-allocating its working memory from the
 * caller's device arena [arena_dev_ptr, arena_dev_ptr + arena_bytes).
 * The arena must stay valid until sk_destroy. */
sk_status sk_create(sk_ctx **out, int device, void *hip_stream, void *arena_dev_ptr,
                    size_t arena_bytes);

/* Waits for all work of the context, stops its serving thread, frees its host
 * resources. */
sk_status sk_destroy(sk_ctx *ctx);

/* Text of the last error recorded on ctx ("" if none). Valid until the next
 * call on ctx. */
const char *sk_last_error(const sk_ctx *ctx);

/* Scales A^(p) for each p of the ladder (Section 3.1 with the logarithmic
 * form of Section 4.1.2), then rechecks the result in FP64 and computes the
 * certificate of Proposition prop:aoc.
 *   n          : 1 <= n <= 65536. Above 16384 only the two-sweep Sinkhorn
 *                iteration on int16 W (storage SK_W_I16, fused = 0, method
 *                SK_SINKHORN), else SK_EINVAL; the same holds for sk_solve,
 *                sk_prune and sk_scale_static. Batches, served requests and
 *                real-valued weights take n <= 16384.
 *   W          : device, n*n int16 (read only).
 *   potentials : device, sk_potentials_bytes(n); output, and input when
 *                params->warm_start = 1.
 *   report     : host, may be NULL.
 * Blocks until done. Returns SK_ENOCONV when a stage hit its cap (the
 * potentials and report are still valid), SK_ENOSUPPORT when a row or column
 * of A is empty. */
sk_status sk_scale(sk_ctx *ctx, const int16_t *W, int32_t n, const sk_params *params,
                   void *potentials, sk_report *report);

/* Builds the reduced matrix of eq. matrixred: B keeps (i, j) iff
 * x_ij(p) >= params->threshold, with x from the potentials and
 * p = the last p of the ladder.
 *   csr : row_ptr, col, w are DEVICE buffers with room for n+1, csr->nnz,
 *         csr->nnz entries; on return csr->nnz is the number kept.
 * Returns SK_ENOMEM (and the needed count in csr->nnz) if the capacity is
 * too small; row_ptr is valid in that case. */
sk_status sk_prune(sk_ctx *ctx, const int16_t *W, int32_t n, const void *potentials,
                   const sk_params *params, sk_csr *csr);

/* Exact maximum-weight perfect matching of a reduced instance (the
 * sequential exact step of Section 4.2), by shortest augmenting paths with
 * potentials on the sparse graph (the O(n (m + n log n)) class of Section 1).
 *   csr  : HOST buffers.
 *   perm : host int32[n]; perm[i] = column assigned to row i.
 *   weight : host; sum_i w[i, perm(i)].
 * Returns SK_EINFEASIBLE if B has no perfect matching. Thread-safe. */
sk_status sk_solve_reduced(const sk_csr *csr, int32_t *perm, int64_t *weight);

/* The path of Algorithm alg:alg1 (Section 4.2) for one instance, natively:
 * the continuation over params->p_ladder (as sk_scale), and at the end of a
 * stage the FP64 certificate ub (Proposition prop:aoc), the reduced matrix B
 * of eq. matrixred at t = params->threshold, an exact optimal assignment of B
 * (as sk_solve_reduced) and log gamma = ub - w(B) (eq. optratio).
 *   params->opt_ratio >= 1: every stage is evaluated; the call stops at the
 *     first stage with gamma <= opt_ratio (the loop condition of the
 *     algorithm, read as "raise p while gamma exceeds the ratio").
 *   params->opt_ratio < 1: only the last stage is evaluated.
 * When B has no perfect matching at the last stage, t is lowered tenfold, at
 * most three times.
 *   W          : DEVICE, n*n int16 row-major, caller-owned, read-only.
 *   potentials : DEVICE, sk_potentials_bytes(n), caller-owned; read first
 *                when params->warm_start; receives the scalings of the
 *                returned stage.
 *   perm       : HOST int32[n]; perm[i] = column assigned to row i.
 *   weight     : HOST; w(B) = sum_i W[i][perm[i]], an optimal weight of B.
 *   report     : HOST, may be NULL; work counters cover all stages run,
 *                the other fields the returned stage.
 * Any storage; the stored-K storages evaluate a stage after folding their
 * scalings into the potentials. Needs an arena of
 * sk_solve_arena_bytes(n, storage, kept), kept >= the entries B keeps
 * (else SK_ENOMEM). Returns SK_OK when the
 * ratio was reached (or, with opt_ratio < 1, B had a perfect matching);
 * SK_ENOCONV when the ladder ended first (the stage with the smallest gamma
 * is returned); SK_EINFEASIBLE when no B had a perfect matching;
 * SK_ENOSUPPORT for an empty row or column of A. Blocks. */
sk_status sk_solve(sk_ctx *ctx, const int16_t *W, int32_t n, const sk_params *params,
                   void *potentials, int32_t *perm, int64_t *weight, sk_report *report);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): sk_scale
 * with its working memory taken from a static device array of the library
 * instead of the context's arena. The array (SK_STATIC_SCRATCH_BYTES, on each
 * GPU the library runs on) is resolved by sk_create and held until the
 * process ends; this call allocates nothing. The caller still passes W and
 * the potentials (as for sk_scale) and may pass a context created with no
 * arena (arena_dev_ptr NULL).
 *   Limit: instances whose working memory (sk_arena_bytes(n, storage))
 *   exceeds SK_STATIC_SCRATCH_BYTES are rejected with SK_ENOMEM before any
 *   work is queued: int16 W up to n = 44016 when n is a multiple of 8 (else
 *   the library's padded copy of W must fit too: n <= 5343), stored BF16 K
 *   up to n = 5336, stored FP32 K up to n = 3888 (n a multiple of 8).
 *   Every call on a GPU shares that GPU's array and leaves its contents
 *   behind (each call initialises what it reads): calls that overlap on one
 *   GPU, from any contexts or threads, race and must be serialised by the
 *   caller. Same arguments, statuses and results as sk_scale. */
#define SK_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
sk_status sk_scale_static(sk_ctx *ctx, const int16_t *W, int32_t n, const sk_params *params,
                          void *potentials, sk_report *report);

/* Real-valued log-weights (Section 5's Euclidean random assignment, and
 * Algorithm alg:alg1 with its own p schedule on the prescaled matrix,
 * Section 4.1.1). W is float32 log A, row-major, pitch n, with -INFINITY for
 * a_ij = 0 (NaN and +inf are rejected). p = p_ladder[k] * (prescale ?
 * 1 / (w_max - w_min) : 1) need not be an integer. Each term
 * exp(p (w_ij - w_max) + log u_i + log v_j) has its exponent formed in FP64
 * and split exactly into a power of two and a fraction in [-1/2, 1/2] whose
 * exp2 is taken in FP32 (about 2 FP32 ulp per term); row and column sums
 * accumulate in FP32, the recheck and certificate in FP64. The potentials
 * have the int16 path's layout, for the shifted weights: x_ij =
 * exp(p (w_ij - w_max) + log u_i + log v_j), w_max the largest finite w.
 * params: storage SK_W_I16 (the sweeps read W), not fused, not deformed,
 * Sinkhorn; ub and weights are in the units of W. One instance per call.
 * Errors as for sk_scale / sk_solve; SK_EINVAL for a NaN or +inf weight. */
typedef struct {
    int32_t n;
    int64_t nnz;
    int64_t *row_ptr;
    int32_t *col;
    float *w;
} sk_csr_real;

/* Device arena bytes sk_scale_real / sk_solve_real need at size n when the
 * reduced matrix keeps at most max_kept entries (0 for sk_scale_real). */
size_t sk_real_arena_bytes(int32_t n, int64_t max_kept);

/* sk_scale for real-valued log-weights. W: DEVICE float[n*n]. */
sk_status sk_scale_real(sk_ctx *ctx, const float *W, int32_t n, const sk_params *params,
                        void *potentials, sk_report *report);

/* sk_solve for real-valued log-weights (Algorithm alg:alg1 with
 * opt_ratio >= 1): per stage the FP64 certificate, the reduced matrix at t,
 * an exact optimum of it on the host (sk_solve_reduced_real) and log gamma =
 * s (ub - w(B)) with s = p_scale when params->prescale (the prescaled
 * matrix's gamma), else 1. *weight = w(B) = sum_i W[i][perm[i]] in FP64.
 * optimal_proved stays 0 (no integrality). */
sk_status sk_solve_real(sk_ctx *ctx, const float *W, int32_t n, const sk_params *params,
                        void *potentials, int32_t *perm, double *weight, sk_report *report);

/* Exact maximum-weight perfect matching of a real-weight reduced instance
 * (HOST buffers), by shortest augmenting paths (Dijkstra with potentials) in
 * FP64: optimal up to the rounding of the sums. SK_EINFEASIBLE without a
 * perfect matching. Thread-safe. */
sk_status sk_solve_reduced_real(const sk_csr_real *csr, int32_t *perm, double *weight);

/* Device arena bytes sk_solve needs for this storage when B keeps at most
 * max_kept entries. */
size_t sk_solve_arena_bytes(int32_t n, int32_t storage, int64_t max_kept);

/* Served path (continuous batching). sk_submit copies W (HOST, n*n int16)
 * into library-owned staging and queues the request; the context's serving
 * thread admits queued requests when their device footprint fits in the
 * arena, sweeps all admitted instances together, and on convergence prunes,
 * solves the reduced instance and checks the certificate. *ticket receives
 * an id for sk_poll. The caller's buffer may be reused when the call
 * returns. Returns SK_EAGAIN when the queue is full or no staging memory is
 * free (a pinned ring of 512 MiB; poll finished requests, then submit again). */
sk_status sk_submit(sk_ctx *ctx, const int16_t *W_host, int32_t n, const sk_params *params,
                    uint64_t *ticket);

/* Completion queue of the served path, for callers that hold many tickets:
 * moves up to `max` tickets of finished, not yet collected requests (in the
 * order they finished) into `tickets` (host uint64[max], caller-owned) and
 * returns how many; collect each with sk_poll. 0 when none is pending or no
 * request was submitted; -1 on a null context or bad arguments. A ticket
 * finished but not listed (the list keeps the last 65536) stays pollable. */
int32_t sk_completed(sk_ctx *ctx, uint64_t *tickets, int32_t max);

/* Non-blocking. Returns SK_EAGAIN while the request runs; otherwise its final
 * status, with perm (host int32[n]), weight and report (may be NULL) filled,
 * and releases the ticket. */
sk_status sk_poll(sk_ctx *ctx, uint64_t ticket, int32_t *perm, int64_t *weight,
                  sk_report *report);

/* Batched scaling of independent instances in one set of launches per sweep
 * (each sweep covers every instance). W[k] device pointers, n[k] sizes,
 * potentials[k] device buffers (sk_potentials_bytes(n[k])), reports[k] host
 * (array may be NULL). All instances share params. Per-instance stopping is
 * exact: an instance that converged is skipped by later sweeps. Blocks. */
sk_status sk_scale_batch(sk_ctx *ctx, int32_t count, const int16_t *const *W,
                         const int32_t *n, const sk_params *params, void *const *potentials,
                         sk_report *reports);

/* Device arena bytes sk_scale_batch needs for these sizes (with the padded
 * copy of each W whose n is not a multiple of 8, as for sk_arena_bytes).
 * 0 when a size is outside [1, 16384] (or [1, 65536] for count = 1). */
size_t sk_batch_arena_bytes(int32_t count, const int32_t *n, int32_t storage);

/* Tile-shape table (process-wide). The column sweep splits the rows of an
 * instance of size n into segments of seg_rows[k] rows for the first k with
 * n <= n_max[k] (n_max ascending; seg_rows a multiple of 16 in [16, 1024]);
 * sizes above the last entry, or an empty table, use the built-in rule.
 * The shape depends only on n, so an instance's result does not depend on
 * what else runs with it. Call before any sk_scale / sk_submit; not
 * thread-safe with running calls. count = 0 restores the built-in rule. */
sk_status sk_set_tile_table(const int32_t *n_max, const int32_t *seg_rows, int32_t count);

/* Kernel timing (measurement aid, off by default). While enabled, the
 * context's kernels are timed with HIP events on its stream: the two sweeps
 * of an iteration share the event between them, the short per-iteration
 * finalise and end-of-iteration launches are not timed, and the other
 * kernels are bracketed one by one; durations accumulate per kernel name
 * (launches that only detected a stage end or came after every instance
 * finished are counted under "<name>:detect" and "<name>:idle") until the
 * next enable. sk_profile_read fills up to `max` entries (host array) and
 * returns how many kernels were seen. */
typedef struct {
    char name[32];
    int64_t launches;
    double total_ms;
} sk_kernel_stat;

sk_status sk_profile_enable(sk_ctx *ctx, int enable);
int32_t sk_profile_read(sk_ctx *ctx, sk_kernel_stat *out, int32_t max);

#ifdef __cplusplus
}
#endif

#endif /* SK_H */
