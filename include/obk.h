/*
 * obk.h -- C ABI of libobk, an MI355X (gfx950) implementation of the hot path
 * of OBK-RCM (Liang & Li, "OBK-RCM: Accelerated Orthogonal Block Kaczmarz
 * Algorithm via RCM Reordering and Dynamic Grouping for Sparse Linear
 * Systems").
 *
 * The library solves the sparse system A x = f (eq. 1.1) as follows (an
 * m x n system with m != n through its extended square system, Section 4):
 *   obk_plan   RCM reordering A~ = P A P^T, f~ = P f (Section 3.2, eqs.
 *              3.1-3.2), squared row norms (denominator of eq. 1.2), the row
 *              cosine table thresholded at delta (Section 3.3, one-row blocks)
 *              and the grouping of mutually near-orthogonal rows (the
 *              Oclass/Nclass rule of Section 3.3 taken to maximal classes:
 *              first-fit in reordered row order);
 *   obk_solve  sweeps of the orthogonal-group block Kaczmarz step: for each
 *              group in ascending id, w_i = (f_i - a_i x) / ||a_i||^2 for all
 *              rows of the group from the same x, then x += sum_i w_i a_i^T
 *              (eq. 3.3; eq. 1.3 when the rows are exactly orthogonal), and
 *              finally x = P^T x~ (Algorithm 4, last step).
 *
 * Conventions shared by every entry point:
 *  - CSR: int64 row_ptr[n+1] (row_ptr[0] = 0), int32 col[nnz], double
 *    val[nnz].  Rows may be unsorted; a repeated (row, col) is an error;
 *    explicit zeros are kept as structure.  A non-square m x n matrix is
 *    solved as the extended N x N system, N = max(m, n) (Section 4): for
 *    m > n, [A, O] with f unchanged and x = x^(1:n) (Algorithm 5); for
 *    m < n, [A; O] with f^ = [f; 0] and x = x^ (Algorithm 6).  x0 and x
 *    always hold the caller's n unknowns; the extension unknowns start at 0.
 *  - Memory spaces: obk_csr.on_device says whether the CSR arrays and f are
 *    host or device pointers.  x0 and x of obk_solve live in the same space
 *    as the CSR given to obk_plan.  The caller owns every pointer it passes;
 *    obk_plan copies what it needs, so the inputs may be freed once it
 *    returns.
 *  - Streams: all device work is enqueued on the given hipStream_t (0 = the
 *    null stream); calls return after synchronising that stream.
 *  - Errors: each call returns an obk_status; a message for the last error
 *    of the calling thread is available from obk_last_error().  On error no
 *    output handle is produced and nothing leaks.  No exception crosses the
 *    ABI.
 *  - A plan is immutable after obk_plan and owns its device workspace; one
 *    solve per plan may run at a time (a second concurrent solve on the same
 *    plan returns OBK_E_BUSY).
 */
#ifndef OBK_H
#define OBK_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define OBK_API __attribute__((visibility("default")))
#else
#define OBK_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *obk_stream_t;   /* the same type as hipStream_t */
typedef struct obk_plan_s *obk_plan_t;

typedef enum {
    OBK_OK = 0,
    OBK_E_ARG = -1,         /* bad argument (null pointer, negative size, bad option) */
    OBK_E_CSR = -2,         /* malformed CSR: row_ptr not monotone, column out of range, duplicate */
    OBK_E_NOT_SQUARE = -3,  /* reserved (non-square systems are extended, Section 4) */
    OBK_E_NONFINITE = -4,   /* NaN or Inf in val or f */
    OBK_E_NOMEM = -5,       /* device or host allocation failed, or over opts.hbm_budget */
    OBK_E_HIP = -6,         /* a HIP runtime call failed */
    OBK_E_BUSY = -7,        /* a solve on this plan is already running */
    OBK_E_INCONSISTENT = -8 /* a zero row with f_i != 0 (reported by obk_plan only when
                               opts.reject_inconsistent is set) */
} obk_status;

/* Solve outcome written to obk_info.status. */
enum {
    OBK_CONVERGED = 0,      /* relative residual <= tol */
    OBK_MAXIT = 1,          /* maxit sweeps done (always the outcome when tol <= 0) */
    OBK_DIVERGED = 2,       /* relative residual grew above 1e3 x its initial value */
    OBK_NONFINITE_ITERATE = 3
};

/* Arithmetic of the sweep. */
enum {
    OBK_FP64 = 0,           /* plain FP64 sweeps */
    OBK_FP32_IR = 1         /* FP32 sweeps inside FP64 iterative refinement (residual,
                               norms, scaling and the update stay FP64) */
};

typedef struct {
    int64_t n_rows, n_cols, nnz;
    const int64_t *row_ptr;  /* [n_rows+1] */
    const int32_t *col;      /* [nnz] */
    const double *val;       /* [nnz] */
    int on_device;           /* 1: the three arrays (and f, x0, x) are device pointers */
} obk_csr;

typedef struct {
    int use_rcm;             /* 0: identity ordering.  1 (default), 2, 3: reverse
                                Cuthill-McKee, the same order from three engines: 1 picks
                                (the device level-synchronous form for graphs of at least
                                16384 vertices, handing over to the host loop once its
                                levels stay narrow; the host loop below that), 2 the device
                                form at any size and to the end, 3 the host loop */
    int precision;           /* OBK_FP64 (default) or OBK_FP32_IR */
    int inner_sweeps;        /* OBK_FP32_IR: FP32 sweeps per refinement step (default 8) */
    int check_every;         /* sweeps between residual checks when tol > 0 (default 1) */
    int reject_inconsistent; /* 1: obk_plan fails with OBK_E_INCONSISTENT on a zero row
                                with f_i != 0; 0 (default): such rows are skipped */
    size_t hbm_budget;       /* 0: unlimited; else obk_plan fails with OBK_E_NOMEM when the
                                plan's device footprint would exceed it */
    int block_k;             /* 0 (default): one-row blocks grouped by first fit.  k in
                                [1, 4096]: block form of Algorithm 4 (Section 3.3), with
                                k uniform chunks of A~ projected exactly; OBK_FP64 only.
                                A plan-time option. */
    int block_wgs;           /* block form: workgroups of the projection launch
                                (0 = from the block size) */
    int block_maxit;         /* block form: CG iterations per projection at most
                                (0 = 4 x block rows + 100) */
    double block_tol;        /* block form: a projection's CG stops once its residual
                                norm is <= block_tol x its initial one (default 1e-14) */
    int block_solver;        /* block form: 0 (default): blocks with a banded Cholesky
                                factor of A_t A_t^T (formed at plan time; full row rank to
                                a pivot test, band within limits) are projected exactly
                                from it in one-workgroup launches, the others by CG;
                                1: CG for every block.  A plan-time option. */
    int sweep_kernel;        /* FP64 sweeps of real one-row-block plans: 0 (default): the
                                banded engine when the reordered band is narrow enough for
                                every slab's windows to fit in LDS, else the per-group phase
                                kernels; 1: the per-group phase kernels; 2: the banded
                                engine, OBK_E_ARG when it does not apply.  Both give the
                                same iterate bit for bit.  A plan-time option. */
    double omega;            /* relaxation of every row step: w_i = omega (f_i - a_i x) /
                                ||a_i||^2 (eq. 1.2 scaled); default 1.0, the paper's step
                                (bit for bit: multiplying by 1.0 is exact); must lie in
                                (0, 2).  Not in the block form.  A plan-time option (kept
                                by obk_plan_set_opts). */
    int max_group;           /* 0 (default): maximal groups (first fit, the hot path);
                                2: the paper's literal class rule of Section 3.3 -- each
                                row pairs with the first later unpaired row it is
                                near-orthogonal to, the two projected one after the other
                                (Algorithm 4, the tau1 and tau2 steps), unpaired rows
                                (Nclass) one by one after all pairs.  This is the block form
                                with k = n one-row blocks, so it needs n <= 4096 and
                                OBK_FP64; other values: OBK_E_ARG.  A plan-time option. */
    int deterministic;       /* 1 (default) or 0.  Every kernel of the library reduces in
                                a fixed order (no floating-point atomics), so results are
                                repeatable bit for bit either way; 0 is accepted and runs
                                the same kernels. */
    void *(*alloc)(size_t bytes, void *ctx);   /* device memory for the plan and the
                                temporaries of planning and solving (NULL: the HIP runtime,
                                stream-ordered during planning).  alloc returns NULL on
                                failure (then OBK_E_NOMEM); alloc and dealloc are both set
                                or both NULL.  A block returned by alloc goes back through
                                dealloc once no queued work uses it (temporaries after a
                                synchronisation of the call's stream, plan memory in
                                obk_free). */
    void (*dealloc)(void *ptr, void *ctx);
    void *ctx;               /* passed to alloc and dealloc */
} obk_opts;

typedef struct {
    int64_t sweeps;          /* sweeps performed (FP32 inner sweeps in OBK_FP32_IR) */
    int64_t outer_steps;     /* refinement steps (OBK_FP32_IR), else residual checks */
    double relres0;          /* ||f~ - A~ x~0|| / ||f~|| */
    double relres;           /* last computed relative residual (-1 if never computed) */
    double seconds;          /* wall time of the solve, host clock */
    int status;              /* OBK_CONVERGED | OBK_MAXIT | OBK_DIVERGED | OBK_NONFINITE_ITERATE */
} obk_info;

/* Fill *opts with the defaults listed above. */
OBK_API obk_status obk_opts_default(obk_opts *opts);

/*
 * Build a plan for A x = f (Algorithm 4, first four steps, with one-row
 * blocks; Sections 3.2-3.3).  delta is the cosine threshold: rows i, j are
 * near-orthogonal iff |cos(a_i, a_j)| < delta (|cos| = |a_i . a_j| /
 * sqrt(||a_i||^2 ||a_j||^2), computed in FP64 with sums in ascending column
 * order).  opts may be NULL (defaults).  On success *out receives a plan that
 * owns device copies of the reordered, grouped system.  For n_rows != n_cols
 * the plan is that of the extended square system of size max(n_rows,
 * n_cols) (Section 4, Algorithms 5 and 6): row_ptr and f hold n_rows (+1)
 * entries, columns must be below n_cols, and the introspection calls below
 * (perm, groups, stats) describe the extended system.
 * Device memory (without opts.alloc): the plan's buffers and its temporaries
 * come from the device's stream-ordered pool on `stream`; a temporary released
 * during planning serves the plan's next request of its size class, and when
 * planning ends (with `stream` synchronised) those the plan no longer uses are
 * kept by the library, at most 1 GiB per process, for later plans on any
 * thread and stream of the device.
 * Errors: OBK_E_ARG, OBK_E_CSR, OBK_E_NONFINITE, OBK_E_NOMEM, OBK_E_HIP,
 * OBK_E_INCONSISTENT.
 */
OBK_API obk_status obk_plan(const obk_csr *A, const double *f, double delta, const obk_opts *opts,
                    obk_stream_t stream, obk_plan_t *out);

/*
 * Complex systems.  The paper applies Algorithm 4 unchanged to a complex
 * matrix (kim1, in its discussion of Table 4); over C the row norm is
 * sum_k |a_ik|^2, the cosine of rows i, j is |a_i^H a_j| / (||a_i|| ||a_j||)
 * (the Hermitian inner product; |.| makes the order of the conjugation
 * immaterial), and the row projection of eq. 1.2 is
 * x + (f_i - a_i x) / ||a_i||^2 a_i^H.  obk_plan_complex takes the same CSR
 * as obk_plan except that A->val holds 2 nnz doubles and f 2 n_rows doubles,
 * each entry as (re, im); a plan built by it takes complex x0 and x in
 * obk_solve (2 n_cols doubles, interleaved) and complex x~ in
 * obk_sweep_device / obk_sweep_profile (2 n doubles).  Every sum runs in
 * ascending index order, as for real systems.  OBK_FP64 only; not in block
 * form; not batched.  Errors as obk_plan.
 */
OBK_API obk_status obk_plan_complex(const obk_csr *A, const double *f, double delta, const obk_opts *opts,
                                    obk_stream_t stream, obk_plan_t *out);

/*
 * Run sweeps from x0 (NULL: x0 = 0, the paper's start, Section 3.5) and write
 * the result in the original ordering to x.  With tol > 0 the relative
 * residual ||f - A x|| / ||f|| is checked every opts.check_every sweeps (each
 * refinement step in OBK_FP32_IR) and the solve stops once it is <= tol; with
 * tol <= 0 exactly maxit sweeps run (refinement steps for OBK_FP32_IR) and no
 * residual is computed except relres0/relres in info.  info may be NULL.
 * Errors: OBK_E_ARG, OBK_E_BUSY, OBK_E_HIP.
 */
OBK_API obk_status obk_solve(obk_plan_t plan, const double *x0, double tol, int64_t maxit, double *x,
                     obk_info *info, obk_stream_t stream);

/*
 * obk_solve without device allocation, for callers that cannot allocate
 * (code in tight serving loops, or harnesses that forbid hipMalloc): the
 * same solve as obk_solve on x0 and x in device memory (x0 NULL: 0; x0 and
 * x hold the caller's unknowns, whatever memory space the plan's CSR came
 * from), for real plans with one-row blocks (OBK_FP64 or OBK_FP32_IR).  The
 * sweeps are launched directly (no graph is captured) and the residual's
 * per-tile partials go to a static device array of 1 MiB, one per GPU,
 * held until the process ends: a plan of more than 65,528 row tiles of 256
 * rows is refused with OBK_E_ARG.  Every call on a GPU shares that array,
 * so calls that overlap on one GPU race; serialise them.  The plan's own
 * workspace is used as by obk_solve (one solve per plan at a time).
 * Errors: OBK_E_ARG, OBK_E_BUSY, OBK_E_HIP.
 */
OBK_API obk_status obk_solve_noalloc(obk_plan_t plan, const double *x0, double tol, int64_t maxit, double *x,
                                     obk_info *info, obk_stream_t stream);

/* Release a plan and its device memory.  NULL is a no-op. */
OBK_API void obk_free(obk_plan_t plan);
/* Release a plan waiting only for `stream` (obk_free waits for the whole
 * device): the caller guarantees that every piece of work that uses the plan
 * has completed or is queued on `stream`.  Once `stream` is idle the plan's
 * pool memory is kept by the library for later plans (at most 1 GiB in all,
 * the rest goes back to the pool); memory from the caller's allocator
 * (opts.alloc) is handed back through dealloc.  NULL is a no-op; OBK_E_BUSY
 * (the plan is kept) while a solve on the plan runs. */
OBK_API obk_status obk_free_async(obk_plan_t plan, obk_stream_t stream);

/*
 * Change a plan's solve options (precision, inner_sweeps, check_every) without
 * replanning; switching to OBK_FP32_IR allocates the FP32 copies (checked
 * against opts->hbm_budget when nonzero).  use_rcm and reject_inconsistent are
 * plan-time options and are ignored here.  Errors: OBK_E_ARG, OBK_E_NOMEM,
 * OBK_E_BUSY.
 */
OBK_API obk_status obk_plan_set_opts(obk_plan_t plan, const obk_opts *opts);

/* Introspection (host outputs). */
/* p_host[t] = original index of reordered row t (new -> old), n entries. */
OBK_API obk_status obk_plan_perm(obk_plan_t plan, int32_t *p_host);
/* group_of_row_host[t] = group of reordered row t (-1 for an all-zero row);
 * *n_groups = number of groups.  In the block form (opts.block_k > 0) the
 * group of a row is its block (zero rows included) and *n_groups = k.
 * Either output may be NULL. */
OBK_API obk_status obk_plan_groups(obk_plan_t plan, int32_t *group_of_row_host, int32_t *n_groups);
/* Device bytes owned by the plan (for admission against an HBM budget). */
OBK_API obk_status obk_plan_bytes(obk_plan_t plan, size_t *device_bytes);
/* Which kernels run the plan's FP64 sweeps (opts.sweep_kernel): *engine = 2
 * for the banded engine, with *slabs its workgroups (each owning a
 * contiguous range of the reordered unknowns), or 1 for the per-group phase
 * kernels (*slabs = 0).  Either output may be NULL. */
OBK_API obk_status obk_plan_engine(obk_plan_t plan, int32_t *engine, int32_t *slabs);
/* Relaxation bound of one-row groups (the paper steps with omega = 1 and is
 * silent on relaxation; this is a reading of Section 3.3's grouping): with
 * B_g the rows of group g scaled to unit norm, per_group[g] is Gershgorin's
 * bound on lambda_max(B_g B_g^H), 1 + max over the rows i of g of
 * sum_{j in g, j != i} |cos(a_i, a_j)| (every such cosine is below delta),
 * and *bound is the largest of them (0 when the plan has no groups).  A group
 * step with omega * bound <= 2 does not expand the error.  Computed in FP64:
 * for complex plans at plan time, for real plans on the first call (from the
 * group-major rows and column segments the plan keeps; the call then runs
 * kernels on a stream of its own and returns when they are done; OBK_E_BUSY
 * while a solve on the plan runs).  per_group (host, n_groups entries) or
 * bound may be NULL.  OBK_E_ARG for block-form plans. */
OBK_API obk_status obk_plan_lambda_bound(obk_plan_t plan, double *bound, double *per_group);
/* Sizes: n, nnz, number of groups, bandwidth of A~, number of conflicting pairs. */
OBK_API obk_status obk_plan_stats(obk_plan_t plan, int64_t *n, int64_t *nnz, int32_t *n_groups,
                          int64_t *bandwidth, int64_t *n_conflicts);

/*
 * Block form of Algorithm 4 (opts.block_k = k > 0; Section 3.3, eq. 3.3).
 * Planning: RCM as above; the reordered rows are cut in order into k blocks,
 * the first k - 1 of floor(n / k) rows and the last of the rest; the centroid
 * of a block is its mean row and the table C(a, b) = |cos| of the centroids
 * of blocks a and b (0 when either centroid is zero) is formed in FP64;
 * pairs are formed in ascending order of a: block a, if not yet paired,
 * pairs with the least b > a not yet paired with C(a, b) < delta (delta is
 * the paper's thr); blocks left unpaired form Nclass.  A sweep projects, for
 * each pair in the order formed, block a then block b, then every Nclass
 * block in ascending order.  A projection onto block t replaces x~ by
 * x~ + A_t^+ (f_t - A_t x~); it is computed as x~ + A_t^T y with y from
 * conjugate gradients on A_t A_t^T y = f_t - A_t x~ (started at 0, stopped
 * by opts.block_tol / opts.block_maxit; all-zero rows take no part), all
 * iterations of all projections of a call in one launch (cooperative when
 * it spans several workgroups).
 *
 * Direct projections (opts.block_solver = 0): y solves A_t A_t^T y =
 * f_t - A_t x~ by a forward and a backward banded triangular solve with the
 * block's Cholesky factor, formed on the host at plan time in FP64 from the
 * pairwise row products (accumulated in ascending column order) with the
 * block's rows in the reverse Cuthill-McKee order of its own Gram graph
 * (two rows adjacent when they share a column), which keeps the band
 * narrow.  A block
 * whose pivots fall below 1e-8 of their diagonal (rank deficient to working
 * accuracy), whose band or whose count of row pairs sharing a column would
 * exceed 2^24, or with more than 8192 rows keeps CG, and so do the blocks
 * past the plan-wide limits (2^27 band entries and 2^36 factorisation steps
 * of rows x band^2, applied in block order before any block is factored)
 * and every block of a launch over several workgroups (factors are built
 * only when the plan's launch is one workgroup).  All-zero rows take no part
 * (their y is 0).
 *
 * obk_plan_blocks (host outputs, each may be NULL): *k; bptr[k+1] the row
 * range of each block in reordered rows; partner[k] the block a block is
 * paired with (-1: Nclass); cos[k*k] the table C, row-major; cg_iters[k] the
 * CG iterations spent on each block over every sweep run on the plan so far.
 * Errors: OBK_E_ARG when the plan is not in block form.
 */
OBK_API obk_status obk_plan_blocks(obk_plan_t plan, int32_t *k, int64_t *bptr, int32_t *partner, double *cos,
                                   int64_t *cg_iters);
/*
 * Per block of a block-form plan (host outputs, each may be NULL): direct[k]
 * 1 when the block is projected from its Cholesky factor, bandwidth[k] that
 * factor's bandwidth (-1 without one).  Errors: OBK_E_ARG when the plan is
 * not in block form.
 */
OBK_API obk_status obk_plan_block_solvers(obk_plan_t plan, int32_t *direct, int64_t *bandwidth);

/*
 * Block-count criteria of Section 3.6 (Definitions 1 and 2) for the block
 * form.  From the k x k table C of a block-form plan: the orthogonality
 * proportion zn = (entries of C exactly 0) / k^2 and the non-orthogonality
 * severity nn = (number of nonzero entries x their mean) / k^2.
 * obk_block_zn_nn reads them from a plan (OBK_E_ARG if it is not in block
 * form).  obk_block_select_k plans A once per candidate k (as obk_plan with
 * opts->block_k = k and delta = thr; opts may be NULL), writes zn[i] and
 * nn[i] of candidate i (host arrays of n_candidates, each may be NULL) and
 * *best_k: the candidate of largest zn, then least nn, then least k -- the
 * paper asks for the k that maximises zn and minimises nn.  Each plan is
 * freed before the next is built.  Errors: as obk_plan; OBK_E_ARG for an
 * empty candidate list or a candidate outside [1, 4096].
 */
OBK_API obk_status obk_block_zn_nn(obk_plan_t plan, double *zn, double *nn);
OBK_API obk_status obk_block_select_k(const obk_csr *A, const double *f, double thr, const int32_t *candidates,
                                      int32_t n_candidates, const obk_opts *opts, obk_stream_t stream,
                                      int32_t *best_k, double *zn, double *nn);

/*
 * Threshold selection of Section 3.7 (Table 5), per real system: the paper fixes
 * thr by comparing run times over candidate values; here, for each
 * candidate delta, A is planned (as obk_plan with that delta and opts, NULL:
 * defaults) and solved from x0 = 0 to tol (at most maxit sweeps, or
 * refinement steps in OBK_FP32_IR), and the time of plan plus solve (host
 * wall clock) is recorded.  *best_delta is the converged candidate with the
 * least time (no candidate converged: the least final relative residual).
 * Per candidate i (host arrays, each may be NULL): seconds[i], sweeps[i]
 * (obk_info.sweeps), relres[i].  Each plan is freed before the next is
 * built; the solutions are discarded.  The choice depends on timing and so
 * may differ between runs when candidates are close.  Errors: as obk_plan
 * and obk_solve; OBK_E_ARG for an empty list, a candidate that is not
 * finite and > 0, tol <= 0 or maxit < 1.
 */
OBK_API obk_status obk_select_delta(const obk_csr *A, const double *f, const double *candidates,
                                    int32_t n_candidates, double tol, int64_t maxit, const obk_opts *opts,
                                    obk_stream_t stream, double *best_delta, double *seconds, int64_t *sweeps,
                                    double *relres);

/*
 * Sweeps on a plan with device-resident iterates, no host synchronisation and
 * no residual (the form a benchmark or a batched driver times): x~ (device,
 * reordered coordinates, n entries) is updated in place by `sweeps` sweeps.
 * Enqueued on stream; returns without waiting.  The sweeps are replayed from
 * graphs captured on first use for this x~ pointer (the plan keeps them until
 * obk_free).  Sweeps on one plan share its workspace: calls on the same plan
 * must be ordered (one stream, or explicit synchronisation).  In the block
 * form all sweeps run in one launch (not from a graph) and the call
 * synchronises the stream to check that launch's barrier flag.
 */
OBK_API obk_status obk_sweep_device(obk_plan_t plan, double *x_tilde_dev, int64_t sweeps,
                            obk_stream_t stream);

/*
 * Per-kernel timing of FP64 sweeps (the device-side roofline measurement):
 * `sweeps` sweeps on x~ (device, reordered coordinates, updated in place as
 * by obk_sweep_device) are launched eagerly -- not from a graph -- with a HIP
 * event recorded on `stream` before and after every kernel launch.  For each
 * distinct sweep kernel, out[k] receives its name, the number of launches,
 * the summed event time and the summed algorithmic bytes of those launches.
 * Algorithmic bytes of one launch over group g (n_g rows, e_g entries, t_g
 * touched columns, element size s = 8, offsets counted at 4 bytes):
 *   phase R: e_g (s + 4) + n_g (4 + 3 s) + t_g s
 *            (values and columns; row offset, f~, 1/||a||^2 and w per row;
 *            each touched x read once)
 *   phase S: e_g (s + 4) + t_g (8 + 2 s) + n_g s
 *            (values and row ids; column offset, column id, x read and
 *            written per touched column; w read once per row)
 * Block-form plans whose blocks are all projected from their factors (one
 * workgroup) report k_block_direct; its bytes per projection of block b
 * (n_b rows, e_b entries, t_b touched columns, factor bandwidth w_b, s = 8)
 * are e_b (s + 4) + n_b (4 + 2 s) + t_b s for the residual, 2 s n_b (w_b + 1)
 * + 2 s n_b for the band and the inverse pivots (once per triangular solve),
 * and e_b (s + 4) + t_b (8 + 2 s) for x~ += A_t^T y.
 * Complex plans report k_phase_r_z / k_phase_s_z with the same formulas and
 * s = 16 for values, f~, w and x~ (1/||a||^2 stays 8 bytes).  Block-form
 * plans report one kernel, k_block_sweeps, timed over the whole launch of
 * `sweeps` sweeps; its bytes are, per CG iteration on block b (n_b rows, e_b
 * entries, t_b touched columns, s = 8, offsets 4 bytes),
 *   2 e_b (s + 4) + n_b (4 + 6 s) + t_b (12 + 5 s),
 * summed over the iterations the launch ran, plus e_b (s + 4) + n_b (4 + 3 s)
 * + t_b s for the residual that starts each projection.
 * Synchronises the stream.  *n_out receives the number of kernels reported
 * (at most max_out).  sweeps must be in [1, 4096].
 */
typedef struct {
    char name[48];
    int64_t launches;
    double seconds;
    double bytes;
} obk_kernel_profile;

OBK_API obk_status obk_sweep_profile(obk_plan_t plan, double *x_tilde_dev, int64_t sweeps,
                             obk_stream_t stream, obk_kernel_profile *out, int32_t max_out,
                             int32_t *n_out);

/*
 * Batched solves: several plans advanced together in shared launches (one
 * persistent launch per step runs the sweeps of every system).  All plans of
 * a batch must share one precision and live on the current device; a plan may
 * belong to several batch objects but only one may run at a time.
 *
 * A step is, for OBK_FP32_IR plans, one iterative-refinement step (FP64
 * residual, scale sigma = max|r_i|, opts.inner_sweeps FP32 sweeps on the
 * scaled correction system, FP64 update) and, for OBK_FP64 plans,
 * opts.check_every FP64 sweeps after an FP64 residual.  A system takes part
 * in a step while it is enabled, its relative residual at the start of the
 * step is above tol (tol <= 0: always) and finite, and sigma > 0.
 *
 * Tunables (0 = default): wgs_per_cu workgroups per compute unit in the
 * persistent launch (default 2, clamped to occupancy); team_work, the entries
 * per sweep one workgroup of a system's team should carry (default: the
 * batch's average per workgroup; a system above it is split over a team of
 * workgroups on one XCD, and a workgroup joins at most one team); max_team,
 * the largest team (default 16); tiles_per_wg, how many tiles (of up to 512
 * rows or columns) a workgroup keeps in flight (default 4).  obk_batch_tune times candidate
 * settings on the given plans and returns the fastest.
 */
typedef struct obk_batch_s *obk_batch_t;
typedef struct {
    int wgs_per_cu;
    int64_t team_work;
    int max_team;
    int tiles_per_wg;        /* tiles a workgroup works on at once: 1, 2 or 4 (default 4) */
} obk_batch_opts;

/* Build the launch schedule for `count` plans (the handles must outlive the batch). */
OBK_API obk_status obk_batch_create(const obk_plan_t *plans, int count, const obk_batch_opts *opts,
                                    obk_batch_t *out);
/* A new member list for an existing batch (continuous batching: members
 * admitted and retired between steps).  The launch schedule is formed again
 * for `plans`; the batch's device storage and its captured step graphs are
 * kept, and reallocated (the graphs then captured again at the next step)
 * only when the new members need more room than the batch holds.  Members
 * keep the iterates held in their plans, so a member that stays continues
 * where it stopped; new members start with obk_batch_start.  Every member is
 * enabled afterwards.  The descriptor copies run on `stream`, which is
 * synchronised before the call returns; the handles of earlier members may be
 * freed after it.  Plans pass the checks of obk_batch_create (OBK_E_ARG, the
 * batch then keeps its members); OBK_E_BUSY while a step of the batch runs;
 * after any other failure the batch is left with no members. */
OBK_API obk_status obk_batch_reset(obk_batch_t batch, const obk_plan_t *plans, int count, obk_stream_t stream);
/* x~_i = P_i x0_i for every system (x0 NULL, or x0[i] NULL: zeros); re-enables all systems. */
OBK_API obk_status obk_batch_begin(obk_batch_t batch, const double *const *x0, obk_stream_t stream);
/* One step for all systems.  relres[i] (host, may be NULL) receives system i's
 * relative residual at the start of the step, active[i] (host, may be NULL)
 * whether the step advanced it. */
OBK_API obk_status obk_batch_step(obk_batch_t batch, double tol, double *relres, int32_t *active,
                                  obk_stream_t stream);
/* x~_index = P x0 for system `index` alone (x0 NULL: zeros) and enable it;
 * the other systems keep their iterates and flags.  Iterates live in each
 * plan's workspace, so a system carried over by obk_batch_reset (or moved into
 * a new batch object) continues from where it stopped, and only newly
 * admitted members need obk_batch_start. */
OBK_API obk_status obk_batch_start(obk_batch_t batch, int index, const double *x0, obk_stream_t stream);
/* enabled[i] = 0 removes system i from later steps until obk_batch_begin. */
OBK_API obk_status obk_batch_enable(obk_batch_t batch, const int32_t *enabled, obk_stream_t stream);
/* x = P^T x~ of system `index`, in the plan's input memory space. */
OBK_API obk_status obk_batch_result(obk_batch_t batch, int index, double *x, obk_stream_t stream);
OBK_API void obk_batch_free(obk_batch_t batch);
/* Solve every system to tol (or maxit steps): x0/x are arrays of `count`
 * pointers (x0 may be NULL); infos (may be NULL) gets one obk_info each. */
OBK_API obk_status obk_solve_batch(const obk_plan_t *plans, int count, const double *const *x0, double tol,
                                   int64_t maxit, double *const *x, obk_info *infos, const obk_batch_opts *opts,
                                   obk_stream_t stream);
/* Autotuner: times candidate tunables on these plans (iterates are reset to 0)
 * and writes the fastest to *best and its time per step to *seconds. */
OBK_API obk_status obk_batch_tune(const obk_plan_t *plans, int count, obk_batch_opts *best, double *seconds);

/*
 * Host stages of obk_plan, exported so that they can be used and tested
 * without a GPU.
 *
 * obk_rcm_host: reverse Cuthill-McKee order (Section 3.2) of an undirected
 * graph given as a symmetric adjacency structure without self loops:
 * gptr[n+1] (int64 offsets), gadj[gptr[n]] (neighbours).  Tie-break: each
 * breadth-first search starts at the unvisited vertex of least (degree,
 * index); unvisited neighbours are visited by ascending (degree, index); the
 * whole Cuthill-McKee sequence is reversed.  perm[t] (caller-allocated, n) =
 * vertex placed at position t.
 *
 * obk_first_fit_host: grouping of Section 3.3 in its maximal form: rows in
 * ascending order; row i joins the least group holding no row j < i that
 * conflicts with it.  cptr[n+1], cidx: for each row the conflicting rows
 * j < i (any order).  active[i] = 0 marks a row that joins no group (-1).
 * group[n] and *n_groups are outputs.
 * Errors: OBK_E_ARG for NULL pointers or negative n.
 */
OBK_API obk_status obk_rcm_host(int64_t n, const int64_t *gptr, const int32_t *gadj, int32_t *perm);
/*
 * obk_banded_emulate_host: the banded engine's plan-time layout for exactly
 * `slabs` slabs and its sweep, run on the host (no device): for the
 * reordered system rp[n+1], col, val (rows sorted by column), f~, inv =
 * 1/||a_i||^2, group[n] (-1: a row in no group) and ngroups, `sweeps`
 * sweeps of eq. 3.3 (groups in ascending order, all rows of a group from the
 * same iterate, each row step relaxed by omega as in obk_opts) update x
 * (reordered coordinates, n entries) in place.  Each
 * slab owns a contiguous range of the unknowns; a slab's rows, and the rows
 * touching its window columns, must lie within its neighbours' ranges.
 * stats (may be NULL, 4 entries): the slab count (0 when that count does not
 * apply; then OBK_E_ARG), the (slab, group, phase) pieces whose data the
 * layout keeps in LDS for a whole launch and those it streams every sweep,
 * and the LDS bytes per workgroup (a budget of 159 KiB is assumed).  The
 * iterate equals the device engine's and the group-phase kernels' bit for
 * bit.
 */
OBK_API obk_status obk_banded_emulate_host(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
                                           const double *f, const double *inv, const int32_t *group,
                                           int32_t ngroups, int32_t slabs, int64_t sweeps, double omega,
                                           double *x, int64_t *stats);
/*
 * obk_validate_layout_host: the plan validator (run inside obk_plan /
 * obk_plan_complex when the environment sets OBK_VALIDATE=1, with the tiles
 * too) on a one-row-block layout given as host arrays: gptr[G+1] and
 * grow[m] (the reordered row of each group-major row; each group's rows
 * ascending), group_of_row[n] (-1: in no group), the group-major CSR
 * rptr[m+1], rcol, rval; the per-group column segments tptr[G+1], tcol[T]
 * (ascending per group), sptr[T+1], srow (group-major rows, ascending per
 * column) and sval.  Complex (cplx = 1): values are (re, im) pairs and the
 * column copies hold conj(a).  Checks that every active row is laid out once
 * in its group, that each entry is owned by exactly one column entry of its
 * group with the same value, and that no two rows of a group have
 * |cos| >= delta (Section 3.3).  OBK_E_ARG names the first violation
 * (obk_last_error); OK when the layout holds.
 */
OBK_API obk_status obk_validate_layout_host(int64_t n, int32_t n_groups, const int64_t *gptr, const int32_t *grow,
                                           const int32_t *group_of_row, const int64_t *rptr, const int32_t *rcol,
                                           const double *rval, const int64_t *tptr, const int32_t *tcol,
                                           const int64_t *sptr, const int32_t *srow, const double *sval,
                                           int32_t cplx, double delta);
OBK_API obk_status obk_first_fit_host(int64_t n, const int64_t *cptr, const int32_t *cidx,
                                      const uint8_t *active, int32_t *group, int32_t *n_groups);

/* Thread-local message for the last failing call of this thread ("" if none). */
OBK_API const char *obk_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* OBK_H */
