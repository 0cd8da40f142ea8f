/*
 * fth.h - C ABI of the f-thermostat (FTH) library for AMD Instinct MI355X
 * (CDNA4, gfx950).
 *
 * Method (Nava, Ceriotti, Dryzun, Parrinello, "Evaluating functions of
 * positive-definite matrices using colored noise thermostats"):
 * a symmetric positive-definite matrix M is used as the Hessian of the
 * harmonic potential V(q) = q^T M q / 2 (Sec. I, Eq. for V), every Cartesian
 * degree of freedom is coupled to an independent copy of a Markovian
 * colored-noise GLE thermostat (Sec. I, extended-momentum SDE with drift
 * matrix A_p and free-particle covariance C_p, related to the diffusion by
 * A_p C_p + C_p A_p^T = B_p B_p^T), and time averages of products of the
 * dynamical variables give elements of a matrix function (Sec. I, covariance
 * identity <x_i x_j> = sum_k U_ik g(eps_k) U_jk).  This library estimates
 * <q_i q_j> = g_h(M)_ij, where g_h(lambda) is the stationary <q^2> of a mode
 * of frequency sqrt(lambda) under the integrated dynamics; a GLE fitted so
 * that g_h(lambda) ~ f(lambda) makes these the elements of f(M).
 *
 * One time step of size h, for every degree of freedom i and replica r:
 *   F = -M q_n                       (dense row or CSR row, stored order)
 *   accumulate q_n products          (selected pairs and/or all diagonals)
 *   p += (h/2) F
 *   (p, s_1..s_ns) <- T (p, s) + S xi,  T = exp(-A_p h),
 *                                       S = chol(C_p - T C_p T^T)
 *   p += (h/2) F
 *   q_{n+1} = q_n + h p
 * (the exact Ornstein-Uhlenbeck step of the GLE between the two half kicks
 * of velocity Verlet; Sec. I, "modified velocity Verlet").
 *
 * Noise xi_j for dof i, replica r, step n, seed K and stream id sigma:
 * Philox4x32-10 (Salmon et al., SC'11) with key (K mod 2^32, K >> 32) and
 * counter (i mod 2^32, n mod 2^32, (j << 16) | (r >> 2), sigma); word r & 3
 * of the block, mapped to u = (2 (x >> 9) + 1) 2^-24, and Box-Muller on the
 * word pairs (0,1), (2,3): even word sqrt(-2 ln u_even) cos(2 pi u_odd), odd
 * word the same radius times sin(2 pi u_odd).  Requirements: n < 2^32 dofs,
 * fewer than 2^32 total steps, R <= 2^18 replicas, ns < 2^16.
 *
 * Conventions
 *  - All pointers passed to fth_create / fth_set_state / fth_read /
 *    fth_get_* are HOST pointers owned by the caller; inputs are deep-copied
 *    (uploaded) before the call returns.  The context owns all device memory.
 *  - Functions return fth_status; nothing throws or aborts across the ABI.
 *    A message describing the last failure on the calling thread is
 *    available from fth_last_error().
 *  - A context is not thread-safe; distinct contexts are independent.
 *  - Work is enqueued on the context's HIP stream; fth_run returns after the
 *    stream has drained (so results and errors are final).
 */
#ifndef FTH_H
#define FTH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fth_ctx fth_ctx;

typedef enum {
    FTH_OK = 0,
    FTH_EINVAL = -1,         /* invalid argument (matrix, GLE, dt, pairs, sizes) */
    FTH_ENOMEM = -2,         /* device or host allocation failed */
    FTH_EDEVICE = -3,        /* HIP runtime error or no usable gfx950 device */
    FTH_ESTATE = -4,         /* call not valid in the context's current state */
    FTH_ENONFINITE = -5,     /* the dynamics produced a non-finite value; the
                                context is poisoned (M not SPD or h too large) */
    FTH_EUNSUPPORTED = -6    /* valid request the library does not implement */
} fth_status;

typedef enum { FTH_DENSE = 0, FTH_CSR = 1 } fth_format;

/* State precision / force form. */
typedef enum {
    FTH_FP64 = 0,            /* FP64 state, FP64 force (plain FP64 form) */
    FTH_FP32 = 1,            /* FP32 state, FP32 force (CSR; dense systems of one
                                workgroup, or with opt.replicas <= 8) */
    FTH_FP32_BF16X3 = 2      /* FP32 state, dense force as split-BF16x3 on MFMA
                                with FP32 accumulation (dense only; with at most 8
                                replicas the force is FP32 matrix-vector products) */
} fth_precision;

/* The matrix M (Sec. I: the Hessian of the harmonic potential).
 * FTH_DENSE: dense[n*n] row-major, symmetric.
 * FTH_CSR:   row_ptr[n+1] (row_ptr[0] == 0, non-decreasing, row_ptr[n] == nnz),
 *            col[nnz] sorted strictly increasing within each row, 0 <= col < n,
 *            val[nnz]; the pattern and values must be symmetric and every
 *            diagonal entry present and positive.
 * Values are double if value_is_f64 != 0, else float.  In the FP32 forms the
 * values are used as float; in FTH_FP64 as double. */
typedef struct {
    int32_t format;
    int32_t value_is_f64;
    int64_t n;
    const void* dense;
    int64_t nnz;
    const int64_t* row_ptr;
    const int32_t* col;
    const void* val;
} fth_matrix;

/* GLE parameters (Sec. I): drift A_p and free-particle covariance C_p,
 * both (ns+1) x (ns+1) row-major doubles, index 0 the physical momentum.
 * Requirements: C_p symmetric positive definite; A_p C_p + C_p A_p^T
 * positive semi-definite; C_p - T C_p T^T positive definite for the
 * requested dt (checked by Cholesky; failure -> FTH_EINVAL). */
typedef struct {
    int32_t ns;
    const double* A_p;
    const double* C_p;
} fth_gle;

/* Device memory provider (e.g. a framework's caching allocator).  alloc
 * returns device memory of at least `bytes` (NULL on failure); release gives
 * it back.  Both are called from the thread that calls into the library. */
typedef struct {
    void* (*alloc)(size_t bytes, void* user);
    void (*release)(void* ptr, void* user);
    void* user;
} fth_allocator;

typedef struct {
    uint64_t seed;           /* Philox key */
    uint32_t stream_id;      /* Philox counter word 3 (distinct per request) */
    int32_t precision;       /* fth_precision */
    int64_t burn_in;         /* steps n < burn_in are not accumulated */
    int64_t block_len;       /* L >= 1: accumulated steps per block average */
    int32_t acc_diag;        /* != 0: also accumulate all n diagonal elements */
    int32_t replicas;        /* R, 0: fixed by the first fth_run */
    void* hip_stream;        /* hipStream_t to enqueue on; NULL: own stream */
    int32_t steps_per_graph; /* steps captured per hipGraph launch, 0: default */
    int32_t tune;            /* != 0: autotune the launch shape at first run */
    int32_t temporal_steps;  /* CSR with half-bandwidth <= 16 and <= 8 entries per row:
                                steps advanced per temporally blocked launch (3 or 5);
                                0: the autotuner decides (one-step kernels if not tuning);
                                -1: never block.  An explicit 3 or 5 on an ineligible
                                matrix makes fth_run fail with FTH_EUNSUPPORTED. */
    int32_t temporal_threads; /* threads per blocked workgroup: 256, 512 or 1024 (0: the largest
                                 allowed for the GLE size and precision) */
    int32_t coded_matrix;    /* CSR with <= 8 entries per row and <= 255 distinct column offsets
                                j - i: 0 also keeps a coded copy (one-byte codes into tables of
                                the distinct offsets and, if <= 256, distinct values) that the
                                one-step kernel reads for R >= 4; -1: plain CSR only.  Results
                                are identical either way. */
    int32_t acc_pp;          /* != 0: also accumulate <p_i p_j> (the momentum form of Eq. 7:
                                p_n sampled with q_n) for the same pairs and diagonal; the
                                estimates then come in two blocks, q-q then p-p */
    int32_t temporal_persistent; /* blocked launches (temporal_steps > 0 or chosen by the autotuner):
                                0: the persistent form when its LDS staging fits the device (one
                                workgroup per resident slot walks a range of row tiles while the
                                next tile's state streams into LDS); -1: one workgroup per tile.
                                Results are identical either way. */
    int32_t acc_trace;       /* != 0: also the trace estimators of Sec. I, appended after the
                                pair blocks: sum_i <q_i^2> (Tr of the position response),
                                <q^T M q> (= -<q . F>, Tr[M g(M)]) and, with acc_pp,
                                sum_i <p_i^2> (the kinetic trace Tr f(M)).  Per-step sums are
                                formed per row tile and folded in a fixed order once per
                                chunk, so they are reproducible. */
    /* Spectral map (Sec. I, scaling of the GLE and of M): the dynamics run on
       M' = scale_r M + scale_m I with A'_p = gle_alpha A_p, C'_p = gle_gamma C_p,
       so the estimates are those of the transformed problem (fth_unscale maps
       them back for the targets where that is possible).  0 for scale_r,
       gle_alpha or gle_gamma means 1.  M' is formed on the host at create and
       must itself pass validation (a shift needs stored diagonal entries). */
    double scale_r;
    double scale_m;
    double gle_alpha;
    double gle_gamma;
    const fth_allocator* allocator; /* NULL: hipMalloc / hipFree; else every device buffer of
                                       the context (and its scratch) comes from it; copied at
                                       create, the functions must stay valid until destroy */
} fth_options;

/* Fill *opt with defaults: seed 0, stream 0, FTH_FP32, burn_in 0,
 * block_len 100, acc_diag 0, replicas 0, own stream, default graph length,
 * no autotuning. */
void fth_default_options(fth_options* opt);

/* Validate and upload M, compute T and S in FP64 on the host, and upload the
 * pair list pairs[2*k], pairs[2*k+1] (k < npairs; 0 <= i, j < n; pairs may
 * be NULL when npairs == 0).  On success *out owns a new context.
 * Errors: FTH_EINVAL (validation), FTH_ENOMEM, FTH_EDEVICE,
 * FTH_EUNSUPPORTED (e.g. FTH_FP32_BF16X3 with a CSR matrix). */
fth_status fth_create(const fth_matrix* M, const fth_gle* gle, double dt,
                      const int32_t* pairs, int64_t npairs,
                      const fth_options* opt, fth_ctx** out);

/* Advance the trajectory and the accumulators by nsteps steps over R
 * replicas (cumulative: continues from the previous call).  The first call
 * fixes R (replicas == 0 uses opt.replicas); a later call with another
 * non-zero R returns FTH_ESTATE.  R must be a power of two <= 512 for the
 * sparse kernels; dense systems beyond one workgroup (N R > 4096) take R in
 * {16, 32, 64, 128} on the matrix cores or R in {1, 2, 4, 8} as
 * matrix-vector products (FTH_EUNSUPPORTED otherwise).  The first call also
 * runs the autotuner when opt.tune is set, so nsteps == 0 fixes R and the
 * launch shape without advancing.
 * Returns FTH_ENONFINITE (and poisons the context) if any state value
 * became non-finite; FTH_ESTATE on a poisoned context. */
fth_status fth_run(fth_ctx* ctx, int64_t nsteps, int32_t replicas);

/* Change the number of steps captured per hipGraph launch (0: default) and
 * drop the current graph; the next fth_run captures one of the new length.
 * A blocked schedule rounds it down to whole blocked launches (at least
 * one).  Errors: FTH_EINVAL. */
fth_status fth_set_steps_per_graph(fth_ctx* ctx, int32_t steps);

/* Number of estimates: npairs, plus n when acc_diag (pairs first, in input
 * order, then the diagonal in index order); twice that with acc_pp, the q-q
 * block followed by the p-p block in the same order; then 2 (3 with acc_pp)
 * trace estimators with acc_trace. */
int64_t fth_num_outputs(const fth_ctx* ctx);

/* Estimates of <q_i q_j> (and <p_i p_j> with acc_pp) and their standard errors (len >= fth_num_outputs,
 * else FTH_EINVAL).  mean = (sum of all accumulated samples) / (R n_acc);
 * stderr from the complete blocks (+inf with fewer than two).  Either output
 * pointer may be NULL.  *nsamples (if not NULL) receives n_acc, the number of
 * accumulated steps.  Does not reset anything. */
fth_status fth_read(fth_ctx* ctx, double* estimates, double* stderr_out,
                    int64_t len, int64_t* nsamples);

/* Raw accumulators, each of length fth_num_outputs: blk = current partial
 * block sum, s1 / s2 = sum / sum of squares of completed block sums (sums
 * over replicas of q_i q_j).  *nblocks = completed blocks, *step = steps
 * taken so far.  Any pointer may be NULL. */
fth_status fth_get_accumulators(fth_ctx* ctx, double* blk, double* s1, double* s2,
                                int64_t* nblocks, int64_t* step);

/* Copy the state to host FP64 arrays: q[n*R], p[n*R] (index i*R + r) and
 * s[ns*n*R] (index (k*n + i)*R + r).  FTH_ESTATE before R is fixed. */
fth_status fth_get_state(fth_ctx* ctx, double* q, double* p, double* s);

/* Overwrite the state from host FP64 arrays (same layout; NULL leaves that
 * part unchanged).  Values are rounded to the state precision. */
fth_status fth_set_state(fth_ctx* ctx, const double* q, const double* p, const double* s);

/* Force check for dense contexts: F = -M q for a host state q[n*R] (index
 * i*R + r, values rounded to the state precision), computed with the same
 * device kernels and partial-sum order as a time step, on scratch buffers
 * (the trajectory is not touched); F[n*R] receives the result as double.
 * FTH_ESTATE before R is fixed; FTH_EUNSUPPORTED for CSR contexts and
 * dense systems of one workgroup. */
fth_status fth_force(fth_ctx* ctx, const double* q, double* F);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the dense
 * force of fth_force, F = -M q, with q and F as DEVICE arrays in the state
 * precision (float for FTH_FP32_BF16X3, double for FTH_FP64; q[n*R] and
 * F[n*R], index i*R + r, caller-owned) and the work buffers (the padded or
 * bf16-split copy of q and the split-K partial sums) in a fixed library
 * array of 64 MiB per GPU instead of per-call allocations.  The result is
 * bit-identical to fth_force's.  Nothing is allocated or freed: the call
 * enqueues four kernels on hip_stream (NULL: the context's stream) and
 * returns; F is ready when that stream reaches them.  Every call on one GPU
 * uses the same array, so calls that overlap on one GPU (other streams,
 * other threads) race; a call's work space keeps its contents afterwards.
 * The first call on a device looks the array up (no allocation).
 * Errors: FTH_EINVAL (NULL pointers, or a system whose work space exceeds
 * the 64 MiB array: 4 (1 + ksplit) P R bytes in the split form, 8 (1 +
 * ksplit) P R in FP64, P = n rounded up to the padded size), FTH_ESTATE
 * before R is fixed, FTH_EUNSUPPORTED for CSR, one-workgroup dense and
 * matrix-vector (R <= 8) dense contexts, FTH_EDEVICE on a launch failure. */
fth_status fth_force_noalloc(fth_ctx* ctx, const void* q, void* F, void* hip_stream);

/* GPU time in milliseconds of the most recent fth_run, measured with HIP
 * events on the context's stream around its launches (0 before any run). */
double fth_last_run_ms(const fth_ctx* ctx);

/* Number of kernel launches per time step of the context's step schedule
 * (for per-launch timing), and a short name of the step kernel variant in
 * use (NUL-terminated, at most len bytes written). */
int32_t fth_launches_per_step(const fth_ctx* ctx);
fth_status fth_kernel_name(const fth_ctx* ctx, char* name, size_t len);

/* Host-only helpers (no device needed). */
/* T = exp(-A_p dt) and S = lower Cholesky factor of C_p - T C_p T^T,
 * (ns+1)^2 row-major doubles.  Errors: FTH_EINVAL. */
fth_status fth_propagator(const fth_gle* gle, double dt, double* T, double* S);

/* Evaluate the noise stream on the device (validation of the generator):
 * out[k] = xi_{j[k]} for dof i[k], replica r[k], step n[k], computed in
 * FTH_FP32 or FTH_FP64 exactly as the step kernels do; if raw != NULL,
 * raw[4k..4k+3] = the Philox4x32-10 block that holds it.  Host arrays of
 * length count (raw: 4*count).  Requires j < 2^16, r < 2^18.  Synchronous.
 * Errors: FTH_EINVAL, FTH_ENOMEM, FTH_EDEVICE. */
fth_status fth_noise_sample(uint64_t seed, uint32_t stream, int64_t count, const uint32_t* i,
                            const uint32_t* r, const uint32_t* n, const uint32_t* j,
                            int32_t precision, double* out, uint32_t* raw);

/* ---- spectral map helpers (host only, Sec. I scaling paragraph) ---- */

/* r and m of M' = r M + m I that send a spectrum [e_min, e_max] onto the
 * window [w_min, w_max] of a fitted GLE:
 *   r = (w_min - w_max) / (e_min - e_max),
 *   m = (e_min w_max - e_max w_min) / (e_min - e_max),
 * so that r e_min + m = w_min and r e_max + m = w_max.
 * FTH_EINVAL unless e_min < e_max and w_min < w_max (all finite). */
fth_status fth_spectral_map(double e_min, double e_max, double w_min, double w_max, double* r, double* m);

/* Gershgorin interval [lo, hi] containing every eigenvalue of M (symmetric). */
fth_status fth_gershgorin(const fth_matrix* M, double* lo, double* hi);

/* Targets whose value on M can be recovered from the transformed problem. */
typedef enum {
    FTH_TARGET_INVSQRT = 0, /* f(x) = x^-1/2: needs m = 0; f(M) = sqrt(r') f(M') */
    FTH_TARGET_LN = 1,      /* f(x) = ln x:   needs m = 0; f(M) = f(M') - ln(r') I */
    FTH_TARGET_EXPNEG = 2   /* f(x) = e^-x:   exp(-r' M) = e^m' f(M') */
} fth_target;

/* Map position-form estimates of a run with (r, m, alpha, gamma) back to
 * f(M).  The q-response of the scaled GLE is (gamma / alpha^2) g(M' / alpha^2)
 * (Sec. I), so first est *= alpha^2 / gamma and r' = r / alpha^2,
 * m' = m / alpha^2; then the target's identity above.  (Momentum-form
 * estimates, acc_pp, scale as gamma g_p(M' / alpha^2): multiply them by
 * alpha^-2 before passing them here, as the server does for its
 * momentum-form requests; with alpha = 1 the two forms unscale alike.)
 * kind_weight[k] is the
 * number of identity entries output k contains: 0 for an off-diagonal
 * element, 1 for a diagonal element, n for a trace over n rows (the ln shift
 * is weighted by it).  est and se (either may be NULL) are updated in place;
 * se scales like est.  FTH_EINVAL for an unknown target, a non-positive r'
 * or a map the target cannot undo. */
fth_status fth_unscale(int32_t target, double r, double m, double alpha, double gamma, int64_t count,
                       const double* kind_weight, double* est, double* se);

/* Device bytes the context holds now (all its buffers, through the allocator). */
size_t fth_device_bytes(const fth_ctx* ctx);

/* Complete state of a solve (q, p, s, accumulators, step counter; the noise
 * is counter-based, so this is all a continuation needs) as a byte image.
 * With buf == NULL, *len receives the size; else len must be at least that.
 * fth_load restores an image into a context created with the same matrix
 * size, GLE size, precision, replicas, outputs, seed and stream id: the
 * continuation is bit-identical to the uninterrupted run.  FTH_EINVAL on a
 * size or parameter mismatch or a damaged image. */
fth_status fth_save(fth_ctx* ctx, void* buf, size_t* len);
fth_status fth_load(fth_ctx* ctx, const void* buf, size_t len);

/* Device bytes a context with these parameters allocates. */
size_t fth_footprint_bytes(const fth_matrix* M, int32_t ns, int32_t replicas,
                           int64_t npairs, int32_t acc_diag, int32_t precision);

/* ------------------------------------------------------------------ */
/* Serving layer: a request loop over many solves that share one GPU.   */
/* ------------------------------------------------------------------ */
/* Requests arrive at any time (fth_server_submit).  Independent
 * simulations of one GPU run concurrently (the paper's remark, Sec. III,
 * that replicas and solves are trivially parallel):
 *  - admission: queued requests get a context (device memory) in arrival
 *    order while their footprint (fth_footprint_bytes) fits the remaining
 *    HBM budget and fewer than max_active run;
 *  - work is issued in chunks, each on its own stream: a running request
 *    that is not packed advances alone on its context's stream; sparse FP32
 *    requests of 4 to 256 replicas with the same ns are packed into one
 *    persistent kernel per step
 *    (a device work list of row and pair tiles of all members, one captured
 *    hipGraph per chunk length) on the group's stream; dense and FP64
 *    requests run their own GEMM and step kernels.  Chunks of different
 *    requests and groups overlap on the device;
 *  - a chunk never crosses a check boundary (a multiple of steps_per_tick
 *    steps of that request) and is shortened (to a divisor of
 *    steps_per_tick) when the previous chunk's measured time says it would
 *    take longer than quantum_ms, so a new arrival waits for the first chunk
 *    that ends, not for the slowest request;
 *  - a new request starts unpacked and joins its packed group at its next
 *    check boundary once the group is also at one;
 *  - at each check boundary the request's estimates and block stderrs are
 *    read (a few KB); it retires at its target (or max_steps), releasing its
 *    memory for the queue.
 * A request's trajectory depends only on its own inputs (matrix, GLE, dt,
 * seed, stream_id, spectral map), and it stops at a check boundary, so its
 * result is the same alone and in any mix.  A server is not thread-safe. */
typedef struct fth_server fth_server;

typedef struct {
    size_t hbm_budget;       /* bytes of device memory for requests; 0: 80% of free */
    int32_t steps_per_tick;  /* steps between stderr checks (the chunk length
                                at most); 0: 200 */
    int32_t max_active;      /* running requests at most; 0: 64 */
    int32_t min_blocks;      /* complete blocks needed before a stderr counts; 0: 8 */
    double quantum_ms;       /* target device time of one chunk (chunks are cut to
                                divisors of steps_per_tick to stay under it);
                                0: 20 ms, < 0: never cut */
} fth_server_options;

typedef struct {
    fth_matrix M;            /* deep-copied at submit */
    fth_gle gle;             /* deep-copied at submit */
    double dt;
    const int32_t* pairs;    /* [npairs][2], deep-copied at submit */
    int64_t npairs;
    int32_t replicas;        /* 0: 32 for CSR, 64 for dense */
    int32_t precision;       /* FTH_FP32 (CSR, packed), FTH_FP64, FTH_FP32_BF16X3 (dense) */
    uint64_t seed;
    uint32_t stream_id;      /* noise stream; 0: the request id */
    int64_t burn_in;
    int64_t block_len;       /* 0: 100 */
    double target_rel_stderr;/* stop when every estimate's stderr / scale <= target;
                                scale = sqrt(est_ii est_jj) when both diagonals are
                                among the request's pairs, else |est| */
    int64_t max_steps;       /* stop at the first check boundary at or after this many
                                steps (0: no limit) */
    /* Spectral map of Sec. I for this request (as in fth_options: the
       dynamics run on M' = scale_r M + scale_m I with (gle_alpha A_p,
       gle_gamma C_p); 0 for scale_r, gle_alpha, gle_gamma means 1), so one
       fitted GLE serves requests of any spectrum.  unscale_target (an
       fth_target, or -1) maps the results back to f(M) with fth_unscale
       (pairs (i, i) count as diagonal entries); -1 returns them as run. */
    double scale_r, scale_m, gle_alpha, gle_gamma;
    int32_t unscale_target;
    /* != 0: the request's estimates are the momentum form <p_i p_j> of Eq. 7
       (acc_pp; for a GLE fitted so that <p^2>(omega) = f(omega^2)) instead
       of <q_i q_j>.  Its stop test, results and unscaling use that block
       (the momentum response scales as gamma g_p(M' / alpha^2), so the
       results are multiplied by alpha^-2 before fth_unscale).  Packs like
       any other request. */
    int32_t momentum_form;
} fth_request;

typedef enum {
    FTH_REQ_QUEUED = 0, FTH_REQ_RUNNING = 1, FTH_REQ_DONE = 2, FTH_REQ_FAILED = 3, FTH_REQ_CANCELLED = 4
} fth_request_state;

typedef struct {
    int32_t state;           /* fth_request_state */
    int32_t status;          /* fth_status of a failure, else FTH_OK */
    int64_t steps;           /* steps taken */
    int64_t nblocks;         /* complete blocks */
    double max_rel_stderr;   /* at the last check (+inf before min_blocks) */
    double t_submit, t_start, t_finish;  /* seconds on the server's clock (-1: not yet) */
    int64_t n_out;           /* number of estimates (= npairs) */
    int32_t replicas;
    int32_t packed;          /* 1 once run by the packed multi-request kernel */
    size_t footprint;        /* device bytes reserved while running */
    double device_ms;        /* device time of the chunks that advanced it (HIP events
                                around each chunk on its stream; a packed chunk counts
                                for every member) */
    int64_t chunks;          /* chunks that advanced it */
    double device_first_ms;  /* device clock (ms since the server was created, from HIP events):
                                start of its first chunk and end of its last (-1: none yet) */
    double device_last_ms;
} fth_request_info;

/* Create a server on the current device.  opt may be NULL (defaults). */
fth_status fth_server_create(const fth_server_options* opt, fth_server** out);
/* Queue a request; *id receives its id (>= 1).  FTH_EINVAL on invalid input,
 * FTH_ENOMEM if its footprint exceeds the whole budget. */
fth_status fth_server_submit(fth_server* srv, const fth_request* req, uint64_t* id);
/* One round of the loop: retire finished chunks (check, retire), admit,
 * issue a chunk to every idle request and packed group, then wait until at
 * least one issued chunk has finished and process it.  Returns at once when
 * nothing is running.  A request that fails (at admission or in a chunk)
 * is marked FTH_REQ_FAILED with its status; the others go on. */
fth_status fth_server_tick(fth_server* srv);
/* State of a request (any state). */
fth_status fth_server_poll(fth_server* srv, uint64_t id, fth_request_info* info);
/* Estimates and standard errors of a finished (or running) request
 * (len >= n_out, either pointer may be NULL). */
fth_status fth_server_result(fth_server* srv, uint64_t id, double* est, double* se, int64_t len);
/* Cancel a queued or running request (its memory is released). */
fth_status fth_server_cancel(fth_server* srv, uint64_t id);
/* Seconds since the server was created (its clock). */
double fth_server_clock(const fth_server* srv);
/* Counts of queued and running requests, and bytes reserved. */
fth_status fth_server_stats(const fth_server* srv, int64_t* queued, int64_t* running, size_t* reserved);
/* Release the server and every request in it.  NULL is accepted. */
fth_status fth_server_destroy(fth_server* srv);

/* Release the context and its device memory.  NULL is accepted. */
fth_status fth_destroy(fth_ctx* ctx);

/* Message for the last failure on the calling thread ("" if none). */
const char* fth_last_error(void);

/* Library version string. */
const char* fth_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FTH_H */
