/*
 * hsma.h -- C ABI of the MI355X (gfx950) triangular-solve library.
 *
 * The operation (paper, Sec. 2.1; the forward-substitution equation of
 * Sec. 4.2.1): left-side, lower-triangular, no-transpose TRSM
 *
 *         B <- alpha * inv(L) * B,    L = lower triangle of A (m x m),
 *
 * i.e. X solves L X = alpha B and overwrites B.  Row i of X is
 *   x_ij = (alpha b_ij - sum_{k<i} l_ik x_kj) / l_ii   (l_ii = 1 for a unit diagonal).
 *
 * Conventions (BLAS TRSM; the paper leaves them open):
 *   - Column-major storage with leading dimensions lda >= max(1, m) and
 *     ldb >= max(1, m), counted in elements of the data type.
 *   - Only the strict lower triangle of A is read, plus the diagonal when
 *     diag == HSMA_NON_UNIT.  The upper triangle is never read.  Rows m..ldb-1
 *     of B are never read or written.
 *   - alpha == 0 sets B to zero and reads neither A nor B.
 *   - No singularity check: a zero or non-finite diagonal propagates IEEE
 *     infinities/NaNs.
 *   - Real data is IEEE double (HSMA_R64F) or float (HSMA_R32F); complex data
 *     is interleaved {re, im} of double (HSMA_C64F, the layout of
 *     hipDoubleComplex and torch.complex128) or of float (HSMA_C32F,
 *     torch.complex64).  FP32 solves compute in FP32 (FP32 matrix cores,
 *     FP32 accumulation), as STRSM/CTRSM do.
 *
 * Memory and streams:
 *   - A and B are DEVICE pointers owned by the caller.  A and B must not
 *     overlap.  The library owns its workspaces (a per-device cache of device
 *     blocks reused in stream order; see hsma_workspace_release).
 *   - Every call is asynchronous on `stream` (a hipStream_t passed as void*;
 *     NULL is the null stream): it returns after enqueueing and the result is
 *     complete when the stream reaches that point.  Exceptions noted per call.
 *   - Calls are thread-safe.  The device used is the caller's current HIP device.
 *
 * Errors: no exception crosses the ABI.  Argument errors are reported before
 * anything is enqueued and leave B untouched.  Check order for one problem:
 *   1. diag or dtype not a listed enumerator        -> HSMA_INVALID_VALUE
 *   2. m < 0 or n < 0                                -> HSMA_INVALID_SIZE
 *   3. lda < max(1, m) or ldb < max(1, m)            -> HSMA_INVALID_SIZE
 *   4. m == 0 or n == 0                              -> HSMA_SUCCESS, nothing done
 *   5. alpha == NULL                                 -> HSMA_INVALID_POINTER
 *   6. B == NULL, or A == NULL with alpha != 0       -> HSMA_INVALID_POINTER
 * A failing HIP runtime call returns HSMA_HIP_ERROR; hsma_last_hip_error()
 * then gives the hipError_t value of the calling thread's last failure.
 */
#ifndef HSMA_H
#define HSMA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Data types.  The paper evaluates all four (Sec. 5).  The FP32 ones
 * (STRSM, CTRSM) are taken by hsma_trsm, hsma_trsm_ex (plain solves) and
 * hsma_trsm_general; the batched, queue and allocation-free calls take FP64
 * data only (HSMA_NOT_SUPPORTED otherwise). */
typedef enum { HSMA_R64F = 0, HSMA_C64F = 1, HSMA_R32F = 2, HSMA_C32F = 3 } hsma_dtype;
typedef enum { HSMA_NON_UNIT = 0, HSMA_UNIT = 1 } hsma_diag;

typedef enum {
    HSMA_SUCCESS = 0,
    HSMA_INVALID_VALUE = 1,
    HSMA_INVALID_SIZE = 2,
    HSMA_INVALID_POINTER = 3,
    HSMA_ALLOC_FAILED = 4,
    HSMA_HIP_ERROR = 5,
    HSMA_NOT_SUPPORTED = 6,
    HSMA_TOO_LARGE = 7,
    HSMA_QUEUE_CLOSED = 8,
    HSMA_PENDING = 9,
    HSMA_TIMEOUT = 10,
    HSMA_NOT_FOUND = 11,
    HSMA_WORKSPACE_TOO_SMALL = 12
} hsma_status;

/* A hipStream_t, passed as an opaque pointer; NULL = the null stream. */
typedef void *hsma_stream_t;

/* Static text for a status code (never NULL). */
const char *hsma_status_string(hsma_status s);

/* hipError_t of this thread's most recent HSMA_HIP_ERROR (0 if none). */
int hsma_last_hip_error(void);

/* Library version string, e.g. "0.1.0 gfx950". */
const char *hsma_version(void);

/*
 * hsma_trsm -- B <- alpha * inv(tril(A)) * B  (paper Sec. 2.1, Sec. 4.1-4.3).
 *
 *   diag   HSMA_NON_UNIT or HSMA_UNIT (diagonal of A taken as 1, not read).
 *   m, n   rows of A and B / columns of B.
 *   alpha  HOST pointer to one scalar of the data type: double (HSMA_R64F),
 *          double[2] = {re, im} (HSMA_C64F), float (HSMA_R32F) or float[2]
 *          (HSMA_C32F); read before the call returns.
 *   A      device pointer, m x m column-major, leading dimension lda.
 *   B      device pointer, m x n column-major, leading dimension ldb; in/out.
 *   dtype  HSMA_R64F, HSMA_C64F, HSMA_R32F or HSMA_C32F.
 *   stream hipStream_t or NULL.
 *
 * Path: m <= 64 uses the register-resident small-solve kernel, one wavefront
 * per 64-column panel of B (Sec. 4.2); m > 64 uses the blocked path (Sec. 4.3):
 * diagonal blocks of edge I_B inverted in parallel, then recursive FP64
 * matrix-core updates and in-place diagonal-block solves, with I_B taken from
 * the compiled-in tuning table (Sec. 4.3.2).
 */
hsma_status hsma_trsm(hsma_diag diag, int64_t m, int64_t n, const void *alpha,
                      const void *A, int64_t lda, void *B, int64_t ldb,
                      hsma_dtype dtype, hsma_stream_t stream);


/*
 * hsma_trsm_noalloc -- hsma_trsm for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same operation, arguments, path choice, I_B and kernels
 * as hsma_trsm, so the result is bit-for-bit the same; it calls no hipMalloc,
 * hipFree or other allocating routine.  The blocked path's workspace comes
 * from a fixed per-device scratch array of hsma_noalloc_scratch_bytes()
 * bytes (64 MiB) inside the library, which each GPU the library runs on
 * holds until the process ends.  A problem whose workspace does not fit
 * (hsma_trsm's blocked workspace: ceil(m/I_B) I_B^2 + (ceil(m/2) + I_B) I_B
 * elements; DTRSM up to m of about 16384 fits) returns
 * HSMA_WORKSPACE_TOO_SMALL before anything is enqueued.  Every call on one
 * GPU uses the same array: calls that overlap in time on one GPU (two
 * streams, two threads) race and give wrong results; serialise them.
 * Asynchronous on `stream`.
 */
hsma_status hsma_trsm_noalloc(hsma_diag diag, int64_t m, int64_t n, const void *alpha,
                              const void *A, int64_t lda, void *B, int64_t ldb,
                              hsma_dtype dtype, hsma_stream_t stream);

/* Bytes of the per-device scratch array of hsma_trsm_noalloc. */
uint64_t hsma_noalloc_scratch_bytes(void);

/* ------------------------------------------------------------------------ */
/* The general BLAS TRSM: either side, either triangle, op(A) = A, A^T, A^H  */
/* ------------------------------------------------------------------------ */

typedef enum { HSMA_LEFT = 0, HSMA_RIGHT = 1 } hsma_side;
typedef enum { HSMA_LOWER = 0, HSMA_UPPER = 1 } hsma_uplo;
typedef enum { HSMA_OP_N = 0, HSMA_OP_T = 1, HSMA_OP_C = 2 } hsma_op;

/*
 * hsma_trsm_general -- the problem as the paper poses it, op(A) X = alpha B
 * (Sec. 2.1), in every BLAS form: X overwrites B, where
 *   side  HSMA_LEFT:  op(A) X = alpha B, A is m x m (lda >= max(1, m));
 *         HSMA_RIGHT: X op(A) = alpha B, A is n x n (lda >= max(1, n));
 *   uplo  which triangle of A is stored (only that one is read);
 *   trans op(A) = A, A^T or A^H (the conjugate transpose; for real data the
 *         same as A^T);
 *   diag  HSMA_UNIT: the diagonal of A is taken as 1 and not read.
 * B is m x n, column-major (ldb >= max(1, m)); alpha is a host pointer as for
 * hsma_trsm (not conjugated by trans).  Left, lower, no transpose is
 * hsma_trsm itself.  Every other case runs the same small and blocked
 * kernels on re-indexed copies (all device work on `stream`): the effective
 * operator (op(A), or op(A)^T for the right side) is copied into a
 * lower-triangular workspace, its indices reversed when it is upper
 * triangular, and B into a workspace with its rows reversed and, for the
 * right side, transposed (for left-side cases whose operator is lower, B is
 * solved in place); the solve's result is copied back.  The workspace holds
 * k^2 (+ m n) elements, k the order of A.
 * Errors, in this order: side, uplo, trans, diag or dtype not an enumerator
 * -> HSMA_INVALID_VALUE; m < 0 or n < 0 -> HSMA_INVALID_SIZE; lda or ldb too
 * small -> HSMA_INVALID_SIZE; m == 0 or n == 0 -> HSMA_SUCCESS, nothing done;
 * alpha NULL -> HSMA_INVALID_POINTER; B NULL, or A NULL with alpha != 0 ->
 * HSMA_INVALID_POINTER.  alpha == 0 zero-fills B without reading A or B.
 * Asynchronous on `stream`.
 */
hsma_status hsma_trsm_general(hsma_side side, hsma_uplo uplo, hsma_op trans, hsma_diag diag,
                              int64_t m, int64_t n, const void *alpha, const void *A,
                              int64_t lda, void *B, int64_t ldb, hsma_dtype dtype,
                              hsma_stream_t stream);

/* ------------------------------------------------------------------------ */
/* Cholesky factorization and solve on the library's TRSM                    */
/* ------------------------------------------------------------------------ */

/*
 * hsma_potrf -- A = L L^H in place (the lower triangle of A is read and
 * overwritten by L; the strict upper triangle is neither read nor written),
 * for real symmetric (HSMA_R64F) or complex Hermitian (HSMA_C64F) positive
 * definite A, n x n column-major with lda >= max(1, n).  TRSM is the core of
 * this factorization (paper Sec. 1): recursion on halves, each step a
 * right-side conjugate-transpose TRSM for the off-diagonal block
 * (hsma_trsm_general) and a lower-triangular update on the FP64 matrix cores,
 * diagonal blocks of <= 64 rows factored in LDS.  No definiteness check: a
 * non-positive pivot gives NaN.  Workspace: about n^2/4 elements.
 * Errors: bad dtype -> HSMA_INVALID_VALUE (FP32 -> HSMA_NOT_SUPPORTED);
 * n < 0 or lda too small -> HSMA_INVALID_SIZE; n == 0 -> success; A NULL ->
 * HSMA_INVALID_POINTER.  Asynchronous on `stream`.
 */
hsma_status hsma_potrf(int64_t n, void *A, int64_t lda, hsma_dtype dtype, hsma_stream_t stream);

/*
 * hsma_potrs -- solve A X = B with A = L L^H from hsma_potrf: L Y = B
 * (hsma_trsm) then L^H X = Y (hsma_trsm_general); X overwrites B (n x nrhs,
 * ldb >= max(1, n)).  L is read from the lower triangle of its array (lda).
 * Errors as hsma_potrf, plus nrhs < 0 or ldb too small -> HSMA_INVALID_SIZE,
 * B NULL -> HSMA_INVALID_POINTER.  Asynchronous on `stream`.
 */
hsma_status hsma_potrs(int64_t n, int64_t nrhs, const void *L, int64_t lda, void *B, int64_t ldb,
                       hsma_dtype dtype, hsma_stream_t stream);

/* Precision of the blocked path's trailing updates. */
typedef enum {
    HSMA_PREC_FP64 = 0,   /* everything in FP64 (FP64 matrix cores) */
    HSMA_PREC_MIXED = 1   /* trailing updates on the FP32 matrix cores with
                             FP64 accumulation of the partial sums, FP64
                             diagonal blocks, then FP64-residual iterative
                             refinement; real data only */
} hsma_precision;

/* Options of hsma_trsm_ex.  Zero-initialise and set what you need. */
typedef struct {
    int32_t block_size;   /* blocked-path diagonal-block edge I_B: 0 = tuning
                             table (Sec. 4.3.2), else 16, 32, 64, 128 or 256 */
    int32_t path;         /* 0 = automatic (m <= 64 small kernel, else blocked);
                             1 = force the small kernel (requires m <= 64);
                             2 = force the blocked path */
    int32_t precision;    /* hsma_precision */
    int32_t refine_steps; /* refinement steps after the first solve, 0..4
                             (each: FP64 residual R = alpha B0 - L X, a solve
                             of L D = R in the chosen precision, X += D);
                             -1 = stop as soon as the backward error is
                             <= refine_tol (at most 4 steps) */
    int32_t want_backward_error; /* 1: compute the normwise backward error of
                             the returned X from an FP64 residual on the GPU,
                             formed by one triangular product whose order of
                             summation is independent of the solve's */
    int32_t use_graph;    /* 1: run the blocked schedule as a HIP graph, one
                             per shape (dtype, diag, m, n, lda, ldb, I_B,
                             precision): captured and instantiated on the
                             shape's first call, replayed with one
                             hipGraphLaunch after that, new A, B and alpha
                             moved into it with hipGraphExecUpdate.  Replays
                             of one shape run one after another on the device
                             (they share the graph-owned workspace that
                             hsma_graph_cache_clear frees).  Ignored with
                             refinement or the small path. */
    int32_t reserved[2];  /* must be zero */
    double refine_tol;    /* target for refine_steps = -1 (0 means 1e-13) */
} hsma_trsm_options;

/* What hsma_trsm_ex did (filled before it returns). */
typedef struct {
    int32_t path;         /* 1 small kernel, 2 blocked path, 0 nothing enqueued */
    int32_t block_size;   /* I_B used by the blocked path, else 0 */
    int32_t refine_steps; /* refinement steps taken */
    int32_t reserved[5];
    double backward_error;/* ||L X - alpha B0||_inf / (||L|| ||X|| + |alpha| ||B0||)
                             of the result, or -1 if not computed */
} hsma_trsm_report;

/*
 * hsma_trsm_ex -- hsma_trsm with explicit options; same operation, arguments
 * and error behaviour.  opts may be NULL (all defaults); report may be NULL.
 * Unknown option values give HSMA_INVALID_VALUE; forcing the small kernel
 * with m > 64 gives HSMA_NOT_SUPPORTED; HSMA_PREC_MIXED with complex data
 * gives HSMA_NOT_SUPPORTED.  Refinement and the backward error work for both
 * FP64 data types (complex: the modulus in every row sum and |alpha|).  FP32
 * data takes plain solves only: the mixed mode, refinement, the backward
 * error or graph replay with HSMA_R32F/HSMA_C32F give HSMA_NOT_SUPPORTED.
 * Asynchronous on `stream` unless a backward error is needed
 * (want_backward_error = 1 or refine_steps = -1): then the call waits for the
 * stream before returning, because the value decides what happens next.
 * Refinement and the backward error need device workspace for two m x n
 * copies (the original right-hand side and the residual).
 */
hsma_status hsma_trsm_ex(hsma_diag diag, int64_t m, int64_t n, const void *alpha,
                         const void *A, int64_t lda, void *B, int64_t ldb,
                         hsma_dtype dtype, const hsma_trsm_options *opts,
                         hsma_trsm_report *report, hsma_stream_t stream);

/*
 * hsma_mfma_peak -- measure the matrix-core rate of the current device: FP64
 * (fp32 == 0, v_mfma_f64_16x16x4_f64) or FP32 (fp32 == 1,
 * v_mfma_f32_16x16x4_f32) instructions on register operands, 16 independent
 * accumulator chains per wavefront, `iters` iterations, 32 wavefronts per CU;
 * *tflops receives the sustained TFLOP/s (2048 flops per instruction per
 * wavefront).  *shader_ghz (may be NULL) receives the clock the CUs ran at
 * during the loop (shader-clock cycles over constant-rate wall-clock time).
 * A measurement aid for the roofline fractions (datasheet peaks: 78.6 FP64,
 * 157.3 FP32 TFLOP/s); synchronises the null stream.  Errors: tflops NULL ->
 * HSMA_INVALID_POINTER; iters outside 1..2^24 -> HSMA_INVALID_SIZE.
 */
hsma_status hsma_mfma_peak(int32_t fp32, int64_t iters, double *tflops, double *shader_ghz);

/* Destroy every cached graph and its workspace (waits for their work). */
hsma_status hsma_graph_cache_clear(void);

/* Graph-cache counters since the library was loaded: graphs instantiated,
 * in-place argument updates, and replays.  Any pointer may be NULL. */
hsma_status hsma_graph_stats(int64_t *captures, int64_t *updates, int64_t *replays);

/*
 * Workspace cache.  The library keeps freed workspace blocks of the current
 * device (binned by size, reused in stream order) instead of returning them;
 * this returns every idle block to the device, after waiting for its last
 * use.  Blocks still in use stay.  The cache also trims itself when an
 * allocation runs out of device memory.
 */
hsma_status hsma_workspace_release(void);

/*
 * hsma_lookup_block_size -- the I_B the tuning table gives for (dtype, m, n):
 * the entry whose tested scale is nearest in log2(m), then log2(n), ties to
 * the smaller scale (Sec. 4.3.2, online phase).  Host-only; no device access.
 */
int32_t hsma_lookup_block_size(hsma_dtype dtype, int64_t m, int64_t n);


/* ------------------------------------------------------------------------ */
/* Batched solves (many independent problems per call)                      */
/* ------------------------------------------------------------------------ */

/* One problem of a batch: the arguments of hsma_trsm in a struct.  For
 * HSMA_R64F alpha_im must be 0.  A and B are device pointers. */
typedef struct {
    int32_t diag;                /* hsma_diag */
    int32_t dtype;               /* hsma_dtype */
    int64_t m, n;
    double alpha_re, alpha_im;
    const void *A;
    int64_t lda;
    void *B;
    int64_t ldb;
} hsma_problem;

/*
 * hsma_trsm_batched -- solve every problem of `probs` (a HOST array of
 * `count` descriptors; read before the call returns).  Shapes, data types,
 * diagonal kinds and alphas may all differ.  Each problem is validated with
 * the hsma_trsm rules first; on the first invalid one its index goes to
 * *first_bad (if non-NULL), its status is returned and nothing is enqueued.
 * Problems with m <= 64 run in grouped launches (one per data type and
 * diagonal kind, one workgroup per 64-column panel, longest first); the rest take the
 * blocked path grouped: every problem keeps the schedule (I_B, inversions,
 * recursion) it gets alone, so its result is bit-for-bit the same, but the
 * k-th operation of all of them shares one launch.  Both parts are forked
 * onto library-owned streams and joined back into `stream`.  Asynchronous on
 * `stream`.  The problems' B matrices must not overlap each other or any A.
 */
hsma_status hsma_trsm_batched(const hsma_problem *probs, int64_t count, int64_t *first_bad,
                              hsma_stream_t stream);

/*
 * A batch prepared once and run many times with the same pointers: create
 * validates like hsma_trsm_batched, builds the work-item table and copies it
 * to device memory owned by the plan (synchronously, on the current device).
 * execute enqueues the whole batch on `stream` (same device as create; no
 * host-to-device copy).  Executions of one plan must not overlap in time
 * (they solve in place in the same B).  destroy frees the plan after the
 * caller has synchronised with its last execution.
 */
typedef struct hsma_batch_plan hsma_batch_plan;
hsma_status hsma_batch_plan_create(const hsma_problem *probs, int64_t count, int64_t *first_bad,
                                   hsma_batch_plan **plan);
hsma_status hsma_batch_plan_execute(hsma_batch_plan *plan, hsma_stream_t stream);
hsma_status hsma_batch_plan_destroy(hsma_batch_plan *plan);

/*
 * Phase accounting (the breakdown of the paper's Sec. 5.3, Table 3).  Between
 * hsma_profile_begin() and hsma_profile_end() every kernel the library
 * launches is bracketed by a pair of HIP events recorded on its own stream
 * and tagged with its phase and algorithmic flop count (2 per real
 * multiply-add of the product it computes; complex counted in its real
 * expansion).  hsma_profile_end() waits for those events (it synchronises
 * with them, not with the whole device), fills out[0..HSMA_PHASE_COUNT-1]
 * and stops recording.  Process-wide; meant for benchmarks and profiling.
 */
typedef enum {
    HSMA_PHASE_DIAG_INV = 0,  /* diagonal-block inversion (base kernel + merges) */
    HSMA_PHASE_UPDATE = 1,    /* trailing updates B_bot -= L_bot,top X_top */
    HSMA_PHASE_LEAF = 2,      /* diagonal solves X_r = alpha inv(D_r) B_r */
    HSMA_PHASE_SMALL = 3,     /* small-regime solves (m <= 64) */
    HSMA_PHASE_OTHER = 4,     /* zero fills, conversions, residuals, norms */
    HSMA_PHASE_FACTOR = 5,    /* Cholesky diagonal blocks and trailing
                                 Hermitian updates (hsma_potrf) */
    HSMA_PHASE_TINY = 6,      /* fused very small solves (m, n <= 16) */
    HSMA_PHASE_COUNT = 7
} hsma_phase;

typedef struct {
    int64_t launches;
    double ms;      /* summed kernel time */
    double flops;   /* summed algorithmic flops */
} hsma_phase_stat;

hsma_status hsma_profile_begin(void);
hsma_status hsma_profile_end(hsma_phase_stat *out, int count);


/* ------------------------------------------------------------------------ */
/* Synthetic inputs and the serving queue                                   */
/* ------------------------------------------------------------------------ */

/*
 * hsma_generate_inputs -- fill a device L (m x m, lda = m) and B (m x n,
 * ldb = m) with the standard synthetic workload, drawn on the GPU from the
 * counter-based generator Philox4x32-10 (Salmon et al., SC'11) under `key`.
 * Element e (column-major index) of L uses counter (e mod 2^32, e div 2^32,
 * 0, 0), of B counter (e mod 2^32, e div 2^32, 1, 0); key words (key mod 2^32,
 * key div 2^32).  The outputs x0..x3 give u1 = ((x1<<32|x0) >> 11) 2^-53 and
 * u2 = ((x3<<32|x2) >> 11) 2^-53.  L: strict lower (2 u1 - 1)/m (complex
 * imaginary part (2 u2 - 1)/m), diagonal 1 + u1 (complex imaginary u2 - 1/2),
 * upper triangle 0.  B: sqrt(-2 ln(1 - u1)) cos(2 pi u2) (complex imaginary
 * part with sin).  Asynchronous on `stream`.  Errors: bad dtype ->
 * HSMA_INVALID_VALUE; m < 0 or n < 0 -> HSMA_INVALID_SIZE; m == 0 -> success,
 * nothing done; L NULL, or B NULL with n > 0 -> HSMA_INVALID_POINTER.
 */
hsma_status hsma_generate_inputs(hsma_dtype dtype, int64_t m, int64_t n, uint64_t key, void *L,
                                 void *B, hsma_stream_t stream);

/*
 * Serving queue (continuous batching; the paper's Sec. 6 outlook on batched
 * TRSM carried to a request loop).  Clients submit solve requests at any
 * time; a scheduler thread owned by the queue
 *   - retires finished work by polling events, returning its memory budget
 *     and recording its latency (arrival to completion),
 *   - admits pending requests strictly in arrival order while the HBM budget
 *     and the in-flight limit allow,
 *   - launches each admission round by size class (m <= 64; 64 < m <= 512;
 *     m > 512; the last two split by data type), each class as one batched
 *     solve (hsma_trsm_batched's work, all of it on the class's stream) with
 *     its own completion event: the small class on the queue's small stream,
 *     the four blocked classes round-robin over the queue's other streams.  Synthetic
 *     inputs of a class are drawn in one launch on the class's stream first.
 * A request's footprint is its blocked-path workspace (a 4 KiB descriptor
 * share for small requests) plus, for synthetic requests, its L and B.
 */
typedef enum { HSMA_BACKEND_HIP = 0, HSMA_BACKEND_SIMULATED = 1 } hsma_backend;
typedef enum { HSMA_INPUT_DEVICE = 0, HSMA_INPUT_SYNTHETIC = 1 } hsma_input_kind;

typedef struct {
    int32_t backend;          /* hsma_backend.  HSMA_BACKEND_SIMULATED runs the
                                 same policy with no device work: each launch
                                 takes sim_fixed_ns + flops / sim_flops_per_ns
                                 of modelled time on its stream (flops = m^2 n,
                                 x4 for complex); for tests of the policy */
    int32_t n_streams;        /* streams for large requests (0 = 8) */
    int32_t max_inflight;     /* admitted, unfinished requests (0 = 8192) */
    int32_t poll_us;          /* completion poll period while work runs (0 = 20) */
    uint64_t hbm_budget_bytes;/* summed footprint limit (0 = 32 GiB) */
    double sim_flops_per_ns;  /* simulated rate (<= 0: 40000, i.e. 40 TFLOP/s) */
    double sim_fixed_ns;      /* simulated per-launch latency */
} hsma_queue_config;

typedef struct {
    hsma_problem prob;        /* the solve; for HSMA_INPUT_SYNTHETIC, A, B, lda
                                 and ldb are ignored (the server allocates
                                 lda = ldb = m and fills them with
                                 hsma_generate_inputs under `key`) */
    int32_t input;            /* hsma_input_kind */
    int32_t release_on_completion; /* 0: a synthetic request keeps L and X,
                                 counted against the budget, and every request
                                 keeps its record until hsma_queue_release;
                                 1: a synthetic request's L and B are freed as
                                 soon as the solve finishes, the record stays
                                 until released;
                                 2 (fire and forget, for load generation): as
                                 1, and the record is dropped too -- poll, wait
                                 and release then give HSMA_NOT_FOUND; the
                                 request still enters the statistics */
    uint64_t key;             /* Philox key of a synthetic request */
    double t_arrival_ns;      /* arrival time on hsma_clock_ns()'s clock for
                                 the latency figure; <= 0 means "now" (an
                                 open-loop generator passes the scheduled
                                 time, so a late submit still counts) */
} hsma_request;

typedef struct {
    int32_t status;           /* HSMA_SUCCESS, HSMA_PENDING or the failure */
    int32_t path;             /* 1 small (batched), 2 blocked, 0 not launched */
    double t_arrival_ns, t_admit_ns, t_done_ns;
    const void *A;            /* where L and X live (server memory for a kept */
    void *B;                  /* synthetic request; the caller's otherwise) */
    int64_t lda, ldb;
} hsma_request_info;

/* Latency (arrival to completion) of the completed requests in the
 * statistics window.  Kept as a histogram of 64 logarithmic bins per doubling
 * from 1 us (and one bin below): percentile q is the bin holding the sample
 * of rank round(q (count - 1)), reported as the bin's geometric midpoint
 * clamped to the observed minimum and maximum, so it is within 0.6 % of the
 * exact order statistic.  max and mean are exact.  Memory and the cost of a
 * statistics call do not grow with the number of requests. */
typedef struct {
    int64_t count;
    double p50_ns, p99_ns, max_ns, mean_ns;
} hsma_latency_summary;

/* Size classes of the per-class latency: m <= 64, 64 < m <= 512, m > 512. */
#define HSMA_LATENCY_CLASSES 3

typedef struct {
    int64_t submitted, rejected, completed, failed, pending, inflight;
    uint64_t bytes_in_use, bytes_peak;  /* budget accounting */
    double p50_ns, p99_ns, max_ns, mean_ns; /* latency over all classes (as in
                                 hsma_latency_summary) */
    double solves_per_s;      /* completed / (last completion - first submit) */
    int64_t rounds;           /* admission rounds that launched work */
    double launch_ms;         /* scheduler time spent enqueueing work */
    double t_first_submit_ns, t_last_done_ns; /* on hsma_clock_ns()'s clock */
    hsma_latency_summary all; /* the same figures as p50_ns .. mean_ns */
    hsma_latency_summary by_class[HSMA_LATENCY_CLASSES];
} hsma_queue_statistics;

typedef struct hsma_queue hsma_queue;

/* Monotonic clock used for arrival and completion times, in ns. */
double hsma_clock_ns(void);

/* Budget footprint of a request in bytes (what admission reserves for it);
 * host-only, no validation beyond the pointers. */
hsma_status hsma_request_footprint(const hsma_request *req, uint64_t *bytes);

/* cfg may be NULL (defaults).  The HIP backend binds the caller's current
 * device.  Negative counts or an unknown backend -> HSMA_INVALID_VALUE. */
hsma_status hsma_queue_create(const hsma_queue_config *cfg, hsma_queue **queue);

/*
 * Submit `count` requests (host array, read before return); tickets[i]
 * receives request i's ticket.  All or nothing: every request is validated
 * first with the hsma_trsm rules (synthetic requests skip the pointer and
 * leading-dimension checks), a request with m == 0 or n == 0 gives
 * HSMA_INVALID_SIZE, a real request with alpha_im != 0 HSMA_INVALID_VALUE,
 * one whose footprint exceeds the whole budget HSMA_TOO_LARGE, and a queue
 * being destroyed HSMA_QUEUE_CLOSED.  Device-input requests must keep A and B
 * alive and untouched until they complete.
 */
hsma_status hsma_queue_submit(hsma_queue *queue, const hsma_request *reqs, int64_t count,
                              uint64_t *tickets);

/* State of one request: HSMA_SUCCESS (done), HSMA_PENDING (queued or
 * running), its failure status, or HSMA_NOT_FOUND (unknown or released).
 * info may be NULL. */
hsma_status hsma_queue_poll(hsma_queue *queue, uint64_t ticket, hsma_request_info *info);

/* Block until the request finishes or timeout_ns passes (< 0: no limit):
 * HSMA_SUCCESS, its failure status, HSMA_TIMEOUT or HSMA_NOT_FOUND. */
hsma_status hsma_queue_wait(hsma_queue *queue, uint64_t ticket, int64_t timeout_ns,
                            hsma_request_info *info);

/* Forget a finished request and free what the server holds for it (a kept
 * synthetic result).  Still running -> HSMA_PENDING, nothing done.  Records of
 * finished requests stay until released (except fire-and-forget requests,
 * release_on_completion = 2, whose records go when they finish). */
hsma_status hsma_queue_release(hsma_queue *queue, uint64_t ticket);

/* Counters, budget and latency statistics (a snapshot; the percentiles are
 * worked out after the queue's lock is released). */
hsma_status hsma_queue_stats(hsma_queue *queue, hsma_queue_statistics *stats);

/* Start a new latency window: clear the latency statistics; from then on
 * only requests whose arrival time is >= t_from_ns enter them (a warm-up
 * period is left out by passing its end).  The counters are not reset. */
hsma_status hsma_queue_stats_reset(hsma_queue *queue, double t_from_ns);

/* Close the queue: later submits fail with HSMA_QUEUE_CLOSED, everything
 * admissible still runs to completion, requests that can no longer be
 * admitted (their budget is held by kept results) fail with
 * HSMA_QUEUE_CLOSED; then the scheduler stops and all server memory is
 * freed.  Waits for the device work the queue launched. */
hsma_status hsma_queue_destroy(hsma_queue *queue);

#ifdef __cplusplus
}
#endif

#endif /* HSMA_H */
