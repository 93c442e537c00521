/*
 * thx.h -- C ABI of libthx: fast polynomial basis conversion  beta = A alpha
 * on AMD Instinct MI355X (gfx950), following Townsend, Webb & Olver, "Fast
 * polynomial transforms based on Toeplitz and Hankel matrices" (arXiv:1604.07486).
 *
 * The conversion matrix is written A = D1 (T o H) D2 (eq. HadamardDecomposition),
 * the Hankel factor H is replaced by a rank-K pivoted-Cholesky approximation
 * (Sec. 2.1, Fig. 3) and each of the K diagonally scaled Toeplitz products of
 * eq. (Cdecomposition) is evaluated with FFTs (Fig. 1, steps 3-5).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - A polynomial of degree N has N+1 coefficients; coefficient vectors are rows
 *   of a row-major [batch][ld] array of doubles with ld >= N+1.  alpha and beta
 *   are DEVICE pointers owned by the caller; beta must not overlap alpha.
 * - All device work is ordered on `stream` (a hipStream_t; 0 = null stream).
 *   Only plan creation synchronises the stream (once, to read the rank K).
 * - No exception or abort crosses this boundary: every call returns a
 *   thx_status.  On THX_HIP_ERROR, thx_last_hip_error() holds the hipError_t.
 * - Plans are immutable after creation; one plan may be executed concurrently
 *   on different streams only if each execution uses its own workspace, which
 *   this library does not provide: serialise executions of a plan.
 */
#ifndef THX_H
#define THX_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    THX_OK = 0,
    THX_INVALID_ARGUMENT = 1, /* bad size, parameter, tolerance or null pointer   */
    THX_UNSUPPORTED = 2,      /* parameters outside the implemented cases         */
    THX_TOL_NOT_REACHED = 3,  /* pivoted Cholesky hit its rank cap before tol, or
                                 tol is below the double-precision floor; the
                                 plan is still created and usable                 */
    THX_OUT_OF_MEMORY = 4,    /* device or host allocation failed                  */
    THX_HIP_ERROR = 5,        /* a HIP runtime call failed                         */
    THX_WORKSPACE_TOO_LARGE = 6 /* thx_execute_noalloc: the execution needs more
                                 workspace than the static scratch holds         */
} thx_status;

typedef enum {
    THX_LEG2CHEB = 0,    /* Legendre -> Chebyshev, eq. (M), Sec. 3                     */
    THX_CHEB2LEG = 1,    /* Chebyshev -> Legendre, eq. (FormulaL), Sec. 5.1            */
    THX_ULTRA2ULTRA = 2, /* C^(l1) -> C^(l2), eq. (UltraSconversion), Sec. 5.2          */
    THX_JAC2JAC = 3,     /* P^(a,b) -> P^(g,d), Sec. 5.3 (reflection, then case 2)      */
    THX_LAG2LAG = 4,     /* L^(a1) -> L^(a2), Sec. 5.4                                  */
    THX_JAC2CHEB = 5,    /* P^(a,b) -> T, Sec. 5.3 (T_k = P_k^(-1/2,-1/2)/P_k^(-1/2,-1/2)(1)) */
    THX_CHEB2JAC = 6     /* T -> P^(g,d), Sec. 5.3                                     */
} thx_kind;

typedef enum {
    THX_FP64 = 0,      /* every step in double precision                              */
    THX_FP32_BULK = 1, /* FFTs and rank accumulation in single precision; Lambda and
                          Gamma ratios, the pivoted Cholesky and D1, D2 in double;
                          the dense path (3) in split bfloat16 with FP32 accumulation */
    THX_FP64_TAIL32 = 2 /* THX_FP64, except that on the three-pass path (2) the
                          trailing ranks whose pivots are at most tol * 2^23 of
                          the largest diagonal of H (Sec. 2.1: the rank-r term of
                          the Hankel approximation is of size pivot_r) run their
                          FFTs and partial sums in single precision: their
                          rounding then adds at most ~tol/4 of ||alpha||_1, below
                          the truncation the tolerance allows, and their
                          intermediates take half the bytes.  On by default for
                          L >= 2^16; thx_plan_autotune decides for its batch from
                          L = 8192 up (and may keep those ranks in double);
                          thx_plan_tail_slots says how many run in single */
} thx_precision;

/* plan flags */
#define THX_FLAG_FORCE_DIRECT 1u /* always use the O(N^2) direct evaluation         */
#define THX_FLAG_FORCE_FFT 2u    /* never use the direct evaluation (testing)        */
#define THX_FLAG_NO_DENSE 4u     /* direct evaluation entry by entry instead of the
                                    materialised dense matrix (testing, plan memory) */
#define THX_FLAG_AUTOTUNE 8u     /* thx_batch_create: tune every bucket for its member
                                    count (thx_plan_autotune); plans: no effect       */

typedef struct thx_plan thx_plan;

/* Plan for converting polynomials of degree <= `degree` (Fig. 1 steps 1-2 and the
 * symbol FFT): fills the Lambda / Gamma-ratio tables, runs the pivoted Cholesky
 * of the Hankel part(s) (Sec. 2.1, Fig. 3), and transforms the Toeplitz symbol.
 * The plan may be reused for any number of executions (Sec. 2.1, last paragraph).
 *   tol: the same target for every kind.  Sec. 2.1 leaves the stopping rule
 *   open; here pivots are chosen on, and the factorisation stopped by, the
 *   residual diagonal d_j weighted by w_j = |D1_j D2_j| (the diagonal pivoting of
 *   S H S with S = diag(sqrt w)), until max_j w_j d_j <= eps max_j w_j H_jj with
 *   eps = 2 tol |t_0| / (amp max_m |t_m|), amp = max_{j <= k} r_j / r_k,
 *   r = sqrt|D1 / D2|.  The truncation then changes beta by at most
 *   2 tol max_j |A_jj| ||alpha||_1, whatever D1 and D2 amplify (for leg2cheb,
 *   max_j |A_jj| = 1 and the rule is "largest residual diagonal <= tol max diag(H)").
 *   eps is never taken below 2^-51 (the double-precision noise of the residual);
 *   a tol that would need less returns THX_TOL_NOT_REACHED with a usable plan.
 *   Multi-stage conversions factorise every stage to the same tol.
 *   params / nparams: kind parameters -- ULTRA2ULTRA (l1, l2) with l1, l2 > 0
 *   (Sec. 5.2: one stage when l1 - l2 <= 1, negative integer differences
 *   banded (case 1); a larger drop goes down in unit steps first (case 3));
 *   JAC2JAC (a, b, g, d), JAC2CHEB (a, b), CHEB2JAC (g, d), all > -1 (Sec.
 *   5.3): a change of the second parameter is done first by the reflection
 *   P_k^(a,b)(-x) = (-1)^k P_k^(b,a)(x), then the first; each change is a
 *   banded stage for a whole-number rise (case 1), unit steps for a
 *   whole-number drop, and otherwise unit steps down to a level in (-1, 0]
 *   (in (0, 1] when both parameters are >= 1), the fractional case-2 stage
 *   there (case 3 with row 0 computed directly when first + second <= -1),
 *   and one banded rise back up (case 4; the order keeps the FFT stage where
 *   D1 and D2 amplify its rounding least);
 *   LAG2LAG (a1, a2) with a1, a2 > -1.  LEG2CHEB / CHEB2LEG take none.
 *   degree >= 0; 0 < tol < 1; flags: THX_FLAG_*.
 * On success *out owns device memory until thx_plan_destroy.  Errors:
 * THX_INVALID_ARGUMENT (out == NULL, degree < 0, tol outside (0,1), bad params),
 * THX_UNSUPPORTED (unknown kind), THX_OUT_OF_MEMORY,
 * THX_HIP_ERROR.  THX_TOL_NOT_REACHED returns a usable plan (rank cap reached
 * first, or tol below the double-precision floor). */
thx_status thx_plan_create(thx_plan **out, thx_kind kind, const double *params, int nparams,
                           int64_t degree, double tol, thx_precision prec, uint32_t flags,
                           hipStream_t stream);

/* beta[b][0..N] = A alpha[b][0..N] for b < batch (Fig. 1 steps 3-5), N = degree
 * with 0 <= degree <= the plan's degree.  alpha, beta: device doubles, row stride
 * ld >= degree+1; entries beyond N in each row are neither read nor written.
 * batch <= 65535 except on the dense path (thx_plan_path 3), which has no limit.
 * Errors: THX_INVALID_ARGUMENT (null plan, null pointers with batch > 0,
 * degree out of range, ld too small, batch < 0 or above the limit), THX_HIP_ERROR. */
thx_status thx_execute(const thx_plan *plan, const double *alpha, double *beta, int64_t degree,
                       int64_t batch, int64_t ld, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): thx_execute with every
 * workspace buffer (packed input, FFT intermediates, partial sums, the
 * intermediates between stages) carved from a static device array of
 * thx_noalloc_scratch_bytes() = 512 MiB, which the library holds on each GPU it
 * runs on until the process ends.  The call allocates nothing (no hipMalloc or
 * hipFree, no events; per-phase timing is not recorded).  Same arguments and
 * errors as thx_execute, plus THX_WORKSPACE_TOO_LARGE when the execution's
 * workspace does not fit (the slot chunks shrink before that happens: one
 * degree-2^20 FP64 vector fits).  Results equal thx_execute's up to rounding
 * (the chunking of the rank slots, and so the order of the partial sums, may
 * differ).  Every call on a GPU uses that GPU's one scratch, which keeps the
 * last call's contents: calls that overlap on one GPU (unordered streams or
 * threads) race and must be ordered by the caller. */
thx_status thx_execute_noalloc(const thx_plan *plan, const double *alpha, double *beta, int64_t degree,
                               int64_t batch, int64_t ld, hipStream_t stream);
int64_t thx_noalloc_scratch_bytes(void);

/* Variable-length members on device offsets (the paper's batches of Sec. 2.1
 * with one factorisation reused for every member): member i occupies
 * alpha[off[i] .. off[i+1] - 1] and beta at the same places, so its degree is
 * off[i+1] - off[i] - 1; d_offsets is a DEVICE array of count + 1 int64 and
 * total is the length of the alpha and beta arrays.  Members whose degree
 * exceeds the plan's, whose range leaves [0, total) or whose offsets decrease
 * are skipped (their beta entries untouched) and, when d_skipped (a DEVICE
 * int64, caller-initialised) is not NULL, counted there with an atomic add;
 * empty members are skipped silently.  The degrees are derived on the device,
 * so nothing synchronises; every member runs at the plan's FFT length (for many
 * members of very different degrees, thx_batch groups them by length instead).
 * count <= 65535 except on the dense path (3).  Errors: THX_INVALID_ARGUMENT
 * (null plan, null pointers with count > 0, count or total negative, count
 * above the limit), THX_OUT_OF_MEMORY, THX_HIP_ERROR. */
thx_status thx_execute_varlen(const thx_plan *plan, const double *alpha, double *beta, const int64_t *d_offsets,
                              int64_t count, int64_t total, int64_t *d_skipped, hipStream_t stream);

/* Release a plan (synchronises nothing; the caller must ensure no execution of
 * it is still running).  NULL is accepted. */
thx_status thx_plan_destroy(thx_plan *plan);

/* Plan introspection (host values; no device work).
 * rank: number of FFT slots K (for parity-split kinds max(K_even, K_odd)).
 * rank_part: rank of Hankel part `part` (0 = even / only, 1 = odd), -1 if absent.
 * fft_length: circulant-embedding length L (0 on the direct path): the smallest
 * of 2^k, 3 * 2^(k-2) and 5 * 2^(k-3) that is >= 2n - 2 for n Toeplitz lanes
 * (Sec. 2: any length >= 2n - 2 embeds the product exactly), the last two only
 * on the three-pass path with columns of at least 6 / 10 entries.
 * path: 0 direct (entries generated per output row), 1 single-workgroup LDS
 * FFT, 2 three-pass FFT, 3 dense: below the FFT crossover (degree + 1 <= 512,
 * THX_FLAG_NO_DENSE not set) the plan materialises the (degree+1)^2 matrix once
 * by the direct evaluation of the unit vectors, and every execution is one
 * matrix-core product with it (double precision for THX_FP64; for
 * THX_FP32_BULK the matrix and alpha as exact sums of three bfloat16 parts,
 * eight partial products summed in single precision), 4 unit step:
 * a parameter lowered by exactly 1 makes T and H constant (Sec. 5.2 and 5.3,
 * case 1), and beta_j = D1_j t_0 h_0 sum_{k >= j} D2_k alpha_k (k - j even for
 * the parity kinds) is a suffix sum, computed by a reverse scan in double
 * precision in O(N).  For a multi-stage plan, path and rank describe the first
 * stage (path 3 the whole conversion). */
int32_t thx_plan_rank(const thx_plan *plan);
/* THX_FP64_TAIL32 plans: FFT slots run in single precision (summed over the
 * stages); 0 for other plans and when every slot runs in double; -1 for NULL. */
int32_t thx_plan_tail_slots(const thx_plan *plan);
int32_t thx_plan_rank_part(const thx_plan *plan, int part);
int64_t thx_plan_fft_length(const thx_plan *plan);
int32_t thx_plan_path(const thx_plan *plan);
/* Three-pass geometry of the (first) stage: L = rows * cols, a row of `rows`
 * points per row-pass workgroup, column tiles of `tile_cols` adjacent columns
 * per column-pass workgroup.  THX_INVALID_ARGUMENT unless thx_plan_path is 2;
 * any output pointer may be NULL. */
thx_status thx_plan_fft_geometry(const thx_plan *plan, int64_t *rows, int64_t *cols,
                                 int64_t *tile_cols);
/* Launch shapes of the (first) stage, as set by thx_plan_autotune (defaults 512
 * and 1024): workgroups targeted per launch of the single-workgroup path and of
 * the inverse column pass.  Any output pointer may be NULL;
 * THX_INVALID_ARGUMENT for a null plan. */
thx_status thx_plan_launch_shape(const thx_plan *plan, int32_t *lds_blocks, int32_t *p3_blocks);
/* Largest FFT radix (8 or 16) of the (first) stage's single-workgroup path, as
 * set by thx_plan_autotune (default 8); -1 for a null plan. */
int32_t thx_plan_lds_radix(const thx_plan *plan);
/* Workgroups targeted per launch of the (first) stage's forward column pass, as
 * set by thx_plan_autotune: 0 (the default) is one workgroup per column tile,
 * slot and vector; a positive value lets each workgroup transform its tile for
 * several consecutive slots.  -1 for a null plan. */
int32_t thx_plan_p1_blocks(const thx_plan *plan);
/* 1 if the (first) stage's three-pass FFT runs its forward column pass inside
 * the row pass (columns of 2 or 4 entries: each row's column DFT is a
 * direct sum over the nonzero half of the zero-padded input, so no
 * intermediate array is written before the row transforms), as chosen by
 * thx_plan_autotune; 0 otherwise; -1 for a null plan. */
int32_t thx_plan_fused_columns(const thx_plan *plan);
/* Partial-sum groups the (first) stage uses for an execution of `batch` vectors
 * (the extra reads of the final D1 step); 0 for paths without them. */
int32_t thx_plan_partial_groups(const thx_plan *plan, int64_t batch);
/* Tune a plan for executions of `batch` vectors of its degree (the launch
 * shapes, row length and crossover that Sec. 2.1's reuse of one plan makes
 * worth choosing once): every FFT stage times its candidate launch shapes
 * (single-workgroup path: workgroups per launch; three-pass path: row length
 * and workgroups of the inverse column pass), then, for degree + 1 <= 2048,
 * the whole conversion times the stages against the materialised dense
 * matrix (path 3) and keeps the faster.  Candidates run on zero inputs with
 * HIP events on `stream` (median of three after a warm-up); the call
 * allocates and synchronises, and the plan must not be executing.  Results are
 * identical up to rounding whichever candidate wins.  THX_FLAG_FORCE_FFT or
 * THX_FLAG_NO_DENSE at creation exclude the dense candidate.  Errors:
 * THX_INVALID_ARGUMENT (null plan, batch < 1), THX_OUT_OF_MEMORY, THX_HIP_ERROR. */
thx_status thx_plan_autotune(thx_plan *plan, int64_t batch, hipStream_t stream);

/* The tolerance the factorisation of Hankel part `part` achieved, in the units
 * of thx_plan_create's tol (<= tol unless the plan returned THX_TOL_NOT_REACHED):
 * the largest weighted residual diagonal at termination, converted by the same
 * factor.  -1 for paths without a factorisation. */
double thx_plan_achieved_tol(const thx_plan *plan, int part);

/* Copy the normalised Cholesky columns of Hankel part `part` to host memory:
 * ell[r*n + i] = l_r[i] / sqrt(a_r) for r < rank_part, i < n, where n is the
 * size of that part (n_out receives it; pass ell = NULL to query n only) and
 * pivots[r] = p_r.  Synchronises `stream`.  For tests and diagnostics. */
thx_status thx_plan_factors(const thx_plan *plan, int part, double *ell, int32_t *pivots,
                            int64_t *n_out, hipStream_t stream);

/* One-shot conversions with an internal plan cache keyed by (kind, params,
 * degree, tol, prec, device): the first call for a key creates the plan
 * (synchronising `stream` once), later calls only execute.  Same buffer
 * conventions as thx_execute with ld = N+1.  Calls with the same key share one
 * workspace and are serialised: a call waits on the host while another thread's
 * call with that key launches, its work waits on the device (an event) for the
 * previous call's work on any stream, and a call with a larger batch than any
 * before it first waits on the host for that work.  Calls with different keys
 * run concurrently.  The paper's commands leg2cheb, cheb2leg, ultra2ultra,
 * jac2jac(v,a,b,g,d), jac2cheb and cheb2jac (Sec. 1, 5.1-5.3) and Laguerre
 * (Sec. 5.4). */
thx_status thx_leg2cheb(const double *alpha, double *beta, int64_t N, int64_t batch, double tol,
                        thx_precision prec, hipStream_t stream);
thx_status thx_cheb2leg(const double *alpha, double *beta, int64_t N, int64_t batch, double tol,
                        thx_precision prec, hipStream_t stream);
thx_status thx_ultra2ultra(const double *alpha, double *beta, int64_t N, int64_t batch,
                           double lambda1, double lambda2, double tol, thx_precision prec,
                           hipStream_t stream);
thx_status thx_lag2lag(const double *alpha, double *beta, int64_t N, int64_t batch, double alpha1,
                       double alpha2, double tol, thx_precision prec, hipStream_t stream);
/* Jacobi P^(a,b) -> P^(g,d) (Sec. 5.3), parameters > -1 (THX_INVALID_ARGUMENT otherwise). */
thx_status thx_jac2jac(const double *alpha, double *beta, int64_t N, int64_t batch, double a, double b, double g,
                       double d, double tol, thx_precision prec, hipStream_t stream);
/* Jacobi P^(a,b) -> Chebyshev T (Sec. 5.3, T_k = P_k^(-1/2,-1/2) / P_k^(-1/2,-1/2)(1)). */
thx_status thx_jac2cheb(const double *alpha, double *beta, int64_t N, int64_t batch, double a, double b,
                        double tol, thx_precision prec, hipStream_t stream);
/* Chebyshev T -> Jacobi P^(g,d) (Sec. 5.3). */
thx_status thx_cheb2jac(const double *alpha, double *beta, int64_t N, int64_t batch, double g, double d,
                        double tol, thx_precision prec, hipStream_t stream);
/* Drop every cached plan: waits for every cached plan's calls (host and device),
 * then synchronises the device.  No one-shot call may start meanwhile. */
thx_status thx_cache_clear(void);

/* Mixed-degree batches (Fig. 1 applied to many polynomials; one pivoted
 * Cholesky per bucket, reused by every member as Sec. 2.1 suggests).
 * Polynomial i has degree degrees[i] (host array of `count`) and its
 * coefficients are stored contiguously: alpha[off_i .. off_i + degrees[i]] with
 * off_i = sum_{m<i} (degrees[m] + 1); beta uses the same layout.  Members are
 * grouped by FFT length; each group gets one plan at its largest degree (the
 * Hankel part for degree N is the leading block of the one for a larger
 * degree, so the factorisation holds for every member).  Degrees up to the
 * direct crossover (THX_DIRECT_MAX, default 512, or flags) form one bucket
 * evaluated directly: by the dense matrix product (path 3) when the largest of
 * them is below 512 and THX_FLAG_NO_DENSE is not set, else entry by entry
 * (buckets of at most 65535 members).  All workspace is allocated here;
 * thx_batch_create synchronises
 * `stream`.  Errors as thx_plan_create, plus THX_INVALID_ARGUMENT for a
 * negative degree or count. */
typedef struct thx_batch thx_batch;
thx_status thx_batch_create(thx_batch **out, thx_kind kind, const double *params, int nparams,
                            const int64_t *degrees, int64_t count, double tol, thx_precision prec,
                            uint32_t flags, hipStream_t stream);
/* Convert every member: device alpha / beta in the layout above.  With
 * use_graph != 0 the launch sequence is captured once into a hipGraph (on the
 * batch's own stream; re-captured when alpha or beta change) and replayed on
 * `stream`; no allocation and no memset node is recorded.  Executions of one
 * batch must be serialised. */
thx_status thx_batch_execute(thx_batch *batch, const double *alpha, double *beta, int use_graph,
                             hipStream_t stream);
thx_status thx_batch_destroy(thx_batch *batch);
/* sum of (degree + 1) over the members; number of buckets; per-bucket facts
 * (fft_length 0 and path 0 for the direct bucket) */
int64_t thx_batch_coefficients(const thx_batch *batch);
int32_t thx_batch_buckets(const thx_batch *batch);
thx_status thx_batch_bucket_info(const thx_batch *batch, int i, int64_t *fft_length, int64_t *members,
                                 int64_t *max_degree, int32_t *path, int32_t *rank);

/* Lambda table (Sec. 1, definition under eq. (M)):
 * out[i] = Lambda(z0 + i) = Gamma(z0 + i + 1/2) / Gamma(z0 + i + 1), i < count;
 * out is a device pointer.  Exposed for tests of the generator. */
thx_status thx_lambda_table(double *out, int64_t count, double z0, hipStream_t stream);
/* General ratio: out[i] = Gamma(z0 + i + a) / Gamma(z0 + i + b), i < count.
 * Poles of the numerator return +-inf; poles of the denominator return 0. */
thx_status thx_gamma_ratio_table(double *out, int64_t count, double z0, double a, double b,
                                 hipStream_t stream);

/* Per-phase GPU timing of thx_execute (tracing).  thx_plan_enable_timing takes
 * a mask of phases (bit 1 << THX_PHASE_x; THX_TIME_ALL for every phase, 0 to
 * stop): each kernel launch of a selected phase is then bracketed by two
 * hipEvents recorded on the execution's stream.  Every recorded event delays
 * the stream by a few microseconds, so a measurement of one kernel should
 * select that phase only.  thx_plan_timings waits for the recorded events and writes, per
 * phase, the summed milliseconds and the number of timed launches since the
 * last reset (ms and launches: host arrays of THX_NPHASES entries, either may
 * be NULL); reset != 0 clears the record.  At most 16384 launches are recorded
 * between resets; later launches run untimed. */
enum {
    THX_PHASE_PACK = 0,     /* v = D2 alpha into complex lanes (Fig. 1 step 3)      */
    THX_PHASE_TOEP_LDS = 1, /* single-workgroup Toeplitz products (step 4)          */
    THX_PHASE_COL_FWD = 2,  /* three-pass FFT, forward column pass (step 4)         */
    THX_PHASE_ROW = 3,      /* three-pass FFT, row pass with the symbol (step 4)    */
    THX_PHASE_COL_INV = 4,  /* three-pass FFT, inverse column pass + rank sum       */
    THX_PHASE_ROW0 = 5,     /* cheb2leg row 0 by a direct dot product               */
    THX_PHASE_UNPACK = 6,   /* beta = D1 w (Fig. 1 step 5)                          */
    THX_PHASE_DIRECT = 7,   /* O(N^2) direct evaluation                             */
    THX_PHASE_DENSE = 8,    /* product with the materialised matrix (path 3)        */
    THX_PHASE_SCAN = 9,     /* unit step by suffix sums (path 4)                    */
    THX_NPHASES = 10
};
#define THX_TIME_ALL ((1u << THX_NPHASES) - 1u)
thx_status thx_plan_enable_timing(thx_plan *plan, uint32_t phases);
thx_status thx_plan_timings(thx_plan *plan, double *ms, int64_t *launches, int reset);

/* Tracing: launch an empty kernel (k_trace_marker) of `id` workgroups of 64
 * threads on `stream`, 1 <= id <= 65535, so that a kernel trace can be cut
 * into regions (the trace shows the grid size id * 64).  THX_INVALID_ARGUMENT
 * outside that range. */
thx_status thx_trace_marker(int id, hipStream_t stream);

const char *thx_status_string(thx_status s);
/* hipError_t of the last failed HIP call made by this thread inside the library */
hipError_t thx_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* THX_H */
