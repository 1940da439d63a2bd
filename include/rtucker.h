/*
 * rtucker.h -- C ABI of the MI355X (gfx950) library for randomized Tucker
 * compression of big dense tensors and FFCP, the CP / nonnegative CP fit
 * computed through the compressed format.
 *
 * Method: G. Zhou, A. Cichocki, S. Xie, "Decomposition of Big Tensors With
 * Low Multilinear Rank" (arXiv 1412.1885).
 *   - rt_tucker_rand : RandTucker2i, Algorithm 3 (Section IV-A), with the
 *                      randomized range finder of Section IV-A, steps 1-3.
 *   - rt_ffcp        : FFCP, Algorithm 1 (Section III-B), eqs. (8), (9),
 *                      (12)-(15).
 *   - rt_ttm, rt_cp_fit_dense : building blocks exported for tests and for
 *                      evaluating a CP model against the dense tensor.
 *   - rt_mlp_*       : the learned FFCP initializer (no counterpart in the
 *                      paper; it proposes the initialization step of
 *                      Algorithm 1).
 *
 * Conventions shared by every entry point
 *   - Tensors are dense, row-major (last index fastest), contiguous.
 *   - Matrices are row-major.  A factor matrix of mode n is I_n x R.
 *   - "device" pointers are HIP device allocations on the current device;
 *     "host" pointers are ordinary host memory.  Arrays of per-mode device
 *     pointers (e.g. `const float* const* U`) are HOST arrays of N device
 *     pointers.
 *   - All device buffers are owned by the caller.  The library allocates no
 *     device memory: temporary storage comes from the caller's workspace,
 *     whose size the matching *_workspace query returns.
 *   - Work is enqueued on the caller's stream `stream` (a hipStream_t passed
 *     as void*; NULL is the default stream) and returns without waiting.
 *     Results and the device-side info structs are valid after the stream
 *     is synchronized.
 *   - Return value: RT_OK (0) or a negative rt_status.  Argument errors are
 *     detected on the host before anything is enqueued; a message is kept
 *     per thread and returned by rt_last_error().  No C++ exception or abort
 *     crosses this ABI.  Conditions the device detects (non-finite input,
 *     ridge applied to a singular Gram matrix) are reported in the info
 *     structs, never as a return code.
 *   - Device pointers must be 16-byte aligned (RT_ERR_INVALID_ARG otherwise).
 */
#ifndef RTUCKER_H
#define RTUCKER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RT_MAX_MODES 8
#define RT_MAX_SKETCH 64 /* largest sketch width R~_n and CP rank R */

typedef enum {
  RT_OK = 0,
  RT_ERR_INVALID_ARG = -1,
  RT_ERR_UNSUPPORTED = -2,
  RT_ERR_WORKSPACE = -3,
  RT_ERR_NONFINITE = -4,
  RT_ERR_NUMERICAL = -5,
  RT_ERR_HIP = -6,
  RT_ERR_NO_DEVICE = -7
} rt_status;

/* Arithmetic of the Y-streaming passes of rt_tucker_rand. */
typedef enum {
  RT_F32 = 0,        /* FP32 Y, FP32 products, FP32 accumulation            */
  RT_BF16_MIXED = 1, /* FP32 Y converted once to a BF16 copy; BF16 products,
                        FP32 accumulation (MFMA); QR/eig stay FP64           */
  RT_F64 = 2         /* FP64 Y, FP64 everywhere                              */
} rt_precision;

/* rt_tucker_desc.flags */
#define RT_FLAG_NO_TRUNCATE 0x1u /* return the R~-sized Q_n and G~         */
#define RT_FLAG_BF16_INPUT 0x2u  /* RT_BF16_MIXED only: Y already holds the
                                    BF16 copy (uint16 bit patterns); no FP32
                                    pass and no conversion                  */
#define RT_FLAG_GAUSS_SEIDEL 0x4u /* the loop order of Algorithm 3 as
                                     printed: mode n's sketch uses the bases
                                     modes < n received in the same sweep
                                     (two passes over Y per sweep instead of
                                     one)                                   */

/*
 * Problem description of rt_tucker_rand.
 *   N              number of modes, 2..RT_MAX_MODES.
 *   dims[n]        I_n >= 1.
 *   ranks_tilde[n] R~_n, sketch width (the paper's R_n + p, Section IV-A),
 *                  1 <= R~_n <= min(I_n, RT_MAX_SKETCH) so that Q_n can
 *                  have R~_n orthonormal columns.
 *   ranks[n]       output Tucker rank R_n, 1..R~_n (ignored with
 *                  RT_FLAG_NO_TRUNCATE).  R~_n -> R_n truncation goes
 *                  through the core's mode-n Gram eigenvectors.
 *   sweeps         1 or 2: how many times the sketch loop of Algorithm 3
 *                  runs (the paper runs it twice; the second sweep is the
 *                  "one additional ALS-like iteration").
 *   precision      rt_precision.
 */
typedef struct {
  int32_t N;
  int32_t sweeps;
  int32_t precision;
  uint32_t flags;
  int64_t dims[RT_MAX_MODES];
  int32_t ranks[RT_MAX_MODES];
  int32_t ranks_tilde[RT_MAX_MODES];
} rt_tucker_desc;

/* Written by the device (caller-owned device memory). */
typedef struct {
  double normY2;    /* ||Y||_F^2 of the input values (FP32, FP64, or the
                       caller's BF16 values), FP64 accumulation           */
  double normG2;    /* ||G||_F^2 of the returned core                    */
  int32_t nonfinite; /* nonzero if a NaN/Inf was seen in Y               */
  int32_t rank_deficient; /* bit n set if Z_n had a zero Householder
                             pivot (exact rank deficiency)               */
  int64_t reserved[2];
} rt_tucker_info;

/* Optional intermediate outputs of rt_tucker_rand (every pointer may be
 * NULL).  Z[s*N+n]: sweep s sketch Z_n, I_n x R~_n FP32 (FP64 for RT_F64).
 * Q[s*N+n]: its orthonormal basis, same shape and type.  Gt: the
 * untruncated core G~, prod R~_n, same type. */
typedef struct {
  void* Z[2 * RT_MAX_MODES];
  void* Q[2 * RT_MAX_MODES];
  void* Gt;
} rt_tucker_trace;

/*
 * Workspace bytes rt_tucker_rand needs for this description (host only; no
 * device work).  Returns RT_ERR_INVALID_ARG for an invalid description.
 */
int rt_tucker_rand_workspace(const rt_tucker_desc* desc, size_t* bytes);

/*
 * Length, in uint16 values, of the Ybf16 buffer rt_tucker_rand needs (host
 * only; no device work): I_1 ... I_{N-1} L with L = I_N rounded up to a
 * multiple of 64, for RT_BF16_MIXED without RT_FLAG_BF16_INPUT; 0 otherwise.
 * Returns RT_ERR_INVALID_ARG for an invalid description or NULL elems.
 */
int rt_tucker_bf16_copy_elems(const rt_tucker_desc* desc, int64_t* elems);

/*
 * RandTucker2i (Algorithm 3, Section IV-A) on a dense tensor.
 *
 * For each sweep s = 1..sweeps and every mode n (Jacobi order: every mode of
 * a sweep uses the bases of the previous sweep; sweep 1 uses Omega_p, the
 * random initial U^(p) that Algorithm 3 starts from; with
 * RT_FLAG_GAUSS_SEIDEL the modes p < n use the bases of the current sweep):
 *     X_n = Y x_{p != n} B_p^T,    Z_n = X_(n) Omega~_n^(s),
 *     Q_n = orth(Z_n)   (FP64 Householder QR, signs so that diag(R) >= 0)
 * then the core G~ = Y x_1 Q_1^T ... x_N Q_N^T (the core projection of Algorithm 3) and,
 * unless RT_FLAG_NO_TRUNCATE, the truncation to R_n:
 *     W_n = top-R_n eigenvectors of G~_(n) G~_(n)^T (descending, each
 *           column's largest-magnitude entry positive),
 *     U_n = Q_n W_n,   G = G~ x_n W_n^T.
 *
 *   Y          device; FP32 (RT_F32, RT_BF16_MIXED), FP64 (RT_F64) or BF16
 *              bit patterns (RT_BF16_MIXED with RT_FLAG_BF16_INPUT);
 *              I_1 x ... x I_N row-major.  Not modified.
 *   Omega      host array of N device FP32 (FP64 for RT_F64) matrices
 *              Omega_n, I_n x R~_n row-major (Gaussian test matrices).
 *   Omega_t    host array of sweeps*N device matrices Omega~_n^(s) (index
 *              s*N + n), (prod_{p != n} R~_p) x R~_n row-major; row index
 *              is the row-major flattening of (j_p)_{p != n}, increasing p.
 *   ws         device workspace of at least ws_bytes >= the query result.
 *   U          host array of N device outputs, I_n x R_n (I_n x R~_n with
 *              RT_FLAG_NO_TRUNCATE), FP32 (FP64 for RT_F64).
 *   G          device output core, R_1 x ... x R_N, same type as U.
 *   Ybf16      RT_BF16_MIXED without RT_FLAG_BF16_INPUT: device buffer of
 *              rt_tucker_bf16_copy_elems(desc) uint16 receiving the scaled
 *              BF16 copy of Y, [I_1 ... I_{N-1}][L] row-major with row
 *              stride L = I_N rounded up to a multiple of 64 (128 bytes):
 *              entry (i_1..i_N) is bf16_rne(Y(i_1..i_N) 2^-e) with one
 *              e per slab of fixed (i_1..i_{N-2}): 0 while the binary
 *              exponent of the slab's largest |Y| lies in [-100, 100], that
 *              exponent otherwise; the L - I_N padding values are zero.
 *              NULL otherwise.
 *   info       device rt_tucker_info (may be NULL).
 *   trace      host struct of optional device outputs (may be NULL).
 *   stream     hipStream_t.
 * Errors: RT_ERR_INVALID_ARG (bad description, NULL required pointer,
 * misalignment), RT_ERR_WORKSPACE (ws_bytes too small), RT_ERR_UNSUPPORTED
 * (a shape the precision form's kernels do not take), RT_ERR_HIP (a launch
 * failed).
 */
int rt_tucker_rand(const rt_tucker_desc* desc, const void* Y,
                   const void* const* Omega, const void* const* Omega_t,
                   void* ws, size_t ws_bytes, void* const* U, void* G,
                   uint16_t* Ybf16, rt_tucker_info* info,
                   const rt_tucker_trace* trace, void* stream);

/*
 * Sequential RandTucker (Algorithm 2, Section IV-A) with dense Gaussian test
 * matrices drawn on the device.  For n = 1..N:
 *     Z_n = Y_(n) Omega_n,  U_n = orth(Z_n)  (FP64 QR, diag(R) >= 0),
 *     Y <- Y x_n U_n^T,
 * where Omega_n has one row per index of the other modes in their current
 * sizes (modes < n already shrunk to R~_k; row-major order of those
 * indices, increasing mode) and R~_n columns.  The last tensor is the core
 * G (R~_1 x ... x R~_N).  Entry (r, k) of Omega_n is produced from
 * (seed, n, r, k) alone by rt_gaussian_matrix's generator.  Two passes over
 * the full tensor; Omega_1 (prod_{k>1} I_k x R~_1) is materialized in the
 * workspace.
 *   N 2..RT_MAX_MODES; precision RT_F32 or RT_F64 (others:
 *   RT_ERR_UNSUPPORTED); dims I_n >= 1; 1 <= R~_n <= min(I_n, RT_MAX_SKETCH).
 */
typedef struct {
  int32_t N;
  int32_t precision;
  uint64_t seed;
  int64_t dims[RT_MAX_MODES];
  int32_t ranks_tilde[RT_MAX_MODES];
} rt_sequential_desc;

int rt_tucker_sequential_workspace(const rt_sequential_desc* desc, size_t* bytes);
/*   Y         device, I_1 x ... x I_N row-major, FP32 or FP64 (precision).
 *   U         host array of N device outputs U_n, I_n x R~_n (same type).
 *   G         device output core, R~_1 x ... x R~_N (same type).
 *   Omega_out NULL, or a host array of N device buffers (entries may be NULL)
 *             receiving each Omega_n as used (rows x R~_n, same type).
 * Errors: RT_ERR_INVALID_ARG, RT_ERR_UNSUPPORTED, RT_ERR_WORKSPACE, RT_ERR_HIP. */
int rt_tucker_sequential(const rt_sequential_desc* desc, const void* Y, void* ws,
                         size_t ws_bytes, void* const* U, void* G, void* const* Omega_out,
                         void* stream);
/*
 * The counter-based Gaussian matrix of Alg. 2's test matrices: out[r][k]
 * (rows x cols row-major, device, dtype RT_F32 or RT_F64) is entry (r, k) for
 * mode `mode`: Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC
 * 2011) on counter (r mod 2^32, r div 2^32, k, mode) and key (seed mod 2^32,
 * seed div 2^32), then Box-Muller in FP64 on the first two output words x0,
 * x1: u1 = (x0 + 1) 2^-32, u2 = (x1 + 1/2) 2^-32,
 * value = sqrt(-2 ln u1) cos(2 pi u2), rounded to dtype.
 */
int rt_gaussian_matrix(int32_t dtype, uint64_t seed, int32_t mode, int64_t rows, int32_t cols,
                       void* out, void* stream);

/* FFCP update rules (the factor update of Algorithm 1). */
typedef enum {
  RT_ALS = 0,  /* eq. (14): A = U G_(n)(KR V) (hadamard A^T A)^{-1}        */
  RT_HALS = 1, /* eq. (8), standard form a_r <- max(eps, a_r + (q_r -
                  A t_r)/t_rr), columns in order, eps = 1e-16            */
  RT_MU = 2    /* eq. (15) with 1e-16 added to the denominator          */
} rt_update;

typedef enum {
  RT_INIT_USER = 0,  /* A_init given                                      */
  RT_INIT_HOSVD = 1, /* V_n = top-R eigenvectors of G_(n) G_(n)^T, padded
                        with the caller's `pad` columns when R > R_n      */
  RT_INIT_COEFF = 2, /* A_init holds N device FP32 R_n x R coefficient
                        matrices V_n (e.g. rt_mlp_forward): A_n = U_n V_n  */
  RT_INIT_COEFF_GUARDED = 3 /* as RT_INIT_COEFF, but the HOSVD start is
                        built too and the one with the higher initial fit
                        is used (ALS without l1; other rules: as COEFF)   */
} rt_init;

/*
 * Problem description of rt_ffcp.
 *   N, dims[n] = I_n, ranks[n] = R_n: the Tucker format [[G; U]].
 *   R        CP rank, 1..RT_MAX_SKETCH.
 *   update   rt_update;  init  rt_init.
 *   max_it   iteration cap (>= 1);  tol  stop at iteration t >= 2 when
 *            |Fit_t - Fit_{t-1}| < tol (Section V-A rule; tol = 0 runs
 *            exactly max_it iterations).
 *   l1       soft-threshold level c of eq. (16) applied after each update
 *            (0 disables); under HALS the shrunk entries are floored at
 *            1e-16 again (HALS's feasible set) so no column vanishes.
 *   normY2   ||[[G;U]]||^2 used by the fit; NaN (or negative) means: compute
 *            <G, G x_n U_n^T U_n> on the device.
 */
typedef struct {
  int32_t N;
  int32_t R;
  int32_t update;
  int32_t init;
  int32_t max_it;
  int32_t reserved;
  double tol;
  double l1;
  double normY2;
  int64_t dims[RT_MAX_MODES];
  int32_t ranks[RT_MAX_MODES];
} rt_ffcp_desc;

/* Written by the device. */
typedef struct {
  int32_t iterations; /* iterations run                                  */
  int32_t converged;  /* 1 if the tolerance test stopped the loop; -1
                         if a grid barrier of the multi-workgroup form
                         gave up (results undefined; not expected: the
                         cooperative launch keeps every workgroup
                         resident)                                       */
  int32_t ridged;     /* 1 if a Cholesky failed and the ridge
                         1e-12 tr(T)/R was added                         */
  int32_t init_used;  /* RT_INIT_COEFF_GUARDED: 1 if the caller's start
                         was kept, 0 if the HOSVD start was; else 0      */
  double fit;         /* final Fit = 1 - ||Yt - Yhat|| / ||Yt||           */
  double fit_prev;    /* fit of the previous iteration                   */
} rt_ffcp_info;

int rt_ffcp_workspace(const rt_ffcp_desc* desc, size_t* bytes);

/*
 * FFCP (Algorithm 1, Section III-B) on a Tucker format [[G; U]].
 * Per iteration, for n = 1..N:
 *     H_n = G_(n) [KR_{p != n} V_p]         (eq. 12-13),
 *     Q_n = U_n H_n,  T_n = hadamard_{p != n} A_p^T A_p   (eq. 9),
 *     A_n <- update (ALS / HALS / MU),  optional S_c (eq. 16),
 *     columns of A_n normalized for n < N (lambda lives in A_N, eq. 2),
 *     V_n = U_n^T A_n                       (eq. 13).
 * Fit after mode N in closed form: ||Yt||^2 - 2 sum(H_N * V_N) +
 * 1^T (hadamard_p A_p^T A_p) 1 (FP64).  Arithmetic is FP64 on the device;
 * U, G, A_init are read as FP32 and the outputs written as FP32.
 * Execution: unconstrained ALS without S_c runs in the compressed space in
 * one workgroup; the other rules run in one workgroup too, or, when the
 * longest mode has 2048 rows or more, in one cooperative launch of up to
 * 256 workgroups (each owning a chunk of every mode's rows, cross products
 * summed from per-workgroup partials in a fixed order).
 *
 *   U        host array of N device FP32 matrices I_n x R_n.
 *   G        device FP32 core R_1 x ... x R_N.
 *   A_init   host array of N device FP32 I_n x R (RT_INIT_USER), or
 *            R_n x R coefficient matrices (RT_INIT_COEFF[_GUARDED]), else
 *            NULL.
 *   pad      RT_INIT_HOSVD with R > R_n: host array of N device FP32
 *            R_n x (R - R_n) matrices (entries for modes with R <= R_n are
 *            ignored and may be NULL); NULL otherwise.
 *   A        host array of N device FP32 outputs I_n x R, unit columns.
 *   lambda   device FP32 output, R weights (||a_r^(N)|| before the final
 *            normalization).
 *   fit_trace device FP64 array of max_it entries receiving the fit of
 *            every iteration run (may be NULL).
 *   info     device rt_ffcp_info (may be NULL).
 * Errors: RT_ERR_INVALID_ARG, RT_ERR_WORKSPACE, RT_ERR_HIP.
 */
int rt_ffcp(const rt_ffcp_desc* desc, const float* const* U, const float* G,
            const float* const* A_init, const float* const* pad,
            void* ws, size_t ws_bytes, float* const* A, float* lambda,
            double* fit_trace, rt_ffcp_info* info, void* stream);

/*
 * rt_ffcp without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, results and errors as
 * rt_ffcp, minus ws / ws_bytes: the scratch is a static 32 MiB array of the
 * library on each GPU (held until the process ends), so the call allocates
 * nothing.  Problems whose rt_ffcp_workspace exceeds 32 MiB are rejected
 * with RT_ERR_UNSUPPORTED before anything is enqueued (R = R_n = 20 needs
 * about 2.9 MiB at I_n = 1000 in 3 modes and 19.0 MiB at I_n = 10^4 in 4).  Every call on one GPU shares
 * that GPU's array: calls that overlap in time on one GPU (other streams or
 * host threads) race and must be serialized by the caller; calls in order on
 * one stream are safe.  Nothing in the array needs to start at zero.
 */
int rt_ffcp_noalloc(const rt_ffcp_desc* desc, const float* const* U, const float* G,
                    const float* const* A_init, const float* const* pad, float* const* A,
                    float* lambda, double* fit_trace, rt_ffcp_info* info, void* stream);

/*
 * Algorithm 1 with the dense tensor as its input (the problem statement
 * "ffcp(Y, R)"): RandTucker2i compresses Y exactly as rt_tucker_rand does,
 * then FFCP runs on the Tucker format it returns exactly as rt_ffcp does.
 * The Tucker format lives in the workspace (the caller does not see it).
 *
 *   tdesc     the compression (rt_tucker_rand's description); precision
 *             RT_F32 or RT_BF16_MIXED (RT_F64: RT_ERR_UNSUPPORTED, FFCP reads
 *             an FP32 format).
 *   fdesc     the fit (rt_ffcp's description); N, dims and ranks must equal
 *             the Tucker output's (R_n, or R~_n with RT_FLAG_NO_TRUNCATE),
 *             else RT_ERR_INVALID_ARG.
 *   Y, Omega, Omega_t, Ybf16, tinfo: as rt_tucker_rand's Y, Omega, Omega_t,
 *             Ybf16, info.
 *   A_init, pad, A, lambda, fit_trace, finfo: as rt_ffcp's A_init, pad, A,
 *             lambda, fit_trace, info.
 *   ws        device workspace of ws_bytes >= rt_ffcp_dense_workspace().
 * Every argument of both stages is checked before anything is enqueued.
 * Errors: those of rt_tucker_rand and rt_ffcp.
 */
int rt_ffcp_dense_workspace(const rt_tucker_desc* tdesc, const rt_ffcp_desc* fdesc,
                            size_t* bytes);
int rt_ffcp_dense(const rt_tucker_desc* tdesc, const rt_ffcp_desc* fdesc, const void* Y,
                  const void* const* Omega, const void* const* Omega_t, uint16_t* Ybf16,
                  const float* const* A_init, const float* const* pad, void* ws,
                  size_t ws_bytes, float* const* A, float* lambda, double* fit_trace,
                  rt_tucker_info* tinfo, rt_ffcp_info* finfo, void* stream);

/*
 * Mode-n product out = X x_n M^T (the contraction the paper writes
 * Y x_n U^T, eq. (1) and Algorithms 2-3): X viewed as [A, I, C] with
 * A = prod_{p<n} I_p, I = I_n, C = prod_{p>n} I_p; M is I x K row-major;
 * out is [A, K, C].  dtype: 0 = FP32, 2 = FP64 (rt_precision values).
 * All pointers device.  K <= RT_MAX_SKETCH.  No workspace.
 */
int rt_ttm(int32_t dtype, int64_t A, int64_t I, int64_t C, int32_t K,
           const void* X, const void* M, void* out, void* stream);

/*
 * One streamed pass over a dense tensor viewed as A slabs of I1 x I2 (the
 * two contractions one Algorithm 3 sweep needs from Y, see rt_tucker_rand):
 *     TA[a, i1, k] = sum_{i2} Y[a, i1, i2] B2[i2, k]     (A x I1 x K2)
 *     TB[a, j, i2] = sum_{i1} B1[i1, j] Y[a, i1, i2]     (A x K1 x I2)
 * TB and B1 may be NULL (core pass: TA only).  norm_out (device FP64[1],
 * may be NULL) receives ||Y||_F^2.  dtype: RT_F32 or RT_F64 (same for all
 * arrays).  All pointers device; K1, K2 <= RT_MAX_SKETCH.  Exported for
 * kernel-level tests; ws: device scratch of >= 8192 bytes.
 */
int rt_stream_pass(int32_t dtype, int64_t A, int64_t I1, int64_t I2,
                   const void* Y, const void* B2, int32_t K2, const void* B1,
                   int32_t K1, void* TA, void* TB, double* norm_out,
                   void* ws, size_t ws_bytes, void* stream);

/*
 * Fit of a CP model against a dense tensor (Section III-B definition,
 * Fit = 1 - ||Y - Yhat|| / ||Y||) through one mode-N contraction of Y:
 * <Y, Yhat> = sum(lambda * A_N * (Y_(N) KR_{p<N} A_p)), ||Yhat||^2 from the
 * Gram identity eq. (9), ||Y||^2 accumulated in FP64.
 *   Y: device FP32 tensor (desc dims/N; R from desc.R); A: host array of N
 *   device FP32 I_n x R; lambda: device FP32 R (NULL = ones);
 *   ws/ws_bytes from rt_cp_fit_workspace; out3: device FP64[3] receiving
 *   {fit, ||Y||^2, <Y,Yhat>}.
 */
int rt_cp_fit_workspace(const rt_ffcp_desc* desc, size_t* bytes);
int rt_cp_fit_dense(const rt_ffcp_desc* desc, const float* Y,
                    const float* const* A, const float* lambda, void* ws,
                    size_t ws_bytes, double* out3, void* stream);

/*
 * Stage timing (tracing).  When enabled, the library brackets each stage it
 * enqueues with HIP events on the caller's stream; rt_profile_read waits for
 * the recorded events and returns per-stage totals.  Host-side only; the
 * events are created by the library (no device memory).
 * Stages (each brackets the launches named): 0 = the streaming kernel of the
 * first sweep,
 * 1 = the streaming kernel of later sweeps, 2 = the core pass's streaming
 * kernel, 3 = intermediate contractions and sketch products, 4 = QR,
 * 5 = truncation (Gram, eig, rotation), 6 = FFCP, 7 = the precision form's
 * per-slab statistics (slab exponents and ||Y||^2 from the conversion's
 * partials, re-conversion of the slabs that need a scale; a caller's BF16
 * input: its statistics pass), 8 = the precision form's FP32 -> BF16
 * conversion, which also yields those partials (the first sweep's streaming
 * kernel then reads the BF16 copy).
 */
#define RT_PROFILE_STAGES 9
typedef struct {
  double ms[RT_PROFILE_STAGES];   /* summed event time per stage          */
  int64_t count[RT_PROFILE_STAGES]; /* number of bracketed launches        */
} rt_profile;

/* Turn stage timing on (1) or off (0); turning it on clears the totals. */
int rt_profile_enable(int on);
/* Synchronize the recorded events and fill *out; returns RT_ERR_HIP if an
 * event query fails. */
int rt_profile_read(rt_profile* out);

/*
 * Learned FFCP initializer (no counterpart in the paper: it supplies the
 * initialization step of Algorithm 1).  A 3-layer MLP maps the normalized
 * core x = vec(G)/||G|| (d0 = prod R_n entries) to compressed factors V_n
 * (R_n x R) of that core:
 *   h1 = gelu(x W1 + b1), h2 = gelu(h1 W2 + b2), y = h2 W3 + b3,
 *   y = [vec V_1, ..., vec V_N] (row-major V_n, d3 = R sum R_n),
 * gelu(z) = z Phi(z).  Training minimizes the CP loss of the core,
 *   L = mean over the batch of ||G/||G|| - [[V_1..V_N]]||^2,
 * whose factor gradient is eq. (5) applied to the core (eq. (17)).  Matrix
 * products take BF16 operands (weights, activations, and in the backward
 * pass the output and pre-activation gradients) with FP32 accumulation;
 * master weights, biases and Adam moments are FP32.  Core order 3 only;
 * R <= 32, R_n <= 32; d0, d3, hidden widths multiples of 8.
 */
typedef struct {
  int32_t batch;                   /* cores per call                          */
  int32_t N;                       /* core order (3)                          */
  int32_t R;                       /* CP rank                                 */
  int32_t hidden1, hidden2;        /* hidden widths                           */
  int32_t core_dims[RT_MAX_MODES]; /* R_1..R_N                                */
} rt_mlp_desc;

/* Device buffers of the network, layer l = 0, 1, 2 with widths
 * (d0, hidden1, hidden2, d3): W[l] d_l x d_{l+1} row-major FP32 (master),
 * Wb[l] its BF16 copy (bit patterns, what the products read), b[l] FP32;
 * Adam moments mW/vW/mb/vb (FP32, same shapes; training only). */
typedef struct {
  float* W[3];
  float* b[3];
  uint16_t* Wb[3];
  float* mW[3];
  float* vW[3];
  float* mb[3];
  float* vb[3];
} rt_mlp_params;

/* Workspace bytes of every rt_mlp_* call with this descriptor. */
int rt_mlp_workspace(const rt_mlp_desc* desc, size_t* bytes);
/* Wb[l] = bf16_rne(W[l]) (after initializing or loading W). */
int rt_mlp_sync_bf16(const rt_mlp_desc* desc, const rt_mlp_params* params,
                     void* stream);
/* Inference: G (device, batch x d0 FP32 cores) -> V (device, batch x d3 FP32),
 * the predicted factors scaled by ||G||^(1/N): FFCP's initial V_n. */
int rt_mlp_forward(const rt_mlp_desc* desc, const rt_mlp_params* params,
                   const float* G, float* V, void* ws, size_t ws_bytes,
                   void* stream);
/* Loss and gradients without updating: gW[l], gb[l] (host arrays of device
 * FP32 buffers shaped like W[l], b[l]); loss (device, batch FP32 per-core
 * losses; their mean is L). */
int rt_mlp_grad(const rt_mlp_desc* desc, const rt_mlp_params* params,
                const float* G, float* const* gW, float* const* gb, float* loss,
                void* ws, size_t ws_bytes, void* stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected with `step`
 * >= 1) on the batch G; updates W, b, the moments and Wb in place; loss as
 * in rt_mlp_grad (may be NULL). */
int rt_mlp_train_step(const rt_mlp_desc* desc, const rt_mlp_params* params,
                      const float* G, float lr, int32_t step, float* loss, void* ws,
                      size_t ws_bytes, void* stream);

/* Human-readable name of a status code (static string). */
const char* rt_status_string(int status);
/* Last error message of the calling thread (static per-thread buffer). */
const char* rt_last_error(void);
/* Library version string. */
const char* rt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RTUCKER_H */
