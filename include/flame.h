/*
 * flame.h -- C ABI of the MI355X (gfx950) blocked Cholesky library.
 *
 * Operation: A := Chol(A) for a symmetric positive definite A, in place, with
 * A = U^T U and U upper triangular with a positive diagonal.  This is the
 * blocked algorithm of Kim et al., "Task Parallel Incomplete Cholesky
 * Factorization using 2D Partitioned-Block Layout" (arXiv 1601.05871),
 * Fig. "dense-chol" (A11 := Chol(A11); A12 := triu(A11)^{-T} A12;
 * A22 := A22 - A12^T A12), and the two other loop invariants of the same
 * partitioned matrix expression (bordered, left-looking).
 *
 * Conventions for every entry point:
 *   - matrices are column-major: element (i, j) of A is A[i + j*lda];
 *   - only the upper triangle (i <= j) of a symmetric operand is read; only
 *     the upper triangle of A is written; the strictly lower triangle is never
 *     referenced (except with FLAME_OPT_LOWER, and by flame_lu and flame_qr,
 *     whose operands are general matrices, read and written whole);
 *   - pointers are DEVICE pointers unless marked "host"; the caller owns all
 *     memory it passes and the library never frees it;
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream);
 *     work is enqueued on it and the call returns without synchronizing,
 *     except where a function says otherwise;
 *   - return value: 0 = enqueued; -i = argument i (1-based) is invalid, checked
 *     on the host before anything is enqueued; > 0 = a FLAME_ERR_* code.
 *   - numerical breakdown is not a return code: it is written to the device
 *     `info` (LAPACK potrf convention): 0 = success; j > 0 = the leading j x j
 *     minor is not positive definite (the first pivot that is not > 0, or NaN,
 *     is at 1-based column j).  The upper triangle then holds partial results
 *     (unspecified); the lower triangle is still untouched.
 */
#ifndef FLAME_H
#define FLAME_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define FLAME_OK 0
#define FLAME_ERR_HIP 1           /* a HIP runtime call failed (see flame_status_string) */
#define FLAME_ERR_NOMEM 2         /* device workspace allocation failed */
#define FLAME_ERR_NOT_CONVERGED 3 /* refinement reached max_iter above tol */
#define FLAME_ERR_UNSUPPORTED 4   /* valid but unsupported combination */
#define FLAME_ERR_BREAKDOWN 5     /* flame_solve_mixed: no factorization attempt succeeded */

/* ---- enumerations ------------------------------------------------------- */
/* FLAME_Z64: complex double, each element two doubles (real part first, the
 * C99 "double complex" / std::complex<double> layout); flame_factor only. */
typedef enum { FLAME_F64 = 0, FLAME_F32 = 1, FLAME_Z64 = 2 } flame_dtype_t;

/* The three loop invariants of A = U^T U after A_TL (k x k) is processed:
 *   BORDERED (1): A_TL = U_TL;                       A_TR, A_BR untouched
 *   LEFT     (2): A_TL = U_TL, A_TR = U_TR;          A_BR untouched
 *   RIGHT    (3): A_TL = U_TL, A_TR = U_TR, A_BR = A_BR - U_TR^T U_TR
 * RIGHT is the loop the paper prints (Fig. "dense-chol").  BY_BLOCKS (4): the
 * paper's Cholesky-by-blocks (Fig. "sparse-chol" with dense 128 x 128
 * blocks), its block operations run as tasks of one persistent kernel in
 * dependence order (flame_factor_by_blocks; FP64, nb ignored).  AUTO (0)
 * lets the library choose (learned selector, else autotuner table, else
 * RIGHT). */
typedef enum {
    FLAME_VAR_AUTO = 0,
    FLAME_VAR_BORDERED = 1,
    FLAME_VAR_LEFT = 2,
    FLAME_VAR_RIGHT = 3,
    FLAME_VAR_BY_BLOCKS = 4
} flame_variant_t;

/* Arithmetic of the trailing update A22 := A22 - A12^T A12 (RIGHT variant).
 * NATIVE: the matrix dtype.  F32 / BF16 (FP64 matrices only): A12 is rounded
 * to FP32 / BF16 (round to nearest even) after its FP64 TRSM, the product is
 * formed on FP32 / BF16 matrix cores with FP32 accumulation and subtracted
 * from the FP64 A22 in FP64.  The diagonal-block factorization and the TRSM
 * stay FP64.  The result is a lower-accuracy factor meant for
 * flame_solve with refinement. */
typedef enum { FLAME_TRAIL_NATIVE = 0, FLAME_TRAIL_F32 = 1, FLAME_TRAIL_BF16 = 2 } flame_trail_t;

/* Options; a NULL pointer means all zeros (= defaults). */
typedef struct {
    int32_t variant;   /* flame_variant_t; 0 = choose */
    int32_t nb;        /* block size b (A11 is b x b, the last block min(b, n-k));
                          0 = choose (selector, else 512); valid range 1..512.
                          RIGHT with lookahead, unless flags has
                          FLAME_OPT_FIXED_NB: the last 8192 columns use
                          min(b, 256) and the last 6144 (4096 with FP32/BF16
                          trailing products) min(b, 128) */
    int32_t trail;     /* flame_trail_t */
    int32_t lookahead; /* RIGHT variant: 0 = default (2), -1 = off.
                          1: the next diagonal block and panel are updated first
                          and factored on a second stream while the rest of the
                          trailing update runs on the caller's stream.
                          2: the same split, with the rest of the trailing update
                          on the second stream and the next CHOL and TRSM on
                          the caller's stream. */
    int32_t graph;     /* 0 = default (off), 1 = capture the loop once per
                          (n, lda, A, info, options, stream) in a HIP graph and
                          replay it on later calls with the same key */
    int32_t flags;     /* bit set of FLAME_OPT_* (0 = none) */
    int32_t reserved[2]; /* must be 0 */
} flame_opts_t;

/* opts.flags: FLAME_OPT_FIXED_NB runs every block of the RIGHT loop at
 * min(nb, n - k), without the smaller blocks of the last columns.
 * FLAME_OPT_LOWER: lower storage, A = L L^T (the "lower" variant the paper's
 * conclusion lists beside the upper one): the lower triangle of A is the
 * input and receives L; the strictly upper triangle is neither used nor
 * changed (it is swapped with the lower one, in place, before and after the
 * factorization of the upper triangle, which is the same factorization of
 * the transpose).  Breakdown columns as for upper storage. */
#define FLAME_OPT_FIXED_NB 1
#define FLAME_OPT_LOWER 2

/* ---- factorization ------------------------------------------------------ */

/* A := Chol(A) (Fig. "dense-chol"), in place, upper triangle.
 *   dtype  FLAME_F64 (A is double*) or FLAME_F32 (A is float*)
 *   n      order of A, n >= 0
 *   A      device, column-major, lda x n, upper triangle read and overwritten
 *   lda    >= max(1, n)
 *   opts   host, may be NULL
 *   info   device, one int32, written asynchronously (see above)
 *   stream hipStream_t or NULL
 * Errors: -1 dtype, -2 n, -3 A (NULL with n > 0), -4 lda, -5 opts (bad field),
 * -6 info (NULL); FLAME_ERR_UNSUPPORTED for trail != NATIVE with dtype F32 or
 * with variant != RIGHT.
 *
 * dtype FLAME_Z64: A complex Hermitian positive definite, A = U^H U with U
 * upper triangular with a real positive diagonal (the loop of Fig.
 * "dense-chol" with the Hermitian update A22 - A12^H A12 it names HERK, and
 * A12 := triu(A11)^{-H} A12; the paper's data are real, complex data is one
 * of the extensions its conclusion lists).  A is element-interleaved
 * (lda counts complex elements); the imaginary parts of the diagonal are not
 * read and are written 0.  Only the right-looking loop at native precision
 * (variant AUTO or RIGHT, trail NATIVE; anything else FLAME_ERR_UNSUPPORTED);
 * opts.nb is the outer block (default 256; rounded to a multiple of 64 in
 * 64..512), opts.graph and opts.lookahead are ignored; FLAME_OPT_LOWER gives
 * A = L L^H in the lower triangle.  Breakdown: info = first column whose
 * pivot's real part is not > 0.  Device workspace of 16 n^2 bytes (two real
 * planes) plus O(nb n) is allocated on the first call and kept. */
int flame_factor(int32_t dtype, int64_t n, void *A, int64_t lda, const flame_opts_t *opts, int32_t *info,
                 void *stream);

/* LU factorization without pivoting, A = L U, in place (L unit lower
 * triangular in the strictly lower triangle, U upper triangular in the upper
 * triangle): the partitioned loop of Fig. "dense-chol" carried over to LU,
 * which the paper's conclusion names among the factorizations its pattern
 * extends to,
 *   A11 := L\U(A11);  A12 := L11^{-1} A12;  A21 := A21 U11^{-1};
 *   A22 := A22 - A21 A12,
 * right-looking at block 64.  No row interchanges: meant for matrices whose
 * LU exists without them (diagonally dominant ones, say).
 *   dtype  FLAME_F64 (FLAME_ERR_UNSUPPORTED for FLAME_F32)
 *   n, A, lda, stream as for flame_factor
 *   info   device, one int32: 0, or the 1-based column of the first pivot
 *          that is zero or not finite (A then holds a partial result)
 * Device workspace of O(64 n) doubles, allocated on the first call and kept.
 * Errors: -1 dtype, -2 n, -3 A, -4 lda, -5 info. */
int flame_lu(int32_t dtype, int64_t n, void *A, int64_t lda, int32_t *info, void *stream);

/* Householder QR factorization, A = Q R, in place, for an m x n matrix with
 * m >= n: the partitioned loop of Fig. "dense-chol" carried over to QR, which
 * the paper's conclusion names among the factorizations its pattern extends
 * to (a panel of columns is reduced by reflectors, their block form
 * I - V T V^T is applied to the columns on its right).  On exit R is in the
 * upper triangle and the reflectors' vectors below the diagonal, with the
 * reflector convention of LAPACK's geqrf: Q = H_0 H_1 ... H_{n-1},
 * H_j = I - tau_j v_j v_j^T, v_j(j) = 1 implied, v_j(0:j) = 0, and
 * R(j,j) = -sign(alpha) ||[alpha; x]|| for the column [alpha; x] it reduces
 * (tau_j = 0 and H_j = I when x = 0).  No rescaling of columns whose squared
 * norm under- or overflows.  Panels of 32 columns, outer blocks of 128.
 *   dtype  FLAME_F64 (FLAME_ERR_UNSUPPORTED for FLAME_F32)
 *   m, n   rows and columns, 0 <= n <= m; m <= 131072 (else
 *          FLAME_ERR_UNSUPPORTED: the panel's rows are spread over
 *          ceil(m / 512) workgroups that must all be resident)
 *   A, lda device, column-major, lda >= max(1, m)
 *   tau    device, n doubles (output)
 *   info   device, one int32: 0, or 1 if a wait between the panel kernel's
 *          workgroups gave up (not expected; A and tau are then invalid;
 *          the environment variable FLAME_QR_SPIN_CAP bounds those waits in
 *          sleep rounds, a negative value makes them give up at once, for
 *          tests of this path)
 *   stream as for flame_factor
 * Device workspace of about 2 KB per row and column (V in two layouts, the
 * block products) plus the split-K buffer of the trailing product, allocated
 * on the first call and kept.  Calls that overlap on one device race on it.
 * Errors: -1 dtype, -2 m, -3 n, -4 A, -5 lda, -6 tau, -7 info. */
int flame_qr(int32_t dtype, int64_t m, int64_t n, void *A, int64_t lda, void *tau, int32_t *info, void *stream);

/* Cholesky-by-blocks (Fig. "sparse-chol" of the paper, the by-blocks form of
 * the loop of Fig. "dense-chol") over 128 x 128 blocks, run as a task DAG by
 * one persistent kernel.  For iteration k the block operations are
 *   A_kk := Chol(A_kk);  A_kj := triu(A_kk)^{-T} A_kj (existing A_kj, j > k);
 *   A_ij := A_ij - A_ki^T A_kj (existing A_ki, A_kj and A_ij, k < i <= j),
 * each a task that starts once the blocks it reads are final and the block
 * it writes has received every update of earlier iterations (per-block
 * counters in device memory play the role of the paper's futures; every wait
 * is bounded).
 *   dtype   FLAME_F64 (FLAME_ERR_UNSUPPORTED for FLAME_F32)
 *   n, A, lda, info  as for flame_factor (info = -1 if a wait gave up)
 *   pattern host, nbt x nbt row-major bytes, nbt = ceil(n / 128): nonzero =
 *           block (i, j) exists (only i <= j is read; diagonal blocks always
 *           exist); NULL = dense.  Blocks that do not exist are neither read
 *           nor written, and an update whose target block does not exist is
 *           dropped: with a pattern that is not closed under fill this is the
 *           block incomplete Cholesky factorization of the pattern.
 * Errors: -1 dtype, -2 n, -3 A, -4 lda, -6 info. */
int flame_factor_by_blocks(int32_t dtype, int64_t n, void *A, int64_t lda, const uint8_t *pattern, int32_t *info,
                           void *stream);

/* The task list flame_factor_by_blocks runs for nbt x nbt blocks and a pattern
 * (as above; NULL = dense), in the order the kernel's workgroups claim it:
 * task q is tasks[4q .. 4q + 3] = (type, k, i, j) with type 0 = CHOL(A_kk),
 * 1 = TRSM(A_kj) (i = k), 2 = update of A_ij from iteration k (HERK when
 * i = j, GEMM else).  *count receives the number of tasks; tasks (host) may
 * be NULL to query it.  Errors: -1 nbt (0..4096), -4 capacity (too small),
 * -5 count. */
int flame_by_blocks_tasks(int64_t nbt, const uint8_t *pattern, int32_t *tasks, int64_t capacity, int64_t *count);

/* ---- solve and iterative refinement ----------------------------------- */

/* Refinement methods (flame_refine_t.method).  The paper uses the factor to
 * solve SPD systems, as a preconditioner; how a low-precision factor is
 * corrected is not in the paper.  All three run in FP64 on the device.
 *   IR   classical iterative refinement: x += (U^T U)^{-1} (b - A0 x); converges
 *        while kappa(A0) times the factor's working precision is well below 1.
 *   CG   conjugate gradients on A0 x = b preconditioned by M = U^T U, from the
 *        current x; when the recursive residual's eta reaches tol the true
 *        residual b - A0 x is formed, and the iteration restarts from it if its
 *        eta is still above tol.
 *   AUTO IR while eta at least halves per step, then CG from the current x. */
#define FLAME_REFINE_IR 0
#define FLAME_REFINE_CG 1
#define FLAME_REFINE_AUTO 2

typedef struct {
    const double *A0; /* device, the original FP64 matrix (upper triangle read), lda0 x n */
    int64_t lda0;     /* >= max(1, n) */
    double tol;       /* stop when eta <= tol (e.g. 1e-13) */
    int32_t max_iter; /* refinement steps allowed (IR corrections + CG iterations), >= 0 */
    int32_t method;   /* FLAME_REFINE_* */
} flame_refine_t;

typedef struct {
    int32_t iters;       /* refinement steps taken */
    int32_t method;      /* FLAME_REFINE_IR or FLAME_REFINE_CG: the method of the last step */
    double eta_max;      /* final normwise backward error, max over the columns:
                            ||b - A0 x||_inf / (||A0||_inf ||x||_inf + ||b||_inf) */
    double shift;        /* flame_solve_mixed: the shift mu of the factorization used (0 = none) */
    int32_t factor_info; /* flame_solve_mixed: info of the last factorization attempt */
    int32_t attempts;    /* flame_solve_mixed: factorizations run (1 + shifted retries) */
} flame_solve_report_t;

/* Solves A X = B with A = U^T U from flame_factor: U^T Y = B, then U X = Y.
 * The paper is silent on the solve: this is the use of the factor it names
 * (solving SPD systems), written as two triangular solves.
 *   dtype  FLAME_F64 or FLAME_F32 (U and B of that type); refinement needs F64
 *   n      order, >= 0;  nrhs  number of right-hand sides, 0 <= nrhs <= 524280
 *   U      device, the factor (upper triangle), ldu x n
 *   B      device, n x nrhs, ldb >= max(1, n); overwritten with X
 *   refine host, NULL = one plain solve.  Otherwise x = solve(U, b), then the
 *          method's steps against A0 until eta <= tol or max_iter steps.  Each
 *          step reads eta back to the host, so this call synchronizes the
 *          stream.  Returns FLAME_ERR_NOT_CONVERGED (X holds the last iterate,
 *          report the last eta) if eta > tol after max_iter steps.
 *   report host, may be NULL; filled when refine is given.
 * Errors: -1 dtype, -2 n, -3 nrhs, -4 U, -5 ldu, -6 B, -7 ldb, -8 refine;
 * FLAME_ERR_UNSUPPORTED for refinement with dtype F32. */
int flame_solve(int32_t dtype, int64_t n, int64_t nrhs, const void *U, int64_t ldu, void *B, int64_t ldb,
                const flame_refine_t *refine, flame_solve_report_t *report, void *stream);

/* Options of flame_solve_mixed. */
typedef struct {
    int32_t trail;      /* flame_trail_t of the factorization (F32 or BF16; NATIVE = FP64) */
    int32_t nb;         /* block size (0 = default) */
    int32_t method;     /* refinement method, FLAME_REFINE_* */
    int32_t max_iter;   /* refinement steps allowed */
    double tol;         /* target eta, e.g. 1e-13 */
    int32_t scale;      /* 1: factor D A0 D, D = diag(A0)^{-1/2} (unit diagonal); 0: A0 */
    int32_t max_shifts; /* retries after a breakdown, each with a larger shift (0..64) */
    double shift;       /* first shift mu added to the (scaled) diagonal; 0 = 2 u_trail */
    int32_t reserved;   /* must be 0 */
    int32_t reserved2;
} flame_mixed_opts_t;

/* Solves A0 X = B to FP64 backward error with a low-precision factor (the
 * mixed-precision use of Fig. "dense-chol"; the paper is silent on mixed
 * precision).  Steps, all on the device:
 *   1. D = diag(A0)^{-1/2} (scale = 1) or D = I;
 *   2. W := D A0 D + mu I (upper triangle; mu = 0 first), W := Chol(W) with
 *      flame_factor (RIGHT, opts.trail); on breakdown retry with mu = shift,
 *      then 4x larger each time, at most max_shifts retries (the scaling and
 *      shift of Higham & Pranesh for low-precision SPD factorizations);
 *   3. W := W D^{-1}, a factor of A0 + mu D^{-2};
 *   4. X from flame_solve with refinement against A0 (method, tol, max_iter).
 *   n, nrhs   order and right-hand sides (>= 0)
 *   A0        device, FP64, lda0 x n, upper triangle read, never written
 *   W         device, FP64, ldw x n: receives the factor (upper triangle)
 *   B         device, n x nrhs, ldb: in the right-hand sides, out X
 *   opts      host, required;  report  host, may be NULL
 * Synchronizes the stream (info and eta are read back).  Returns
 * FLAME_ERR_BREAKDOWN if A0 has a diagonal entry that is not positive or every
 * attempt broke down (report->factor_info holds the column),
 * FLAME_ERR_NOT_CONVERGED as flame_solve.
 * Errors: -1 n, -2 nrhs, -3 A0, -4 lda0, -5 W, -6 ldw, -7 B, -8 ldb, -9 opts. */
int flame_solve_mixed(int64_t n, int64_t nrhs, const double *A0, int64_t lda0, double *W, int64_t ldw, double *B,
                      int64_t ldb, const flame_mixed_opts_t *opts, flame_solve_report_t *report, void *stream);

/* ---- batched factorization ---------------------------------------------- */

/* Factors `batch` independent matrices A_i := Chol(A_i) in one persistent
 * kernel launch (replayed from a HIP graph after the first call with the same
 * arguments).  All arrays are device arrays of length `batch`:
 *   n[i]    order of A_i, 0 <= n[i] <= 1024 (larger: info[i] = -1, untouched)
 *   A[i]    device pointer to A_i (column-major), dtype as given
 *   lda[i]  >= max(1, n[i]) (else info[i] = -1)
 *   info[i] per-matrix breakdown index (as for flame_factor)
 *   opts    host, may be NULL (nb is ignored; variant must be AUTO or RIGHT)
 * A breakdown in one matrix leaves every other matrix's result unaffected.
 * Errors: -1 dtype, -2 batch (< 0), -3 n, -4 A, -5 lda, -6 info, -7 opts. */
int flame_batched_factor(int32_t dtype, int32_t batch, const int32_t *n, void *const *A, const int32_t *lda,
                         int32_t *info, const flame_opts_t *opts, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * factorization as flame_batched_factor, launched directly (no graph), with
 * its sort workspace in a fixed device array instead of library-allocated
 * memory.  It calls no hipMalloc / hipFree.  The array holds
 * FLAME_NOALLOC_MAX_BATCH + 1090 int32 (about 1 MiB) on every GPU the
 * library runs on, until the process ends; the first call on a device looks
 * its address up.  Every call on one GPU uses that GPU's array: calls that
 * overlap on one GPU (on different streams) race and must be ordered by the
 * caller.  Launches are not recorded by flame_trace_enable.
 * Errors: -1 dtype, -2 batch (< 0 or > FLAME_NOALLOC_MAX_BATCH), -3 n, -4 A,
 * -5 lda, -6 info; the arrays as for flame_batched_factor. */
#define FLAME_NOALLOC_MAX_BATCH 262144
int flame_batched_factor_noalloc(int32_t dtype, int32_t batch, const int32_t *n, void *const *A,
                                 const int32_t *lda, int32_t *info, void *stream);

/* ---- block operations of the loop body (Fig. "dense-chol") ------------- */
/* Exposed so each kernel of the loop can be checked on its own.  Same
 * conventions as above; `dtype` selects double or float operands. */

/* A := Chol(A) for one diagonal block, 0 <= n <= 256, one kernel.  Breakdown
 * writes info = info_base + j (j the 1-based local column) if *info == 0.
 * Errors: -1 dtype, -2 n, -3 A, -4 lda, -5 info. */
int flame_op_chol(int32_t dtype, int64_t n, void *A, int64_t lda, int32_t *info, int64_t info_base,
                  void *stream);

/* X := triu(U)^{-T} X: U is b x b (upper triangle read), X is b x m,
 * 0 <= b <= 256.  Errors: -1 dtype, -2 b, -3 m, -4 U, -5 ldu, -6 X, -7 ldx. */
int flame_op_trsm(int32_t dtype, int64_t b, int64_t m, const void *U, int64_t ldu, void *X, int64_t ldx,
                  void *stream);

/* C := C - X^T Y on the upper triangle (i <= j) if `upper`, else on all of C.
 * C is mr x nc, X is k x mr, Y is k x nc (columns of X and Y contiguous in k).
 * With X == Y and mr == nc this is the SYRK/HERK step.  `trail` selects the
 * product arithmetic for dtype F64 as in flame_trail_t; for F32 / BF16 the
 * operands X, Y are float / bfloat16 (uint16 storage) and C is double.
 * Errors: -1 dtype, -2 trail, -3 mr, -4 nc, -5 k, -6 X, -7 ldx, -8 Y, -9 ldy,
 * -10 C, -11 ldc. */
int flame_op_gemm_tn(int32_t dtype, int32_t trail, int32_t upper, int64_t mr, int64_t nc, int64_t k,
                     const void *X, int64_t ldx, const void *Y, int64_t ldy, void *C, int64_t ldc,
                     void *stream);

/* ---- selector and autotuner ---------------------------------------------- */

/* The selector's classes are the library's distinct ways to solve an SPD
 * system A x = b (or a batch of them, all of order n) to the accuracy of the
 * data: FP64 factorizations reach backward error <= 1e-13, the mixed classes
 * refine to it.  (The paper chooses its task granularity by hand; this is the
 * learned replacement for that choice.)
 *   class  program
 *    0     flame_factor RIGHT nb 512 (512 / 256 / 128 by position) + flame_solve
 *    1     RIGHT nb 256, FLAME_OPT_FIXED_NB            + flame_solve
 *    2     RIGHT nb 128, FLAME_OPT_FIXED_NB            + flame_solve
 *    3     RIGHT nb 64, FLAME_OPT_FIXED_NB             + flame_solve
 *    4     LEFT nb 128                                 + flame_solve
 *    5     LEFT nb 256                                 + flame_solve
 *    6     BORDERED nb 256                             + flame_solve
 *    7     flame_batched_factor (n <= 1024)            + flame_solve per matrix
 *    8     flame_solve_mixed, FP32 products, FLAME_REFINE_AUTO   (FP64 only)
 *    9     flame_solve_mixed, BF16 products, FLAME_REFINE_AUTO   (FP64 only)
 *   10     flame_solve_mixed, FP32 products, FLAME_REFINE_CG     (FP64 only)
 *   11     flame_solve_mixed, BF16 products, FLAME_REFINE_CG     (FP64 only) */
typedef struct {
    int32_t cls;       /* class number */
    int32_t variant;   /* flame_variant_t */
    int32_t nb;        /* block size (0 = the library's default schedule) */
    int32_t trail;     /* flame_trail_t: NATIVE, or the mixed solve's products */
    int32_t flags;     /* FLAME_OPT_* for flame_factor */
    int32_t method;    /* FLAME_REFINE_* of the mixed solve (classes 8..11) */
    int32_t batched;   /* 1: flame_batched_factor */
    int32_t reserved;
} flame_choice_t;

/* Loads the weights of the learned selector: a 3-layer FP32 MLP
 * in -> 64 -> 64 -> FLAME_SEL_CLASSES with ReLU, features (log2 n, log2 batch,
 * is_f64, is_f32, log10 kappa).  `w` (host) holds W1[64][5], b1[64],
 * W2[64][64], b2[64], W3[12][64], b3[12], row-major, count = FLAME_SEL_NPARAM
 * floats.  Copied to each device on first use.  w == NULL with count == 0
 * unloads the weights (VAR_AUTO then uses the autotuner's table).
 * Errors: -1 w, -2 count. */
#define FLAME_SEL_FEATURES 5
#define FLAME_SEL_HIDDEN 64
#define FLAME_SEL_CLASSES 12
#define FLAME_SEL_NPARAM (64 * 5 + 64 + 64 * 64 + 64 + 12 * 64 + 12)
int flame_selector_load(const float *w, int64_t count);

/* The program of class `cls` (host).  Errors: -1 cls, -2 choice. */
int flame_select_class(int32_t cls, flame_choice_t *choice);

/* Runs the selector's inference kernel for one shape (batch matrices of order
 * n, condition estimate kappa, 0 = unknown) and returns the highest-ranked
 * class that can run it (host).  Synchronous.  Without loaded weights returns
 * FLAME_ERR_UNSUPPORTED.  Errors: -1 n, -2 batch, -3 dtype, -4 kappa,
 * -5 choice. */
int flame_select(int64_t n, int64_t batch, int32_t dtype, double kappa, flame_choice_t *choice);

/* Batch inference: `count` feature rows (host, count x FLAME_SEL_FEATURES)
 * -> class logits (host, count x FLAME_SEL_CLASSES).  Synchronous. */
int flame_select_logits(const float *features, int64_t count, float *logits);

/* Exhaustive autotuner: times every class that can run (see above) for
 * solving A x = b, b = (1, ..., 1), with A the given n x n SPD matrix (left
 * unchanged): milliseconds per matrix, the median of `reps` runs after a
 * warm-up (the warm-up alone when it takes more than 2 s), into times_ms
 * (host, 12 doubles; +inf for a class that cannot run, breaks down or does
 * not converge).  The batched class factors min(batch, 2 GiB / matrix)
 * replicas of A in one launch; its time per matrix adds class 0's plain
 * solve.  Records the fastest of classes 0..6 in the library's tuning table
 * used by VAR_AUTO.  Synchronous.
 * Errors: -1 dtype, -2 n, -3 A, -4 lda, -5 batch (< 1), -6 reps, -7 times_ms. */
int flame_autotune(int32_t dtype, int64_t n, void *A, int64_t lda, int64_t batch, int32_t reps, double *times_ms,
                   void *stream);

/* ---- per-kernel timing (instrumentation) --------------------------------- */

/* Kernel classes of the loop body. */
#define FLAME_KC_CHOL 0  /* diagonal block, A11 := Chol(A11) */
#define FLAME_KC_TRSM 1  /* panel, A12 := triu(A11)^{-T} A12 */
#define FLAME_KC_GEMM 2  /* trailing update, C := C - X^T Y (SYRK/HERK and GEMM) */
#define FLAME_KC_OTHER 3 /* solves, residuals, casts, fills */
#define FLAME_KC_COUNT 4

/* Instrumentation, not part of the factorization.  While enabled (on != 0),
 * every kernel launch made by this library on the calling thread is
 * bracketed with HIP events on the stream it is launched on, and its
 * algorithmic work is recorded: flops (a trailing update of an M x N block
 * with inner dimension K counts 2*K per updated element) and bytes (each
 * operand element read once plus each result element written once).
 * Enabling clears previous records.  Not available inside a HIP graph
 * capture (graph replays are not recorded).  Errors: none. */
int flame_trace_enable(int32_t on);

/* Synchronizes the recorded events and sums them per kernel class: launches,
 * milliseconds (sum of per-launch event durations), flops and bytes (host
 * arrays of FLAME_KC_COUNT entries each; any may be NULL).
 * Errors: FLAME_ERR_HIP if an event query fails. */
int flame_trace_collect(int64_t *launches, double *ms, double *flops, double *bytes);

/* Busy time per kernel class: the length of the union of the recorded
 * launches' [start, end] intervals on one clock (launches of one class that
 * overlap on different streams count once), host array of FLAME_KC_COUNT;
 * span_ms (host, may be NULL): from the first record's start to the last end.
 * Synchronizes the recorded events.  Errors: FLAME_ERR_HIP if an event query
 * fails. */
int flame_trace_busy(double *busy_ms, double *span_ms);

/* ---- measurement probes ---------------------------------------------------- */

/* The device rates the roofline fractions are read against, measured with
 * plain loops on the calling device (instrumentation, not part of the
 * factorization).  kind:
 *   FLAME_PROBE_MFMA_F64   v_mfma_f64_16x16x4f64 chains, work = rounds per wavefront
 *                          (a round is 64 instructions: 16 steps of 4 chains)
 *   FLAME_PROBE_MFMA_F32   v_mfma_f32_16x16x4f32 chains, work = rounds
 *   FLAME_PROBE_MFMA_BF16  v_mfma_f32_16x16x32_bf16 chains, work = rounds
 *   FLAME_PROBE_COPY       device copy of work bytes (multiple of 16) from the
 *                          first half of buf to the second
 * wg_per_cu: workgroups of four wavefronts per compute unit in the grid
 * (1..8, 0 = 2).  buf: device scratch of buf_bytes (MFMA: >= wg_per_cu * CUs
 * * 256 floats, written; copy: >= 2 * work).  The best of `reps` timed runs
 * (after one warm-up) is returned in *rate (host): TFLOP/s for MFMA, GB/s
 * (read + write) for copy.  Synchronous.  Errors: -1 kind, -2 work,
 * -3 wg_per_cu, -4 buf, -5 buf_bytes, -6 reps, -7 rate. */
#define FLAME_PROBE_MFMA_F64 0
#define FLAME_PROBE_MFMA_F32 1
#define FLAME_PROBE_MFMA_BF16 2
#define FLAME_PROBE_COPY 3
int flame_probe(int32_t kind, int64_t work, int32_t wg_per_cu, void *buf, int64_t buf_bytes, int32_t reps,
                double *rate, void *stream);

/* ---- teardown -------------------------------------------------------------- */

/* Waits for every device the library has used, then releases its state there:
 * cached HIP graphs, streams, events and workspaces.  Call it before the HIP
 * runtime is torn down (the Python binding registers it with atexit).  Later
 * calls re-create the state on demand.  Returns FLAME_ERR_HIP if a device
 * could not be synchronized (the state is released anyway). */
int flame_shutdown(void);

/* ---- level(k) incomplete Cholesky by blocks ----------------------------------
 * The paper's own method (Sec. "Symbolic factorization", Alg. symb_fact;
 * Sec. "2D sparse partitioned-block matrix"; the numeric Cholesky-by-blocks
 * of Fig. "sparse-chol"): A ~= U^T U for a sparse SPD A, U restricted to the
 * level-k fill pattern (the entries of A have level 0; eliminating a pivot
 * gives (i, j) the level lev(k,i) + lev(k,j) + 1; entries above level k are
 * dropped).
 *
 * flame_ichol_analyze (host only, no device call): the symbolic phase.  The
 * plan's device memory (block pool, masks, task list, entry maps) is
 * allocated on the device current at its first flame_ichol_factor /
 * flame_ichol_values, which binds the plan to that device.
 *   n          order of A.
 *   rp, ci     host CSR of A's pattern: rp[n + 1] (int64), ci[rp[n]] (int32);
 *              both triangles or one, any column order, no duplicate
 *              entries; the same arrays (and value order) are the input of
 *              flame_ichol_factor.
 *   level      k >= 0 (a large k gives the complete factor of the ordered A).
 *   order      host int64[n], order[new] = old index, or NULL: the library's
 *              nested dissection (breadth-first level-structure bisection,
 *              leaves of at most `leaf` vertices).
 *   bounds     host int64[nranges + 1] (0 = bounds[0] < ... = n): the ranges
 *              of the 2D block layout in the new numbering; NULL with an
 *              `order`: ranges of 128.  Ranges longer than 128 are cut.
 *   leaf       leaf size of the dissection (0 = 128).
 *   plan       receives the plan (free it with flame_ichol_destroy).
 * Returns 0, -i for an invalid argument (an `order` that is not a
 * permutation: -5; bounds that do not tile [0, n): -6), FLAME_ERR_UNSUPPORTED
 * beyond 4096 blocks per side, FLAME_ERR_NOMEM. */
typedef struct flame_ichol_plan_s *flame_ichol_plan;
int flame_ichol_analyze(int64_t n, const int64_t *rp, const int32_t *ci, int32_t level, const int64_t *order,
                        const int64_t *bounds, int64_t nranges, int32_t leaf, flame_ichol_plan *plan);

/* Sizes of a plan (host): nnz_u = entries of U's pattern, nbt = blocks per
 * side, nblocks = existing blocks (upper), ntasks = tasks of the DAG,
 * pool_bytes = device bytes of the block pool, flops = the factorization's
 * floating-point operations (a multiply and a subtraction per update whose
 * target is in the pattern, the row scalings and square roots). */
typedef struct {
    int64_t n, nnz_a, nnz_u, nbt, nblocks, ntasks, pool_bytes;
    double flops;
} flame_ichol_stats_t;
int flame_ichol_stats(flame_ichol_plan plan, flame_ichol_stats_t *stats);

/* Copies the plan's structure to host arrays (each may be NULL): order[n],
 * bounds[nbt + 1], U's pattern in the new numbering urp[n + 1] / uci[nnz_u]
 * (rows, columns increasing, the diagonal first), the block pattern
 * pattern[nbt * nbt] (row-major, upper), the task list tasks[4 * ntasks]
 * (type 0 CHOL / 1 TRSM / 2 HERK-GEMM, k, i, j per task, in claim order). */
int flame_ichol_structure(flame_ichol_plan plan, int64_t *order, int64_t *bounds, int64_t *urp, int32_t *uci,
                          uint8_t *pattern, int32_t *tasks);

/* The numeric phase on `stream`: A's values vals[rp[n]] (device, float64, in
 * the order of the ci given to flame_ichol_analyze; only the entries with
 * new row <= new column are read) are scattered into the plan's block pool
 * and the task DAG runs there (one persistent launch; CHOL and TRSM of a
 * block drop fill outside the pattern as each row of U becomes final).
 * info (device int32): 0, the 1-based new-numbering column of the first
 * pivot that is not > 0, or -1 if a wait gave up.  The plan holds U until the
 * next call; calls on one plan must not overlap.  FLAME_ERR_UNSUPPORTED if
 * the current device is not the plan's. */
int flame_ichol_factor(flame_ichol_plan plan, const double *vals, int32_t *info, void *stream);
/* (FLAME_ERR_NOMEM if the plan's first upload fails.) */

/* U's values on its pattern (device uvals[nnz_u], the order of
 * flame_ichol_structure's urp / uci), from the last flame_ichol_factor. */
int flame_ichol_values(flame_ichol_plan plan, double *uvals, void *stream);

/* z := M^{-1} r with M = P^T U^T U P, the incomplete factor of the last
 * flame_ichol_factor (P the plan's ordering): device vectors of n doubles in
 * the original numbering (r and z may not overlap).  One forward and one
 * backward block-triangular solve, each a single launch over the blocks. */
int flame_ichol_apply(flame_ichol_plan plan, const double *r, double *z, void *stream);

/* Preconditioned conjugate gradients for A x = b with M (the paper's use of
 * the incomplete factor, Sec. "Introduction": a preconditioner for SPD
 * systems).  vals: A's values (device, the order of the analysed ci); the
 * analysed pattern must hold both triangles (else FLAME_ERR_UNSUPPORTED:
 * the product uses every stored entry).  b, x: device n-vectors, x the
 * starting guess on entry, the solution on exit.  Stops when
 * ||b - A x||_2 <= tol ||b||_2 (recursive residual) or after max_iter
 * iterations (report->status = FLAME_ERR_NOT_CONVERGED, the return value
 * stays 0).  Call flame_ichol_factor on the same values first.
 * Synchronizes `stream` once per iteration. */
typedef struct {
    double tol;          /* > 0; default 1e-10 when opts is NULL */
    int32_t max_iter;    /* >= 0; default 1000 */
    int32_t reserved[2]; /* must be 0 */
} flame_pcg_opts_t;
typedef struct {
    int32_t iters;  /* iterations taken */
    int32_t status; /* FLAME_OK or FLAME_ERR_NOT_CONVERGED */
    double relres;  /* ||r||_2 / ||b||_2 at exit */
    double bnorm;   /* ||b||_2 */
} flame_pcg_report_t;
int flame_ichol_pcg(flame_ichol_plan plan, const double *vals, const double *b, double *x, const flame_pcg_opts_t *opts,
                    flame_pcg_report_t *report, void *stream);

/* Frees a plan (synchronizes nothing: no call on it may be in flight). */
int flame_ichol_destroy(flame_ichol_plan plan);

/* ---- status -------------------------------------------------------------- */
const char *flame_status_string(int status);
const char *flame_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FLAME_H */
