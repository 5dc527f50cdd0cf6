// Internal declarations shared by the kernels, the loop drivers and the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>

#include "flame.h"

namespace flame {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Result of a HIP call inside the library; the last failing code is kept for
// flame_status_string.
void set_last_hip_error(hipError_t e);
hipError_t last_hip_error();

#define FLAME_HIP(call)                                  \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) {                          \
            ::flame::set_last_hip_error(e_);             \
            return FLAME_ERR_HIP;                        \
        }                                                \
    } while (0)

#define FLAME_CHECK_LAUNCH()                                 \
    do {                                                     \
        hipError_t e_ = hipGetLastError();                   \
        if (e_ != hipSuccess) {                              \
            ::flame::set_last_hip_error(e_);                 \
            return FLAME_ERR_HIP;                            \
        }                                                    \
    } while (0)

// Instrumentation: trace_begin returns a record id (or -1 when tracing is
// off or the stream is capturing); trace_end closes it with the launch's
// algorithmic flops and bytes.
int trace_begin(int kclass, hipStream_t s);
void trace_end(int id, hipStream_t s, double flops, double bytes);

// ---- kernel launchers (each returns 0 or a FLAME_ERR_* code) --------------

// info[0] := 0 (a fill kernel, so that the loop can be captured in a graph).
int launch_zero_i32(int32_t *p, int64_t count, hipStream_t s);
// Swaps the strict lower and upper triangles of A in place (lower storage).
template <typename T>
int launch_swap_triangles(int64_t n, T *A, int64_t lda, hipStream_t s);

// Diagonal block A := Chol(A), n <= 256, one workgroup.  Skips all work if
// *info != 0 on entry; on breakdown at local column j writes
// info = info_base + j.
template <typename T>
int launch_chol_block(int n, T *A, int64_t lda, int32_t *info, int64_t info_base, hipStream_t s);

// X := triu(U)^{-T} X, U b x b (b <= 256), X b x m.  Skips if info && *info.
template <typename T>
int launch_trsm_panel(int b, int64_t m, const T *U, int64_t ldu, T *X, int64_t ldx, const int32_t *info,
                      hipStream_t s);

// Operand precisions of the trailing product.
enum class Prec { F64, F32, BF16 };

// C := C - X^T Y (upper: only i <= j written), X k x M, Y k x N, C M x N.
//   F64:  X, Y, C double
//   F32:  X, Y float;  C float (cfloat) or double (!cfloat)
//   BF16: X, Y bf16 (uint16 storage); C double
// Skips if info && *info.
// reserve_cus > 0: leave that many compute units free of this launch (for
// kernels running concurrently on another stream).
int launch_gemm_tn(Prec p, bool c_is_double, bool upper, int64_t M, int64_t N, int64_t K, const void *X,
                   int64_t ldx, const void *Y, int64_t ldy, void *C, int64_t ldc, const int32_t *info,
                   hipStream_t s, int reserve_cus = 0);

// Y (rows x cols, ldy) := round(X) to float / bf16, column by column.
// C -= X^T Y with the K range split over slices that run as one launch,
// each writing its partial product to W, then added to C in slice order
// (deterministic).  Falls back to launch_gemm_tn when a split does not pay
// or the operands are not 16-byte aligned.  W: splitk_workspace_bytes().
template <typename CT>
int launch_gemm_splitk(bool upper, int64_t M, int64_t N, int64_t K, const CT *X, int64_t ldx, const CT *Y,
                       int64_t ldy, CT *C, int64_t ldc, CT *W, const int32_t *info, hipStream_t s);
size_t splitk_workspace_bytes();
int launch_round_panel(Prec p, int64_t rows, int64_t cols, const double *X, int64_t ldx, void *Y, int64_t ldy,
                       const int32_t *info, hipStream_t s);

// ---- solve and residual kernels -------------------------------------------
// Dt_q = U_qq^{-T} for the diagonal blocks of order bs (<= 128); Dt must hold
// identity blocks on entry (see launch_identity_blocks).
int launch_diag_inverse_t(int64_t n, int bs, const double *U, int64_t ldu, double *Dt, hipStream_t s);
int launch_identity_blocks(int64_t nblk, int bs, double *Dt, hipStream_t s);
// One right-hand side: U^T y = b (fwd) and U x = y (bwd) in place on x, one
// persistent launch each, using the block inverses Dt; flags: nblk ints
// (cleared here), err: one int set to 1 if a wait gave up.
int launch_trsv1(bool forward, int64_t n, const double *U, int64_t ldu, const double *Dt, double *x, int32_t *flags,
                 int32_t *err, hipStream_t s);
// Residual R = B - A0 X (A0 symmetric from its upper triangle; B == nullptr:
// the product R = A0 X), nrhs <= 8,
// through per-tile partial sums (deterministic); also rowsums of |A0| when
// rowsums != nullptr.  part: workspace of tiles^2 * 128 * (nrhs + 1) doubles.
int launch_residual_tiled(int64_t n, int64_t nrhs, const double *A0, int64_t lda0, const double *X, int64_t ldx,
                          const double *B, int64_t ldb, double *R, int64_t ldr, double *rowsums, double *part,
                          hipStream_t s);
size_t residual_workspace_doubles(int64_t n, int64_t nrhs);
// Many right-hand sides, FP64, one persistent launch per direction
// (k_trsm_chain.hip): forward U^T Y = B or backward U X = Y in place on X,
// with the block inverses Dt; column chunks side by side.  flags:
// trsm_chain_flags(n, nrhs) ints (cleared here), err: one int set to 1 if a
// wait gave up (the results are then NaN).
int trsm_chain_flags(int64_t n, int64_t nrhs);
int launch_trsm_chain(bool forward, int64_t n, int64_t nrhs, const double *U, int64_t ldu, const double *Dt,
                      double *X, int64_t ldx, int32_t *flags, int32_t *err, hipStream_t s);
template <typename T>
int launch_trsv_fwd(int64_t n, int64_t nrhs, const T *U, int64_t ldu, T *B, int64_t ldb, hipStream_t s);
template <typename T>
int launch_trsv_bwd(int64_t n, int64_t nrhs, const T *U, int64_t ldu, T *B, int64_t ldb, hipStream_t s);

// R := B - A0 X with A0 symmetric from its upper triangle (FP64); with
// want_rowsums also rowsums[i] = sum_j |A0(i, j)| (for ||A0||_inf).
int launch_residual(int64_t n, int64_t nrhs, const double *A0, int64_t lda0, const double *X, int64_t ldx,
                    const double *B, int64_t ldb, double *R, int64_t ldr, double *rowsums, bool want_rowsums,
                    hipStream_t s);
// R := beta B + alpha A0 X (A0 symmetric from its upper triangle; B may be
// nullptr when beta is unused), any nrhs, with |A0| row sums when rowsums !=
// nullptr.  Deterministic.
int launch_symm(int64_t n, int64_t nrhs, double alpha, const double *A0, int64_t lda0, const double *X, int64_t ldx,
                double beta, const double *B, int64_t ldb, double *R, int64_t ldr, double *rowsums, hipStream_t s);
// out[c] = X(:, c) . Y(:, c), deterministic.
int launch_dot_cols(int64_t n, int64_t nrhs, const double *X, int64_t ldx, const double *Y, int64_t ldy, double *out,
                    hipStream_t s);
// Conjugate-gradient updates per column: P := Z + (rho / rho_old) P (P := Z
// when first); X += alpha P, R -= alpha Q with alpha = rho / pq.
int launch_cg_direction(int64_t n, int64_t nrhs, const double *Z, int64_t ldz, double *P, int64_t ldp,
                        const double *rho, const double *rho_old, bool first, hipStream_t s);
int launch_cg_step(int64_t n, int64_t nrhs, double *X, int64_t ldx, double *R, int64_t ldr, const double *P,
                   int64_t ldp, const double *Q, int64_t ldq, const double *rho, const double *pq, hipStream_t s);
// Diagonal scaling: d = 1 / sqrt(diag(A0)), *bad = first 1-based column whose
// diagonal is not > 0 (0x7fffffff if none); W := D A0 D + mu I (upper; d ==
// nullptr: no scaling); U := U D^{-1} (columns).
int launch_diag_scale(int64_t n, const double *A0, int64_t lda0, double *d, int32_t *bad, hipStream_t s);
int launch_scale_copy_upper(int64_t n, const double *A0, int64_t lda0, double *W, int64_t ldw, const double *d,
                            double mu, hipStream_t s);
int launch_unscale_cols(int64_t n, double *U, int64_t ldu, const double *d, hipStream_t s);
int launch_axpy_cols(int64_t n, int64_t nrhs, const double *D, int64_t ldd, double *X, int64_t ldx,
                     hipStream_t s);
int launch_copy_cols(int64_t n, int64_t nrhs, const double *S, int64_t lds, double *D, int64_t ldd,
                     hipStream_t s);
// eta[c] = ||r_c||_inf / (||A0||_inf ||x_c||_inf + ||b_c||_inf), eta[nrhs] = max.
int launch_eta_full(int64_t n, int64_t nrhs, const double *R, int64_t ldr, const double *X, int64_t ldx,
                    const double *B, int64_t ldb, const double *rowsums, double *eta, hipStream_t s);

// ---- batched -------------------------------------------------------------
// ws: batched_workspace_ints(batch) ints (order, counter, histogram), cleared
// here by a fill kernel.  traced: record the launch when tracing is on.
template <typename T>
int launch_batched(int32_t batch, const int32_t *n, void *const *A, const int32_t *lda, int32_t *info, int32_t *ws,
                   hipStream_t s, bool traced = true);
size_t batched_workspace_ints(int32_t batch);

// ---- complex Hermitian factorization (k_complex.hip, zfactor.cpp) ---------
// One complex double: two doubles, real part first (the interleaved layout).
struct zdouble {
    double re, im;
    zdouble() = default;
    __host__ __device__ constexpr zdouble(double v) : re(v), im(0.0) {}
};
// Real and imaginary planes (column-major, ld) := upper triangle of the
// interleaved complex A, and back (the diagonal's imaginary part written 0).
int launch_z_split(int64_t n, const void *A, int64_t lda, double *R, double *I, int64_t ld, hipStream_t s);
int launch_z_merge(int64_t n, const double *R, const double *I, int64_t ld, void *A, int64_t lda, hipStream_t s);
// dst := scale * src (skipped if info && *info) and dst := 0 (rows x cols,
// real).
int launch_scaled_copy(int64_t rows, int64_t cols, const double *src, int64_t lds, double *dst, int64_t ldd,
                       double scale, const int32_t *info, hipStream_t s);
int launch_fill0(int64_t rows, int64_t cols, double *dst, int64_t ldd, hipStream_t s);
// Complex diagonal block (n <= 64, planes): A := Chol(A) (on breakdown
// *info = info_base + column) and V := -U^{-1} (planes Vr, Vi, ldv >= n), in
// one launch.  Skips if *info.
int launch_zchol_lds(int n, double *R, double *I, int64_t ld, int32_t *info, int64_t info_base, double *Vr,
                     double *Vi, int64_t ldv, hipStream_t s);
// C -= P^H Q on planes in one matrix-core pass (P K x M, Q K x N, C M x N;
// upper: i <= j only).  Skips if *info.
int launch_zgemm_h(bool upper, int64_t M, int64_t N, int64_t K, const double *Pr, const double *Pi, int64_t ldp,
                   const double *Qr, const double *Qi, int64_t ldq, double *Cr, double *Ci, int64_t ldc,
                   const int32_t *info, hipStream_t s);
// X := -P^H X in place (M <= 64 rows; P is K x M, planes), one row of
// workgroup tiles.
int launch_zgemm_h_inplace(int64_t M, int64_t N, int64_t K, const double *Pr, const double *Pi, int64_t ldp,
                           double *Xr, double *Xi, int64_t ldx, const int32_t *info, hipStream_t s);
// The complex factorization of flame_factor (dtype FLAME_Z64), upper storage.
int zfactor(int64_t n, void *A, int64_t lda, int nb, int32_t *info, hipStream_t s);

// ---- LU without pivoting (k_lu.hip, lu.cpp) ---------------------------------
// Diagonal block (n <= 64) := L\U in place (on a zero or non-finite pivot
// *info = info_base + column) and, unless P1 and P2 are null, P1 :=
// -(L^{-1})^T, P2 := -U^{-1} (n x n, ld 64), in one launch.  dst (cols x rows)
// := src^T, and z1, z2 (null or shaped as dst) := 0.  Both skip if *info (the
// transpose only when info is given).
int launch_lu_diag(int n, double *A, int64_t lda, int32_t *info, int64_t info_base, double *P1, double *P2,
                   hipStream_t s);
int launch_transpose_copy(int64_t rows, int64_t cols, const double *src, int64_t lds, double *dst, int64_t ldd,
                          const int32_t *info, hipStream_t s, double *z1 = nullptr, double *z2 = nullptr);
int lu_factor(int64_t n, double *A, int64_t lda, int32_t *info, hipStream_t s);

// ---- Householder QR (k_qr.hip, qr.cpp) -----------------------------------
// A = Q R in place (m >= n): R in the upper triangle, the reflectors below
// the diagonal, tau (n, device); *info := 0, or 1 if a device-side wait of
// the panel kernel gave up.
int qr_factor(int64_t m, int64_t n, double *A, int64_t lda, double *tau, int32_t *info, hipStream_t s);

// ---- selector --------------------------------------------------------------
int launch_selector(const float *w, const float *feat, int64_t count, float *logits, hipStream_t s);

// ---- per-device context: side stream, events, workspace, graph cache ------
struct DevCtx;
DevCtx *ctx_for_current_device();
// Workspace slot `slot` (factor panel, solve, batched, selector) of
// at least `bytes` (grown under a lock, kept until the process ends).
enum {
    kWsFactor = 0,
    kWsSolve = 1,
    kWsBatched = 2,
    kWsSelector = 3,
    kWsTune = 4,
    kWsSplit = 5,
    kWsMixed = 6,
    kWsDag = 7,
    kWsComplex = 8,
    kWsLu = 9,
    kWsQr = 10,
    kWsQrSplit = 11,
    kWsSlots = 12
};
int ctx_workspace(DevCtx *c, int slot, size_t bytes, void **out);
// Generation of a slot's buffer: changes every time ctx_workspace replaces it
// (a graph that captured the old pointer must not be replayed).
uint64_t ctx_workspace_gen(DevCtx *c, int slot);
// Teardown helpers of flame_shutdown: each drops its module's device state.
void drop_factor_graphs();
void drop_batched_graphs();
void drop_dag_lists();
// Cholesky-by-blocks on the device task DAG (by_blocks.cpp), FP64; pattern:
// host nbt x nbt block mask or nullptr (dense).
int by_blocks_factor(int64_t n, double *A, int64_t lda, const uint8_t *pattern, int32_t *info, hipStream_t s);
void selector_forget_devices();
hipStream_t ctx_side_stream(DevCtx *c);
hipStream_t ctx_aux_stream(DevCtx *c);
// Variant, block size and flags for FLAME_VAR_AUTO (o->nb kept when set): the
// single-matrix factorization the learned selector ranks highest when its
// weights are loaded, else the autotuner's table, else RIGHT with nb 512.
void choose_variant(int32_t dtype, int64_t n, int64_t batch, flame_opts_t *o);
hipEvent_t ctx_event(DevCtx *c, int i);

// Loop drivers (driver.cpp).
int factor_dispatch(int32_t dtype, int64_t n, void *A, int64_t lda, const flame_opts_t &o, int32_t *info,
                    hipStream_t s);

}  // namespace flame
