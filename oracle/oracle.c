/*
 * oracle.c -- plain, slow, FP64 CPU oracle for the dense Cholesky of
 * Kim, Rajamanickam, Stelle, Edwards, Olivier, "Task Parallel Incomplete
 * Cholesky Factorization using 2D Partitioned-Block Layout" (arXiv 1601.05871).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library links, loads or calls this
 * file; only the tests, the smoke check and the benchmark's CPU-baseline leg
 * do.  It shares no code, header or constant with the GPU path.
 *
 * Conventions (all functions):
 *   - column-major storage, element (i, j) at A[i + j*lda];
 *   - only the upper triangle (i <= j) of a symmetric operand is read, and
 *     only the upper triangle of the factor is written; the strictly lower
 *     triangle is never touched;
 *   - IEEE binary64, round to nearest even, no contraction (the build uses
 *     -ffp-contract=off -fno-fast-math); sqrt is the correctly rounded libm
 *     sqrt;
 *   - the operation is A := Chol(A) with A = U^T U and U upper triangular with
 *     a positive diagonal (Fig. "dense-chol" and its caption: the update
 *     A22 - A12^T A12 and triu() fix the upper-triangular form).
 *
 * Every update below applies the rank-1 terms of the Schur complement one at a
 * time, in increasing pivot order, each product rounded and then subtracted.
 * With that choice the blocked variants perform, element by element, exactly
 * the same sequence of floating-point operations as the unblocked loop, so they
 * agree with it bit for bit at every block size (the paper notes the blocked
 * algorithm works equally for scalar entries, b = 1: blocking only regroups
 * the same arithmetic).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define AT(A, lda, i, j) ((A)[(int64_t)(i) + (int64_t)(j) * (int64_t)(lda)])

/* nthreads <= 0: the OpenMP default (all cores); otherwise that many threads. */
static int pick_threads(int nthreads) {
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * O1: unblocked right-looking Cholesky, the loop of Fig. "dense-chol" with
 * block size b = 1 (Sec. "Numeric factorization: Cholesky-by-blocks").
 * Runs the first `jstop` pivot steps (jstop >= n: the whole factorization).
 * After s steps, rows 0..s-1 of the upper triangle hold the final rows of U
 * and the trailing upper triangle holds the Schur complement.
 *
 * Step j, with alpha11 = A(j,j), a12 = A(j, j+1:n), A22 = A(j+1:n, j+1:n):
 *   alpha11 := sqrt(alpha11)                       CHOL of a 1x1 block
 *   a12     := a12 / alpha11                       TRSM (triu(alpha11)^{-T} a12)
 *   A22     := A22 - a12^T a12   (upper part)      HERK (real: SYRK)
 * Breakdown (the paper is silent): the first pivot that is not > 0 (this also
 * catches NaN) stops the loop and returns its 1-based column index.
 * Returns 0 on success.
 */
int oracle_potrf_upper_steps(int64_t n, double *A, int64_t lda, int64_t jstop, int nthreads) {
    int nt = pick_threads(nthreads);
    (void)nt;
    if (jstop > n) jstop = n;
    double *row = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!row) return -1;
    for (int64_t j = 0; j < jstop; ++j) {
        double a = AT(A, lda, j, j);
        if (!(a > 0.0)) {
            free(row);
            return (int)(j + 1);
        }
        double d = sqrt(a);
        AT(A, lda, j, j) = d;
        /* a12 := a12 / alpha11, and keep a copy of row j of U */
        for (int64_t c = j + 1; c < n; ++c) {
            AT(A, lda, j, c) = AT(A, lda, j, c) / d;
            row[c] = AT(A, lda, j, c);
        }
        /* A22(i, c) -= U(j, i) * U(j, c) for j < i <= c (upper triangle) */
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt)
        for (int64_t c = j + 1; c < n; ++c) {
            double ujc = row[c];
            double *col = &AT(A, lda, 0, c);
            for (int64_t i = j + 1; i <= c; ++i) {
                double p = row[i] * ujc;
                col[i] = col[i] - p;
            }
        }
    }
    free(row);
    return 0;
}

int oracle_potrf_upper(int64_t n, double *A, int64_t lda, int nthreads) {
    return oracle_potrf_upper_steps(n, A, lda, n, nthreads);
}

/*
 * X := triu(U)^{-T} X, U is b x b upper triangular, X is b x m.
 * This is the TRSM of Fig. "dense-chol", A12 := triu(A11)^{-T} A12 (the figure
 * prints ^{-1}; only the transposed solve satisfies A = U^T U, see the
 * readings list).  Solves U^T X_new = X_old by forward substitution, row by
 * row: x_s := x_s / U(s,s); then x_r -= U(s,r) * x_s for r > s.
 */
void oracle_trsm_upper_t(int64_t b, int64_t m, const double *U, int64_t ldu, double *X, int64_t ldx) {
    for (int64_t c = 0; c < m; ++c) {
        double *x = &AT(X, ldx, 0, c);
        for (int64_t s = 0; s < b; ++s) {
            x[s] = x[s] / AT(U, ldu, s, s);
            for (int64_t r = s + 1; r < b; ++r) {
                double p = AT(U, ldu, s, r) * x[s];
                x[r] = x[r] - p;
            }
        }
    }
}

/*
 * C := C - P^T P on the upper triangle of the m x m matrix C; P is k x m.
 * The HERK of Fig. "dense-chol" (real arithmetic: SYRK); off-diagonal blocks
 * of the by-blocks form are the same formula (GEMM).  The k rank-1 terms are
 * subtracted one by one in increasing row order of P.
 */
void oracle_syrk_upper(int64_t m, int64_t k, const double *P, int64_t ldp, double *C, int64_t ldc) {
    for (int64_t j = 0; j < m; ++j)
        for (int64_t i = 0; i <= j; ++i) {
            double acc = AT(C, ldc, i, j);
            for (int64_t r = 0; r < k; ++r) {
                double p = AT(P, ldp, r, i) * AT(P, ldp, r, j);
                acc = acc - p;
            }
            AT(C, ldc, i, j) = acc;
        }
}

/*
 * C := C - X^T Y, C is mr x nc (full), X is k x mr, Y is k x nc.
 * Terms subtracted one by one in increasing row order of X and Y.
 */
void oracle_gemm_tn(int64_t mr, int64_t nc, int64_t k, const double *X, int64_t ldx, const double *Y,
                    int64_t ldy, double *C, int64_t ldc) {
    for (int64_t j = 0; j < nc; ++j)
        for (int64_t i = 0; i < mr; ++i) {
            double acc = AT(C, ldc, i, j);
            for (int64_t r = 0; r < k; ++r) {
                double p = AT(X, ldx, r, i) * AT(Y, ldy, r, j);
                acc = acc - p;
            }
            AT(C, ldc, i, j) = acc;
        }
}

/*
 * O2: the blocked loop of Fig. "dense-chol" in FLAME partition/repartition
 * form, for the three loop invariants of A = U^T U.  At iteration start A_TL is
 * k x k; A11 is bk x bk with bk = min(b, n - k) (the "Determine block size b"
 * step; the last block takes what is left).  With m = n - k - bk:
 *
 *   A00 = A(0:k, 0:k)      A01 = A(0:k, k:k+bk)      A02 = A(0:k, k+bk:n)
 *                          A11 = A(k:k+bk, k:k+bk)   A12 = A(k:k+bk, k+bk:n)
 *                                                    A22 = A(k+bk:n, k+bk:n)
 *
 * variant 3 (right-looking, the one the paper prints):
 *   A11 := Chol(A11);  A12 := triu(A11)^{-T} A12;  A22 := A22 - A12^T A12
 * variant 2 (left-looking):
 *   A11 := A11 - A01^T A01;  A11 := Chol(A11);
 *   A12 := A12 - A01^T A02;  A12 := triu(A11)^{-T} A12
 * variant 1 (bordered):
 *   A01 := triu(A00)^{-T} A01;  A11 := A11 - A01^T A01;  A11 := Chol(A11)
 *
 * `iters` < 0 runs to completion; otherwise the loop stops after that many
 * iterations so a test can inspect the loop invariant.  Returns the LAPACK-style
 * breakdown index (k + local index) or 0.
 */
int oracle_potrf_blocked(int64_t n, double *A, int64_t lda, int64_t b, int variant, int64_t iters) {
    if (b <= 0) return -4;
    int64_t it = 0;
    for (int64_t k = 0; k < n; k += b) {
        if (iters >= 0 && it >= iters) break;
        ++it;
        int64_t bk = (n - k < b) ? (n - k) : b;
        int64_t m = n - k - bk;
        double *A01 = &AT(A, lda, 0, k);
        double *A02 = &AT(A, lda, 0, k + bk);
        double *A11 = &AT(A, lda, k, k);
        double *A12 = &AT(A, lda, k, k + bk);
        double *A22 = &AT(A, lda, k + bk, k + bk);
        const double *A00 = &AT(A, lda, 0, 0);
        int info;
        if (variant == 3) {
            info = oracle_potrf_upper(bk, A11, lda, 1);
            if (info) return (int)(k + info);
            oracle_trsm_upper_t(bk, m, A11, lda, A12, lda);
            oracle_syrk_upper(m, bk, A12, lda, A22, lda);
        } else if (variant == 2) {
            oracle_syrk_upper(bk, k, A01, lda, A11, lda);
            info = oracle_potrf_upper(bk, A11, lda, 1);
            if (info) return (int)(k + info);
            oracle_gemm_tn(bk, m, k, A01, lda, A02, lda, A12, lda);
            oracle_trsm_upper_t(bk, m, A11, lda, A12, lda);
        } else if (variant == 1) {
            oracle_trsm_upper_t(k, bk, A00, lda, A01, lda);
            oracle_syrk_upper(bk, k, A01, lda, A11, lda);
            info = oracle_potrf_upper(bk, A11, lda, 1);
            if (info) return (int)(k + info);
        } else {
            return -5;
        }
    }
    return 0;
}

/*
 * O3: solve A X = B with A = U^T U, in place on B (n x nrhs): forward
 * substitution U^T Y = B, then back substitution U X = Y, column by column.
 * Terms are subtracted one by one in increasing (forward) or decreasing (back)
 * index order.  The paper does not state a solve; it is the use of the factor
 * (preconditioned iterative methods for SPD systems, Sec. "Introduction").
 */
void oracle_solve_upper(int64_t n, int64_t nrhs, const double *U, int64_t ldu, double *B, int64_t ldb) {
    for (int64_t c = 0; c < nrhs; ++c) {
        double *x = &AT(B, ldb, 0, c);
        /* U^T y = b: y_r = (b_r - sum_{s<r} U(s,r) y_s) / U(r,r) */
        for (int64_t r = 0; r < n; ++r) {
            double acc = x[r];
            for (int64_t s = 0; s < r; ++s) {
                double p = AT(U, ldu, s, r) * x[s];
                acc = acc - p;
            }
            x[r] = acc / AT(U, ldu, r, r);
        }
        /* U x = y: x_r = (y_r - sum_{s>r} U(r,s) x_s) / U(r,r) */
        for (int64_t r = n - 1; r >= 0; --r) {
            double acc = x[r];
            for (int64_t s = n - 1; s > r; --s) {
                double p = AT(U, ldu, r, s) * x[s];
                acc = acc - p;
            }
            x[r] = acc / AT(U, ldu, r, r);
        }
    }
}

/*
 * O6: level(k) fill pattern of the upper factor (Sec. "Symbolic
 * factorization"; the level of an entry is set during elimination: the
 * entries of A have level 0, and eliminating k gives entry (i, j), k < i <= j,
 * the level lev(k,i) + lev(k,j) + 1 when that is lower; entries whose level
 * would exceed K are not created and take no part in later eliminations).
 *
 * Input: the upper pattern of the (already reordered) symmetric matrix as
 * rows: arp[n + 1], aci (row i holds its columns j >= i, any order; the
 * diagonal is added if missing).  Row i of U receives contributions only from
 * the rows k < i that hold column i, and those are final when row i is
 * formed, so rows are formed in increasing order: a dense work row holds the
 * levels of row i, and column lists record, for each column j, the rows k < j
 * holding it (with the position of (k, j) in row k).
 * Output: rp[n + 1], ci and lev (row i: columns increasing, the diagonal
 * first, with their levels), written when the entry count fits `cap`;
 * returns the entry count (call again with a larger cap when it exceeds
 * cap), -1 on allocation failure.
 */
typedef struct {
    int64_t k, pos;
} kpos_t;

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

int64_t oracle_fill_pattern(int64_t n, const int64_t *arp, const int32_t *aci, int32_t K, int64_t *rp, int32_t *ci,
                            int32_t *lev, int64_t cap) {
    const int32_t INF = 0x7fffffff;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t *w = (int32_t *)malloc(sizeof(int32_t) * nn);
    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * nn);
    int64_t *urp = (int64_t *)malloc(sizeof(int64_t) * (nn + 1));
    int64_t ucap = 8 * (int64_t)nn, ucount = 0;
    int32_t *uci = (int32_t *)malloc(sizeof(int32_t) * (size_t)ucap);
    int32_t *ulev = (int32_t *)malloc(sizeof(int32_t) * (size_t)ucap);
    kpos_t **col = (kpos_t **)calloc(nn, sizeof(kpos_t *));
    int64_t *ccnt = (int64_t *)calloc(nn, sizeof(int64_t));
    int64_t *ccap = (int64_t *)calloc(nn, sizeof(int64_t));
    int64_t result = -1;
    if (!w || !touched || !urp || !uci || !ulev || !col || !ccnt || !ccap) goto done;
    for (int64_t j = 0; j < n; ++j) w[j] = INF;
    urp[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t nt = 0;
        w[i] = 0; /* the diagonal always exists */
        touched[nt++] = (int32_t)i;
        for (int64_t e = arp[i]; e < arp[i + 1]; ++e) {
            int32_t j = aci[e];
            if (j <= i) continue;
            if (w[j] == INF) touched[nt++] = j;
            w[j] = 0;
        }
        /* eliminate every k < i whose row holds column i */
        for (int64_t q = 0; q < ccnt[i]; ++q) {
            const int64_t k = col[i][q].k, pos = col[i][q].pos;
            const int32_t lki = ulev[pos];
            for (int64_t e = pos + 1; e < urp[k + 1]; ++e) { /* columns j > i of row k */
                const int32_t j = uci[e];
                const int64_t cand = (int64_t)lki + ulev[e] + 1;
                if (cand <= K && cand < w[j]) {
                    if (w[j] == INF) touched[nt++] = j;
                    w[j] = (int32_t)cand;
                }
            }
        }
        qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
        if (ucount + nt > ucap) {
            while (ucount + nt > ucap) ucap *= 2;
            int32_t *a = (int32_t *)realloc(uci, sizeof(int32_t) * (size_t)ucap);
            if (!a) goto done;
            uci = a;
            int32_t *b = (int32_t *)realloc(ulev, sizeof(int32_t) * (size_t)ucap);
            if (!b) goto done;
            ulev = b;
        }
        for (int64_t t = 0; t < nt; ++t) {
            const int32_t j = touched[t];
            uci[ucount] = j;
            ulev[ucount] = w[j];
            if (j > i) { /* row i holds column j: record it for row j */
                if (ccnt[j] == ccap[j]) {
                    ccap[j] = ccap[j] ? 2 * ccap[j] : 8;
                    kpos_t *c = (kpos_t *)realloc(col[j], sizeof(kpos_t) * (size_t)ccap[j]);
                    if (!c) goto done;
                    col[j] = c;
                }
                col[j][ccnt[j]].k = i;
                col[j][ccnt[j]].pos = ucount;
                ++ccnt[j];
            }
            w[j] = INF;
            ++ucount;
        }
        urp[i + 1] = ucount;
    }
    if (ucount <= cap) {
        for (int64_t i = 0; i <= n; ++i) rp[i] = urp[i];
        for (int64_t e = 0; e < ucount; ++e) {
            ci[e] = uci[e];
            lev[e] = ulev[e];
        }
    }
    result = ucount;
done:
    if (col)
        for (int64_t j = 0; j < n; ++j) free(col[j]);
    free(w); free(touched); free(urp); free(uci); free(ulev); free(col); free(ccnt); free(ccap);
    return result;
}

/*
 * O7: level(k) incomplete Cholesky, A ~= U^T U on a fixed pattern (the
 * numeric factorization the paper runs by blocks, Sec. "Numeric
 * factorization: Cholesky-by-blocks", on the pattern of O6): the loop of
 * O1 (b = 1), where every update whose target is not in the pattern is
 * dropped.  Pattern and values as rows: rp[n + 1], ci (row i: columns
 * increasing, the diagonal first), val (A's upper entries on the pattern, 0
 * on fill), overwritten with U.  Step k: u_kk := sqrt(a_kk); u_kj := a_kj /
 * u_kk for j in row k; a_ij -= u_ki u_kj for i <= j, both in row k, (i, j) in
 * the pattern (found by bisection in row i).  With the complete pattern these
 * are O1's operations in O1's order.  Returns 0 or the 1-based column of the
 * first pivot that is not > 0.
 */
int oracle_ichol_rows(int64_t n, const int64_t *rp, const int32_t *ci, double *val) {
    for (int64_t k = 0; k < n; ++k) {
        const int64_t b = rp[k], e = rp[k + 1];
        if (e <= b || ci[b] != k) return -1; /* the diagonal must lead the row */
        const double a = val[b];
        if (!(a > 0.0)) return (int)(k + 1);
        const double piv = sqrt(a);
        val[b] = piv;
        for (int64_t q = b + 1; q < e; ++q) val[q] = val[q] / piv;
        for (int64_t qc = b + 1; qc < e; ++qc) {
            const int32_t c = ci[qc];
            const double ukc = val[qc];
            for (int64_t qi = b + 1; qi <= qc; ++qi) {
                const int32_t i = ci[qi];
                /* (i, c) in row i? */
                int64_t lo = rp[i], hi = rp[i + 1] - 1;
                while (lo <= hi) {
                    const int64_t mid = (lo + hi) / 2;
                    if (ci[mid] < c)
                        lo = mid + 1;
                    else if (ci[mid] > c)
                        hi = mid - 1;
                    else {
                        double p = val[qi] * ukc;
                        val[mid] = val[mid] - p;
                        break;
                    }
                }
            }
        }
    }
    return 0;
}

/*
 * O8 -- the loop of Fig. "dense-chol" at b = 1 for a complex Hermitian
 * positive definite A = U^H U (the HERK the figure names is the Hermitian
 * rank-k update; the conclusion lists complex data among the extensions).
 * A holds interleaved (real, imaginary) doubles, element (i, j) at
 * A[2 (i + j lda)] and A[2 (i + j lda) + 1] (lda counts complex elements);
 * only the upper triangle is read and written.
 *
 * Step j, with alpha11 = A(j,j), a12 = A(j, j+1:n), A22 = A(j+1:n, j+1:n):
 *   alpha11 := sqrt(re alpha11)                      CHOL (its imaginary part,
 *                                                    zero for Hermitian A, is
 *                                                    not read; U(j,j) is real)
 *   a12     := a12 / alpha11                         TRSM (triu(alpha11)^{-H})
 *   A22     := A22 - a12^H a12   (upper part)        HERK
 * element-wise A(i,c) -= conj(U(j,i)) U(j,c) for j < i <= c, with
 *   conj(x) y = (xr yr + xi yi) + i (xr yi - xi yr),
 * each product rounded, the two summed, then subtracted.  Breakdown: the
 * first pivot whose real part is not > 0 (NaN included) stops the loop and
 * returns its 1-based column.  Returns 0 on success.
 */
#define ZR(A, lda, i, j) ((A)[2 * ((int64_t)(i) + (int64_t)(j) * (int64_t)(lda))])
#define ZI(A, lda, i, j) ((A)[2 * ((int64_t)(i) + (int64_t)(j) * (int64_t)(lda)) + 1])

int oracle_zpotrf_upper(int64_t n, double *A, int64_t lda) {
    for (int64_t j = 0; j < n; ++j) {
        double ar = ZR(A, lda, j, j);
        if (!(ar > 0.0)) return (int)(j + 1);
        double dr = sqrt(ar);
        ZR(A, lda, j, j) = dr;
        ZI(A, lda, j, j) = 0.0;
        for (int64_t c = j + 1; c < n; ++c) {
            ZR(A, lda, j, c) = ZR(A, lda, j, c) / dr;
            ZI(A, lda, j, c) = ZI(A, lda, j, c) / dr;
        }
        for (int64_t c = j + 1; c < n; ++c) {
            double yr = ZR(A, lda, j, c), yi = ZI(A, lda, j, c);
            for (int64_t i = j + 1; i <= c; i++) {
                double xr = ZR(A, lda, j, i), xi = ZI(A, lda, j, i);
                double pr = xr * yr + xi * yi;
                double pi = xr * yi - xi * yr;
                ZR(A, lda, i, c) = ZR(A, lda, i, c) - pr;
                ZI(A, lda, i, c) = ZI(A, lda, i, c) - pi;
            }
        }
    }
    return 0;
}

/*
 * O9 -- LU factorization without pivoting, A = L U (L unit lower triangular,
 * U upper triangular), in place: the same partitioned loop as the Cholesky
 * loop of Fig. "dense-chol" (the conclusion names LU among the factorizations
 * the by-blocks pattern carries over to), at b = 1.  Step j, with
 * alpha11 = A(j,j), a21 = A(j+1:n, j), a12 = A(j, j+1:n):
 *   a21 := a21 / alpha11          (the column of L below its unit diagonal)
 *   A22 := A22 - a21 a12          (each product rounded, then subtracted)
 * alpha11 and a12 are final as they stand (the row of U).  Breakdown (no
 * pivoting: the paper does not treat it): the first pivot that is zero or not
 * finite stops the loop and returns its 1-based column.  Returns 0 on success.
 */
int oracle_getrf_nopiv(int64_t n, double *A, int64_t lda) {
    for (int64_t j = 0; j < n; ++j) {
        double piv = AT(A, lda, j, j);
        if (piv == 0.0 || !isfinite(piv)) return (int)(j + 1);
        for (int64_t r = j + 1; r < n; ++r) AT(A, lda, r, j) = AT(A, lda, r, j) / piv;
        for (int64_t c = j + 1; c < n; ++c) {
            double ujc = AT(A, lda, j, c);
            for (int64_t r = j + 1; r < n; ++r) {
                double q = AT(A, lda, r, j) * ujc;
                AT(A, lda, r, c) = AT(A, lda, r, c) - q;
            }
        }
    }
    return 0;
}

/*
 * O10 -- Householder QR, A = Q R (m >= n), in place: the partitioned loop of
 * Fig. "dense-chol" carried over to QR (the conclusion names QR among the
 * factorizations the by-blocks pattern carries over to), at b = 1.  Step j,
 * with alpha = A(j,j) and x = A(j+1:m, j):
 *   sigma = x^T x.  sigma == 0: tau_j = 0 (H_j = I), column j stays.
 *   Otherwise beta = -sign(alpha) sqrt(alpha^2 + sigma) (sign(0) = +),
 *     tau_j = (beta - alpha) / beta, x := x / (alpha - beta) (so that
 *     v_j = [1; x]), A(j,j) := beta, and every later column c is reflected:
 *     w = A(j,c) + x^T A(j+1:m, c);  A(j,c) -= tau_j w;
 *     A(j+1:m, c) -= tau_j w x.
 * On exit R is the upper triangle, v_j below the diagonal of column j (unit
 * entry implied), Q = H_0 H_1 ... H_{n-1} with H_j = I - tau_j v_j v_j^T (the
 * reflector convention of LAPACK's geqrf).  No rescaling of columns whose
 * squared norm under- or overflows.
 */
void oracle_geqrf(int64_t m, int64_t n, double *A, int64_t lda, double *tau) {
    for (int64_t j = 0; j < n && j < m; ++j) {
        double alpha = AT(A, lda, j, j);
        double sigma = 0.0;
        for (int64_t r = j + 1; r < m; ++r) sigma += AT(A, lda, r, j) * AT(A, lda, r, j);
        if (sigma == 0.0) {
            tau[j] = 0.0;
            continue;
        }
        double mag = sqrt(alpha * alpha + sigma);
        double beta = alpha >= 0.0 ? -mag : mag;
        double tj = (beta - alpha) / beta;
        double den = alpha - beta;
        for (int64_t r = j + 1; r < m; ++r) AT(A, lda, r, j) = AT(A, lda, r, j) / den;
        AT(A, lda, j, j) = beta;
        tau[j] = tj;
        for (int64_t c = j + 1; c < n; ++c) {
            double w = AT(A, lda, j, c);
            for (int64_t r = j + 1; r < m; ++r) w += AT(A, lda, r, j) * AT(A, lda, r, c);
            AT(A, lda, j, c) = AT(A, lda, j, c) - tj * w;
            double tw = tj * w;
            for (int64_t i = j + 1; i < m; ++i) AT(A, lda, i, c) = AT(A, lda, i, c) - tw * AT(A, lda, i, j);
        }
    }
}
