/*
 * oracle.c -- CPU FP64 oracle for the delayed-update Cholesky / LU library.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain C, IEEE binary64, built with
 * -O2 -ffp-contract=off and without fast-math, so every sum is evaluated in the
 * order written.  Where OpenMP is used, only independent rows are spread over
 * threads; each row's arithmetic is unchanged, so the results are bitwise the
 * same for any thread count.
 *
 * Paper: C. Camarero, arXiv 1812.02056 (Sec. 2: Algorithms 1, 2 and 3 and the
 * discussion of their special cases s = 1 and s = n).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Cholesky, plain definition: the lower-triangular L with positive diagonal and
 * A = L L^T (Introduction).  Computed as the Cholesky-Crout algorithm, which is
 * Algorithm 1 with s = n (Sec. 2): column j is formed from the original A and
 * all previously computed columns,
 *     L[j,j] = sqrt(A[j,j] - sum_{k<j} L[j,k]^2),
 *     L[i,j] = (A[i,j] - sum_{k<j} L[i,k] L[j,k]) / L[j,j]      (i > j).
 * The factor is kept in a row-major working array so each sum runs over
 * contiguous memory; that is a storage choice only, the operations and their
 * order are exactly the ones above.
 */
int oracle_chol(int64_t n, const double *A, int64_t lda, double *L, int64_t ldl)
{
    if (n <= 0) return 0;
    double *W = (double *)calloc((size_t)n * (size_t)n, sizeof(double));
    if (!W) return -1;
    int info = 0;
    for (int64_t j = 0; j < n; ++j) {
        const double *wj = W + (size_t)j * (size_t)n;
        double d = A[IDX(j, j, lda)];
        for (int64_t k = 0; k < j; ++k) d -= wj[k] * wj[k];
        if (!(d > 0.0)) {           /* non-positive or NaN pivot */
            info = (int)(j + 1);
            break;
        }
        const double ljj = sqrt(d);
        W[(size_t)j * (size_t)n + (size_t)j] = ljj;
#pragma omp parallel for schedule(static)
        for (int64_t i = j + 1; i < n; ++i) {
            const double *wi = W + (size_t)i * (size_t)n;
            double t = A[IDX(i, j, lda)];
            for (int64_t k = 0; k < j; ++k) t -= wi[k] * wj[k];
            W[(size_t)i * (size_t)n + (size_t)j] = t / ljj;
        }
    }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i)
            L[IDX(i, j, ldl)] = (i >= j) ? W[(size_t)i * (size_t)n + (size_t)j] : 0.0;
    free(W);
    return info;
}

/*
 * LU without pivoting, Doolittle form (unit lower L, upper U), the unique
 * factorisation when all leading principal minors are nonzero (Sec. 2,
 * Algorithm 2's data requirement).  For k = 0..n-1:
 *     U[k,j] = A[k,j] - sum_{p<k} L[k,p] U[p,j]            (j >= k)
 *     L[i,k] = (A[i,k] - sum_{p<k} L[i,p] U[p,k]) / U[k,k]  (i > k)
 * L is held row-major and U column-major so each sum is contiguous.
 */
int oracle_lu(int64_t n, const double *A, int64_t lda, double *LU, int64_t ldlu)
{
    if (n <= 0) return 0;
    double *Lr = (double *)calloc((size_t)n * (size_t)n, sizeof(double)); /* Lr[i*n+p] = L[i,p] */
    double *Uc = (double *)calloc((size_t)n * (size_t)n, sizeof(double)); /* Uc[j*n+p] = U[p,j] */
    if (!Lr || !Uc) { free(Lr); free(Uc); return -1; }
    int info = 0;
    for (int64_t k = 0; k < n; ++k) {
        const double *lk = Lr + (size_t)k * (size_t)n;
#pragma omp parallel for schedule(static)
        for (int64_t j = k; j < n; ++j) {
            const double *uj = Uc + (size_t)j * (size_t)n;
            double t = A[IDX(k, j, lda)];
            for (int64_t p = 0; p < k; ++p) t -= lk[p] * uj[p];
            Uc[(size_t)j * (size_t)n + (size_t)k] = t;
        }
        const double ukk = Uc[(size_t)k * (size_t)n + (size_t)k];
        if (ukk == 0.0 || !isfinite(ukk)) {
            info = (int)(k + 1);
            break;
        }
        const double *uk = Uc + (size_t)k * (size_t)n;
#pragma omp parallel for schedule(static)
        for (int64_t i = k + 1; i < n; ++i) {
            const double *li = Lr + (size_t)i * (size_t)n;
            double t = A[IDX(i, k, lda)];
            for (int64_t p = 0; p < k; ++p) t -= li[p] * uk[p];
            Lr[(size_t)i * (size_t)n + (size_t)k] = t / ukk;
        }
    }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i)
            LU[IDX(i, j, ldlu)] = (i > j) ? Lr[(size_t)i * (size_t)n + (size_t)j]
                                          : Uc[(size_t)j * (size_t)n + (size_t)i];
    free(Lr);
    free(Uc);
    return info;
}

/* Forward substitution L y = b, then backward L^T x = y, per right-hand side. */
void oracle_chol_solve(int64_t n, int64_t nrhs, const double *L, int64_t ldl,
                       const double *B, int64_t ldb, double *X, int64_t ldx)
{
    double *y = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    for (int64_t r = 0; r < nrhs; ++r) {
        const double *b = B + (size_t)r * (size_t)ldb;
        double *x = X + (size_t)r * (size_t)ldx;
        for (int64_t i = 0; i < n; ++i) {
            double t = b[i];
            for (int64_t k = 0; k < i; ++k) t -= L[IDX(i, k, ldl)] * y[k];
            y[i] = t / L[IDX(i, i, ldl)];
        }
        for (int64_t i = n - 1; i >= 0; --i) {
            double t = y[i];
            for (int64_t k = i + 1; k < n; ++k) t -= L[IDX(k, i, ldl)] * x[k];
            x[i] = t / L[IDX(i, i, ldl)];
        }
    }
    free(y);
}

/* Forward substitution with the unit lower L, then backward with U. */
void oracle_lu_solve(int64_t n, int64_t nrhs, const double *LU, int64_t ldlu,
                     const double *B, int64_t ldb, double *X, int64_t ldx)
{
    double *y = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    for (int64_t r = 0; r < nrhs; ++r) {
        const double *b = B + (size_t)r * (size_t)ldb;
        double *x = X + (size_t)r * (size_t)ldx;
        for (int64_t i = 0; i < n; ++i) {
            double t = b[i];
            for (int64_t k = 0; k < i; ++k) t -= LU[IDX(i, k, ldlu)] * y[k];
            y[i] = t;
        }
        for (int64_t i = n - 1; i >= 0; --i) {
            double t = y[i];
            for (int64_t k = i + 1; k < n; ++k) t -= LU[IDX(i, k, ldlu)] * x[k];
            x[i] = t / LU[IDX(i, i, ldlu)];
        }
    }
    free(y);
}

/*
 * The step-s algorithms of Sec. 2 (Algorithms 1 and 2) in block terms.  With
 * the columns cut into consecutive blocks of w = min(s, columns left), the
 * columns of one block are formed from the working matrix, which already holds
 * every earlier block's deferred product, and from the block's own earlier
 * columns only.  For a block starting at column c0 that is
 *   (i)   the factorisation of its w x w diagonal block,
 *   (ii)  the triangular solve of the rows below it against that factor (LU:
 *         also of the columns to its right),
 *   (iii) if rows remain, the deferred product of the block's m x w columns
 *         with their transposed partner, subtracted from the whole m x m
 *         trailing square of the working matrix (one "update").
 * Each entry is one running difference started from the working matrix and
 * taken over the block's columns in ascending order, followed by one division.
 */

/* Working-matrix helpers shared by the two step-s routines below. */
static double *copy_square(int64_t n, const double *A, int64_t lda)
{
    double *W = (double *)malloc((size_t)n * (size_t)n * sizeof(double));
    for (int64_t j = 0; j < n; ++j)
        memcpy(W + (size_t)j * (size_t)n, A + (size_t)j * (size_t)lda, (size_t)n * sizeof(double));
    return W;
}

/* Aw[r.., r..] -= X Y over the whole trailing square, where X(i, k) = Lw[r+i, c0+k]
 * and Y(k, j) = Rw[c0+k, r+j] (k < w); each entry's product is summed first. */
static void subtract_block_product(int64_t n, int64_t c0, int64_t w, double *Aw,
                                   const double *Lw, const double *Rw)
{
    const int64_t r = c0 + w;
    for (int64_t j = r; j < n; ++j)
        for (int64_t i = r; i < n; ++i) {
            double prod = 0.0;
            for (int64_t k = c0; k < r; ++k) prod += Lw[IDX(i, k, n)] * Rw[IDX(k, j, n)];
            Aw[IDX(i, j, n)] -= prod;
        }
}

/*
 * Algorithm 1 of Sec. 2 with step s.  Per block: (i) Cholesky of the diagonal
 * block, (ii) rows below divided through by the block's factor transposed,
 * (iii) the symmetric deferred product R R^T.  Rt holds the transposed factor
 * so that (iii) has the same shape as the LU product.
 */
int64_t oracle_chol_alg1(int64_t n, int64_t s, const double *A, int64_t lda,
                         double *L, int64_t ldl)
{
    if (n <= 0) return 0;
    double *Aw = copy_square(n, A, lda);
    double *Lw = (double *)calloc((size_t)n * (size_t)n, sizeof(double));
    double *Rt = (double *)calloc((size_t)n * (size_t)n, sizeof(double));
    int64_t updates = 0;
    for (int64_t c0 = 0; c0 < n; c0 += s) {
        const int64_t w = (n - c0 < s) ? n - c0 : s;
        /* (i) + (ii): column by column over the block; the pivot comes from the
         * diagonal entry, the rows below (inside and under the block) share it. */
        for (int64_t c = c0; c < c0 + w; ++c) {
            double piv = Aw[IDX(c, c, n)];
            for (int64_t k = c0; k < c; ++k) piv -= Lw[IDX(c, k, n)] * Lw[IDX(c, k, n)];
            const double root = sqrt(piv);
            Lw[IDX(c, c, n)] = root;
            for (int64_t i = c + 1; i < n; ++i) {
                double v = Aw[IDX(i, c, n)];
                for (int64_t k = c0; k < c; ++k) v -= Lw[IDX(i, k, n)] * Lw[IDX(c, k, n)];
                Lw[IDX(i, c, n)] = v / root;
            }
        }
        if (c0 + w >= n) break;
        /* (iii) */
        for (int64_t k = c0; k < c0 + w; ++k)
            for (int64_t j = c0 + w; j < n; ++j) Rt[IDX(k, j, n)] = Lw[IDX(j, k, n)];
        subtract_block_product(n, c0, w, Aw, Lw, Rt);
        ++updates;
    }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) L[IDX(i, j, ldl)] = Lw[IDX(i, j, n)];
    free(Aw);
    free(Lw);
    free(Rt);
    return updates;
}

/*
 * Algorithm 2 of Sec. 2 with step s, Crout form (L lower with its diagonal, U
 * unit upper).  Per block, column c of L and then row c of U, ascending:
 * L(i, c) for rows i >= c (the diagonal block and the rows below it, solved
 * against the block's unit U), then U(c, j) for columns j >= c (solved against
 * the block's L and divided by L(c, c)); then (iii) S = R_L R_U.
 */
int64_t oracle_lu_alg2(int64_t n, int64_t s, const double *A, int64_t lda,
                       double *L, int64_t ldl, double *U, int64_t ldu)
{
    if (n <= 0) return 0;
    double *Aw = copy_square(n, A, lda);
    double *Lw = (double *)calloc((size_t)n * (size_t)n, sizeof(double));
    double *Uw = (double *)calloc((size_t)n * (size_t)n, sizeof(double));
    int64_t updates = 0;
    for (int64_t c0 = 0; c0 < n; c0 += s) {
        const int64_t w = (n - c0 < s) ? n - c0 : s;
        for (int64_t c = c0; c < c0 + w; ++c) {
            for (int64_t i = c; i < n; ++i) {
                double v = Aw[IDX(i, c, n)];
                for (int64_t k = c0; k < c; ++k) v -= Lw[IDX(i, k, n)] * Uw[IDX(k, c, n)];
                Lw[IDX(i, c, n)] = v;
            }
            const double piv = Lw[IDX(c, c, n)];
            for (int64_t j = c; j < n; ++j) {
                double v = Aw[IDX(c, j, n)];
                for (int64_t k = c0; k < c; ++k) v -= Lw[IDX(c, k, n)] * Uw[IDX(k, j, n)];
                Uw[IDX(c, j, n)] = v / piv;
            }
        }
        if (c0 + w >= n) break;
        subtract_block_product(n, c0, w, Aw, Lw, Uw);
        ++updates;
    }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) {
            L[IDX(i, j, ldl)] = Lw[IDX(i, j, n)];
            U[IDX(i, j, ldu)] = Uw[IDX(i, j, n)];
        }
    free(Aw);
    free(Lw);
    free(Uw);
    return updates;
}

/* The deferred update of Algorithm 1 (Sec. 2), lower triangle only: the entries
 * i < j of the trailing square are never read again by the algorithm. */
void oracle_syrk_update(int64_t m, int64_t w, double *C, int64_t ldc,
                        const double *P, int64_t ldp)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < m; ++j)
        for (int64_t i = j; i < m; ++i) {
            double t = 0.0;
            for (int64_t k = 0; k < w; ++k) t += P[IDX(i, k, ldp)] * P[IDX(j, k, ldp)];
            C[IDX(i, j, ldc)] -= t;
        }
}

/* The deferred update of Algorithm 2 (Sec. 2) over the full trailing square. */
void oracle_gemm_update(int64_t m, int64_t w, double *C, int64_t ldc,
                        const double *X, int64_t ldx, const double *Y, int64_t ldy)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m; ++j)
        for (int64_t i = 0; i < m; ++i) {
            double t = 0.0;
            for (int64_t k = 0; k < w; ++k) t += X[IDX(i, k, ldx)] * Y[IDX(k, j, ldy)];
            C[IDX(i, j, ldc)] -= t;
        }
}

/*
 * The block projection of Algorithm 3 (Sec. 2): with the finished columns
 * Bq = Q[:, z..c-1] (w of them) and the columns still to come Bm = M[:, c..n],
 *     C = Bq^T Bm          (w x k; each entry a sum over the m rows, ascending)
 *     S = Bq C, Bm -= S    (each entry of S a sum over the w columns, ascending)
 * Columns of Bm are independent, so they are spread over threads.
 */
void oracle_qr_project(int64_t m, int64_t w, int64_t k, const double *Bq, int64_t ldq,
                       double *Bm, int64_t ldm, double *C, int64_t ldc)
{
#pragma omp parallel
    {
        double *cj = (double *)malloc((size_t)(w > 0 ? w : 1) * sizeof(double));
#pragma omp for schedule(dynamic, 4)
        for (int64_t j = 0; j < k; ++j) {
            double *bm = Bm + (size_t)j * (size_t)ldm;
            for (int64_t t = 0; t < w; ++t) {
                const double *q = Bq + (size_t)t * (size_t)ldq;
                double d = 0.0;
                for (int64_t i = 0; i < m; ++i) d += q[i] * bm[i];
                cj[t] = d;
            }
            for (int64_t i = 0; i < m; ++i) {
                double sv = 0.0;
                for (int64_t t = 0; t < w; ++t) sv += Bq[IDX(i, t, ldq)] * cj[t];
                bm[i] -= sv;
            }
            if (C)
                for (int64_t t = 0; t < w; ++t) C[IDX(t, j, ldc)] = cj[t];
        }
        free(cj);
    }
}

/*
 * Algorithm 3 of Sec. 2 with step s, organised by blocks.  M starts as a copy
 * of A.  For each block of w = min(s, n - c0) columns starting at c0:
 *   (i)  the block's columns are orthonormalised among themselves by modified
 *        Gram-Schmidt: column c loses its component along each finished column
 *        q_j of the block (j = c0, ..., c-1, in that order, every product taken
 *        with the vector as updated so far) and is divided by its norm (a sum
 *        of squares in row order, then sqrt);
 *   (ii) the finished block is projected out of every later column at once
 *        (oracle_qr_project), so later blocks start from columns already free
 *        of it.
 * Then R = Q^T A in full.  With s = 1 every column is projected out as soon as
 * it is finished, and with s >= n no block projection happens; the two are the
 * right- and left-looking orderings of modified Gram-Schmidt and perform the
 * same operations on every column.
 */
static int qr_orthonormalise_block(int64_t m, int64_t c0, int64_t w, double *M, double *Q, int64_t ldq)
{
    for (int64_t c = c0; c < c0 + w; ++c) {
        double *v = M + (size_t)c * (size_t)m;
        for (int64_t j = c0; j < c; ++j) {
            const double *qj = Q + (size_t)j * (size_t)ldq;
            double d = 0.0;
            for (int64_t i = 0; i < m; ++i) d += qj[i] * v[i];
            for (int64_t i = 0; i < m; ++i) v[i] -= qj[i] * d;
        }
        double ss = 0.0;
        for (int64_t i = 0; i < m; ++i) ss += v[i] * v[i];
        const double nrm = sqrt(ss);
        if (!(nrm > 0.0)) return (int)(c + 1);
        double *qc = Q + (size_t)c * (size_t)ldq;
        for (int64_t i = 0; i < m; ++i) qc[i] = v[i] / nrm;
    }
    return 0;
}

int64_t oracle_qr_alg3(int64_t m, int64_t n, int64_t s, const double *A, int64_t lda,
                       double *Q, int64_t ldq, double *R, int64_t ldr, int *info)
{
    *info = 0;
    if (n <= 0) return 0;
    double *M = (double *)malloc((size_t)m * (size_t)n * sizeof(double));
    if (!M) return -1;
    for (int64_t j = 0; j < n; ++j) {
        memcpy(M + (size_t)j * (size_t)m, A + (size_t)j * (size_t)lda, (size_t)m * sizeof(double));
        memset(Q + (size_t)j * (size_t)ldq, 0, (size_t)m * sizeof(double));
    }
    int64_t projections = 0;
    for (int64_t c0 = 0; c0 < n; c0 += s) {
        const int64_t w = (n - c0 < s) ? n - c0 : s;
        *info = qr_orthonormalise_block(m, c0, w, M, Q, ldq);
        if (*info) break;
        if (c0 + w >= n) break;
        oracle_qr_project(m, w, n - c0 - w, Q + (size_t)c0 * (size_t)ldq, ldq,
                          M + (size_t)(c0 + w) * (size_t)m, m, NULL, 0);
        ++projections;
    }
    if (*info == 0) {
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i) {
                const double *qi = Q + (size_t)i * (size_t)ldq;
                const double *aj = A + (size_t)j * (size_t)lda;
                double d = 0.0;
                for (int64_t k = 0; k < m; ++k) d += qi[k] * aj[k];
                R[IDX(i, j, ldr)] = d;
            }
    }
    free(M);
    return projections;
}

double oracle_round_f32(double x) { return (double)(float)x; }

/*
 * bfloat16 keeps binary32's 8-bit exponent and 8 significant bits.  Round the
 * binary32 value f to the nearer of its two bfloat16 neighbours, taking the one
 * with an even last significand bit on a tie; magnitudes at or beyond the
 * midpoint above the largest finite bfloat16 become infinity.
 */
double oracle_round_bf16(double x)
{
    const double f = (double)(float)x;
    if (isnan(f) || isinf(f) || f == 0.0) return f;
    int e;
    (void)frexp(fabs(f), &e);                 /* 2^(e-1) <= |f| < 2^e */
    int ulp_exp = e - 8;                      /* spacing of 8-bit significands */
    if (ulp_exp < -133) ulp_exp = -133;       /* bfloat16 subnormal spacing */
    const double q = ldexp(fabs(f), -ulp_exp);/* exact: scaling by a power of two */
    const double lo = floor(q);
    const double frac = q - lo;
    double r;
    if (frac > 0.5) r = lo + 1.0;
    else if (frac < 0.5) r = lo;
    else r = (fmod(lo, 2.0) == 0.0) ? lo : lo + 1.0;
    double mag = ldexp(r, ulp_exp);
    const double bf16_max = ldexp(255.0, 120);  /* (2 - 2^-7) * 2^127 */
    if (mag > bf16_max) mag = INFINITY;
    return copysign(mag, f);
}
