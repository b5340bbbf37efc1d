/*
 * oracle.h -- CPU FP64 oracle for the delayed-update Cholesky / LU library.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this code: only the test suite, the package's smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no source with the GPU library.
 *
 * Every routine is the plain definition of what the library computes, written
 * as the textbook algorithm in IEEE binary64 (compiled with -ffp-contract=off,
 * no fast-math, sums taken in ascending index order).  Matrices are
 * column-major with a leading dimension; all pointers are host memory owned by
 * the caller.
 *
 * Paper: C. Camarero, "Simple, Fast and Practicable Algorithms for Cholesky,
 * LU and QR Decomposition Using Fast Rectangular Matrix Multiplication"
 * (arXiv 1812.02056).
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Cholesky factor (Introduction: A = L L^T; Sec. 2, Algorithm 1 with s = n,
 * the Cholesky-Crout special case).  Reads tril(A) only.  Writes the lower
 * triangle of L (including the diagonal) and zeros its strict upper triangle.
 * Returns 0, or the 1-based column j whose pivot A[j,j] - sum L[j,k]^2 is not
 * > 0 (NaN included); columns >= j of L are then unspecified. */
int oracle_chol(int64_t n, const double *A, int64_t lda, double *L, int64_t ldl);

/* LU without pivoting, Doolittle convention (unit lower L, upper U), packed
 * in LU: strict lower = L, upper incl. diagonal = U.  Definition: the unique
 * factorisation A = L U when every leading principal minor is nonzero
 * (Sec. 2, Algorithm 2 data requirements).  Returns 0, or the 1-based k whose
 * pivot U[k,k] is zero or non-finite. */
int oracle_lu(int64_t n, const double *A, int64_t lda, double *LU, int64_t ldlu);

/* Solve A X = B given the Cholesky factor L (forward then backward
 * substitution).  B, X are n x nrhs. */
void oracle_chol_solve(int64_t n, int64_t nrhs, const double *L, int64_t ldl,
                       const double *B, int64_t ldb, double *X, int64_t ldx);

/* Solve A X = B given Doolittle-packed LU. */
void oracle_lu_solve(int64_t n, int64_t nrhs, const double *LU, int64_t ldlu,
                     const double *B, int64_t ldb, double *X, int64_t ldx);

/* Algorithm 1 (Sec. 2) with an arbitrary step s, with the deferred product
 * S = R R^T formed classically and subtracted over the full trailing square.
 * A is the full symmetric matrix (read only; a working copy is made).
 * Returns the number of deferred updates performed. */
int64_t oracle_chol_alg1(int64_t n, int64_t s, const double *A, int64_t lda,
                         double *L, int64_t ldl);

/* Algorithm 2 (Sec. 2) with step s: Crout factors, L lower with its diagonal,
 * U unit upper.  Returns the number of deferred updates performed. */
int64_t oracle_lu_alg2(int64_t n, int64_t s, const double *A, int64_t lda,
                       double *L, int64_t ldl, double *U, int64_t ldu);

/* One deferred update of Algorithm 1: S = P P^T, then C -= S on the lower
 * triangle (i >= j) of the m x m matrix C.  P is m x w. */
void oracle_syrk_update(int64_t m, int64_t w, double *C, int64_t ldc,
                        const double *P, int64_t ldp);

/* One deferred update of Algorithm 2: S = X Y, then C -= S on all of the
 * m x m matrix C.  X is m x w, Y is w x m. */
void oracle_gemm_update(int64_t m, int64_t w, double *C, int64_t ldc,
                        const double *X, int64_t ldx, const double *Y, int64_t ldy);

/* Round a binary64 value to the nearest binary32 value (ties to even), and
 * to the nearest bfloat16 value (8-bit significand; ties to even) of its
 * binary32 rounding, both returned as binary64. */
/* QR by Gram-Schmidt with deferred block projections (Sec. 2, Algorithm 3),
 * for an m x n matrix A with m >= n >= 0.  Writes the m x n Q (orthonormal
 * columns) and the full n x n product R = Q^T A (its strict lower triangle is
 * rounding noise; the algorithm states R upper triangular).  *info = 0, or the
 * 1-based column c whose norm after the projections is not > 0 (zero or NaN);
 * the routine then stops: columns >= c of Q are zero and R is not written.
 * Returns the number of block projections, floor((n-1)/s) when info = 0. */
int64_t oracle_qr_alg3(int64_t m, int64_t n, int64_t s, const double *A, int64_t lda,
                       double *Q, int64_t ldq, double *R, int64_t ldr, int *info);

/* One block projection of Algorithm 3 (Sec. 2) on its own: C = Bq^T Bm
 * (w x k, Bq m x w, Bm m x k), then Bm -= Bq C.  C may be NULL. */
void oracle_qr_project(int64_t m, int64_t w, int64_t k, const double *Bq, int64_t ldq,
                       double *Bm, int64_t ldm, double *C, int64_t ldc);

double oracle_round_f32(double x);
double oracle_round_bf16(double x);

/* Number of OpenMP threads the oracle uses (1 when built without OpenMP). */
int oracle_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
