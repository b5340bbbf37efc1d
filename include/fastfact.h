/*
 * fastfact.h -- C ABI of the MI355X (gfx950) delayed-update Cholesky / LU library.
 *
 * The method is C. Camarero, "Simple, Fast and Practicable Algorithms for
 * Cholesky, LU and QR Decomposition Using Fast Rectangular Matrix
 * Multiplication" (arXiv 1812.02056), Sec. 2, Algorithms 1 and 2: columns are
 * produced Crout-style and, every s columns, the pending block R of the factor
 * is folded into the rest of the matrix with one rectangular product
 * S = R R^T (LU: S = R_L R_U) that is subtracted from the trailing square.
 * Over one block of w <= s columns that is, in the usual vocabulary, a w x w
 * diagonal factorisation, a triangular solve of the m x w panel below it and
 * the rank-w trailing update A22 -= L21 L21^T (LU: A22 -= L21 U12).
 *
 * Conventions shared by every entry point
 *  - Matrices are column-major with a leading dimension ld >= max(1, rows);
 *    element (i, j) of A is A[i + j*lda].
 *  - Matrix pointers are DEVICE pointers (HIP device memory on the current
 *    device) unless stated otherwise.  The library never allocates, frees or
 *    retains caller memory; the caller owns every buffer.
 *  - `stream` is a hipStream_t passed as void* (NULL = the legacy default
 *    stream).  Work is enqueued on it; nothing is synchronised unless stated.
 *  - Return value: 0 = enqueued; -k = argument k (1-based) is invalid;
 *    FF_ERR_HIP (-100) = a HIP runtime call failed; FF_ERR_WORKSPACE (-101) =
 *    workspace too small; FF_ERR_UNSUPPORTED (-102) = valid but unsupported
 *    combination (e.g. a dtype an entry point does not implement).
 *    ff_status_string() names each code.
 *  - Numerical failure is reported asynchronously through *d_info, a device
 *    int32 that the call first sets to 0: k > 0 means the 1-based column k had
 *    a pivot that was not > 0 (Cholesky, NaN included) or was zero or not
 *    finite (LU).  The factorisation stops at the block containing column k;
 *    entries from that block on are unspecified.
 *  - Calls are reentrant: different streams may run different calls at once
 *    provided their buffers do not overlap.
 */
#ifndef FASTFACT_H
#define FASTFACT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Arithmetic of the trailing update (and storage type of the factored matrix). */
typedef enum {
    FF_F64 = 0,  /* storage double, every step in binary64 */
    FF_F32 = 1,  /* storage float; update and panel solve in binary32 MFMA;
                    diagonal blocks factored in binary64 and rounded back */
    FF_BF16 = 2  /* storage float; update operands rounded to bfloat16 (nearest,
                    ties to even), products accumulated in binary32; panel solve
                    in binary32; diagonal blocks in binary64 */
} ff_dtype;

/* Flags for the factorisations. */
enum {
    FF_FLAG_STRASSEN1 = 1u << 0,  /* one Strassen level in the trailing update
                                      (Sec. 2, Strassen on rectangles): every
                                      128 x 128 output super-tile takes the 7
                                      half-K products of its 64 x 64 quadrants
                                      instead of 8; under Cholesky, super-tiles
                                      on the diagonal keep the 6 classical ones.
                                      Binary64 only (FF_ERR_UNSUPPORTED for
                                      other dtypes).  Results differ from the
                                      classical update by rounding only; the
                                      bound grows as K^2 u max|X| max|Y|
                                      instead of K u sum|X||Y|. */
    FF_FLAG_NO_LOOKAHEAD = 1u << 1, /* keep every step on `stream` in strict order.
                                      Without it (Cholesky and LU), the next
                                      block's diagonal factorisation and panel
                                      solves run on a second, library-owned
                                      stream (default priority, ordered by
                                      events; the call still returns with all
                                      work ordered before later work on
                                      `stream`) while the rest of the update
                                      runs on all but a few CUs; the last
                                      min(1536, n/4) columns are factored in
                                      order on `stream`.  Both schedules give
                                      bitwise identical factors. */
    FF_FLAG_ESCALATE = 1u << 3,     /* chol_solve only: when the factor in the
                                      requested precision fails (info > 0) or
                                      its refinement ends neither converged nor
                                      at a backward error <= tol, factor A again
                                      in the next precision (bfloat16 ->
                                      binary32 -> binary64) and refine with
                                      that; see chol_solve. */
    FF_FLAG_GMRES_IR = 1u << 4,     /* chol_solve only: each refinement step
                                      solves its correction equation A d = r
                                      by GMRES in binary64, preconditioned on
                                      the left by the factor (M = W W^T in W's
                                      precision), instead of by one pair of
                                      triangular solves; see chol_solve. */
    FF_FLAG_STRASSEN2 = 1u << 5,    /* lu_nopiv_factor only: two Strassen levels
                                      (the paper times its Strassen variant with
                                      two and three recursions, Sec. 2 timing
                                      paragraph): on trailing products of
                                      m >= 2048 rows a matrix-level level splits
                                      m and the step in halves into Strassen's
                                      7 products, each computed by the one-level
                                      kernel of FF_FLAG_STRASSEN1 (odd last rows,
                                      columns or steps are applied classically);
                                      smaller products take one level.  Needs
                                      the workspace of ff_lu_workspace_size
                                      (n/2 x n/2 + n x s/2 doubles).  Binary64
                                      only; not combinable with
                                      FF_FLAG_STRASSEN1; FF_ERR_UNSUPPORTED for
                                      chol_factor. */
    FF_FLAG_FIXED_STEP = 1u << 2    /* every block exactly s columns wide (the
                                      step of Sec. 2 Algorithms 1 and 2
                                      verbatim).  Without it, the first block
                                      and the blocks near the end are narrower
                                      when s is wide: Cholesky 192 columns over
                                      the last 6144 when s > 192, LU 128 over
                                      the last 4096 when s > 128 (see
                                      chol_factor, lu_nopiv_factor).  Factors
                                      differ by rounding only. */
};

enum {
    FF_ERR_HIP = -100,
    FF_ERR_WORKSPACE = -101,
    FF_ERR_UNSUPPORTED = -102,
    FF_ERR_SCRATCH = -103   /* larger than the static scratch of chol_trisolve_noalloc */
};

const char *ff_status_string(int code);

/* Library version string, e.g. "fastfact 0.1 gfx950". */
const char *ff_version(void);

/*
 * Cholesky factorisation A = L L^T in place (Introduction; Sec. 2 Algorithm 1
 * with step s).  Reads only the lower triangle of the n x n matrix A and
 * overwrites it with L; the strict upper triangle is neither read nor written.
 *   n      order, >= 0 (n = 0 is a no-op)
 *   s      step size (columns per deferred update), >= 1; s >= n means no update.
 *          For the first block and over the last 6144 columns a step above 192
 *          is cut to 192, the widest diagonal block one workgroup factors in LDS
 *          (there the block factorisation, not the update, is on the critical
 *          path); FF_FLAG_FIXED_STEP keeps every block s wide.
 *   A      device pointer, double* for FF_F64, float* for FF_F32 / FF_BF16
 *   lda    >= max(1, n)
 *   dtype  ff_dtype
 *   flags  FF_FLAG_*
 *   ws     device workspace of ws_bytes bytes, >= ff_chol_workspace_size(...)
 *          (may be NULL when that size is 0)
 *   d_info device int32, see above
 *   stream hipStream_t
 */
size_t ff_chol_workspace_size(int64_t n, int64_t s, int dtype, unsigned flags);
int chol_factor(int64_t n, int64_t s, void *A, int64_t lda, int dtype, unsigned flags,
                void *ws, size_t ws_bytes, int32_t *d_info, void *stream);

/*
 * LU factorisation without pivoting A = L U in place (Sec. 2 Algorithm 2 with
 * step s; every leading principal minor of A must be nonzero).  The result is
 * Doolittle-packed: the strict lower triangle holds the unit-lower L, the upper
 * triangle including the diagonal holds U.  (Algorithm 2 returns the Crout form
 * L_c = L D, U_c = D^-1 U with D = diag(U); the deferred products are equal in
 * both forms.)  Only FF_F64 is implemented.  For the first block and over the
 * last 4096 columns a step above 128 is cut to 128, the widest diagonal block
 * one workgroup factors in LDS; FF_FLAG_FIXED_STEP keeps every block s wide.
 */
size_t ff_lu_workspace_size(int64_t n, int64_t s, int dtype, unsigned flags);
int lu_nopiv_factor(int64_t n, int64_t s, void *A, int64_t lda, int dtype, unsigned flags,
                    void *ws, size_t ws_bytes, int32_t *d_info, void *stream);

/*
 * QR factorisation A = Q R by Gram-Schmidt with deferred block projections
 * (Sec. 2 Algorithm 3 with step s), for an m x n matrix with m >= n.  A is read
 * only; Q (m x n, orthonormal columns) and R (n x n upper triangular with a
 * positive diagonal; its strict lower triangle is written as zero) are outputs
 * and must not overlap A or each other.  Per block of ws = min(s, n,
 * ff_qr_step-limit) columns: modified Gram-Schmidt inside the block (every
 * column projected against the block's earlier columns one at a time, then
 * divided by its norm), then C = B_Q^T M[:, c..] and M[:, c..] -= B_Q C for the
 * block's columns B_Q and the columns M[:, c..] after it; finally R = Q^T A.
 * The working matrix M of the algorithm lives in Q.  Only FF_F64.
 *   m, n   m >= n >= 0; m is limited to 128 rows per compute unit (256 rows per
 *          compute unit with blocks of at most 71 columns), else FF_ERR_UNSUPPORTED
 *   s      step, >= 1; the block width actually used is ff_qr_step(m, n, s)
 *          (at most 142 columns for m <= 128 * compute units: the block lives in
 *          the LDS of the workgroups that run its Gram-Schmidt)
 *   A      device double*, lda >= max(1, m)
 *   Q      device double*, ldq >= max(1, m)
 *   R      device double*, ldr >= max(1, n)
 *   flags  must be 0
 *   ws     device workspace, >= ff_qr_workspace_size(m, n, s, dtype, flags)
 *   d_info device int32: 0, or the 1-based column whose norm after its
 *          projections is not > 0 (zero or NaN; Q and R are then incomplete), or
 *          -1 if a wait between the co-resident workgroups of the Gram-Schmidt
 *          kernel expired (the device was shared with other work that kept
 *          compute units busy; Q and R are then invalid)
 *   stream hipStream_t; the call is asynchronous.
 * The Gram-Schmidt kernel keeps one workgroup per compute unit resident and
 * synchronises them through device memory; it must not share the device with
 * work that holds compute units indefinitely.  While it runs, tiles of R whose
 * columns of Q are final are formed (over chunks of rows, added in order) on a
 * second, library-owned stream of default priority, on the compute units it
 * leaves idle; events order that stream, and the call still returns with all of
 * its work ordered before later work on `stream`.
 */
size_t ff_qr_workspace_size(int64_t m, int64_t n, int64_t s, int dtype, unsigned flags);
int ff_qr_step(int64_t m, int64_t n, int64_t s);
int qr_factor(int64_t m, int64_t n, int64_t s, const void *A, int64_t lda, void *Q, int64_t ldq, void *R,
              int64_t ldr, int dtype, unsigned flags, void *ws, size_t ws_bytes, int32_t *d_info, void *stream);

/* Outcome of chol_solve (host struct). */
typedef struct {
    int32_t info;          /* info of the factorisation that produced X (0 = ok), as d_info above */
    int32_t iters;         /* refinement iterations performed with that factor */
    int32_t converged;     /* 1 if the correction test was met */
    int32_t dtype_used;    /* update precision of the factor that produced X */
    double last_correction;/* ||dX||_inf / ||X||_inf of the last iteration */
    double backward_err;   /* max_j ||b_j - A x_j||_inf / (||A||_inf ||x_j||_inf + ||b_j||_inf) */
    int32_t escalated_to;  /* -1, or (with FF_FLAG_ESCALATE) the ff_dtype escalated to (== dtype_used) */
    int32_t escalations;   /* refactorisations after the first */
    int32_t total_iters;   /* refinement iterations over all factors tried */
    int32_t first_info;    /* info of the factorisation in the requested precision */
    int32_t krylov_iters;  /* with FF_FLAG_GMRES_IR: GMRES steps over all columns and factors */
    int32_t reserved;      /* 0 */
} ff_solve_info;

/*
 * Solve A X = B for SPD A (solving linear systems being the use of the
 * factorisation, Introduction) with mixed-precision iterative refinement.
 *   A64   n x n binary64 SPD matrix (lower triangle read, never written)
 *   W     n x n working factor in `dtype` storage (double* for FF_F64, float*
 *         otherwise), leading dimension ldw.  If w_is_factored == 0 the call
 *         copies tril(A64) into W (rounded for float storage) and factors it
 *         with chol_factor(n, s, W, ldw, dtype, flags); otherwise W must hold
 *         such a factor already (e.g. kept from an earlier request).
 *   B     n x nrhs binary64 right-hand sides (read only), ldb >= n
 *   X     n x nrhs binary64 solution (written), ldx >= n
 *   tol   refinement stops once ||dX||_inf <= tol * ||X||_inf (per call, over
 *         all columns); also on stagnation (the correction shrank by less
 *         than half) or after max_iter iterations.  max_iter = 0 returns the
 *         plain triangular-solve result.
 *   flags FF_FLAG_* of the factorisations, plus FF_FLAG_ESCALATE: a result
 *         is accepted when the correction test was met, or when refinement
 *         stopped with backward error <= tol (the accuracy the conditioning
 *         allows); otherwise, or when the factorisation failed, A64 is
 *         factored again in the next precision (bfloat16 -> binary32, in W;
 *         binary32 -> binary64, in the workspace) and refined again.  out
 *         then describes the last attempt; escalated_to, escalations,
 *         total_iters and first_info record the way there.
 *         FF_FLAG_GMRES_IR refines each column on its own: a step computes
 *         r = b - A x in binary64 and runs one GMRES cycle (at most 30
 *         steps, stopping when the preconditioned residual has fallen by
 *         1e-8) on M^-1 A d = M^-1 r, Gram-Schmidt applied twice, then x += d;
 *         iters is then the most steps any column took, the stop rules are
 *         those above applied per column, and converged needs every column.
 *   ws    device workspace, >= ff_solve_workspace_size(n, s, nrhs, dtype,
 *         flags) (with FF_FLAG_ESCALATE and float storage it includes an n x n
 *         binary64 factor)
 *   out   host pointer, filled on return.
 * The residual B - A X and the update X += dX are binary64; the triangular
 * solves with W run in W's storage precision.  This call SYNCHRONISES `stream`
 * (the stop test runs on the host) and returns 0 even if refinement did not
 * converge (out->converged = 0) or the factorisation failed (out->info > 0).
 */
size_t ff_solve_workspace_size(int64_t n, int64_t s, int64_t nrhs, int dtype, unsigned flags);
int chol_solve(int64_t n, int64_t s, int64_t nrhs, const double *A64, int64_t lda,
               void *W, int64_t ldw, int dtype, unsigned flags, int w_is_factored,
               const double *B, int64_t ldb, double *X, int64_t ldx,
               double tol, int max_iter, void *ws, size_t ws_bytes, void *stream,
               ff_solve_info *out);

/*
 * Triangular solve with a Cholesky factor: X = L^-T L^-1 X in place (forward
 * then back substitution, in the storage precision of L: double for FF_F64,
 * float otherwise; X has the same type).  L is n x n lower (only tril read);
 * used to solve A x = b once A = L L^T is known (Introduction).  The solve
 * works on 64-row blocks: it first forms, in the workspace, the inverses of
 * the 64 x 64 diagonal blocks (binary64 arithmetic, stored in L's precision)
 * and copies of the tiles next to the diagonal, then runs one forward and one
 * backward sweep per group of at most 16 right-hand sides.  Asynchronous.
 *   ws   device workspace >= ff_trisolve_workspace_size(n, dtype).  Its first
 *        int32 is an error word: the call sets it to 0, and it becomes
 *        nonzero if a bounded wait between the workgroups of a sweep expired
 *        (which does not happen unless the device is shared with work that
 *        starves the launch); X is then unspecified.  Read it after the stream
 *        has reached the end of the call.
 */
size_t ff_trisolve_workspace_size(int64_t n, int dtype);
int chol_trisolve(int64_t n, int64_t nrhs, const void *L, int64_t ldl, int dtype,
                  void *X, int64_t ldx, void *ws, size_t ws_bytes, void *stream);

/*
 * chol_trisolve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same solve, with its workspace in a static device array of
 * FF_NOALLOC_SCRATCH_BYTES bytes that the library holds on every device it
 * runs on until the process ends.  No allocation of any kind is made.
 *   Arguments as chol_trisolve, without the workspace;
 *   d_status  device int32 or NULL: receives the error word (0, or nonzero if
 *             a bounded wait expired and X is unspecified).
 * Returns FF_ERR_SCRATCH when ff_trisolve_workspace_size(n, dtype) exceeds
 * FF_NOALLOC_SCRATCH_BYTES (binary64: n <= 9344; binary32: n <= 18688).
 * Every call on one device uses that device's one array, which keeps the last
 * call's contents (everything the solve needs is rewritten at its start):
 * calls that overlap on one device (different streams or host threads) race
 * and give wrong results; serialise them.
 */
#define FF_NOALLOC_SCRATCH_BYTES (32u << 20)
int chol_trisolve_noalloc(int64_t n, int64_t nrhs, const void *L, int64_t ldl, int dtype,
                          void *X, int64_t ldx, int32_t *d_status, void *stream);

/*
 * The deferred update on its own (Sec. 2: S = R R^T, then A -= S over the
 * trailing square), the library's hot kernel, exposed for tests and timing.
 *   ff_update_syrk: C -= P P^T on the lower triangle (i >= j) of the m x m C;
 *                   P is m x w.  The strict upper triangle of C is untouched.
 *   ff_update_gemm: C -= X Y on all of the m x m C; X is m x w, Y is w x m
 *                   (Algorithm 2's S = R_L R_U).
 * C and the operands share the storage type of dtype (double for FF_F64,
 * float otherwise).  Operands must not overlap C.  Asynchronous.
 */
int ff_update_syrk(int64_t m, int64_t w, void *C, int64_t ldc, const void *P, int64_t ldp,
                   int dtype, unsigned flags, void *stream);
int ff_update_gemm(int64_t m, int64_t w, void *C, int64_t ldc, const void *X, int64_t ldx,
                   const void *Y, int64_t ldy, int dtype, unsigned flags, void *stream);

/*
 * Measurement aid (not part of the method): while enabled, every trailing
 * update launched by chol_factor on the caller's stream is bracketed by a pair
 * of HIP events recorded on that stream, and tallied by the kernel that ran:
 * for binary64 by kernel shape, FF_UPD_SHAPE_64 (64 x 64 tiles),
 * FF_UPD_SHAPE_128 (128 x 128 tiles, two workgroups per CU) and
 * FF_UPD_SHAPE_256x128 (256 x 128 tiles, one workgroup per CU: the lookahead
 * update); FF_UPD_SHAPE_F32 and FF_UPD_SHAPE_BF16 collect the binary32 and the
 * bfloat16-operand updates of every shape.  Events are created per launch, so
 * leave it off outside timing runs.
 *   ff_update_profile_enable(1) clears the tallies and starts recording;
 *   ff_update_profile_enable(0) stops recording (tallies are kept).
 *   ff_update_profile_read waits for the recorded events and fills out[shape];
 *   flops are the algorithmic 2 K x (entries written) of each launch, bytes
 *   its algorithmic HBM traffic (each entry written read and written once, the
 *   M x K panel rows of the region read once, at the storage element size).
 *   Host-synchronous; the tallies are process-wide.  Returns 0 or FF_ERR_HIP.
 */
enum { FF_UPD_SHAPE_64 = 0, FF_UPD_SHAPE_128 = 1, FF_UPD_SHAPE_256x128 = 2, FF_UPD_SHAPE_F32 = 3,
       FF_UPD_SHAPE_BF16 = 4, FF_UPD_NSHAPES = 5 };
typedef struct {
    int64_t launches;
    double total_ms;
    double total_flops;
    double total_bytes;
} ff_kernel_profile;
int ff_update_profile_enable(int enable);
int ff_update_profile_read(ff_kernel_profile out[FF_UPD_NSHAPES]);

/*
 * Serving: many independent SPD systems A_i X_i = B_i (binary64 A, B, X), each
 * factored by Algorithm 1 (Sec. 2) with step s = min(n, 192) (the widest
 * diagonal block one workgroup factors) and solved with the factor.  A server
 * keeps every admitted factorisation in flight: each ff_server_step advances
 * all of them by one block of s columns with three grouped launches (the
 * diagonal blocks of every matrix, then their panel solves, then their trailing
 * updates), and starts the solves of those that finished.  Factors live in the
 * caller's device arena; a finished factor stays resident under its nonzero
 * key, so a later request with the same key (and n) is solved without
 * refactoring (a cache hit).  Requests are admitted in arrival order while the
 * arena has room for the factor and the solve workspace, evicting least
 * recently used resident factors that no request is using.
 *
 * Precision (dtype at creation):
 *   FF_F64  binary64 factors (8 n^2 bytes), one forward and one back solve;
 *   FF_F32  binary32 factors (4 n^2 bytes; diagonal blocks factored in
 *           binary64, panel solves and updates in binary32) and binary64
 *           iterative refinement against the request's A: an iteration is
 *           enqueued per scheduler iteration after the previous one's
 *           correction ||dX||_inf / ||X||_inf has reached the host; it stops at
 *           <= 1e-12, on stagnation (the correction shrank by less than half)
 *           or after 30 iterations.  The request's A must stay valid until it
 *           is returned (it is read by every iteration, also on a cache hit).
 *   FF_BF16 is not served (FF_ERR_UNSUPPORTED).
 *
 *   ff_server_create: arena = device buffer of arena_bytes (the HBM budget),
 *     owned by the caller and untouched by anything else while the server
 *     lives; stream = HIP stream for all server work.  Returns NULL on error
 *     (*status < 0).  The server allocates its own small job tables and pinned
 *     host slots.
 *   ff_server_submit: A (lda >= n), B and X (n x nrhs, ldb, ldx >= n) are
 *     device buffers that must stay valid, and B / A unmodified, until the
 *     request is returned by ff_server_poll; key = 0 means never cache.
 *     The arrival time is stamped when submit is called.  Returns 0,
 *     -(argument index) or FF_ERR_WORKSPACE if the request can never fit.
 *   ff_server_step: one scheduler iteration (admission, one block step of
 *     every active factorisation, solves and refinement decisions).  Enqueues
 *     only, except that it waits for the step 4 iterations back before reusing
 *     its job table.  Returns the number of requests not yet finished (>= 0),
 *     or an error (FF_ERR_WORKSPACE if the oldest queued request cannot be
 *     admitted although nothing runs).
 *   ff_server_poll: up to max_out finished requests (their work has completed
 *     on the device): id, info (as chol_factor's; FF_ERR_HIP if a bounded wait
 *     of the triangular solves expired), cache_hit, latency_ms (device time
 *     from the submit stamp to the end of the solve), iters and converged (the
 *     refinement of FF_F32 servers; 0 for FF_F64).  A request whose
 *     factorisation failed reports info > 0 and its X is unspecified.
 *     Non-blocking.
 * A server is not thread safe; use one per host thread.
 */
typedef struct ff_server ff_server;
typedef struct {
    int64_t id;
    int32_t info;
    int32_t cache_hit;
    double latency_ms;
    int32_t iters;
    int32_t converged;
} ff_server_result;
typedef struct {
    int64_t submitted, completed, steps, grouped_launches, cache_hits, evictions;
    int64_t arena_free, resident_factors, queued, active;
} ff_server_stats;
ff_server *ff_server_create(void *arena, size_t arena_bytes, int dtype, void *stream, int *status);
int ff_server_destroy(ff_server *srv);
int ff_server_submit(ff_server *srv, uint64_t key, int64_t n, const double *A, int64_t lda, const double *B,
                     int64_t nrhs, int64_t ldb, double *X, int64_t ldx, int64_t *req_id);
int ff_server_step(ff_server *srv);
int ff_server_poll(ff_server *srv, ff_server_result *out, int max_out, int *n_out);
int ff_server_get_stats(ff_server *srv, ff_server_stats *out);

#ifdef __cplusplus
}
#endif
#endif /* FASTFACT_H */
