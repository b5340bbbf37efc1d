// internal.hpp -- launchers shared between the kernel files and the host driver.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ff {

// Largest diagonal blocks the single-workgroup diagonal kernels take, the block
// held in LDS (Cholesky: its lower triangle; LU: the whole square); larger
// blocks are factored recursively by the host driver.  TRSM_MAX bounds the
// columns of one panel-solve launch; wider panels are solved in column chunks
// by the host.
constexpr int LDS_DIAG_MAX = 192;
constexpr int LU_LDS_MAX = 128;
constexpr int TRSM_MAX = 192;

hipError_t launch_set_int(int* p, int v, hipStream_t st);

// QR (qr.hip).  In-block modified Gram-Schmidt of w columns of Mp (m rows) on
// co-resident workgroups of qr_panel_rows(m) rows each (0: m too large);
// w <= qr_panel_max_width(m).  part: qr_panel_part_elems(m, w) doubles of
// hand-off slots, filled with the sentinel by launch_qr_part_clear once before
// the first panel of a factorisation (panels take increasing col0); info: 0 on
// entry or the kernel does nothing; set to col0 + j + 1 when column j's norm is
// not > 0, to -1 when a wait between the workgroups expired.
constexpr int QR_PANEL_LDS_DOUBLES = 18432;   // 144 KB of LDS per workgroup
constexpr int QR_PANEL_WMAX = 256;
constexpr int QR_PANEL_MAXWG = 256;
hipError_t launch_qr_part_clear(int64_t m, double* part, hipStream_t st);
int qr_panel_rows(int64_t m);
int qr_panel_max_width(int64_t m);
size_t qr_panel_part_elems(int64_t m, int w);
hipError_t launch_qr_panel(int m, int w, int col0, double* Mp, int64_t ldm, double* part, int* info, hipStream_t st);
// D = X^T Y (M x N) with X(k, i) = X[k + i*ldx], Y(k, j) = Y[k + j*ldy], k < K.
// upper: M == N and only the upper triangle is formed, the strict lower
// triangle of D is set to zero.  part: tn_gemm_part_elems(M, N, K, upper)
// doubles (may be null when that is 0).  Nothing happens when *info != 0.
// max_wg > 0: at most that many workgroups walk the tiles (no K split, part
// unused), so that the launch leaves the other CUs to concurrent work.
size_t tn_gemm_part_elems(int M, int N, int K, bool upper);
bool tn_gemm_fits(int64_t K, int64_t ldx, int64_t ldy);
hipError_t launch_tn_gemm(int M, int N, int K, const double* X, int64_t ldx, const double* Y, int64_t ldy, double* D,
                          int64_t ldd, bool upper, double* part, const int* info, hipStream_t st, int max_wg = 0);
int qr_panel_workgroups(int64_t m);
// R = Q^T A by slabs (qr.hip): tiles of r_slab_tile() x r_slab_tile() in the upper
// triangle of R's tile grid, numbered row by row (tile row r holds the tiles
// (r, r) ... (r, T - 1)); r_slab_tiles_before(n, rows) counts the tiles of the
// first `rows` tile rows.  launch_r_slab forms tiles [t0, t1) over the K range
// [k0, k1): stored when k0 == 0, added otherwise (the earlier K ranges of those
// tiles must precede it in stream order); at most max_wg workgroups (0: one per
// tile).  Entries below the diagonal are not written.
int r_slab_tile();
int64_t r_slab_tiles_before(int n, int rows);
hipError_t launch_r_slab(int n, int64_t t0, int64_t t1, int k0, int k1, const double* Q, int64_t ldq, const double* A,
                         int64_t lda, double* R, int64_t ldr, const int* info, hipStream_t st, int max_wg);
hipError_t launch_zero_strict_lower(int n, double* D, int64_t ldd, const int* info, hipStream_t st);
hipError_t launch_copy_int(const int* src, int* dst, hipStream_t st);

// Trailing updates (update.hip).
// C(i, j) -= sum_k X(i, k) Y(j, k) for i < M, j < N; X column-major M x K;
// Y(j, k) = Y[j + k*ldy] when yrows, else Y[k + j*ldy]; with `lower` only
// entries with i - j >= shift are written.  `info` (may be null): the kernels do
// nothing when *info != 0.  reserve_cus: number of CUs the (persistent) update
// leaves free for work on other streams.  max_cus (> 0): the launch sizes its
// grid for that many CUs (work on a stream that owns only the reserved CUs).
// [f0, f1): the part of the region's tile order this launch covers (two launches
// with the same shape arguments and adjoining ranges cover the region once);
// hipErrorInvalidValue when the region is too small to have a split order.
template <typename T>
hipError_t launch_update(int M, int N, int K, T* C, int64_t ldc, const T* X, int64_t ldx, const T* Y, int64_t ldy,
                         bool yrows, bool lower, int shift, const int* info, hipStream_t st, int reserve_cus = 0,
                         int max_cus = 0, double f0 = 0.0, double f1 = 1.0);
// bfloat16-operand form (yrows only), binary32 storage and accumulation.
hipError_t launch_update_bf16(int M, int N, int K, float* C, int64_t ldc, const float* X, int64_t ldx,
                              const float* Y, int64_t ldy, bool lower, int shift, const int* info, hipStream_t st,
                              int reserve_cus = 0);
// The same from a transposed bfloat16 copy of the panel: launch_panel_bf16t
// writes Pt[r * bf16t_width(w) + k] = bf16(P[r + k*ldp]) (zero-padded K) for
// r < m; launch_update_bf16t then takes X rows from Xt and Y rows from Yt
// (pointers into that copy, a row of bf16t_width(w) values each).
int bf16t_width(int w);
hipError_t launch_panel_bf16t(int m, int w, const float* P, int64_t ldp, __bf16* Pt, hipStream_t st);
hipError_t launch_update_bf16t(int M, int N, int w, float* C, int64_t ldc, const __bf16* Xt, const __bf16* Yt,
                               bool lower, int shift, const int* info, hipStream_t st, int reserve_cus = 0);
// Persistent workgroups an update launch uses when reserve_cus CUs are kept free.
int update_workers(int reserve_cus);
// Kernel shape launch_update picks for an M x N region (FF_UPD_SHAPE_*).
int update_shape(int M, int N, int reserve_cus);
// Whether launch_update can split that region's tile order ([f0, f1) ranges).
bool update_splittable(int M, int N, bool lower, int shift, int reserve_cus);
// Entries of C that the [f0, f1) part of that split order writes (-1: no split order).
double update_range_entries(int M, int N, bool lower, int shift, int reserve_cus, double f0, double f1);
// Tiles in that split order (0: no split order).
int update_order_tiles(int M, int N, bool lower, int shift, int reserve_cus);
// One Strassen level over 128 x 128 super-tiles of 64 x 64 quadrants
// (strassen.hip): C -= P P^T on the lower triangle of the m x m C (P m x w), or
// C -= X Y on all of it (X m x w, Y w x m column-major).  One workgroup per CU on
// all but reserve_cus CUs.
hipError_t launch_update_syrk_strassen_f64(int m, int w, double* C, int64_t ldc, const double* P, int64_t ldp,
                                           const int* info, hipStream_t st, int reserve_cus = 0);
// Two Strassen levels for the LU product (a matrix-level level over the
// one-level kernel) once m >= STRASSEN2_MIN_M; ws: strassen2_ws_doubles(m, w).
constexpr int STRASSEN2_MIN_M = 2048;
size_t strassen2_ws_doubles(int m, int w);
hipError_t launch_update_gemm_strassen2_f64(int m, int w, double* C, int64_t ldc, const double* X, int64_t ldx,
                                            const double* Y, int64_t ldy, double* ws, const int* info, hipStream_t st,
                                            int reserve_cus = 0);
hipError_t launch_update_gemm_strassen_f64(int m, int w, double* C, int64_t ldc, const double* X, int64_t ldx,
                                           const double* Y, int64_t ldy, const int* info, hipStream_t st,
                                           int reserve_cus = 0);

// Job tables of the grouped (many-matrix) kernels, device resident.  Matrix
// pointers are untyped: the launch's storage type S (double or float) gives
// their element type.
//   GroupDiag: factor the w x w block at a (binary64 arithmetic, w <= LDS_DIAG_MAX).
//   GroupTrsm: solve the m x w panel x against the factored block t (both with
//              leading dimension ld); workgroups [wg_begin, wg_begin + nwg).
//   GroupUpd:  c -= p p^T on the lower triangle of the m x m square c, p m x w;
//              lower-triangle 128 x 128 tiles [tiles_begin, tiles_begin + tiles).
struct GroupDiag {
    void* a;
    int64_t ld;
    int w;
    int col_base;
    int* info;
};
struct GroupTrsm {
    void* x;
    const void* t;
    int64_t ld;
    int m, w;
    int wg_begin, nwg;
    const int* info;
};
struct GroupUpd {
    void* c;
    const void* p;
    int64_t ld;
    int m, w;
    int tiles_begin;
    const int* info;
};
template <typename S>
hipError_t launch_potrf_grouped(int njobs, const GroupDiag* d_jobs, hipStream_t st);
template <typename S>
hipError_t launch_trsm_grouped(int njobs, int total_wg, const GroupTrsm* d_jobs, hipStream_t st);
int trsm_rows_per_wg();
template <typename S>
hipError_t launch_update_grouped(int njobs, int total_tiles, const GroupUpd* d_jobs, hipStream_t st);
int grouped_update_tile();

// Diagonal factorisations and panel solves (panel.hip).
template <typename S>
hipError_t launch_potrf_diag(int w, S* blk, int64_t ldb, int* info, int col_base, hipStream_t st);
hipError_t launch_getrf_lds(int w, double* a, int64_t ld, int* info, int col_base, hipStream_t st);
template <typename T>
hipError_t launch_trsm(int m, int w, T* x, int64_t xi, int64_t xj, const T* t, int64_t tk, int64_t tj,
                       int unit, const int* info, hipStream_t st, int max_wg = 0);

// Solve-side kernels (solve.hip).
template <typename S>
hipError_t launch_copy_lower_from_f64(int n, const double* A, int64_t lda, S* W, int64_t ldw, hipStream_t st);
template <typename S>
hipError_t launch_convert_from_f64(int n, int nrhs, const double* B, int64_t ldb, S* X, int64_t ldx, hipStream_t st);
// Triangular solves with a Cholesky factor (solve.hip).  X = L^-T L^-1 X in
// place, 64-row blocks, at most TRI_RC right-hand sides per sweep.  Memory:
//   fac   per-factor data, trisolve_fac_elems(n) elements of the factor's
//         type: the inverses of the 64 x 64 diagonal blocks, the same
//         transposed, and the tiles L(j, j-f) and L(j+f, j)^T, f = 1..TRI_F,
//         that the solving workgroup folds itself, all laid out in the order
//         its threads read them.  Formed when make_fac is set, reusable while
//         L is unchanged.
//   pub   hand-off area of trisolve_pub_elems(n) elements (solved blocks and
//         partial sums, pre-filled with a sentinel before every sweep).
//   ctl   TRI_CTL ints: [0] error word (nonzero once a bounded wait of any
//         sweep expired; never cleared here, callers clear it once per call),
//         [1, 1 + TRI_GROUPS) and [1 + TRI_GROUPS, 1 + 2 TRI_GROUPS) the two
//         sweeps' workgroup tickets, one per group of right-hand sides.
// One right-hand side is solved by one chain of workgroups; 2..16 by
// independent chains of 2 columns in the same launch (binary64 with more than
// 8 right-hand sides: chains of 4, fewer chains re-reading L).
constexpr int TRI_TB = 64;          // row block
constexpr int TRI_RC = 16;          // right-hand sides per sweep
constexpr int TRI_F = 2;            // newest solved blocks the solving workgroup folds itself
constexpr int TRI_GC = 2;           // right-hand sides per chain when several chains run (narrowest)
constexpr int TRI_GC_WIDE = 4;      // the same for binary64 with more than 8 right-hand sides
constexpr int TRI_GROUPS = TRI_RC / TRI_GC;
constexpr int TRI_CTL = 1 + 2 * TRI_GROUPS;
constexpr int RESIDUAL_SEG = 4;     // 64-row blocks per residual segment (side of a workgroup's tile square)
inline int trisolve_nblk(int n) { return (n + TRI_TB - 1) / TRI_TB; }
inline size_t trisolve_fac_elems(int n) { return (size_t)trisolve_nblk(n) * (2 + 2 * TRI_F) * TRI_TB * TRI_TB; }
inline size_t trisolve_pub_elems(int n) { return (size_t)4 * trisolve_nblk(n) * TRI_TB * TRI_RC; }
template <typename S>
struct TriWs {
    int* ctl;
    S* fac;
    S* pub;
};
template <typename S>
hipError_t trisolve_impl(int n, int nrhs, const S* L, int64_t ldl, S* X, int64_t ldx, const TriWs<S>& w,
                         bool make_fac, hipStream_t st);
// part: residual_part_doubles(n) doubles of scratch (two partial sums per
// segment of RESIDUAL_SEG row blocks, for 16 right-hand sides and the absolute
// row sums).
inline int residual_segments(int n) { return (trisolve_nblk(n) + RESIDUAL_SEG - 1) / RESIDUAL_SEG; }
inline size_t residual_part_doubles(int n) { return 17 * ((size_t)residual_segments(n) + 1) * (size_t)n; }
hipError_t launch_residual_f64(int n, int nrhs, const double* A, int64_t lda, const double* X, int64_t ldx,
                               const double* B, int64_t ldb, double* R, int64_t ldr, double* rowsum, double* part,
                               hipStream_t st);
template <typename S>
hipError_t launch_axpy_update(int n, int nrhs, const S* D, int64_t ldd, double* X, int64_t ldx, hipStream_t st);
// X += D, out[0] = max|D|, out[1] = max|X|.
template <typename S>
hipError_t launch_axpy_max(int n, int nrhs, const S* D, int64_t ldd, double* X, int64_t ldx, double* out,
                           hipStream_t st);
template <typename S>
hipError_t launch_widen(int n, int nrhs, const S* D, int64_t ldd, double* X, int64_t ldx, hipStream_t st);
template <typename S>
hipError_t launch_widen_lower(int w, const S* a, int64_t lda, double* d, int64_t ldd, hipStream_t st);
template <typename S>
hipError_t launch_narrow_lower(int w, const double* d, int64_t ldd, S* a, int64_t lda, hipStream_t st);
hipError_t launch_norms(int n, int nrhs, const double* rowsum, const double* X, int64_t ldx, const double* D,
                        int64_t ldd, const double* R, int64_t ldr, const double* B, int64_t ldb, double* out,
                        hipStream_t st);

// GMRES pieces (solve.hip): Krylov basis V n x k (k <= 32) column-major binary64.
// GMRES pieces, batched over nc columns: column c's basis is V + c*vs (ld ldv),
// its vectors w + c*ws, its scalars out / h / sq + c*os (hs, ss).
// out_c[i] = V_c[:, i] . w_c, i < k <= 32 (part: nc * multidot_part_doubles(n)
// doubles of scratch); w_c += alpha V_c h_c; y_c = x_c / sqrt(sq_c) (sq_c > 0);
// y_c = -x_c.
size_t multidot_part_doubles(int n);
hipError_t launch_multidot(int n, int nc, int k, const double* V, int64_t ldv, int64_t vs, const double* w, int64_t ws,
                           double* part, double* out, int64_t os, hipStream_t st);
hipError_t launch_gemv_add(int n, int nc, int k, const double* V, int64_t ldv, int64_t vs, const double* h,
                           int64_t hs, double alpha, double* w, int64_t ws, hipStream_t st);
hipError_t launch_normalize(int n, int nc, const double* x, int64_t xs, const double* sq, int64_t ss, double* y,
                            int64_t ys, hipStream_t st);
hipError_t launch_negate(int n, int nc, const double* x, int64_t xs, double* y, int64_t ys, hipStream_t st);
// X += D with per-column norms out[2j] = max|D_j|, out[2j + 1] = max|X_j|.
template <typename S>
hipError_t launch_axpy_max_cols(int n, int nrhs, const S* D, int64_t ldd, double* X, int64_t ldx, double* out,
                                hipStream_t st);
hipError_t launch_fill_double(int n, double* y, double v, hipStream_t st);

}  // namespace ff
