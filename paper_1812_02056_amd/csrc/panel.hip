// panel.hip -- the per-block steps between two deferred updates.
//
// Sec. 2 of arXiv 1812.02056, Algorithm 1: after an update, the next s columns
// are formed Crout-style from the updated matrix and the columns pending since
// the update:
//     L[c,c] = sqrt(A[c,c] - sum_{k=z}^{c-1} L[c,k]^2)
//     L[i,c] = (A[i,c] - sum_{k=z}^{c-1} L[i,k] L[c,k]) / L[c,c]      (i > c)
// For the w pending columns of one block, the rows inside the block form the
// w x w diagonal factorisation (potrf_lds_kernel) and the rows below it are a
// triangular solve L21 = A21 L11^-T (trsm_reg_kernel, rows independent).
// Algorithm 2 (LU) splits the same way into getrf_lds_kernel and two
// triangular solves L21 = A21 U11^-1 and U12 = L11^-1 A12.
//
// Both diagonal kernels run in ONE workgroup that holds the block in LDS as
// 16 x 16 tiles and factors it right-looking over tile columns (potrf_block,
// getrf_lds_kernel).  Diagonal blocks are always binary64; for binary32 storage
// they are widened into a workspace, factored, and rounded back.
#include <math.h>

#include "common.hpp"
#include "internal.hpp"

namespace ff {

namespace {

__global__ void set_int_kernel(int* p, int v) { if (threadIdx.x == 0) *p = v; }
__global__ void copy_int_kernel(const int* src, int* dst) { if (threadIdx.x == 0) *dst = *src; }

// value of v in lane l (l uniform across the wave)
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)bits, l);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// ---------------------------------------------------------------------------
// MFMA output layout of a 16 x 16 tile: for the transposed tile D'[a][b] = M(b, a),
// lane l holds row b = l % 16 and, in register r, column a = acc_traits<T>::col(l, r).
template <typename T>
__device__ __forceinline__ int tcol(int lane, int r) { return acc_traits<T>::col(lane, r); }

// Row-layout 16 x 16 tile primitives: lane l holds row i = l % 16 of the tile in
// x[0..15] (x[c] = M(i, c)); the four lane groups hold the same rows and do the
// same work, so only lanes 0..15 need to store.


// In-register Cholesky of a 16 x 16 tile in row layout (lane l holds row
// i = l % 16), with the rows of L^-T formed alongside.  Column j: the pivot
// d = M(j, j) is read from lane j, L(j, j) = sqrt(d) (returned in ljj[j]), every row
// is scaled by the correctly rounded reciprocal r_j = 1 / L(j, j), and
// M(i, c) -= L(i, j) L(c, j) for c > j, L(c, j) read from lane c.  Every entry below
// the diagonal receives exactly these operations; the diagonal and the entries
// above it are left with meaningless values (the caller stores ljj), and nothing
// else reads them, so no lane masks are needed.
// y enters as row i of the identity and leaves as row i of L^-T: the row-wise
// substitution y L^T = e_i takes column j's step (y_j *= r_j, then
// y_c -= y_j L(c, j) for c > j) with the same broadcast values.
// Returns the first column j whose pivot was not > 0, or -1 (uniform).
__device__ __forceinline__ int row_potrf(double (&x)[16], double (&y)[16], double (&ljj)[16]) {
    int bad = -1;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const double d = readlane_f64(x[j], j);
        if (!(d > 0.0) && bad < 0) bad = j;
        ljj[j] = sqrt(d);
        const double rj = 1.0 / ljj[j];
        const double lij = x[j] * rj;
        x[j] = lij;
        y[j] = y[j] * rj;
#pragma unroll
        for (int c = j + 1; c < 16; ++c) {
            const double lcj = readlane_f64(lij, c);
            x[c] -= lij * lcj;
            y[c] -= y[j] * lcj;
            // y is stored only at the end: without this the compiler sinks its
            // updates there, and the 120 broadcasts they need exhaust the
            // scalar registers
            asm volatile("" : "+v"(y[c]));
        }
    }
    return bad;
}

// ---------------------------------------------------------------------------
// Cholesky of the w x w diagonal block (w <= LDS_DIAG_MAX) in ONE workgroup of
// 1024 threads.  The lower triangle is held in LDS as 16 x 16 tiles (tile (i, j),
// i >= j, at index i(i+1)/2 + j, element (r, c) at r + 16 c) padded with the
// identity beyond w, and factored right-looking over tile columns: the waves
// solve the tiles below the factored diagonal tile, then update the trailing
// tiles with 16 x 16 x 16 MFMA products.  Wave 0 updates the next diagonal tile
// first and factors it while the other waves finish the trailing update, so the
// serial diagonal factorisation overlaps the update of the step before.  S is the
// storage type; the arithmetic is binary64 in every case.
constexpr int DT = 16;
constexpr int LDS_TMAX = LDS_DIAG_MAX / DT;
constexpr int LDS_NTILE = LDS_TMAX * (LDS_TMAX + 1) / 2;
constexpr int PT = 1024;
constexpr int PW = PT / 64;

__device__ __forceinline__ int ltile(int i, int j) { return (i * (i + 1) / 2 + j) * 256; }

// Staging and write-back of the block: the PT / 256 thread quarters take every
// fourth tile, so PSTG slots per thread cover the largest block and all its
// global loads are in flight at once.
constexpr int PSTG = (LDS_NTILE + PT / 256 - 1) / (PT / 256);

// (i, j) of packed lower-triangle tile t + 4, given (i, j) of tile t
__device__ __forceinline__ void tile_step4(int& i, int& j) {
    j += 4;
    while (j > i) { j -= i + 1; ++i; }
}

// Orders this wave's LDS stores before its later LDS loads from other lanes.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// c -= li lj^T for 16 x 16 tiles in LDS (one wave, MFMA layout)
__device__ __forceinline__ void tile_syrk(double* c, const double* li, const double* lj, int lane) {
    const int b = lane & 15;
    d4_t acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = c[b + 16 * tcol<double>(lane, r)];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int k = tcol<double>(lane, i);
        acc = mfma_f64(-lj[b + 16 * k], li[b + 16 * k], acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) c[b + 16 * tcol<double>(lane, r)] = acc[r];
}

// Factors diagonal tile kt in place (one wave) and leaves Y = L_kk^-T in yt
// (Y(r, c) at c + 16 r).  A pivot that is not > 0 sets fail and, inside the block,
// the info word.
__device__ __forceinline__ void diag_tile(double* tl, int kt, double* yt, int* fail, int lane, int w,
                                          int* info, int col_base) {
    double* dtile = tl + ltile(kt, kt);
    const int b = lane & 15;
    // the identity row is formed here, not kept from an earlier step: hoisted out
    // of the caller's loop, its 16 lane masks would take 32 scalar registers
    int bi = b;
    asm volatile("" : "+v"(bi));
    double x[16], y[16], ljj[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        x[c] = dtile[b + 16 * c];
        y[c] = bi == c ? 1.0 : 0.0;
    }
    const int bad = row_potrf(x, y, ljj);
    if (lane < 16) {
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            dtile[b + 16 * c] = x[c];
            yt[c + 16 * b] = y[c];
        }
    }
    // the diagonal, over what the row stores left there (LDS operations of one
    // wave complete in order)
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < 16; ++j) dtile[17 * j] = ljj[j];
        if (bad >= 0) {
            *fail = bad;
            if (DT * kt + bad < w) *info = col_base + DT * kt + bad + 1;
        }
    }
}

// t <- t Y for a 16 x 16 tile t in LDS (one wave, MFMA layout); yt as above
__device__ __forceinline__ void tile_mul_yt(double* t, const double* yt, int lane) {
    const int b = lane & 15;
    d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int k = tcol<double>(lane, s);
        acc = mfma_f64(yt[b + 16 * k], t[b + 16 * k], acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) t[b + 16 * tcol<double>(lane, r)] = acc[r];
}

template <typename S>
__device__ __forceinline__ void potrf_block(int w, S* __restrict__ blk, int64_t ldb, int* info, int col_base)
{
    if (*info != 0) return;
    __shared__ double tl[LDS_NTILE * 256];
    __shared__ double yt[256];        // L_kk^-T of the last factored diagonal tile
    __shared__ int fail;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int T = (w + DT - 1) / DT;
    const int ntile = T * (T + 1) / 2;
    // thread's entry rc of tiles q0 + 4u; (i0, j0) is tile q0 (q0 < 4)
    const int rc = tid & 255, q0 = wave >> 2;
    const int i0 = q0 == 0 ? 0 : (q0 == 3 ? 2 : 1), j0 = q0 - i0 * (i0 + 1) / 2;
    if (tid == 0) fail = -1;
    // Stage the lower triangle.  Entries outside the block read a valid address
    // and are replaced by the identity.
    {
        double v[PSTG];
        int i = i0, j = j0;
#pragma unroll
        for (int u = 0; u < PSTG; ++u) {
            if (q0 + 4 * u < ntile) {
                const int gr = DT * i + (rc & 15), gc = DT * j + (rc >> 4);
                const bool in = gr < w && gc < w && gr >= gc;
                const double x = (double)blk[in ? gr + (int64_t)gc * ldb : 0];
                v[u] = in ? x : (gr == gc ? 1.0 : 0.0);
            }
            tile_step4(i, j);
        }
#pragma unroll
        for (int u = 0; u < PSTG; ++u)
            if (q0 + 4 * u < ntile) tl[(q0 + 4 * u) * 256 + rc] = v[u];
    }
    __syncthreads();
    if (wave == 0) diag_tile(tl, 0, yt, &fail, lane, w, info, col_base);
    __syncthreads();
    for (int kt = 0; kt + 1 < T; ++kt) {
        if (fail >= 0) return;
        // tiles below: X L_kk^T = A, i.e. X = A L_kk^-T, one wave per tile
        for (int it = kt + 1 + wave; it < T; it += PW) tile_mul_yt(tl + ltile(it, kt), yt, lane);
        __syncthreads();
        // trailing tiles (it, jt), kt < jt <= it: A -= L_it,kt L_jt,kt^T.  Pair p = 0
        // is the next diagonal tile: wave 0 updates and factors it, the other waves
        // take the remaining pairs.
        if (wave == 0) {
            tile_syrk(tl + ltile(kt + 1, kt + 1), tl + ltile(kt + 1, kt), tl + ltile(kt + 1, kt), lane);
            wave_lds_sync();
            diag_tile(tl, kt + 1, yt, &fail, lane, w, info, col_base);
        } else {
            const int nr = T - kt - 1;
            const int npair = nr * (nr + 1) / 2;
            for (int p = wave; p < npair; p += PW - 1) {
                const int ii = tri_row(p);
                const int jj = p - ii * (ii + 1) / 2;
                const int it = kt + 1 + ii, jt = kt + 1 + jj;
                tile_syrk(tl + ltile(it, jt), tl + ltile(it, kt), tl + ltile(jt, kt), lane);
            }
        }
        __syncthreads();
    }
    if (fail >= 0) return;
    {
        double v[PSTG];
#pragma unroll
        for (int u = 0; u < PSTG; ++u)
            if (q0 + 4 * u < ntile) v[u] = tl[(q0 + 4 * u) * 256 + rc];
        int i = i0, j = j0;
        // walked again rather than kept from the staging loop, where the 2 PSTG
        // tile coordinates would hold scalar registers through the whole kernel
        asm volatile("" : "+s"(i), "+s"(j));
#pragma unroll
        for (int u = 0; u < PSTG; ++u) {
            if (q0 + 4 * u < ntile) {
                const int gr = DT * i + (rc & 15), gc = DT * j + (rc >> 4);
                if (gr < w && gc < w && gr >= gc) blk[gr + (int64_t)gc * ldb] = (S)v[u];
            }
            tile_step4(i, j);
        }
    }
}

// ---------------------------------------------------------------------------
// LU (Doolittle, no pivoting) of the w x w diagonal block, w <= LU_LDS_MAX, in
// ONE workgroup, the block held in LDS as 16 x 16 tiles (tile (i, j) at index
// i * LU_TMAX + j, element (r, c) at r + 16 c) padded with the identity beyond w.
// Right-looking over tile columns: one wave factors the diagonal tile, forming
// U_kk^-1 and L_kk^-1 alongside; the waves solve the tiles below (A U_kk^-1) and
// to the right (L_kk^-1 A) with one MFMA product each, then update the trailing
// tiles; wave 0 updates the next diagonal tile first and factors it while the
// other waves finish the update.
constexpr int LU_TMAX = LU_LDS_MAX / DT;
constexpr int LU_PT = 512;
constexpr int LU_PW = LU_PT / 64;
constexpr int LSTG = LU_TMAX * LU_TMAX / (LU_PT / 256);

__device__ __forceinline__ int utile(int i, int j) { return (i * LU_TMAX + j) * 256; }

// In-register LU of a 16 x 16 tile in row layout (lane l holds row i = l % 16 in
// x; bi is i), with the rows of U^-1 (in z) and of L^-T (in y) formed alongside.
// Column j: the pivot u = U(j, j) and U's row j are read from lane j, and rows
// i > j take l = x_j / u, x_k -= l U(j, k) for k > j.  z enters as row i of the
// identity and takes column j's step of z U = e_i (z_j /= u, z_k -= z_j U(j, k));
// y enters as row i of the identity and takes column j's step of y L^T = e_i
// (y_c -= y_j L(c, j) for c > j, L(c, j) read from lane c).  Returns the first
// column whose pivot was zero or not finite, or -1 (uniform across the wave).
__device__ __forceinline__ int row_getrf(double (&x)[16], double (&z)[16], double (&y)[16], int bi) {
    int bad = -1;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if (bad < 0) {
            const double u = readlane_f64(x[j], j);
            if (u == 0.0 || !isfinite(u)) {
                bad = j;
            } else {
                double ur[16];
#pragma unroll
                for (int k = j + 1; k < 16; ++k) ur[k] = readlane_f64(x[k], j);
                z[j] = z[j] / u;
#pragma unroll
                for (int k = j + 1; k < 16; ++k) {
                    z[k] -= z[j] * ur[k];
                    // kept next to its broadcast (sunk to the end, the
                    // broadcasts it needs exhaust the scalar registers)
                    asm volatile("" : "+v"(z[k]));
                }
                if (bi > j) {
                    const double l = x[j] / u;
                    x[j] = l;
#pragma unroll
                    for (int k = j + 1; k < 16; ++k) x[k] -= l * ur[k];
                }
#pragma unroll
                for (int c = j + 1; c < 16; ++c) {
                    y[c] -= y[j] * readlane_f64(x[j], c);
                    asm volatile("" : "+v"(y[c]));
                }
            }
        }
    }
    return bad;
}

// Factors diagonal tile kt in place (one wave) and leaves Z = U_kk^-1 in zt
// (Z(r, c) at c + 16 r) and W = L_kk^-1 in wt (W(r, c) at r + 16 c).  A pivot
// that is zero or not finite sets fail and, inside the block, the info word.
__device__ __forceinline__ void lu_diag_tile(double* tl, int kt, double* zt, double* wt, int* fail, int lane, int w,
                                             int* info, int col_base) {
    double* dtile = tl + utile(kt, kt);
    const int b = lane & 15;
    // lane masks are formed here, not kept across the caller's loop
    int bi = b;
    asm volatile("" : "+v"(bi));
    double x[16], z[16], y[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        x[c] = dtile[b + 16 * c];
        z[c] = bi == c ? 1.0 : 0.0;
        y[c] = z[c];
    }
    const int bad = row_getrf(x, z, y, bi);
    if (lane < 16) {
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            dtile[b + 16 * c] = x[c];
            zt[c + 16 * b] = z[c];
            wt[c + 16 * b] = y[c];
        }
    }
    if (lane == 0 && bad >= 0) {
        *fail = bad;
        if (DT * kt + bad < w) *info = col_base + DT * kt + bad + 1;
    }
}

// t <- W t for a 16 x 16 tile t in LDS (one wave, MFMA layout); wt as above
__device__ __forceinline__ void tile_lmul_wt(double* t, const double* wt, int lane) {
    const int b = lane & 15;
    d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int k = tcol<double>(lane, s);
        acc = mfma_f64(t[k + 16 * b], wt[b + 16 * k], acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) t[b + 16 * tcol<double>(lane, r)] = acc[r];
}

// c -= l u for 16 x 16 tiles in LDS (one wave, MFMA layout)
__device__ __forceinline__ void tile_gemm_sub(double* c, const double* l, const double* u, int lane) {
    const int b = lane & 15;
    d4_t acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = c[b + 16 * tcol<double>(lane, r)];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int k = tcol<double>(lane, s);
        acc = mfma_f64(-u[k + 16 * b], l[b + 16 * k], acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) c[b + 16 * tcol<double>(lane, r)] = acc[r];
}

__global__ __launch_bounds__(LU_PT)
void getrf_lds_kernel(int w, double* __restrict__ blk, int64_t ldb, int* info, int col_base)
{
    if (*info != 0) return;
    __shared__ double tl[LU_TMAX * LU_TMAX * 256];
    __shared__ double zt[256], wt[256];
    __shared__ int fail;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int T = (w + DT - 1) / DT;
    // thread's entry rc of tile slots q0 + 2u (slot q is tile (q / LU_TMAX, q % LU_TMAX))
    const int rc = tid & 255, q0 = wave >> 2;
    if (tid == 0) fail = -1;
    {
        double v[LSTG];
#pragma unroll
        for (int u = 0; u < LSTG; ++u) {
            const int q = q0 + 2 * u, i = q / LU_TMAX, j = q % LU_TMAX;
            if (i < T && j < T) {
                const int gr = DT * i + (rc & 15), gc = DT * j + (rc >> 4);
                const bool in = gr < w && gc < w;
                const double x = blk[in ? gr + (int64_t)gc * ldb : 0];
                v[u] = in ? x : (gr == gc ? 1.0 : 0.0);
            }
        }
#pragma unroll
        for (int u = 0; u < LSTG; ++u) {
            const int q = q0 + 2 * u;
            if (q / LU_TMAX < T && q % LU_TMAX < T) tl[q * 256 + rc] = v[u];
        }
    }
    __syncthreads();
    if (wave == 0) lu_diag_tile(tl, 0, zt, wt, &fail, lane, w, info, col_base);
    __syncthreads();
    for (int kt = 0; kt + 1 < T; ++kt) {
        if (fail >= 0) return;
        const int nr = T - kt - 1;
        // the tiles below (A U_kk^-1) and to the right (L_kk^-1 A), one wave each
        for (int t = wave; t < 2 * nr; t += LU_PW) {
            if (t < nr) tile_mul_yt(tl + utile(kt + 1 + t, kt), zt, lane);
            else tile_lmul_wt(tl + utile(kt, kt + 1 + (t - nr)), wt, lane);
        }
        __syncthreads();
        // trailing tiles (it, jt), it, jt > kt: A -= L_it,kt U_kt,jt.  Pair p = 0
        // is the next diagonal tile: wave 0 updates and factors it, the other
        // waves take the remaining pairs.
        if (wave == 0) {
            tile_gemm_sub(tl + utile(kt + 1, kt + 1), tl + utile(kt + 1, kt), tl + utile(kt, kt + 1), lane);
            wave_lds_sync();
            lu_diag_tile(tl, kt + 1, zt, wt, &fail, lane, w, info, col_base);
        } else {
            for (int p = wave; p < nr * nr; p += LU_PW - 1) {
                const int it = kt + 1 + p / nr, jt = kt + 1 + p % nr;
                tile_gemm_sub(tl + utile(it, jt), tl + utile(it, kt), tl + utile(kt, jt), lane);
            }
        }
        __syncthreads();
    }
    if (fail >= 0) return;
#pragma unroll
    for (int u = 0; u < LSTG; ++u) {
        const int q = q0 + 2 * u, i = q / LU_TMAX, j = q % LU_TMAX;
        if (i < T && j < T) {
            const int gr = DT * i + (rc & 15), gc = DT * j + (rc >> 4);
            if (gr < w && gc < w) blk[gr + (int64_t)gc * ldb] = tl[q * 256 + rc];
        }
    }
}

template <typename S>
__global__ __launch_bounds__(PT)
void potrf_lds_kernel(int w, S* __restrict__ blk, int64_t ldb, int* info, int col_base)
{
    potrf_block<S>(w, blk, ldb, info, col_base);
}

// ---------------------------------------------------------------------------
// Triangular solve X T = B in place (X overwrites B), T upper triangular w x w
// (w <= TRSM_MAX): row by row, x_j = (b_j - sum_{k<j} x_k T(k, j)) / T(j, j)
// (unit: no division).  X(i, j) = x[i*xi + j*xj] (m rows), T(k, j) = t[k*tk + j*tj].
// T's upper tiles are staged in LDS (tile (j, t), j <= t, at index t(t+1)/2 + j,
// element (k, a) = T(16j + k, 16t + a) at a + 16 k), and each diagonal tile is
// replaced by its inverse, formed once per workgroup by back substitution with
// the correctly rounded reciprocals of the pivots.  Waves walk 16-row blocks of
// X, kept in registers as 16-column tiles, right-looking over tile columns:
// tile j becomes (B_j - sum_{k<j} X_k T_kj) T_jj^-1 (one 16 x 16 x 16 MFMA
// product with the inverse), then its contribution is subtracted from the later
// tile columns (MFMA products, K = 16).  With integer data and pivots 1 or 2 the
// tile inverses are dyadic rationals of fewer than 53 significant bits, so every
// intermediate stays exact.
constexpr int TRSM_TMAX = TRSM_MAX / DT;
constexpr int TRSM_NTILE = TRSM_TMAX * (TRSM_TMAX + 1) / 2;
// Four waves, one per SIMD: the row-block solves are MFMA-bound, and a second
// wave on a SIMD only queues behind the first.
constexpr int TRSM_NT = 256;

// The row blocks of the solve with NTT >= Tn tile columns, a compile-time count
// so that every MFMA of the unrolled loops is unconditional.  Tile columns past
// Tn are staged as the identity (diagonal tiles) and zeros, and their X entries
// load as zero and are never stored, so they change nothing.
template <typename T, bool XCOL, int NTT>
__device__ __forceinline__ void trsm_rows(int m, int w, T* x, int64_t xi, int64_t xj, const T* tu, int lane,
                                          int wave, int wg, int nwg)
{
    typedef acc_traits<T> AT;
    typedef typename AT::vec V;
    const int b = lane & 15;
    constexpr int SZ = sizeof(T);
    for (int r0 = (wg * (TRSM_NT / 64) + wave) * DT; r0 < m; r0 += nwg * (TRSM_NT / 64) * DT) {
        const int row = r0 + b;
        const bool rok = row < m;
        V xr[NTT];
        // every entry's whole offset is in the lane's register offset, out of
        // range (loads read zero, stores are dropped) past row m and column w
        const rsrc_t rx = make_rsrc(x + (int64_t)r0 * xi);
        auto xoff = [&](int q, int r) -> int {
            const int col = DT * q + tcol<T>(lane, r);
            return (rok && col < w) ? (int)((b * xi + col * xj) * SZ) : BUF_OOB;
        };
#pragma unroll
        for (int q = 0; q < NTT; ++q) {
#pragma unroll
            for (int r = 0; r < 4; ++r) xr[q][r] = buf_load<T>(rx, xoff(q, r), 0);
        }
#pragma unroll
        for (int jq = 0; jq < NTT; ++jq) {
            const T* vt = tu + (jq * (jq + 1) / 2 + jq) * 256;
            V y = zero_vec<V>();
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = tcol<T>(lane, i);
                y = AT::mfma(vt[b + 16 * k], xr[jq][i], y);
            }
            xr[jq] = y;
            // one 4-deep K step at a time across all later tile columns: the MFMAs
            // of a step are independent, so they issue back to back
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = tcol<T>(lane, i);
#pragma unroll
                for (int q = jq + 1; q < NTT; ++q)
                    xr[q] = AT::mfma(-tu[(q * (q + 1) / 2 + jq) * 256 + b + 16 * k], xr[jq][i], xr[q]);
            }
            // one tile column's LDS operands at a time: hoisting them all spills
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int q = 0; q < NTT; ++q) {
#pragma unroll
            for (int r = 0; r < 4; ++r) buf_store<T>(rx, xoff(q, r), xr[q][r], 0);
        }
    }
}

// Workgroup wg of nwg solving one panel (the row-block loop strides by nwg).
template <typename T, bool XCOL>
__device__ __forceinline__ void trsm_block(int m, int w, T* x, int64_t xi, int64_t xj, const T* __restrict__ t,
                                           int64_t tk, int64_t tj, int unit, const int* info, int wg, int nwg)
{
    if (info && *info != 0) return;
    __shared__ T tu[TRSM_TMAX * (TRSM_TMAX + 1) / 2 * 256];
    __shared__ T tinv[TRSM_MAX];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int Tn = (w + DT - 1) / DT;
    // Stage T's upper tiles: thread tid owns entry tid of every tile, and all its
    // loads are in flight at once.  Tile coordinates are compile-time constants,
    // so each load is one buffer instruction: the thread's own offset, the tile's
    // scalar offset, and an out-of-range offset (reading zero) outside the upper
    // triangle of the w x w block.  The pivots' reciprocals (1 past w, where the
    // padding is the identity, and for a unit diagonal) come from the staged values.
    static_assert(TRSM_NT == 256, "one tile entry per thread");
    {
        const int ko = tid >> 4, ao = tid & 15;
        const rsrc_t rt = make_rsrc(t);
        const int vo = (int)((ko * tk + ao * tj) * (int64_t)sizeof(T));
        T v[TRSM_NTILE];
        int tt = 0, jj = 0;
#pragma unroll
        for (int q = 0; q < TRSM_NTILE; ++q) {
            const int gk = DT * jj + ko, ga = DT * tt + ao;
            const bool in = gk < w && ga < w && gk <= ga;
            const int so = (int)((DT * jj * tk + DT * tt * tj) * (int64_t)sizeof(T));
            v[q] = buf_load<T>(rt, in ? vo : BUF_OOB, so);
            if (++jj > tt) { jj = 0; ++tt; }
        }
        tt = 0; jj = 0;
#pragma unroll
        for (int q = 0; q < TRSM_NTILE; ++q) {
            const int gk = DT * jj + ko, ga = DT * tt + ao;
            const bool in = gk < w && ga < w && gk <= ga;
            const T x = in ? v[q] : (gk == ga ? T(1) : T(0));
            tu[q * 256 + tid] = x;
            if (jj == tt && ko == ao) tinv[gk] = (gk < w && !unit) ? T(1) / x : T(1);
            if (++jj > tt) { jj = 0; ++tt; }
        }
    }
    __syncthreads();
    // Invert the diagonal tiles, one 16-lane group per tile (all of them in one
    // round), lane a owning column a of the inverse:
    // v_a = 1/U(a,a), v_k = -(sum_{j>k} U(k,j) v_j) / U(k,k) for k < a.
    static_assert(TRSM_NT / 16 >= TRSM_TMAX, "a lane group per diagonal tile");
    {
        const int jq = tid >> 4, a = lane & 15;
        if (jq < Tn) {
            T* dt = tu + (jq * (jq + 1) / 2 + jq) * 256;
            const T* ri = tinv + DT * jq;
            T v[16];
#pragma unroll
            for (int k = 15; k >= 0; --k) {
                T acc = T(0);
#pragma unroll
                for (int j = k + 1; j < 16; ++j) acc += dt[j + 16 * k] * v[j];   // v_j = 0 for j > a
                v[k] = k > a ? T(0) : (k == a ? ri[k] : -acc * ri[k]);
            }
#pragma unroll
            for (int k = 0; k < 16; ++k) dt[a + 16 * k] = v[k];
        }
    }
    __syncthreads();
    // Each wave walks 16-row blocks grid-stride; T stays staged for all of them.
    if (Tn <= 4) trsm_rows<T, XCOL, 4>(m, w, x, xi, xj, tu, lane, wave, wg, nwg);
    else if (Tn <= 8) trsm_rows<T, XCOL, 8>(m, w, x, xi, xj, tu, lane, wave, wg, nwg);
    else trsm_rows<T, XCOL, TRSM_TMAX>(m, w, x, xi, xj, tu, lane, wave, wg, nwg);
}

template <typename T, bool XCOL>
__global__ __launch_bounds__(TRSM_NT)
void trsm_reg_kernel(int m, int w, T* x, int64_t xi, int64_t xj, const T* __restrict__ t, int64_t tk,
                     int64_t tj, int unit, const int* info)
{
    trsm_block<T, XCOL>(m, w, x, xi, xj, t, tk, tj, unit, info, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Grouped forms for many independent factorisations at once (serving): one
// launch covers the diagonal blocks, or the panel solves, of every job.
template <typename S>
__global__ __launch_bounds__(PT)
void potrf_grouped_kernel(const GroupDiag* __restrict__ jobs)
{
    const GroupDiag jb = jobs[blockIdx.x];
    potrf_block<S>(jb.w, static_cast<S*>(jb.a), jb.ld, jb.info, jb.col_base);
}

template <typename S>
__global__ __launch_bounds__(TRSM_NT)
void trsm_grouped_kernel(const GroupTrsm* __restrict__ jobs, int njobs)
{
    // the job whose workgroup range holds this workgroup
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].wg_begin <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const GroupTrsm jb = jobs[lo];
    trsm_block<S, true>(jb.m, jb.w, static_cast<S*>(jb.x), 1, jb.ld, static_cast<const S*>(jb.t), jb.ld, 1, 0, jb.info,
                        blockIdx.x - jb.wg_begin, jb.nwg);
}

}  // namespace

hipError_t launch_set_int(int* p, int v, hipStream_t st) {
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, st, p, v);
    return hipGetLastError();
}

hipError_t launch_copy_int(const int* src, int* dst, hipStream_t st) {
    hipLaunchKernelGGL(copy_int_kernel, dim3(1), dim3(64), 0, st, src, dst);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_potrf_diag(int w, S* blk, int64_t ldb, int* info, int col_base, hipStream_t st) {
    if (w <= 0) return hipSuccess;
    if (w > LDS_DIAG_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL((potrf_lds_kernel<S>), dim3(1), dim3(PT), 0, st, w, blk, ldb, info, col_base);
    return hipGetLastError();
}

hipError_t launch_getrf_lds(int w, double* a, int64_t ld, int* info, int col_base, hipStream_t st) {
    if (w <= 0) return hipSuccess;
    if (w > LU_LDS_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(getrf_lds_kernel, dim3(1), dim3(LU_PT), 0, st, w, a, ld, info, col_base);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_trsm(int m, int w, T* x, int64_t xi, int64_t xj, const T* t, int64_t tk, int64_t tj,
                       int unit, const int* info, hipStream_t st, int max_wg) {
    if (m <= 0 || w <= 0) return hipSuccess;
    if (w > TRSM_MAX) return hipErrorInvalidValue;
    // byte offsets inside one 16-row block (padded to whole tiles) must fit the buffer records
    const int64_t span = (16 * xi + (int64_t)(w + 16) * xj) * (int64_t)sizeof(T);
    if (span >= (int64_t)BUF_RECORDS) return hipErrorInvalidValue;
    // T is read through one buffer resource: its w x w block must lie within the records
    if ((int64_t)(w + DT) * (tk + tj) * (int64_t)sizeof(T) >= (int64_t)BUF_RECORDS) return hipErrorInvalidValue;
    int grid = (m + TRSM_NT / 4 - 1) / (TRSM_NT / 4);     // 16 rows per wave
    if (max_wg > 0 && grid > max_wg) grid = max_wg;
    if (xi == 1)
        hipLaunchKernelGGL((trsm_reg_kernel<T, true>), dim3(grid), dim3(TRSM_NT), 0, st, m, w, x, xi, xj, t, tk, tj,
                           unit, info);
    else
        hipLaunchKernelGGL((trsm_reg_kernel<T, false>), dim3(grid), dim3(TRSM_NT), 0, st, m, w, x, xi, xj, t, tk,
                           tj, unit, info);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_potrf_grouped(int njobs, const GroupDiag* d_jobs, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL((potrf_grouped_kernel<S>), dim3(njobs), dim3(PT), 0, st, d_jobs);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_trsm_grouped(int njobs, int total_wg, const GroupTrsm* d_jobs, hipStream_t st) {
    if (njobs <= 0 || total_wg <= 0) return hipSuccess;
    hipLaunchKernelGGL((trsm_grouped_kernel<S>), dim3(total_wg), dim3(TRSM_NT), 0, st, d_jobs, njobs);
    return hipGetLastError();
}

template hipError_t launch_potrf_grouped<double>(int, const GroupDiag*, hipStream_t);
template hipError_t launch_potrf_grouped<float>(int, const GroupDiag*, hipStream_t);
template hipError_t launch_trsm_grouped<double>(int, int, const GroupTrsm*, hipStream_t);
template hipError_t launch_trsm_grouped<float>(int, int, const GroupTrsm*, hipStream_t);

int trsm_rows_per_wg() { return TRSM_NT / 4; }

template hipError_t launch_potrf_diag<double>(int, double*, int64_t, int*, int, hipStream_t);
template hipError_t launch_potrf_diag<float>(int, float*, int64_t, int*, int, hipStream_t);
template hipError_t launch_trsm<double>(int, int, double*, int64_t, int64_t, const double*, int64_t, int64_t, int,
                                        const int*, hipStream_t, int);
template hipError_t launch_trsm<float>(int, int, float*, int64_t, int64_t, const float*, int64_t, int64_t, int,
                                       const int*, hipStream_t, int);

}  // namespace ff
