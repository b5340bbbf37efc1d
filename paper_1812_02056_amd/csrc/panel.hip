// panel.hip -- the per-block steps between two deferred updates.
//
// Sec. 2 of arXiv 1812.02056, Algorithm 1: after an update, the next s columns
// are formed Crout-style from the updated matrix and the columns pending since
// the update:
//     L[c,c] = sqrt(A[c,c] - sum_{k=z}^{c-1} L[c,k]^2)
//     L[i,c] = (A[i,c] - sum_{k=z}^{c-1} L[i,k] L[c,k]) / L[c,c]      (i > c)
// For the w pending columns of one block, the rows inside the block form the
// w x w diagonal factorisation (potrf_diag_kernel) and the rows below it are a
// triangular solve L21 = A21 L11^-T (trsm_kernel, rows independent).
// Algorithm 2 (LU) splits the same way into getrf_diag_kernel and two
// triangular solves L21 = A21 U11^-1 and U12 = L11^-1 A12.
//
// Both diagonal kernels run in ONE workgroup: the block is processed in panels
// of 16 columns, each first brought up to date with the columns left of it by an
// MFMA product (left-looking), then factored column by column with each thread
// owning whole rows in registers.  Diagonal blocks are always binary64; for
// binary32 storage they are widened into a workspace, factored, and rounded back.
#include <math.h>

#include "common.hpp"
#include "internal.hpp"

namespace ff {

namespace {

constexpr int PNT = 256;     // threads of the single-workgroup diagonal kernels
constexpr int PB = 16;       // panel width
constexpr int MAXR = DIAG_MAX / PNT;   // rows per thread in the diagonal kernels

__global__ void set_int_kernel(int* p, int v) { if (threadIdx.x == 0) *p = v; }

// a[rows r0.., cols q0..] -= Lsrc[r0.., 0:c] * Usrc[0:c, q0..] for one 16 x 16
// tile (one wave), with element accessors L(i, k) = a[i + k*ld] and
// U(k, j) = ub[k*uk + j*uj].  Rows >= rmax, cols >= qmax, and (lower_only)
// entries above the diagonal are not written.
__device__ __forceinline__ void tile_update_f64(double* a, int64_t ld, const double* ub, int64_t uk, int64_t uj,
                                                int r0, int q0, int c, int rmax, int qmax, bool lower_only,
                                                int lane) {
    d4_t acc0 = zero_vec<d4_t>(), acc1 = zero_vec<d4_t>();
    const int ra = r0 + (lane & 15), qa = q0 + (lane & 15);
    const bool rok = ra < rmax, qok = qa < qmax;
    int k = 0;
    for (; k + 8 <= c; k += 8) {
        const int k1 = k + (lane >> 4), k2 = k1 + 4;
        const double fa1 = qok ? ub[(int64_t)k1 * uk + (int64_t)qa * uj] : 0.0;
        const double fb1 = rok ? a[(int64_t)ra + (int64_t)k1 * ld] : 0.0;
        const double fa2 = qok ? ub[(int64_t)k2 * uk + (int64_t)qa * uj] : 0.0;
        const double fb2 = rok ? a[(int64_t)ra + (int64_t)k2 * ld] : 0.0;
        acc0 = mfma_f64(fa1, fb1, acc0);
        acc1 = mfma_f64(fa2, fb2, acc1);
    }
    for (; k < c; k += 4) {
        const int k1 = k + (lane >> 4);
        const double fa1 = (qok && k1 < c) ? ub[(int64_t)k1 * uk + (int64_t)qa * uj] : 0.0;
        const double fb1 = (rok && k1 < c) ? a[(int64_t)ra + (int64_t)k1 * ld] : 0.0;
        acc0 = mfma_f64(fa1, fb1, acc0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int gi = r0 + (lane & 15);
        const int gj = q0 + acc_traits<double>::col(lane, r);
        if (gi < rmax && gj < qmax && (!lower_only || gi >= gj))
            a[(int64_t)gi + (int64_t)gj * ld] -= (acc0[r] + acc1[r]);
    }
}

// Cholesky of the w x w diagonal block (w <= DIAG_MAX).  S is the storage type;
// for float storage the lower triangle is widened into ws (w x w, ld = w).
template <typename S>
__global__ __launch_bounds__(PNT)
void potrf_diag_kernel(int w, S* blk, int64_t ldb, double* ws, int* info, int col_base)
{
    if (*info != 0) return;
    __shared__ double top[PB][PB + 1];
    __shared__ int fail;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    double* a;
    int64_t ld;
    if constexpr (sizeof(S) == sizeof(double)) {
        a = reinterpret_cast<double*>(blk);
        ld = ldb;
    } else {
        a = ws;
        ld = w;
        for (int j = 0; j < w; ++j)
            for (int i = j + tid; i < w; i += PNT) a[i + (int64_t)j * ld] = (double)blk[i + (int64_t)j * ldb];
    }
    if (tid == 0) fail = 0;
    __syncthreads();

    for (int c = 0; c < w; c += PB) {
        const int nbc = min(PB, w - c);
        const int pe = c + nbc;
        if (c > 0) {
            const int ntile = (w - c + 15) / 16;
            for (int t = wave; t < ntile; t += PNT / 64)
                tile_update_f64(a, ld, a, ld, 1, c + 16 * t, c, c, w, pe, true, lane);  // U(k,j) = L(j,k)
        }
        __syncthreads();
        // factor panel columns c..pe-1 over rows c..w-1; thread owns rows c+tid, c+tid+PNT, ...
        double p[MAXR][PB];
#pragma unroll
        for (int q = 0; q < MAXR; ++q) {
            const int i = c + tid + q * PNT;
#pragma unroll
            for (int j = 0; j < PB; ++j)
                p[q][j] = (i < w && j < nbc && (i - c) >= j) ? a[i + (int64_t)(c + j) * ld] : 0.0;
        }
bool failed = false;
#pragma unroll
        for (int j = 0; j < PB; ++j) {
            if (j < nbc && !failed) {
                if (tid == j) {
                    const double d = p[0][j];
                    if (!(d > 0.0)) {
                        fail = 1;
                        *info = col_base + c + j + 1;
                    } else {
                        p[0][j] = sqrt(d);
                        top[j][j] = p[0][j];
                    }
                }
                __syncthreads();
                failed = fail != 0;
                if (!failed) {
                    const double ljj = top[j][j];
#pragma unroll
                    for (int q = 0; q < MAXR; ++q) {
                        const int li = tid + q * PNT;
                        if (c + li < w && li > j) {
                            p[q][j] = p[q][j] / ljj;
                            if (li < PB) top[li][j] = p[q][j];
                        }
                    }
                    __syncthreads();
#pragma unroll
                    for (int q = 0; q < MAXR; ++q) {
                        const int li = tid + q * PNT;
                        if (c + li < w && li > j) {
                            const double lij = p[q][j];
#pragma unroll
                            for (int k = 0; k < PB; ++k)
                                if (k > j && k < nbc && k <= li) p[q][k] -= lij * top[k][j];
                        }
                    }
                }
            }
        }
        if (failed) return;
#pragma unroll
        for (int q = 0; q < MAXR; ++q) {
            const int li = tid + q * PNT;
            const int i = c + li;
            if (i < w) {
#pragma unroll
                for (int j = 0; j < PB; ++j)
                    if (j < nbc && li >= j) a[i + (int64_t)(c + j) * ld] = p[q][j];
            }
        }
        __syncthreads();
    }
    if constexpr (sizeof(S) != sizeof(double)) {
        for (int j = 0; j < w; ++j)
            for (int i = j + tid; i < w; i += PNT) blk[i + (int64_t)j * ldb] = (S)a[i + (int64_t)j * ld];
    }
}

// Doolittle LU without pivoting of the w x w diagonal block, in place (binary64).
__global__ __launch_bounds__(PNT)
void getrf_diag_kernel(int w, double* a, int64_t ld, int* info, int col_base)
{
    if (*info != 0) return;
    __shared__ double top[PB][PB + 1];
    __shared__ int fail;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) fail = 0;
    __syncthreads();

    for (int c = 0; c < w; c += PB) {
        const int nbc = min(PB, w - c);
        const int pe = c + nbc;
        if (c > 0) {
            // column panel: rows c..w-1, cols c..pe-1; row panel: rows c..pe-1, cols pe..w-1
            const int ncol_t = (w - c + 15) / 16;
            const int nrow_t = (w - pe + 15) / 16;
            for (int t = wave; t < ncol_t + nrow_t; t += PNT / 64) {
                if (t < ncol_t)
                    tile_update_f64(a, ld, a, 1, ld, c + 16 * t, c, c, w, pe, false, lane);
                else
                    tile_update_f64(a, ld, a, 1, ld, c, pe + 16 * (t - ncol_t), c, pe, w, false, lane);
            }
        }
        __syncthreads();
        double p[MAXR][PB];
#pragma unroll
        for (int q = 0; q < MAXR; ++q) {
            const int i = c + tid + q * PNT;
#pragma unroll
            for (int j = 0; j < PB; ++j) p[q][j] = (i < w && j < nbc) ? a[i + (int64_t)(c + j) * ld] : 0.0;
        }
bool failed = false;
#pragma unroll
        for (int j = 0; j < PB; ++j) {
            if (j < nbc && !failed) {
                if (tid == j) {
#pragma unroll
                    for (int k = 0; k < PB; ++k)
                        if (k >= j) top[j][k] = p[0][k];
                    const double u = p[0][j];
                    if (u == 0.0 || !isfinite(u)) {
                        fail = 1;
                        *info = col_base + c + j + 1;
                    }
                }
                __syncthreads();
                failed = fail != 0;
                if (!failed) {
                    const double u = top[j][j];
#pragma unroll
                    for (int q = 0; q < MAXR; ++q) {
                        const int li = tid + q * PNT;
                        if (c + li < w && li > j) {
                            const double l = p[q][j] / u;
                            p[q][j] = l;
                            if (li < PB) top[li][j] = l;
#pragma unroll
                            for (int k = 0; k < PB; ++k)
                                if (k > j && k < nbc) p[q][k] -= l * top[j][k];
                        }
                    }
                    __syncthreads();
                }
            }
        }
        if (failed) return;
#pragma unroll
        for (int q = 0; q < MAXR; ++q) {
            const int i = c + tid + q * PNT;
            if (i < w) {
#pragma unroll
                for (int j = 0; j < PB; ++j)
                    if (j < nbc) a[i + (int64_t)(c + j) * ld] = p[q][j];
            }
        }
        __syncthreads();
        // U row panel: U[c+j, q] = A[c+j, q] - sum_{k<j} L[c+j, c+k] U[c+k, q], q >= pe
        for (int q = pe + tid; q < w; q += PNT) {
            double u[PB];
#pragma unroll
            for (int j = 0; j < PB; ++j) {
                if (j < nbc) {
                    double x = a[(int64_t)(c + j) + (int64_t)q * ld];
#pragma unroll
                    for (int k = 0; k < PB; ++k)
                        if (k < j) x -= top[j][k] * u[k];
                    u[j] = x;
                    a[(int64_t)(c + j) + (int64_t)q * ld] = x;
                }
            }
        }
        __syncthreads();
    }
}

// Triangular solve X T = B in place (B overwritten by X), T upper triangular
// w x w: x_j = (b_j - sum_{k<j} x_k T(k,j)) / T(j,j) (no division if unit).
// X(i, j) = x[i*xi + j*xj] (m rows), T(k, j) = t[k*tk + j*tj].
// Each wave owns 16 rows and walks the w columns in panels of 16: an MFMA product
// brings the panel up to date with the solved columns left of it, then 16 lanes
// finish the panel by substitution, one row each.
template <typename T>
__global__ __launch_bounds__(256)
void trsm_kernel(int m, int w, T* x, int64_t xi, int64_t xj, const T* t, int64_t tk, int64_t tj,
                 int unit, const int* info)
{
    if (info && *info != 0) return;
    typedef acc_traits<T> AT;
    typedef typename AT::vec V;
    __shared__ T tile[4][PB][PB + 1];
    __shared__ T tdg[4][PB][PB + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r0 = (blockIdx.x * 4 + wave) * PB;
    if (r0 >= m) return;
    const int ra = r0 + (lane & 15);
    const bool rok = ra < m;

    for (int c = 0; c < w; c += PB) {
        const int nbc = min(PB, w - c);
        const int qa = c + (lane & 15);
        const bool qok = qa < w;
        V acc0 = zero_vec<V>(), acc1 = zero_vec<V>();
        int k = 0;
        for (; k + 8 <= c; k += 8) {
            const int k1 = k + (lane >> 4), k2 = k1 + 4;
            const T fa1 = qok ? t[(int64_t)k1 * tk + (int64_t)qa * tj] : T(0);
            const T fb1 = rok ? x[(int64_t)ra * xi + (int64_t)k1 * xj] : T(0);
            const T fa2 = qok ? t[(int64_t)k2 * tk + (int64_t)qa * tj] : T(0);
            const T fb2 = rok ? x[(int64_t)ra * xi + (int64_t)k2 * xj] : T(0);
            acc0 = AT::mfma(fa1, fb1, acc0);
            acc1 = AT::mfma(fa2, fb2, acc1);
        }
        for (; k < c; k += 4) {
            const int k1 = k + (lane >> 4);
            const T fa1 = (qok && k1 < c) ? t[(int64_t)k1 * tk + (int64_t)qa * tj] : T(0);
            const T fb1 = (rok && k1 < c) ? x[(int64_t)ra * xi + (int64_t)k1 * xj] : T(0);
            acc0 = AT::mfma(fa1, fb1, acc0);
        }
        // stage the partially reduced panel rows and the diagonal block of T
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int a = AT::col(lane, r);
            if (rok && a < nbc)
                tile[wave][lane & 15][a] = x[(int64_t)ra * xi + (int64_t)(c + a) * xj] - (acc0[r] + acc1[r]);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = lane + 64 * e;
            const int kk = idx & 15, jj = idx >> 4;
            if (kk < nbc && jj < nbc && kk <= jj)
                tdg[wave][kk][jj] = t[(int64_t)(c + kk) * tk + (int64_t)(c + jj) * tj];
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (lane < 16 && rok) {
            for (int j = 0; j < nbc; ++j) {
                T v = tile[wave][lane][j];
                for (int kq = 0; kq < j; ++kq) v -= tile[wave][lane][kq] * tdg[wave][kq][j];
                if (!unit) v = v / tdg[wave][j][j];
                tile[wave][lane][j] = v;
            }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // write the solved panel back: lane group g writes columns g, g+4, ...
        for (int j = (lane >> 4); j < nbc; j += 4)
            if (rok) x[(int64_t)ra * xi + (int64_t)(c + j) * xj] = tile[wave][lane & 15][j];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
}

}  // namespace

hipError_t launch_set_int(int* p, int v, hipStream_t st) {
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, st, p, v);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_potrf_diag(int w, S* blk, int64_t ldb, double* ws, int* info, int col_base, hipStream_t st) {
    if (w <= 0) return hipSuccess;
    if (w > DIAG_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL((potrf_diag_kernel<S>), dim3(1), dim3(PNT), 0, st, w, blk, ldb, ws, info, col_base);
    return hipGetLastError();
}

hipError_t launch_getrf_diag(int w, double* a, int64_t ld, int* info, int col_base, hipStream_t st) {
    if (w <= 0) return hipSuccess;
    if (w > DIAG_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(getrf_diag_kernel, dim3(1), dim3(PNT), 0, st, w, a, ld, info, col_base);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_trsm(int m, int w, T* x, int64_t xi, int64_t xj, const T* t, int64_t tk, int64_t tj,
                       int unit, const int* info, hipStream_t st) {
    if (m <= 0 || w <= 0) return hipSuccess;
    const int grid = (m + 63) / 64;
    hipLaunchKernelGGL((trsm_kernel<T>), dim3(grid), dim3(256), 0, st, m, w, x, xi, xj, t, tk, tj, unit, info);
    return hipGetLastError();
}

template hipError_t launch_potrf_diag<double>(int, double*, int64_t, double*, int*, int, hipStream_t);
template hipError_t launch_potrf_diag<float>(int, float*, int64_t, double*, int*, int, hipStream_t);
template hipError_t launch_trsm<double>(int, int, double*, int64_t, int64_t, const double*, int64_t, int64_t, int, const int*, hipStream_t);
template hipError_t launch_trsm<float>(int, int, float*, int64_t, int64_t, const float*, int64_t, int64_t, int, const int*, hipStream_t);

}  // namespace ff
