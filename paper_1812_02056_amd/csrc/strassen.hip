// strassen.hip -- the trailing update with one level of Strassen's multiplication.
//
// Sec. 2 of arXiv 1812.02056 notes that the rectangular product R R^T (R_L R_U
// for LU) of the delayed update may use Strassen's algorithm on rectangles
// (Knight): the n x s by s x n product is cut into square-block products.  Here
// one Strassen level is applied per 128 x 128 super-tile of the output: with
//     X = [X1; X2] (rows of the super-tile's two 64-row quadrants),
//     Y = [Y1; Y2] (rows of Y for its two 64-column quadrants),
// and K split into halves k1 = [0, K2), k2 = [K2, K) with K2 = ceil(K / 2)
// (the odd column of k2 is a zero), the blocks
//     A11 = X1(k1)  A12 = X1(k2)  A21 = X2(k1)  A22 = X2(k2)
//     B11 = Y1(k1)^T  B12 = Y2(k1)^T  B21 = Y1(k2)^T  B22 = Y2(k2)^T
// give S = X Y^T from Strassen's seven products
//     M1 = (A11 + A22)(B11 + B22)   M2 = (A21 + A22) B11   M3 = A11 (B12 - B22)
//     M4 = A22 (B21 - B11)          M5 = (A11 + A12) B22   M6 = (A21 - A11)(B11 + B12)
//     M7 = (A12 - A22)(B21 + B22)
//     S11 = M1 + M4 - M5 + M7   S12 = M3 + M5   S21 = M2 + M4   S22 = M1 - M2 + M3 + M6
// which take 7 of the 8 half-K quadrant products of the classical form.
//
// Cholesky (lower part of R R^T only): a super-tile on the diagonal needs just
// S11, S21 and S22 (6 half-K products classically), which is fewer than
// Strassen's 7, so diagonal super-tiles take the classical products
//     S11 = A11 B11 + A12 B21   S21 = A21 B11 + A22 B21   S22 = A21 B12 + A22 B22
// through the same seven product slots (the seventh is zero) and the strictly
// upper quadrant is not written.
//
// Kernel: one workgroup of 8 waves per super-tile (persistent, one per CU, two
// waves per SIMD), the seven 64 x 64 products accumulated together in registers
// (each wave holds a 32 x 16 part of all seven: 112 accumulator registers), so C
// is read and written once per super-tile as in the classical kernels and the
// operands are loaded once: each thread loads the four X blocks (and four Y
// blocks) at the same position, forms the seven operand sums in registers while
// staging, and writes them to LDS.  Stages of 8 K positions are double-buffered
// in LDS and loaded one stage ahead.
#include <algorithm>

#include "common.hpp"
#include "grid.hpp"
#include "internal.hpp"

namespace ff {

namespace {

constexpr int SQ = 64;          // quadrant edge
constexpr int ST = 2 * SQ;      // super-tile edge
constexpr int SBK = 8;          // K positions per LDS stage (of each half)
constexpr int SNT = 512;        // 2 x 4 waves, each a 32 x 16 part of every product
constexpr int NPROD = 7;
constexpr int NBR = 2;          // 16-row MFMA blocks per wave (one 16-column block)
// LDS row pitch: for a K-by-N operand (Y[k + j*ldy]) two doubles of padding put
// the 8 K positions that 8 lanes store for one column in distinct banks.
template <bool YROWS> struct lds_pitch { static constexpr int P = YROWS ? SQ : SQ + 2; };

// Operand sums of the seven product slots; `dg` selects the classical products
// of a diagonal super-tile.
__device__ __forceinline__ void x_sums(double a11, double a12, double a21, double a22, bool dg, double (&x)[NPROD]) {
    x[0] = dg ? a11 : a11 + a22;
    x[1] = dg ? a12 : a21 + a22;
    x[2] = dg ? a21 : a11;
    x[3] = a22;
    x[4] = dg ? a21 : a11 + a12;
    x[5] = dg ? a22 : a21 - a11;
    x[6] = dg ? 0.0 : a12 - a22;
}
__device__ __forceinline__ void y_sums(double b11, double b12, double b21, double b22, bool dg, double (&y)[NPROD]) {
    y[0] = dg ? b11 : b11 + b22;
    y[1] = dg ? b21 : b11;
    y[2] = dg ? b11 : b12 - b22;
    y[3] = dg ? b21 : b21 - b11;
    y[4] = dg ? b12 : b22;
    y[5] = dg ? b22 : b11 + b12;
    y[6] = dg ? 0.0 : b21 + b22;
}

// One super-tile (bi, bj): the K loop over both halves and the write-back.  DG:
// a diagonal super-tile of the lower region (classical products, upper
// quadrant skipped).  Ends with a barrier so the caller may start another
// super-tile on the same LDS buffers.
template <bool YROWS, bool LOWER, bool DG>
__device__ __forceinline__ void strassen_tile(int M, int N, int K, double* __restrict__ C, int64_t ldc,
                                              const double* __restrict__ X, int64_t ldx, const double* __restrict__ Y,
                                              int64_t ldy, int bi, int bj, double (&As)[2][NPROD][SBK][lds_pitch<YROWS>::P],
                                              double (&Bs)[2][NPROD][SBK][lds_pitch<YROWS>::P])
{
    constexpr int SZ = 8;
    constexpr bool dg = DG;
    typedef acc_traits<double> AT;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave & 1, wc = wave >> 1;     // 32-row half, 16-column quarter
    const int K2 = (K + 1) / 2;
    const int nk = (K2 + SBK - 1) / SBK;
    const int xs = (int)ldx * SZ, ys = (int)ldy * SZ;
    // staging of row-indexed operands: row sr of both quadrants, K position sk
    const int sr = tid & 63, sk = wave;
    // staging of Y when K runs down its columns: column yc, K position yk
    const int yc = tid >> 3, yk = tid & 7;

    {
        const int row0 = bi * ST, col0 = bj * ST;
        const int mrem = M - row0, nrem = N - col0;
        const int vx1 = sr < mrem ? sr * SZ : BUF_OOB;
        const int vx2 = sr + SQ < mrem ? (sr + SQ) * SZ : BUF_OOB;
        const int vy1 = YROWS ? (sr < nrem ? sr * SZ : BUF_OOB) : (yc < nrem ? yc * ys : BUF_OOB);
        const int vy2 = YROWS ? (sr + SQ < nrem ? (sr + SQ) * SZ : BUF_OOB) : (yc + SQ < nrem ? (yc + SQ) * ys : BUF_OOB);
        const double* Xt = X + row0;
        const double* Yt = YROWS ? Y + col0 : Y + (int64_t)col0 * ldy;

        // raw blocks at this thread's K position: [11, 12, 21, 22]
        double xa[4], ya[4];
        auto load = [&](int kt) {
            const int k0 = kt * SBK;
            int kv1 = K2 - k0, kv2 = K - K2 - k0;
            kv1 = kv1 < 0 ? 0 : (kv1 > SBK ? SBK : kv1);
            kv2 = kv2 < 0 ? 0 : (kv2 > SBK ? SBK : kv2);
            // wave-uniform, so the resources below live in scalar registers (a
            // clamp computed on the vector unit would make every load a loop
            // over distinct resources)
            kv1 = __builtin_amdgcn_readfirstlane(kv1);
            kv2 = __builtin_amdgcn_readfirstlane(kv2);
            // resources end at the half's last column: later positions read zero
            const rsrc_t rx1 = make_rsrc_n(Xt + (int64_t)k0 * ldx, kv1 * xs);
            const rsrc_t rx2 = make_rsrc_n(Xt + (int64_t)(K2 + k0) * ldx, kv2 * xs);
            const int sox = sk * xs;
            xa[0] = buf_load<double>(rx1, vx1, sox);
            xa[1] = buf_load<double>(rx2, vx1, sox);
            xa[2] = buf_load<double>(rx1, vx2, sox);
            xa[3] = buf_load<double>(rx2, vx2, sox);
            if (YROWS) {
                const rsrc_t ry1 = make_rsrc_n(Yt + (int64_t)k0 * ldy, kv1 * ys);
                const rsrc_t ry2 = make_rsrc_n(Yt + (int64_t)(K2 + k0) * ldy, kv2 * ys);
                const int soy = sk * ys;
                ya[0] = buf_load<double>(ry1, vy1, soy);   // B11: Y1, k1
                ya[1] = buf_load<double>(ry1, vy2, soy);   // B12: Y2, k1
                ya[2] = buf_load<double>(ry2, vy1, soy);   // B21: Y1, k2
                ya[3] = buf_load<double>(ry2, vy2, soy);   // B22: Y2, k2
            } else {
                const rsrc_t ry1 = make_rsrc(Yt + k0);
                const rsrc_t ry2 = make_rsrc(Yt + K2 + k0);
                const bool in1 = yk < kv1, in2 = yk < kv2;
                ya[0] = buf_load<double>(ry1, in1 && vy1 != BUF_OOB ? vy1 + yk * SZ : BUF_OOB, 0);
                ya[1] = buf_load<double>(ry1, in1 && vy2 != BUF_OOB ? vy2 + yk * SZ : BUF_OOB, 0);
                ya[2] = buf_load<double>(ry2, in2 && vy1 != BUF_OOB ? vy1 + yk * SZ : BUF_OOB, 0);
                ya[3] = buf_load<double>(ry2, in2 && vy2 != BUF_OOB ? vy2 + yk * SZ : BUF_OOB, 0);
            }
        };
        auto store = [&](int buf) {
            double x[NPROD], y[NPROD];
            x_sums(xa[0], xa[1], xa[2], xa[3], dg, x);
            y_sums(ya[0], ya[1], ya[2], ya[3], dg, y);
#pragma unroll
            for (int p = 0; p < NPROD; ++p) As[buf][p][sk][sr] = x[p];
            if (YROWS) {
#pragma unroll
                for (int p = 0; p < NPROD; ++p) Bs[buf][p][sk][sr] = y[p];
            } else {
#pragma unroll
                for (int p = 0; p < NPROD; ++p) Bs[buf][p][yk][yc] = y[p];
            }
        };

        d4_t acc[NPROD][NBR];
#pragma unroll
        for (int p = 0; p < NPROD; ++p)
#pragma unroll
            for (int b = 0; b < NBR; ++b) acc[p][b] = zero_vec<d4_t>();

        // fragments of product slot p at 4-deep step k4: fa column operand (this
        // wave's 16 columns), fb row operand (its 32 rows)
        auto frags = [&](int buf, int k4, int p, double& fa, double (&fb)[NBR]) {
            const int kk = 4 * k4 + (lane >> 4);
            fa = Bs[buf][p][kk][16 * wc + (lane & 15)];
#pragma unroll
            for (int b = 0; b < NBR; ++b) fb[b] = As[buf][p][kk][32 * wr + 16 * b + (lane & 15)];
        };
        auto compute = [&](int buf) {
            constexpr int NS = (SBK / 4) * NPROD;      // (k4, product) steps of one stage
            double fa[2], fb[2][NBR];
            frags(buf, 0, 0, fa[0], fb[0]);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (s + 1 < NS) frags(buf, (s + 1) / NPROD, (s + 1) % NPROD, fa[(s + 1) & 1], fb[(s + 1) & 1]);
                const int p = s % NPROD;
#pragma unroll
                for (int r4 = 0; r4 < NBR; ++r4) acc[p][r4] = AT::mfma(fa[s & 1], fb[s & 1][r4], acc[p][r4]);
            }
        };

        load(0);
        store(0);
        __syncthreads();
        for (int kt = 0; kt + 1 < nk; ++kt) {
            load(kt + 1);
            compute(kt & 1);
            store((kt + 1) & 1);
            __syncthreads();
        }
        compute((nk - 1) & 1);    // positions past each half's end hold zeros

        // Write-back C - S quadrant by quadrant; lanes hold 16 consecutive rows.
        const int li0 = 32 * wr + (lane & 15);
        const int lj0 = 16 * wc + AT::col_lane(lane);
        auto put = [&](int qi, int qj, const d4_t (&sq)[NBR]) {
            const int r0 = row0 + SQ * qi, c0 = col0 + SQ * qj;
            const int mq = M - r0, nq = N - c0;
            const rsrc_t rc = make_rsrc(C + r0 + (int64_t)c0 * ldc);
            const bool full = mq >= SQ && nq >= SQ && (!LOWER || r0 - (c0 + SQ - 1) >= 0);
            const int cbase = (li0 + lj0 * (int)ldc) * SZ;
            double cv[NBR][4];
            int off[NBR][4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int r4 = 0; r4 < NBR; ++r4) {
                    const int li = li0 + 16 * r4, lj = lj0 + AT::col_reg(r);
                    const bool ok = full || (li < mq && lj < nq && (!LOWER || (r0 + li) - (c0 + lj) >= 0));
                    off[r4][r] = ok ? cbase + (16 * r4 + AT::col_reg(r) * (int)ldc) * SZ : BUF_OOB;
                    cv[r4][r] = bufop<double, AUX_NT>::load(rc, off[r4][r], 0);
                }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int r4 = 0; r4 < NBR; ++r4)
                    bufop<double, AUX_NT>::store(rc, off[r4][r], cv[r4][r] - sq[r4][r], 0);
        };
        d4_t sq[NBR];
        if constexpr (DG) {
#pragma unroll
            for (int b = 0; b < NBR; ++b) sq[b] = acc[0][b] + acc[1][b];
            put(0, 0, sq);
#pragma unroll
            for (int b = 0; b < NBR; ++b) sq[b] = acc[2][b] + acc[3][b];
            put(1, 0, sq);
#pragma unroll
            for (int b = 0; b < NBR; ++b) sq[b] = acc[4][b] + acc[5][b];
            put(1, 1, sq);
        } else {
#pragma unroll
            for (int b = 0; b < NBR; ++b) sq[b] = ((acc[0][b] + acc[3][b]) - acc[4][b]) + acc[6][b];
            put(0, 0, sq);
#pragma unroll
            for (int b = 0; b < NBR; ++b) sq[b] = acc[2][b] + acc[4][b];
            put(0, 1, sq);
#pragma unroll
            for (int b = 0; b < NBR; ++b) sq[b] = acc[1][b] + acc[3][b];
            put(1, 0, sq);
#pragma unroll
            for (int b = 0; b < NBR; ++b) sq[b] = ((acc[0][b] - acc[1][b]) + acc[2][b]) + acc[5][b];
            put(1, 1, sq);
        }
        __syncthreads();   // the next super-tile's first stage reuses buffer 0
    }
}

template <bool YROWS, bool LOWER>
__global__ __launch_bounds__(SNT, 1)
void strassen_kernel(int M, int N, int K, double* __restrict__ C, int64_t ldc, const double* __restrict__ X,
                     int64_t ldx, const double* __restrict__ Y, int64_t ldy, Grid g, const int* __restrict__ info)
{
    if (info && *info != 0) return;
    __shared__ double As[2][NPROD][SBK][lds_pitch<YROWS>::P];    // X-side sums, [k][row]
    __shared__ double Bs[2][NPROD][SBK][lds_pitch<YROWS>::P];    // Y-side sums, [k][column]
    int it0, it1, itd;
    tile_walk(g, it0, it1, itd);
    for (int it = it0; it < it1; it += itd) {
        int bi, bj;
        if (g.balanced) tile_of_index(g, LOWER, it, bi, bj);
        else if (!tile_of_slot(g, it, LOWER, bi, bj)) continue;
        if (LOWER && bi == bj)
            strassen_tile<YROWS, LOWER, true>(M, N, K, C, ldc, X, ldx, Y, ldy, bi, bj, As, Bs);
        else
            strassen_tile<YROWS, LOWER, false>(M, N, K, C, ldc, X, ldx, Y, ldy, bi, bj, As, Bs);
    }
}

hipError_t launch_strassen(int M, int N, int K, double* C, int64_t ldc, const double* X, int64_t ldx,
                           const double* Y, int64_t ldy, bool yrows, bool lower, const int* info, hipStream_t st,
                           int reserve_cus) {
    if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
    if (lower && M != N) return hipErrorInvalidValue;
    if (!ld_fits(ldc, sizeof(double)) || !ld_fits(ldx, sizeof(double)) || !ld_fits(ldy, sizeof(double)))
        return hipErrorInvalidValue;
    Grid g = make_grid(ST, M, N, lower, 0);
    const int nwg = persistent_grid(g, update_workers(reserve_cus));   // one workgroup per CU
#define FF_STRASSEN_LAUNCH(YR, LO)                                                                                 \
    hipLaunchKernelGGL((strassen_kernel<YR, LO>), dim3(nwg), dim3(SNT), 0, st, M, N, K, C, ldc, X, ldx, Y, ldy, g, \
                       info)
    if (yrows) {
        if (lower) FF_STRASSEN_LAUNCH(true, true);
        else FF_STRASSEN_LAUNCH(true, false);
    } else {
        FF_STRASSEN_LAUNCH(false, false);
    }
#undef FF_STRASSEN_LAUNCH
    return hipGetLastError();
}

}  // namespace

hipError_t launch_update_syrk_strassen_f64(int m, int w, double* C, int64_t ldc, const double* P, int64_t ldp,
                                           const int* info, hipStream_t st, int reserve_cus) {
    return launch_strassen(m, m, w, C, ldc, P, ldp, P, ldp, true, true, info, st, reserve_cus);
}

hipError_t launch_update_gemm_strassen_f64(int m, int w, double* C, int64_t ldc, const double* X, int64_t ldx,
                                           const double* Y, int64_t ldy, const int* info, hipStream_t st,
                                           int reserve_cus) {
    return launch_strassen(m, m, w, C, ldc, X, ldx, Y, ldy, false, false, info, st, reserve_cus);
}

// ---------------------------------------------------------------- a second level
// The paper's experiments apply Strassen recursively (Sec. 2, timing paragraph).
// A second level at matrix scale on the LU product C -= X Y (C m x m, X m x w,
// Y w x m): with mh = floor(m / 2), kh = floor(w / 2) the leading 2mh x 2mh part
// of C takes Strassen's seven half-size products over the leading 2kh columns of
// X, each product computed by the one-level kernel above (so every output takes
// two levels); an odd last row, column or K index is applied classically first.
// Products that feed one quadrant are subtracted into it directly (M6 into C22,
// M7 into C11); the other five are formed into a scratch T (T = 0, T -= .., so
// T = -Mi) and added to, or subtracted from, the quadrants they feed:
//     C11 -= M1 + M4 - M5 + M7   C12 -= M3 + M5   C21 -= M2 + M4
//     C22 -= M1 - M2 + M3 + M6
// Workspace: strassen2_ws_doubles(m, w) doubles (operand sums and T).
namespace {
__global__ void s2_sum_kernel(int m, int n, const double* __restrict__ A, int64_t lda, const double* __restrict__ B,
                              int64_t ldb, double beta, double* __restrict__ D, int64_t ldd,
                              const int* __restrict__ info) {
    if (info && *info != 0) return;
    for (int j = blockIdx.y; j < n; j += gridDim.y)
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
            D[i + (int64_t)j * ldd] = A[i + (int64_t)j * lda] + beta * B[i + (int64_t)j * ldb];
}
__global__ void s2_axpy_kernel(int m, int n, const double* __restrict__ T, int64_t ldt, double alpha,
                               double* __restrict__ C, int64_t ldc, const int* __restrict__ info) {
    if (info && *info != 0) return;
    for (int j = blockIdx.y; j < n; j += gridDim.y)
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
            C[i + (int64_t)j * ldc] += alpha * T[i + (int64_t)j * ldt];
}
__global__ void s2_zero_kernel(int m, int n, double* __restrict__ T, int64_t ldt, const int* __restrict__ info) {
    if (info && *info != 0) return;
    for (int j = blockIdx.y; j < n; j += gridDim.y)
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
            T[i + (int64_t)j * ldt] = 0.0;
}
dim3 s2_grid(int m, int n) { return dim3((unsigned)std::min(4, (m + 255) / 256), (unsigned)std::min(n, 4096)); }
}  // namespace

size_t strassen2_ws_doubles(int m, int w) {
    const size_t mh = (size_t)(m / 2), kh = (size_t)(w / 2);
    return 2 * mh * kh + mh * mh;
}

hipError_t launch_update_gemm_strassen2_f64(int m, int w, double* C, int64_t ldc, const double* X, int64_t ldx,
                                            const double* Y, int64_t ldy, double* ws, const int* info, hipStream_t st,
                                            int reserve_cus) {
    if (m <= 0 || w <= 0) return hipSuccess;
    if (m < STRASSEN2_MIN_M || w < 2 || ws == nullptr)
        return launch_update_gemm_strassen_f64(m, w, C, ldc, X, ldx, Y, ldy, info, st, reserve_cus);
    const int mh = m / 2, kh = w / 2;
    hipError_t e = hipSuccess;
    // classical remainders: the odd K index over all of C, then an odd last row and column
    if (w > 2 * kh)
        e = launch_update<double>(m, m, w - 2 * kh, C, ldc, X + (int64_t)2 * kh * ldx, ldx, Y + 2 * kh, ldy, false,
                                  false, 0, info, st, reserve_cus);
    if (e == hipSuccess && m > 2 * mh) {
        e = launch_update<double>(m - 2 * mh, m, 2 * kh, C + 2 * mh, ldc, X + 2 * mh, ldx, Y, ldy, false, false, 0,
                                  info, st, reserve_cus);
        if (e == hipSuccess)
            e = launch_update<double>(2 * mh, m - 2 * mh, 2 * kh, C + (int64_t)2 * mh * ldc, ldc, X, ldx,
                                      Y + (int64_t)2 * mh * ldy, ldy, false, false, 0, info, st, reserve_cus);
    }
    if (e != hipSuccess) return e;
    double* TX = ws;
    double* TY = ws + (size_t)mh * kh;
    double* T = TY + (size_t)kh * mh;
    const double *X11 = X, *X12 = X + (int64_t)kh * ldx, *X21 = X + mh, *X22 = X + mh + (int64_t)kh * ldx;
    const double *Y11 = Y, *Y12 = Y + (int64_t)mh * ldy, *Y21 = Y + kh, *Y22 = Y + kh + (int64_t)mh * ldy;
    double *C11 = C, *C12 = C + (int64_t)mh * ldc, *C21 = C + mh, *C22 = C + mh + (int64_t)mh * ldc;
    auto sumx = [&](const double* A, const double* B, double beta) {
        hipLaunchKernelGGL(s2_sum_kernel, s2_grid(mh, kh), dim3(256), 0, st, mh, kh, A, ldx, B, ldx, beta, TX,
                           (int64_t)mh, info);
        return hipGetLastError();
    };
    auto sumy = [&](const double* A, const double* B, double beta) {
        hipLaunchKernelGGL(s2_sum_kernel, s2_grid(kh, mh), dim3(256), 0, st, kh, mh, A, ldy, B, ldy, beta, TY,
                           (int64_t)kh, info);
        return hipGetLastError();
    };
    auto zero_t = [&]() {
        hipLaunchKernelGGL(s2_zero_kernel, s2_grid(mh, mh), dim3(256), 0, st, mh, mh, T, (int64_t)mh, info);
        return hipGetLastError();
    };
    auto add_t = [&](double* Cq, double alpha) {
        hipLaunchKernelGGL(s2_axpy_kernel, s2_grid(mh, mh), dim3(256), 0, st, mh, mh, (const double*)T, (int64_t)mh,
                           alpha, Cq, ldc, info);
        return hipGetLastError();
    };
    auto prod = [&](double* Cq, int64_t ldcq, const double* A, int64_t lda, const double* B, int64_t ldb) {
        return launch_update_gemm_strassen_f64(mh, kh, Cq, ldcq, A, lda, B, ldb, info, st, reserve_cus);
    };
#define S2_TRY(x)                          \
    do {                                   \
        hipError_t e_ = (x);               \
        if (e_ != hipSuccess) return e_;   \
    } while (0)
    // M1 = (X11 + X22)(Y11 + Y22): C11, C22
    S2_TRY(sumx(X11, X22, 1.0));
    S2_TRY(sumy(Y11, Y22, 1.0));
    S2_TRY(zero_t());
    S2_TRY(prod(T, mh, TX, mh, TY, kh));
    S2_TRY(add_t(C11, 1.0));
    S2_TRY(add_t(C22, 1.0));
    // M2 = (X21 + X22) Y11: C21, C22 (-)
    S2_TRY(sumx(X21, X22, 1.0));
    S2_TRY(zero_t());
    S2_TRY(prod(T, mh, TX, mh, Y11, ldy));
    S2_TRY(add_t(C21, 1.0));
    S2_TRY(add_t(C22, -1.0));
    // M3 = X11 (Y12 - Y22): C12, C22
    S2_TRY(sumy(Y12, Y22, -1.0));
    S2_TRY(zero_t());
    S2_TRY(prod(T, mh, X11, ldx, TY, kh));
    S2_TRY(add_t(C12, 1.0));
    S2_TRY(add_t(C22, 1.0));
    // M4 = X22 (Y21 - Y11): C11, C21
    S2_TRY(sumy(Y21, Y11, -1.0));
    S2_TRY(zero_t());
    S2_TRY(prod(T, mh, X22, ldx, TY, kh));
    S2_TRY(add_t(C11, 1.0));
    S2_TRY(add_t(C21, 1.0));
    // M5 = (X11 + X12) Y22: C11 (-), C12
    S2_TRY(sumx(X11, X12, 1.0));
    S2_TRY(zero_t());
    S2_TRY(prod(T, mh, TX, mh, Y22, ldy));
    S2_TRY(add_t(C11, -1.0));
    S2_TRY(add_t(C12, 1.0));
    // M6 = (X21 - X11)(Y11 + Y12): into C22
    S2_TRY(sumx(X21, X11, -1.0));
    S2_TRY(sumy(Y11, Y12, 1.0));
    S2_TRY(prod(C22, ldc, TX, mh, TY, kh));
    // M7 = (X12 - X22)(Y21 + Y22): into C11
    S2_TRY(sumx(X12, X22, -1.0));
    S2_TRY(sumy(Y21, Y22, 1.0));
    S2_TRY(prod(C11, ldc, TX, mh, TY, kh));
#undef S2_TRY
    return hipSuccess;
}

}  // namespace ff
