// qr.hip -- QR factorisation by Gram-Schmidt with deferred block projections.
//
// Sec. 2 of arXiv 1812.02056, Algorithm 3.  M starts as a copy of A; here M lives
// in the output Q (column c of M is not read again once column c of Q exists).
// Per block of w columns:
//   (1) in-block modified Gram-Schmidt: each column is projected against the
//       block's earlier columns one at a time, every product taken with the
//       vector as updated so far, and divided by its norm;
//   (2) block projection of the finished block B_Q out of the later columns:
//       C = B_Q^T M[:, c..], then M[:, c..] -= B_Q C.
// Finally R = Q^T A (its upper triangle; the strict lower triangle is zero).
//
// Kernels:
//   qr_panel_kernel  (1) on P co-resident workgroups, each holding RR rows of the
//                    block in LDS.  MGS runs right-looking: in round j column j
//                    is normalised and projected out of the block's later
//                    columns.  Every column still receives the same projections
//                    in the same order as in the left-looking form.  A round
//                    needs one grid-wide sum (the norm of v_j and the products
//                    v_j . v_c), taken in a fixed order so that every workgroup
//                    holds bitwise the same values.
//   tn_gemm_kernel   D = X^T Y with both operands K-major (the product of (2)
//                    and R = Q^T A), v_mfma_f64_16x16x4f64 on 128 x 128 tiles,
//                    split over K into partial products that tn_reduce_kernel
//                    sums in a fixed order.
//   r_slab_kernel    R = Q^T A tile by tile over a K range, stored or added, so
//                    that R's tiles can be formed on the CUs the panel leaves
//                    idle as soon as the columns of Q they need are final.
// The subtraction of (2) is the LU trailing-update kernel (update.hip).
#include <algorithm>

#include "common.hpp"
#include "fastfact.h"
#include "grid.hpp"
#include "internal.hpp"

namespace ff {

namespace {

// ---------------------------------------------------------------- products
constexpr int TG_T = 128;          // output tile edge
constexpr int TG_BK = 16;          // K depth of one LDS stage
constexpr int TG_P = TG_T + 4;     // LDS row pitch: the staging writes of a wave
                                   // (8 columns x 8 K pairs) then cover every bank pair once
constexpr int TG_NT = 256;         // 2 x 2 waves, each a 64 x 64 part of the tile

__device__ __forceinline__ void load2(rsrc_t r, int off, double& a, double& b) {
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    const u4 v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    u2 lo, hi;
    lo.x = v.x; lo.y = v.y;
    hi.x = v.z; hi.y = v.w;
    a = __builtin_bit_cast(double, lo);
    b = __builtin_bit_cast(double, hi);
}

// Tile (bi, bj) of D = X^T Y over the K range [kb, kb + kc):
// D(i, j) (+)= sum over k of X(k, i) Y(k, j), for i < M, j < N, where
// X(k, i) = X[k + i*ldx] and Y(k, j) = Y[k + j*ldy].  ADD: the sum is added to
// D(i, j) instead of stored.  UPPER: only entries with i <= j are written.  Ends
// with a barrier so the next tile may reuse the LDS buffers.
template <bool UPPER, bool ADD>
__device__ __forceinline__ void tn_tile(int bi, int bj, int kb, int kc, int M, int N, const double* __restrict__ X,
                                        int64_t ldx, const double* __restrict__ Y, int64_t ldy,
                                        double* __restrict__ D, int64_t ldd, double (&As)[2][TG_BK][TG_P],
                                        double (&Bs)[2][TG_BK][TG_P]);

// Workgroup item b of a K-split product: K part q = b % ks of tile b / ks,
// written to D + q * dstride (ks = 1: D itself).  UPPER: tiles are the upper
// triangle of the tile grid (column-major triangle order).
template <bool UPPER>
__device__ __forceinline__ void tn_item(int b, int M, int N, int K, int kchunk, int ks, int tiles_m,
                                        const double* __restrict__ X, int64_t ldx, const double* __restrict__ Y,
                                        int64_t ldy, double* __restrict__ D, int64_t ldd, int64_t dstride,
                                        double (&As)[2][TG_BK][TG_P], double (&Bs)[2][TG_BK][TG_P])
{
    const int q = b % ks, tile = b / ks;
    int bi, bj;
    if (UPPER) {
        bj = tri_row(tile);
        bi = tile - bj * (bj + 1) / 2;
    } else {
        bi = tile % tiles_m;
        bj = tile / tiles_m;
    }
    const int kb = q * kchunk;
    tn_tile<UPPER, false>(bi, bj, kb, min(K, kb + kchunk) - kb, M, N, X, ldx, Y, ldy, D + (int64_t)q * dstride, ldd,
                          As, Bs);
}

template <bool UPPER>
__global__ __launch_bounds__(TG_NT, 2)
void tn_gemm_kernel(int M, int N, int K, int kchunk, int ks, int tiles_m, int nitems, const double* __restrict__ X,
                    int64_t ldx, const double* __restrict__ Y, int64_t ldy, double* __restrict__ D, int64_t ldd,
                    int64_t dstride, const int* __restrict__ info)
{
    if (info && *info != 0) return;
    __shared__ double As[2][TG_BK][TG_P];   // As[k][i] = X(k0 + k, row0 + i)
    __shared__ double Bs[2][TG_BK][TG_P];   // Bs[k][j] = Y(k0 + k, col0 + j)
    for (int b = blockIdx.x; b < nitems; b += gridDim.x)
        tn_item<UPPER>(b, M, N, K, kchunk, ks, tiles_m, X, ldx, Y, ldy, D, ldd, dstride, As, Bs);
}

// R's rows by slabs: tiles [t0, t1) of the upper triangle of R's tile grid in
// row-major order (tile row r holds tiles (r, r), ..., (r, T - 1)), each over the
// K range [kb, kb + kc) of R = Q^T A; ADD: added to R (a later K range of tiles
// whose earlier ranges a previous launch stored).  Grid-stride over the tiles.
template <bool ADD>
__global__ __launch_bounds__(TG_NT, 2)
void r_slab_kernel(int n, int T, int t0, int t1, int kb, int kc, const double* __restrict__ X, int64_t ldx,
                   const double* __restrict__ Y, int64_t ldy, double* __restrict__ D, int64_t ldd,
                   const int* __restrict__ info)
{
    if (info && *info != 0) return;
    __shared__ double As[2][TG_BK][TG_P];
    __shared__ double Bs[2][TG_BK][TG_P];
    // tile row r starts at index r T - r (r - 1) / 2
    auto start = [&](int64_t r) { return r * T - r * (r - 1) / 2; };
    const double a = 2.0 * T + 1.0;
    for (int t = t0 + (int)blockIdx.x; t < t1; t += (int)gridDim.x) {
        int r = (int)((a - sqrt(fmax(a * a - 8.0 * t, 0.0))) * 0.5);
        r = r < 0 ? 0 : (r > T - 1 ? T - 1 : r);
        while (r > 0 && start(r) > t) --r;
        while (r + 1 < T && start(r + 1) <= t) ++r;
        const int bj = r + (int)(t - start(r));
        tn_tile<true, ADD>(r, bj, kb, kc, n, n, X, ldx, Y, ldy, D, ldd, As, Bs);
    }
}

template <bool UPPER, bool ADD>
__device__ __forceinline__ void tn_tile(int bi, int bj, int kb, int kc, int M, int N, const double* __restrict__ X,
                                        int64_t ldx, const double* __restrict__ Y, int64_t ldy,
                                        double* __restrict__ D, int64_t ldd, double (&As)[2][TG_BK][TG_P],
                                        double (&Bs)[2][TG_BK][TG_P])
{
    const int row0 = bi * TG_T, col0 = bj * TG_T;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave & 1, wc = wave >> 1;

    // Staging: 8 lanes read one 128-byte run (16 K values) of a column; a
    // thread owns K pair kp and columns sc + 32 u, u = 0..3.
    const int kp = 2 * (tid & 7), sc = tid >> 3;
    const rsrc_t rx = make_rsrc(X + kb + (int64_t)row0 * ldx);
    const rsrc_t ry = make_rsrc(Y + kb + (int64_t)col0 * ldy);
    int ox[4], oy[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int c = sc + 32 * u;
        ox[u] = row0 + c < M ? (kp + c * (int)ldx) * 8 : BUF_OOB;
        oy[u] = col0 + c < N ? (kp + c * (int)ldy) * 8 : BUF_OOB;
    }
    double xa[4][2], ya[4][2];
    const int nk = (kc + TG_BK - 1) / TG_BK;
    auto load = [&](int kt) {
        const int k0 = kt * TG_BK;
        if (k0 + TG_BK <= kc) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                load2(rx, ox[u] == BUF_OOB ? BUF_OOB : ox[u] + k0 * 8, xa[u][0], xa[u][1]);
                load2(ry, oy[u] == BUF_OOB ? BUF_OOB : oy[u] + k0 * 8, ya[u][0], ya[u][1]);
            }
        } else {
            // last, partial stage: K values at or past kc read as zero
            const bool v0 = k0 + kp < kc, v1 = k0 + kp + 1 < kc;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                xa[u][0] = buf_load<double>(rx, v0 && ox[u] != BUF_OOB ? ox[u] + k0 * 8 : BUF_OOB);
                xa[u][1] = buf_load<double>(rx, v1 && ox[u] != BUF_OOB ? ox[u] + k0 * 8 + 8 : BUF_OOB);
                ya[u][0] = buf_load<double>(ry, v0 && oy[u] != BUF_OOB ? oy[u] + k0 * 8 : BUF_OOB);
                ya[u][1] = buf_load<double>(ry, v1 && oy[u] != BUF_OOB ? oy[u] + k0 * 8 + 8 : BUF_OOB);
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            As[buf][kp][sc + 32 * u] = xa[u][0];
            As[buf][kp + 1][sc + 32 * u] = xa[u][1];
            Bs[buf][kp][sc + 32 * u] = ya[u][0];
            Bs[buf][kp + 1][sc + 32 * u] = ya[u][1];
        }
    };

    d4_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = zero_vec<d4_t>();
    // Transposed product tile (lanes along output rows): the MFMA A input is the
    // column operand, the B input the row operand.
    auto frags = [&](int buf, int k4, double (&fa)[4], double (&fb)[4]) {
        const int kk = 4 * k4 + (lane >> 4);
#pragma unroll
        for (int u = 0; u < 4; ++u) fa[u] = Bs[buf][kk][64 * wc + 16 * u + (lane & 15)];
#pragma unroll
        for (int u = 0; u < 4; ++u) fb[u] = As[buf][kk][64 * wr + 16 * u + (lane & 15)];
    };
    auto mma = [&](const double (&fa)[4], const double (&fb)[4]) {
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) acc[cb][r4] = mfma_f64(fa[cb], fb[r4], acc[cb][r4]);
    };
    auto compute = [&](int buf) {
        double fa0[4], fb0[4], fa1[4], fb1[4];
        __builtin_amdgcn_s_setprio(1);
        frags(buf, 0, fa0, fb0);
#pragma unroll
        for (int k4 = 0; k4 < TG_BK / 4; k4 += 2) {
            frags(buf, k4 + 1, fa1, fb1);
            mma(fa0, fb0);
            if (k4 + 2 < TG_BK / 4) frags(buf, k4 + 2, fa0, fb0);
            mma(fa1, fb1);
        }
        __builtin_amdgcn_s_setprio(0);
    };

    if (nk > 0) {
        load(0);
        store(0);
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            if (kt + 1 < nk) load(kt + 1);
            compute(kt & 1);      // zero-filled K positions add nothing
            if (kt + 1 < nk) store((kt + 1) & 1);
            __syncthreads();
        }
    }

#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = col0 + 64 * wc + 16 * cb + 4 * r + (lane >> 4);
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                const int i = row0 + 64 * wr + 16 * r4 + (lane & 15);
                if (i < M && j < N && (!UPPER || i <= j)) {
                    double* d = D + i + (int64_t)j * ldd;
                    *d = ADD ? *d + acc[cb][r4][r] : acc[cb][r4][r];
                }
            }
        }
    __syncthreads();
}

// D(i, j) = sum_q P[q * pstride + i + j * M] for q = 0, 1, ... in order
// (UPPER: entries with i > j are set to zero instead).
__global__ void tn_reduce_kernel(int M, int N, int ks, const double* __restrict__ P, int64_t pstride,
                                 double* __restrict__ D, int64_t ldd, int upper, const int* __restrict__ info)
{
    if (info && *info != 0) return;
    const int64_t total = (int64_t)M * N;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % M), j = (int)(e / M);
        double v = 0.0;
        if (!upper || i <= j)
            for (int q = 0; q < ks; ++q) v += P[q * pstride + e];
        D[i + (int64_t)j * ldd] = v;
    }
}

// D(i, j) = 0 for i > j (the strict lower triangle of an n x n matrix).
__global__ void zero_strict_lower_kernel(int n, double* __restrict__ D, int64_t ldd, const int* __restrict__ info)
{
    if (info && *info != 0) return;
    const int64_t total = (int64_t)n * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % n), j = (int)(e / n);
        if (i > j) D[i + (int64_t)j * ldd] = 0.0;
    }
}

// ---------------------------------------------------------------- in-block MGS
constexpr int QR_LDS = QR_PANEL_LDS_DOUBLES;   // panel slab, doubles
constexpr int QR_NT = 256;
constexpr int QR_SPIN_LIMIT = 1 << 20;

// Hand-off words of the panel: SENT marks a share not written yet; a share whose
// bits equal SENT (a NaN) is stored as the canonical quiet NaN instead.
constexpr unsigned long long QR_SENT = 0xFFFFFFFFFFFFFFFFull;
constexpr unsigned long long QR_QNAN = 0x7FF8000000000000ull;

__device__ __forceinline__ void share_put(double* p, double v) {
    unsigned long long b = (unsigned long long)__double_as_longlong(v);
    if (b == QR_SENT) b = QR_QNAN;
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void share_clear(double* p) {
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), QR_SENT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long share_peek(const double* p) {
    return __hip_atomic_load(reinterpret_cast<unsigned long long*>(const_cast<double*>(p)), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

// Step (b) of a panel round for one wave: the sums over workgroups [g_lo, g_hi)
// of the shares of columns lane + 64 u, u < NG, into accv (in workgroup order).
// GB shares per column are loaded at once and polled until none is SENT;
// out-of-range workgroups load a clamped (valid) address and are ignored.
template <int NG, int GB>
__device__ __forceinline__ bool gather_shares(const double* pj, int WS, int g_lo, int g_hi, int lane, int nc,
                                              double (&accv)[4]) {
    for (int gg0 = g_lo; gg0 < g_hi; gg0 += GB) {
        unsigned long long v[NG][GB];
        int spins = 0;
        while (true) {
            bool pending = false;
#pragma unroll
            for (int u = 0; u < NG; ++u)
#pragma unroll
                for (int e = 0; e < GB; ++e) {
                    const int gg = min(gg0 + e, g_hi - 1);
                    const int ci = min(lane + 64 * u, nc - 1);
                    v[u][e] = share_peek(pj + (size_t)gg * WS + ci);
                }
#pragma unroll
            for (int u = 0; u < NG; ++u)
#pragma unroll
                for (int e = 0; e < GB; ++e)
                    pending |= (gg0 + e < g_hi && lane + 64 * u < nc && v[u][e] == QR_SENT);
            if (!__any(pending)) break;
            if (++spins > QR_SPIN_LIMIT) return false;
            __builtin_amdgcn_s_sleep(1);
        }
#pragma unroll
        for (int u = 0; u < NG; ++u)
#pragma unroll
            for (int e = 0; e < GB; ++e)
                if (gg0 + e < g_hi) accv[u] += __longlong_as_double((long long)v[u][e]);
    }
    return true;
}

// Block columns [0, w) of Mp (m rows, leading dimension ldm) are replaced by the
// orthonormal columns of modified Gram-Schmidt.  Workgroup g holds rows
// [g RR, (g+1) RR) in LDS (column pitch RR + 1); gridDim.x = P = ceil(m / RR)
// workgroups, all resident at once (one per CU, by their LDS).
//
// Round j (global round G = col0 + j): (a) each workgroup forms its rows' share
// of v_j . v_c, c = j..w-1 (wave h sums rows [h RR/4, (h+1) RR/4) in row order,
// the four waves' sums are added in wave order); it clears its own slots of
// buffer (G + 1) % 3 and then publishes the shares in its slots of buffer G % 3,
// part[G % 3][g][c - j]; (b) each workgroup reads the P shares of every column,
// polling each slot until it no longer holds SENT, and adds them in workgroup
// order (wave h over workgroups [h P/4, (h+1) P/4) in order, then the four in
// wave order): all workgroups obtain the same sums S_c; (c) ||v_j|| = sqrt(S_j),
// q_j = v_j / ||v_j||, and v_c -= q_j (S_c / ||v_j||) for c > j (S_c / ||v_j|| is
// q_j . v_c up to rounding).
// The shares are their own ready flags, so no separate count is needed.  A
// workgroup clears buffer (G + 1) % 3, last used in round G - 2, only after it has
// read every share of round G - 1, which every workgroup published after it had
// read round G - 2; and it clears before it publishes round G (the same thread
// writes both, with a completion wait between), so whoever reads round G + 1
// finds SENT or the new share.  Global round numbers keep the rotation going
// across the panels of one factorisation; the slots are cleared once per call.
// Shares are agent-scope atomics, which gfx950 serves at the device's coherence
// point (no stale per-XCD L2 copy), so no cache-wide write-back or invalidate is
// needed.
// A norm that is not > 0 (zero or NaN) sets *info = col0 + j + 1 and ends the
// kernel in every workgroup (all hold the same sums); a wait that exceeds its
// bound sets *info = -1.  The panel is at most QR_PANEL_WMAX = 256 columns wide,
// so a lane holds at most 4 of them.
template <int RR>
__global__ __launch_bounds__(QR_NT, 1)
void qr_panel_kernel(int m, int w, int col0, double* __restrict__ Mp, int64_t ldm, double* part, int* info)
{
    static_assert(RR % 4 == 0 && RR <= QR_NT && QR_NT % RR == 0, "row split");
    constexpr int RP = RR + 1;
    constexpr int RQ = RR / 4;
    constexpr int CSTEP = QR_NT / RR;
    constexpr int WS = QR_PANEL_WMAX;      // slot row length (fixed across panels)
    __shared__ double slab[QR_LDS];
    __shared__ double red[4][QR_PANEL_WMAX];
    __shared__ double dv[QR_PANEL_WMAX];
    __shared__ double dq[QR_PANEL_WMAX];
    __shared__ int bad;
    if (__hip_atomic_load(info, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
    const int P = gridDim.x, g = blockIdx.x;
    const int t = threadIdx.x, lane = t & 63, h = t >> 6;
    const int r0 = g * RR;
    const size_t bstride = (size_t)P * WS;
    for (int idx = t; idx < w * RR; idx += QR_NT) {
        const int c = idx / RR, r = idx % RR;
        slab[c * RP + r] = r0 + r < m ? Mp[r0 + r + (int64_t)c * ldm] : 0.0;
    }
    if (t == 0) bad = 0;
    const int g_lo = h * P / 4, g_hi = (h + 1) * P / 4;
    const int ur = t % RR, uc = t / RR;
    __syncthreads();

    for (int j = 0; j < w; ++j) {
        const int nc = w - j;
        const int G = col0 + j;
        double* pj = part + (size_t)(G % 3) * bstride;
        double* pn = part + (size_t)((G + 1) % 3) * bstride;
        // (a)
        for (int ci = lane; ci < nc; ci += 64) {
            const double* vj = slab + j * RP + h * RQ;
            const double* vc = slab + (j + ci) * RP + h * RQ;
            double acc = 0.0;
#pragma unroll 8
            for (int r = 0; r < RQ; ++r) acc += vj[r] * vc[r];
            red[h][ci] = acc;
        }
        __syncthreads();
        if (t < WS) {
            share_clear(pn + (size_t)g * WS + t);
            __builtin_amdgcn_s_waitcnt(0);   // the clear lands before this round's share
            if (t < nc) share_put(pj + (size_t)g * WS + t, ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t]);
        }
        __syncthreads();   // every share is read from red before (b) overwrites it
        // (b) a lane sums the shares of columns lane + 64 u; the gather is
        // specialised on the number of 64-column groups so that no load goes to
        // a column past nc, and a wave's whole workgroup range is loaded in one
        // batch when it spans at most 32 workgroups (two column groups or fewer)
        {
            double accv[4] = {0.0, 0.0, 0.0, 0.0};
            const int ng = (nc + 63) / 64;
            bool ok;
            if (ng == 1) ok = gather_shares<1, 32>(pj, WS, g_lo, g_hi, lane, nc, accv);
            else if (ng == 2) ok = gather_shares<2, 32>(pj, WS, g_lo, g_hi, lane, nc, accv);
            else if (ng == 3) ok = gather_shares<3, 16>(pj, WS, g_lo, g_hi, lane, nc, accv);
            else ok = gather_shares<4, 16>(pj, WS, g_lo, g_hi, lane, nc, accv);
            if (!ok) bad = 1;
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (lane + 64 * u < nc) red[h][lane + 64 * u] = accv[u];
        }
        __syncthreads();
        if (bad) {
            if (t == 0) __hip_atomic_store(info, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        if (t < nc) dv[t] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
        __syncthreads();
        // (c)
        const double nrm = sqrt(dv[0]);
        if (!(nrm > 0.0)) {
            if (g == 0 && t == 0) __hip_atomic_store(info, col0 + j + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        if (t > 0 && t < nc) dq[t] = dv[t] / nrm;
        const double qv = slab[j * RP + ur] / nrm;
        __syncthreads();                     // every read of v_j is done, dq is complete
        if (uc == 0) slab[j * RP + ur] = qv;
        for (int c = j + 1 + uc; c < w; c += CSTEP) slab[c * RP + ur] -= qv * dq[c - j];
        __syncthreads();
    }
    for (int idx = t; idx < w * RR; idx += QR_NT) {
        const int c = idx / RR, r = idx % RR;
        if (r0 + r < m) Mp[r0 + r + (int64_t)c * ldm] = slab[c * RP + r];
    }
}

__global__ void qr_part_clear_kernel(double* part, size_t count) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        reinterpret_cast<unsigned long long*>(part)[i] = QR_SENT;
}


}  // namespace

// ---------------------------------------------------------------- host side
int qr_panel_rows(int64_t m) {
    // 128 rows per workgroup while that needs at most one workgroup per CU,
    // else 256 (then the panel is at most 71 columns wide)
    const int64_t cus = std::min(cu_count(), QR_PANEL_MAXWG);
    if ((m + 127) / 128 <= cus) return 128;
    if ((m + 255) / 256 <= cus) return 256;
    return 0;
}

int qr_panel_workgroups(int64_t m) {
    const int rr = qr_panel_rows(m);
    return rr == 0 ? 0 : (int)((m + rr - 1) / rr);
}

int qr_panel_max_width(int64_t m) {
    const int rr = qr_panel_rows(m);
    if (rr == 0) return 0;
    return std::min(QR_PANEL_WMAX, QR_PANEL_LDS_DOUBLES / (rr + 1));
}

// Three rotating buffers of P x QR_PANEL_WMAX slots (independent of the panel width).
size_t qr_panel_part_elems(int64_t m, int w) {
    (void)w;
    const int rr = qr_panel_rows(m);
    if (rr == 0) return 0;
    return 3 * (size_t)((m + rr - 1) / rr) * (size_t)QR_PANEL_WMAX;
}

hipError_t launch_qr_part_clear(int64_t m, double* part, hipStream_t st) {
    const size_t count = qr_panel_part_elems(m, 0);
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(qr_part_clear_kernel, dim3((unsigned)std::min<size_t>(1024, (count + 255) / 256)), dim3(256),
                       0, st, part, count);
    return hipGetLastError();
}

hipError_t launch_qr_panel(int m, int w, int col0, double* Mp, int64_t ldm, double* part, int* info, hipStream_t st) {
    if (m <= 0 || w <= 0) return hipSuccess;
    const int rr = qr_panel_rows(m);
    if (rr == 0 || w > qr_panel_max_width(m)) return hipErrorInvalidValue;
    const int P = (m + rr - 1) / rr;
    if (P > QR_PANEL_MAXWG) return hipErrorInvalidValue;
    if (rr == 128)
        hipLaunchKernelGGL(qr_panel_kernel<128>, dim3(P), dim3(QR_NT), 0, st, m, w, col0, Mp, ldm, part, info);
    else
        hipLaunchKernelGGL(qr_panel_kernel<256>, dim3(P), dim3(QR_NT), 0, st, m, w, col0, Mp, ldm, part, info);
    return hipGetLastError();
}

namespace {
struct TnPlan {
    int tiles_m, tiles, ks, kchunk;
};

TnPlan tn_plan(int M, int N, int K, bool upper) {
    TnPlan p;
    p.tiles_m = (M + TG_T - 1) / TG_T;
    const int tn = (N + TG_T - 1) / TG_T;
    p.tiles = upper ? tn * (tn + 1) / 2 : p.tiles_m * tn;
    const int target = 2 * cu_count();
    int ks = 1;
    while (ks < 16 && (int64_t)p.tiles * ks < target && K / (2 * ks) >= 512) ks *= 2;
    int kchunk = (K + ks - 1) / ks;
    kchunk = (kchunk + TG_BK - 1) / TG_BK * TG_BK;
    p.kchunk = std::max(kchunk, TG_BK);
    p.ks = (K + p.kchunk - 1) / p.kchunk;
    if (p.ks < 1) p.ks = 1;
    return p;
}
TnPlan tn_plan_unsplit(int M, int N, int K, bool upper) {
    TnPlan p = tn_plan(M, N, K, upper);
    p.ks = 1;
    p.kchunk = (K + TG_BK - 1) / TG_BK * TG_BK;
    return p;
}
}  // namespace

hipError_t launch_zero_strict_lower(int n, double* D, int64_t ldd, const int* info, hipStream_t st) {
    if (n <= 1) return hipSuccess;
    hipLaunchKernelGGL(zero_strict_lower_kernel, dim3(std::min<int64_t>(4096, ((int64_t)n * n + 255) / 256)),
                       dim3(256), 0, st, n, D, ldd, info);
    return hipGetLastError();
}

size_t tn_gemm_part_elems(int M, int N, int K, bool upper) {
    if (M <= 0 || N <= 0 || K <= 0) return 0;
    const TnPlan p = tn_plan(M, N, K, upper);
    return p.ks > 1 ? (size_t)p.ks * (size_t)M * (size_t)N : 0;
}

bool tn_gemm_fits(int64_t K, int64_t ldx, int64_t ldy) {
    const int64_t span = (int64_t)K + (int64_t)TG_T * std::max(ldx, ldy);
    return span * 8 < (int64_t)BUF_RECORDS - 64;
}

int r_slab_tile() { return TG_T; }

int64_t r_slab_tiles_before(int n, int rows) {
    const int64_t T = (n + TG_T - 1) / TG_T;
    const int64_t r = std::min<int64_t>(std::max(rows, 0), T);
    return r * T - r * (r - 1) / 2;
}

hipError_t launch_r_slab(int n, int64_t t0, int64_t t1, int k0, int k1, const double* Q, int64_t ldq, const double* A,
                         int64_t lda, double* R, int64_t ldr, const int* info, hipStream_t st, int max_wg) {
    if (t1 <= t0 || k1 <= k0) return hipSuccess;
    if (t0 < 0 || t1 > r_slab_tiles_before(n, n) || k0 < 0) return hipErrorInvalidValue;
    const int T = (n + TG_T - 1) / TG_T;
    const int64_t nt = t1 - t0;
    const int nwg = (int)std::min<int64_t>(nt, max_wg > 0 ? max_wg : nt);
    if (k0 > 0)
        hipLaunchKernelGGL(r_slab_kernel<true>, dim3(nwg), dim3(TG_NT), 0, st, n, T, (int)t0, (int)t1, k0, k1 - k0, Q,
                           ldq, A, lda, R, ldr, info);
    else
        hipLaunchKernelGGL(r_slab_kernel<false>, dim3(nwg), dim3(TG_NT), 0, st, n, T, (int)t0, (int)t1, k0, k1 - k0,
                           Q, ldq, A, lda, R, ldr, info);
    return hipGetLastError();
}

hipError_t launch_tn_gemm(int M, int N, int K, const double* X, int64_t ldx, const double* Y, int64_t ldy, double* D,
                          int64_t ldd, bool upper, double* part, const int* info, hipStream_t st, int max_wg) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (upper && M != N) return hipErrorInvalidValue;
    if (K <= 0) {
        // an empty sum: zeros (and the strict lower triangle for UPPER)
        hipLaunchKernelGGL(tn_reduce_kernel, dim3(std::min<int64_t>(4096, ((int64_t)M * N + 255) / 256)), dim3(256),
                           0, st, M, N, 0, (const double*)nullptr, (int64_t)0, D, ldd, upper ? 1 : 0, info);
        return hipGetLastError();
    }
    if (!tn_gemm_fits(K, ldx, ldy)) return hipErrorInvalidValue;
    const TnPlan p = max_wg > 0 ? tn_plan_unsplit(M, N, K, upper) : tn_plan(M, N, K, upper);
    const int nitems = p.tiles * p.ks;
    const int nwg = max_wg > 0 ? std::min(nitems, max_wg) : nitems;
    if (p.ks == 1) {
        if (upper)
            hipLaunchKernelGGL(tn_gemm_kernel<true>, dim3(nwg), dim3(TG_NT), 0, st, M, N, K, p.kchunk, 1, p.tiles_m,
                               nitems, X, ldx, Y, ldy, D, ldd, (int64_t)0, info);
        else
            hipLaunchKernelGGL(tn_gemm_kernel<false>, dim3(nwg), dim3(TG_NT), 0, st, M, N, K, p.kchunk, 1, p.tiles_m,
                               nitems, X, ldx, Y, ldy, D, ldd, (int64_t)0, info);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || !upper) return e;
        hipLaunchKernelGGL(zero_strict_lower_kernel, dim3(std::min<int64_t>(4096, ((int64_t)M * N + 255) / 256)),
                           dim3(256), 0, st, M, D, ldd, info);
        return hipGetLastError();
    }
    if (part == nullptr) return hipErrorInvalidValue;
    const int64_t ps = (int64_t)M * N;
    if (upper)
        hipLaunchKernelGGL(tn_gemm_kernel<true>, dim3(nwg), dim3(TG_NT), 0, st, M, N, K, p.kchunk, p.ks, p.tiles_m,
                           nitems, X, ldx, Y, ldy, part, (int64_t)M, ps, info);
    else
        hipLaunchKernelGGL(tn_gemm_kernel<false>, dim3(nwg), dim3(TG_NT), 0, st, M, N, K, p.kchunk, p.ks, p.tiles_m,
                           nitems, X, ldx, Y, ldy, part, (int64_t)M, ps, info);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(tn_reduce_kernel, dim3(std::min<int64_t>(4096, (ps + 255) / 256)), dim3(256), 0, st, M, N,
                       p.ks, (const double*)part, ps, D, ldd, upper ? 1 : 0, info);
    return hipGetLastError();
}

}  // namespace ff
