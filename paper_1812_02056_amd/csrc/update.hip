// update.hip -- the deferred trailing update of the delayed-update factorisations.
//
// Sec. 2 of arXiv 1812.02056, Algorithm 1: every s columns the pending block
// R = L[c.., z..c-1] of the factor gives S = R R^T, subtracted from the trailing
// square A[c.., c..]; Algorithm 2 uses S = R_L R_U.  Here S is never stored: each
// workgroup forms one 128 x 128 output tile of S with MFMA instructions, K-loop
// over the pending columns staged through LDS, and subtracts it from C in the
// write-back.
//
// One kernel template covers every product the library needs:
//     C(i, j) -= sum_k X(i, k) Y(j, k)      i < M, j < N
// with C and X column-major (C[i + j*ldc], X[i + k*ldx]) and Y either the rows of
// a column-major N x K matrix (YROWS: Y[j + k*ldy], Algorithm 1's R R^T) or a
// column-major K x N matrix (Y[k + j*ldy], Algorithm 2's R_L R_U).  With LOWER
// only entries with i - j >= shift are written (the lower triangle of the
// trailing square, or of a region of it); tiles wholly above that line are
// skipped, and for a square lower region (shift 0) the grid enumerates only the
// tiles on or below the diagonal.
//
// Variants by element type:
//   double   binary64 operands and accumulation (v_mfma_f64_16x16x4f64)
//   float    binary32 (v_mfma_f32_16x16x4f32)
//   bf16     binary32 storage, operands rounded to bfloat16 while staged into
//            LDS, binary32 accumulation (v_mfma_f32_16x16x32_bf16); YROWS only.
#include "common.hpp"
#include "internal.hpp"

namespace ff {

namespace {

constexpr int NT = 256;    // 4 waves; wave (wr, wc) owns a 64 x 64 quarter of the tile
constexpr int TM = UPD_TILE;

struct Grid {
    int nbm, nbn;      // tiles along M and N
    int nsm, nsn;      // super-tiles along M and N
    int tri;           // 1: square lower region enumerated as a triangle of super-tiles
    int shift;         // LOWER: write only i - j >= shift
};

// Map the flat workgroup index to an output tile (bi, bj).  Returns false when
// the slot is empty.  Workgroups are dealt to the 8 XCDs round-robin; each XCD
// works through whole 8 x 8 super-tiles so the 16 operand blocks of a
// super-tile stay in that XCD's L2.
__device__ __forceinline__ bool tile_of_block(const Grid& g, bool lower, int& bi, int& bj) {
    const int bid = blockIdx.x;
    const int xcd = bid % N_XCD;
    const int k = bid / N_XCD;
    int u = (k / UPD_WG_PER_SUPER) * N_XCD + xcd;
    const int within = k % UPD_WG_PER_SUPER;
    int SI, SJ;
    if (g.tri) {
        const int nsup = g.nsm * (g.nsm + 1) / 2;
        if (u >= nsup) return false;
        SJ = 0;
        while (u >= g.nsm - SJ) { u -= g.nsm - SJ; ++SJ; }
        SI = SJ + u;
    } else {
        if (u >= g.nsm * g.nsn) return false;
        SI = u % g.nsm;
        SJ = u / g.nsm;
    }
    bi = SI * UPD_GROUP + (within % UPD_GROUP);
    bj = SJ * UPD_GROUP + (within / UPD_GROUP);
    if (bi >= g.nbm || bj >= g.nbn) return false;
    if (lower && (bi * TM + TM - 1) - bj * TM < g.shift) return false;   // wholly above the line
    return true;
}

template <typename T> struct upd_cfg { static constexpr int BK = 16; };

template <typename T, bool YROWS, bool LOWER>
__global__ __launch_bounds__(NT, 2)
void update_kernel(int M, int N, int K, T* __restrict__ C, int64_t ldc,
                   const T* __restrict__ X, int64_t ldx,
                   const T* __restrict__ Y, int64_t ldy, Grid g, const int* __restrict__ info)
{
    if (info && *info != 0) return;
    constexpr int BK = upd_cfg<T>::BK;
    constexpr int NLD = BK * TM / NT;          // operand elements each thread stages per K step
    typedef acc_traits<T> AT;
    typedef typename AT::vec V;

    __shared__ T As[2][BK][TM];   // row operand  X[row0 + r, k]       stored [k][r]
    __shared__ T Bs[2][BK][TM];   // column operand                    stored [k][c ^ (k % 16)]

    int bi, bj;
    if (!tile_of_block(g, LOWER, bi, bj)) return;
    const int row0 = bi * TM, col0 = bj * TM;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave & 1, wc = wave >> 1;
    // a quarter wholly above the line computes nothing
    const bool active = !LOWER || (row0 + 64 * wr + 63) - (col0 + 64 * wc) >= g.shift;

    V acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = zero_vec<V>();

    T ra[NLD], rb[NLD];
    auto load = [&](int kt) {
        const int k0 = kt * BK;
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            const int idx = tid + NT * q;
            const int kk = idx / TM, r = idx % TM;
            const int gr = row0 + r, gk = k0 + kk;
            ra[q] = (gr < M && gk < K) ? X[(int64_t)gr + (int64_t)gk * ldx] : T(0);
        }
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            const int idx = tid + NT * q;
            if (YROWS) {
                const int kk = idx / TM, c = idx % TM;
                const int gc = col0 + c, gk = k0 + kk;
                rb[q] = (gc < N && gk < K) ? Y[(int64_t)gc + (int64_t)gk * ldy] : T(0);
            } else {
                const int kk = idx % BK, c = idx / BK;
                const int gc = col0 + c, gk = k0 + kk;
                rb[q] = (gc < N && gk < K) ? Y[(int64_t)gk + (int64_t)gc * ldy] : T(0);
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            const int idx = tid + NT * q;
            As[buf][idx / TM][idx % TM] = ra[q];
        }
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            const int idx = tid + NT * q;
            int kk, c;
            if (YROWS) { kk = idx / TM; c = idx % TM; }
            else { kk = idx % BK; c = idx / BK; }
            Bs[buf][kk][c ^ (kk & 15)] = rb[q];
        }
    };

    const int nk = (K + BK - 1) / BK;
    load(0);
    store(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) load(kt + 1);
        if (active) {
#pragma unroll
            for (int k4 = 0; k4 < BK / 4; ++k4) {
                const int kk = 4 * k4 + (lane >> 4);
                T fa[4], fb[4];
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
                    fa[cb] = Bs[buf][kk][(64 * wc + 16 * cb + (lane & 15)) ^ (kk & 15)];
#pragma unroll
                for (int r4 = 0; r4 < 4; ++r4)
                    fb[r4] = As[buf][kk][64 * wr + 16 * r4 + (lane & 15)];
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                    for (int r4 = 0; r4 < 4; ++r4)
                        acc[cb][r4] = AT::mfma(fa[cb], fb[r4], acc[cb][r4]);
            }
        }
        if (kt + 1 < nk) store(buf ^ 1);
        __syncthreads();
    }
    if (!active) return;

    // Fused write-back: C[i, j] -= S[i, j].
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) {
            const int gi = row0 + 64 * wr + 16 * r4 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gj = col0 + 64 * wc + 16 * cb + AT::col(lane, r);
                if (gi < M && gj < N && (!LOWER || gi - gj >= g.shift)) {
                    T* p = C + (int64_t)gi + (int64_t)gj * ldc;
                    *p = *p - acc[cb][r4][r];
                }
            }
        }
    }
}

// bfloat16-operand variant (YROWS form, optional LOWER); binary32 storage and
// accumulation.  Operand tiles are stored row-major [row][k] with a 40-element
// row pitch (80 bytes) so the 16-byte fragment reads of a lane group hit
// distinct LDS banks.
constexpr int BF_BK = 32;
constexpr int BF_PITCH = 40;

template <bool LOWER>
__global__ __launch_bounds__(NT, 2)
void update_bf16_kernel(int M, int N, int K, float* __restrict__ C, int64_t ldc,
                        const float* __restrict__ X, int64_t ldx, const float* __restrict__ Y, int64_t ldy,
                        Grid g, const int* __restrict__ info)
{
    if (info && *info != 0) return;
    __shared__ __attribute__((aligned(16))) __bf16 As[2][TM][BF_PITCH];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[2][TM][BF_PITCH];

    int bi, bj;
    if (!tile_of_block(g, LOWER, bi, bj)) return;
    const int row0 = bi * TM, col0 = bj * TM;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave & 1, wc = wave >> 1;
    const bool active = !LOWER || (row0 + 64 * wr + 63) - (col0 + 64 * wc) >= g.shift;

    f4_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = zero_vec<f4_t>();

    // thread t stages row (t % 128), k-half (t / 128) of both operands
    const int sr = tid % TM, sh = tid / TM;
    float ra[16], rb[16];
    auto load = [&](int kt) {
        const int k0 = kt * BF_BK + 16 * sh;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int gk = k0 + e;
            const int gr = row0 + sr, gc = col0 + sr;
            ra[e] = (gr < M && gk < K) ? X[(int64_t)gr + (int64_t)gk * ldx] : 0.0f;
            rb[e] = (gc < N && gk < K) ? Y[(int64_t)gc + (int64_t)gk * ldy] : 0.0f;
        }
    };
    auto store = [&](int buf) {
        bf8_t a0, a1, b0, b1;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            a0[e] = to_bf16(ra[e]);
            a1[e] = to_bf16(ra[8 + e]);
            b0[e] = to_bf16(rb[e]);
            b1[e] = to_bf16(rb[8 + e]);
        }
        *reinterpret_cast<bf8_t*>(&As[buf][sr][16 * sh]) = a0;
        *reinterpret_cast<bf8_t*>(&As[buf][sr][16 * sh + 8]) = a1;
        *reinterpret_cast<bf8_t*>(&Bs[buf][sr][16 * sh]) = b0;
        *reinterpret_cast<bf8_t*>(&Bs[buf][sr][16 * sh + 8]) = b1;
    };

    const int nk = (K + BF_BK - 1) / BF_BK;
    load(0);
    store(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) load(kt + 1);
        if (active) {
            bf8_t fa[4], fb[4];
            const int ko = 8 * (lane >> 4);
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
                fa[cb] = *reinterpret_cast<const bf8_t*>(&Bs[buf][64 * wc + 16 * cb + (lane & 15)][ko]);
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4)
                fb[r4] = *reinterpret_cast<const bf8_t*>(&As[buf][64 * wr + 16 * r4 + (lane & 15)][ko]);
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int r4 = 0; r4 < 4; ++r4)
                    acc[cb][r4] = mfma_bf16(fa[cb], fb[r4], acc[cb][r4]);
        }
        if (kt + 1 < nk) store(buf ^ 1);
        __syncthreads();
    }
    if (!active) return;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) {
            const int gi = row0 + 64 * wr + 16 * r4 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gj = col0 + 64 * wc + 16 * cb + acc_traits<float>::col(lane, r);
                if (gi < M && gj < N && (!LOWER || gi - gj >= g.shift)) {
                    float* p = C + (int64_t)gi + (int64_t)gj * ldc;
                    *p = *p - acc[cb][r4][r];
                }
            }
        }
    }
}

Grid make_grid(int M, int N, bool lower, int shift, int& nwg) {
    Grid g;
    g.nbm = (M + TM - 1) / TM;
    g.nbn = (N + TM - 1) / TM;
    g.nsm = (g.nbm + UPD_GROUP - 1) / UPD_GROUP;
    g.nsn = (g.nbn + UPD_GROUP - 1) / UPD_GROUP;
    g.tri = (lower && M == N && shift == 0) ? 1 : 0;
    g.shift = shift;
    const int nsup = g.tri ? g.nsm * (g.nsm + 1) / 2 : g.nsm * g.nsn;
    nwg = ((nsup + N_XCD - 1) / N_XCD) * N_XCD * UPD_WG_PER_SUPER;
    return g;
}

}  // namespace

template <typename T>
hipError_t launch_update(int M, int N, int K, T* C, int64_t ldc, const T* X, int64_t ldx, const T* Y, int64_t ldy,
                         bool yrows, bool lower, int shift, const int* info, hipStream_t st) {
    if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
    int nwg;
    const Grid g = make_grid(M, N, lower, shift, nwg);
    if (yrows) {
        if (lower)
            hipLaunchKernelGGL((update_kernel<T, true, true>), dim3(nwg), dim3(NT), 0, st, M, N, K, C, ldc, X, ldx, Y,
                               ldy, g, info);
        else
            hipLaunchKernelGGL((update_kernel<T, true, false>), dim3(nwg), dim3(NT), 0, st, M, N, K, C, ldc, X, ldx,
                               Y, ldy, g, info);
    } else {
        if (lower)
            hipLaunchKernelGGL((update_kernel<T, false, true>), dim3(nwg), dim3(NT), 0, st, M, N, K, C, ldc, X, ldx,
                               Y, ldy, g, info);
        else
            hipLaunchKernelGGL((update_kernel<T, false, false>), dim3(nwg), dim3(NT), 0, st, M, N, K, C, ldc, X, ldx,
                               Y, ldy, g, info);
    }
    return hipGetLastError();
}

hipError_t launch_update_bf16(int M, int N, int K, float* C, int64_t ldc, const float* X, int64_t ldx,
                              const float* Y, int64_t ldy, bool lower, int shift, const int* info, hipStream_t st) {
    if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
    int nwg;
    const Grid g = make_grid(M, N, lower, shift, nwg);
    if (lower)
        hipLaunchKernelGGL(update_bf16_kernel<true>, dim3(nwg), dim3(NT), 0, st, M, N, K, C, ldc, X, ldx, Y, ldy, g,
                           info);
    else
        hipLaunchKernelGGL(update_bf16_kernel<false>, dim3(nwg), dim3(NT), 0, st, M, N, K, C, ldc, X, ldx, Y, ldy, g,
                           info);
    return hipGetLastError();
}

template hipError_t launch_update<double>(int, int, int, double*, int64_t, const double*, int64_t, const double*,
                                          int64_t, bool, bool, int, const int*, hipStream_t);
template hipError_t launch_update<float>(int, int, int, float*, int64_t, const float*, int64_t, const float*,
                                         int64_t, bool, bool, int, const int*, hipStream_t);

}  // namespace ff
