// update.hip -- the deferred trailing update of the delayed-update factorisations.
//
// Sec. 2 of arXiv 1812.02056, Algorithm 1: every s columns the pending block
// R = L[c.., z..c-1] of the factor gives S = R R^T, subtracted from the trailing
// square A[c.., c..]; Algorithm 2 uses S = R_L R_U.  Here S is never stored: each
// workgroup forms one 128 x 128 output tile of S with MFMA instructions, K-loop
// over the w pending columns staged through LDS, and subtracts it from C in the
// write-back.  Cholesky updates only the lower triangle (tiles with bi >= bj;
// inside diagonal tiles only i >= j is written), LU the whole square.
//
// Variants:
//   update_kernel<double>   binary64 operands and accumulation (v_mfma_f64_16x16x4f64)
//   update_kernel<float>    binary32 (v_mfma_f32_16x16x4f32)
//   update_bf16_kernel      binary32 storage, operands rounded to bfloat16 while
//                           staged into LDS, binary32 accumulation
//                           (v_mfma_f32_16x16x32_bf16)
#include "common.hpp"
#include "internal.hpp"

namespace ff {

namespace {

constexpr int NT = 256;    // 4 waves; wave (wr, wc) owns a 64 x 64 quarter of the tile
constexpr int TM = UPD_TILE;

// Map the flat workgroup index to an output tile (bi, bj).  Returns false when
// the slot is empty (outside the matrix, or above the diagonal for Cholesky).
__device__ __forceinline__ bool tile_of_block(bool lower_only, int nb, int nsb, int& bi, int& bj) {
    const int bid = blockIdx.x;
    const int xcd = bid % N_XCD;
    const int k = bid / N_XCD;
    int u = (k / UPD_WG_PER_SUPER) * N_XCD + xcd;
    const int within = k % UPD_WG_PER_SUPER;
    int SI, SJ;
    if (lower_only) {
        const int nsup = nsb * (nsb + 1) / 2;
        if (u >= nsup) return false;
        SJ = 0;
        while (u >= nsb - SJ) { u -= nsb - SJ; ++SJ; }
        SI = SJ + u;
    } else {
        if (u >= nsb * nsb) return false;
        SI = u % nsb;
        SJ = u / nsb;
    }
    bi = SI * UPD_GROUP + (within % UPD_GROUP);
    bj = SJ * UPD_GROUP + (within / UPD_GROUP);
    if (bi >= nb || bj >= nb) return false;
    if (lower_only && bi < bj) return false;
    return true;
}

template <typename T> struct upd_cfg;
template <> struct upd_cfg<double> { static constexpr int BK = 16; };
template <> struct upd_cfg<float> { static constexpr int BK = 16; };

// C -= X * Y^T-ish product, see the file header.  GEMM selects Algorithm 2's
// form (Y is w x m, column operand Y[k, j]); otherwise the column operand is
// X itself (rows j of X), Algorithm 1's R R^T.
template <typename T, bool GEMM>
__global__ __launch_bounds__(NT, 2)
void update_kernel(int m, int w, T* __restrict__ C, int64_t ldc,
                   const T* __restrict__ X, int64_t ldx,
                   const T* __restrict__ Y, int64_t ldy, int nb, int nsb, const int* __restrict__ info)
{
    if (info && *info != 0) return;
    constexpr int BK = upd_cfg<T>::BK;
    constexpr int NLD = BK * TM / NT;          // operand elements each thread stages per K step
    typedef acc_traits<T> AT;
    typedef typename AT::vec V;

    __shared__ T As[2][BK][TM];   // row operand  X[row0 + r, k]       stored [k][r]
    __shared__ T Bs[2][BK][TM];   // column operand                    stored [k][c ^ (k % 16)]

    int bi, bj;
    if (!tile_of_block(!GEMM, nb, nsb, bi, bj)) return;
    const int row0 = bi * TM, col0 = bj * TM;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave & 1, wc = wave >> 1;
    const bool diag = !GEMM && (bi == bj);
    const bool active = !(diag && wr == 0 && wc == 1);   // that quarter lies above the diagonal

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
            ra[q] = (gr < m && gk < w) ? X[(int64_t)gr + (int64_t)gk * ldx] : T(0);
        }
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            const int idx = tid + NT * q;
            if (GEMM) {
                const int kk = idx % BK, c = idx / BK;
                const int gc = col0 + c, gk = k0 + kk;
                rb[q] = (gc < m && gk < w) ? Y[(int64_t)gk + (int64_t)gc * ldy] : T(0);
            } else {
                const int kk = idx / TM, c = idx % TM;
                const int gc = col0 + c, gk = k0 + kk;
                rb[q] = (gc < m && gk < w) ? X[(int64_t)gc + (int64_t)gk * ldx] : T(0);
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
            if (GEMM) { kk = idx % BK; c = idx / BK; }
            else { kk = idx / TM; c = idx % TM; }
            Bs[buf][kk][c ^ (kk & 15)] = rb[q];
        }
    };

    const int nk = (w + BK - 1) / BK;
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
                if (gi < m && gj < m && (GEMM || gi >= gj)) {
                    T* p = C + (int64_t)gi + (int64_t)gj * ldc;
                    *p = *p - acc[cb][r4][r];
                }
            }
        }
    }
}

// bfloat16-operand variant of the lower-triangle update; binary32 storage and
// accumulation.  Operand tiles are stored row-major [row][k] with a 40-element
// row pitch (80 bytes) so the 16-byte fragment reads of a lane group hit
// distinct LDS banks.
constexpr int BF_BK = 32;
constexpr int BF_PITCH = 40;

__global__ __launch_bounds__(NT, 2)
void update_bf16_kernel(int m, int w, float* __restrict__ C, int64_t ldc,
                        const float* __restrict__ X, int64_t ldx, int nb, int nsb,
                        const int* __restrict__ info)
{
    if (info && *info != 0) return;
    __shared__ __attribute__((aligned(16))) __bf16 As[2][TM][BF_PITCH];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[2][TM][BF_PITCH];

    int bi, bj;
    if (!tile_of_block(true, nb, nsb, bi, bj)) return;
    const int row0 = bi * TM, col0 = bj * TM;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave & 1, wc = wave >> 1;
    const bool diag = (bi == bj);
    const bool active = !(diag && wr == 0 && wc == 1);

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
            ra[e] = (gr < m && gk < w) ? X[(int64_t)gr + (int64_t)gk * ldx] : 0.0f;
            rb[e] = (gc < m && gk < w) ? X[(int64_t)gc + (int64_t)gk * ldx] : 0.0f;
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

    const int nk = (w + BF_BK - 1) / BF_BK;
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
                if (gi < m && gj < m && gi >= gj) {
                    float* p = C + (int64_t)gi + (int64_t)gj * ldc;
                    *p = *p - acc[cb][r4][r];
                }
            }
        }
    }
}

inline int grid_for(int nb, bool lower_only, int& nsb) {
    nsb = (nb + UPD_GROUP - 1) / UPD_GROUP;
    const int nsup = lower_only ? nsb * (nsb + 1) / 2 : nsb * nsb;
    return ((nsup + N_XCD - 1) / N_XCD) * N_XCD * UPD_WG_PER_SUPER;
}

}  // namespace

template <typename T>
hipError_t launch_update_syrk(int m, int w, T* C, int64_t ldc, const T* P, int64_t ldp, const int* info,
                              hipStream_t st) {
    if (m <= 0 || w <= 0) return hipSuccess;
    const int nb = (m + TM - 1) / TM;
    int nsb;
    const int grid = grid_for(nb, true, nsb);
    hipLaunchKernelGGL((update_kernel<T, false>), dim3(grid), dim3(NT), 0, st, m, w, C, ldc, P, ldp, P, ldp, nb, nsb, info);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_update_gemm(int m, int w, T* C, int64_t ldc, const T* X, int64_t ldx,
                              const T* Y, int64_t ldy, const int* info, hipStream_t st) {
    if (m <= 0 || w <= 0) return hipSuccess;
    const int nb = (m + TM - 1) / TM;
    int nsb;
    const int grid = grid_for(nb, false, nsb);
    hipLaunchKernelGGL((update_kernel<T, true>), dim3(grid), dim3(NT), 0, st, m, w, C, ldc, X, ldx, Y, ldy, nb, nsb, info);
    return hipGetLastError();
}

hipError_t launch_update_syrk_bf16(int m, int w, float* C, int64_t ldc, const float* P, int64_t ldp,
                                   const int* info, hipStream_t st) {
    if (m <= 0 || w <= 0) return hipSuccess;
    const int nb = (m + TM - 1) / TM;
    int nsb;
    const int grid = grid_for(nb, true, nsb);
    hipLaunchKernelGGL(update_bf16_kernel, dim3(grid), dim3(NT), 0, st, m, w, C, ldc, P, ldp, nb, nsb, info);
    return hipGetLastError();
}

template hipError_t launch_update_syrk<double>(int, int, double*, int64_t, const double*, int64_t, const int*,
                                               hipStream_t);
template hipError_t launch_update_syrk<float>(int, int, float*, int64_t, const float*, int64_t, const int*, hipStream_t);
template hipError_t launch_update_gemm<double>(int, int, double*, int64_t, const double*, int64_t, const double*,
                                               int64_t, const int*, hipStream_t);
template hipError_t launch_update_gemm<float>(int, int, float*, int64_t, const float*, int64_t, const float*, int64_t,
                                              const int*, hipStream_t);

}  // namespace ff
