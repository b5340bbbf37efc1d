// update.hip -- the deferred trailing update of the delayed-update factorisations.
//
// Sec. 2 of arXiv 1812.02056, Algorithm 1: every s columns the pending block
// R = L[c.., z..c-1] of the factor gives S = R R^T, subtracted from the trailing
// square A[c.., c..]; Algorithm 2 uses S = R_L R_U.  Here S is never stored: a
// workgroup forms one output tile of S with MFMA instructions, K-loop over the
// pending columns staged through LDS, and subtracts it from C in the write-back.
//
// One kernel template covers every product the library needs:
//     C(i, j) -= sum_k X(i, k) Y(j, k)      i < M, j < N
// with C and X column-major (C[i + j*ldc], X[i + k*ldx]) and Y either the rows of
// a column-major N x K matrix (YROWS: Y[j + k*ldy], Algorithm 1's R R^T) or a
// column-major K x N matrix (Y[k + j*ldy], Algorithm 2's R_L R_U).  With LOWER
// only entries with i - j >= shift are written (the lower triangle of the
// trailing square, or of a region of it); tiles wholly above that line are
// skipped, and for a square lower region (shift 0) the tiles on or below the
// diagonal are enumerated as a triangle.
//
// Shapes of the one kernel template (every wave computes a WW x WW part of the
// tile with 16 x 16 MFMA blocks):
//   128 x 128 tiles, 4 waves, two workgroups per CU: wide regions;
//   256 x 128 tiles, 8 waves, one workgroup per CU: wide regions while another
//     stream needs whole CUs (the grid is sized to leave them free);
//   64 x 64 tiles of 32 x 32 wave parts: narrow regions, where wider tiles would
//     leave most of the chip idle.
//
// Element types: double (v_mfma_f64_16x16x4f64), float (v_mfma_f32_16x16x4f32),
// and bf16 operands (binary32 storage, operands rounded to bfloat16 while staged
// into LDS, binary32 accumulation, v_mfma_f32_16x16x32_bf16; YROWS only).
#include <algorithm>

#include "common.hpp"
#include "fastfact.h"
#include "grid.hpp"
#include "internal.hpp"

namespace ff {

namespace {

constexpr int NT = 256;    // threads of the bfloat16 shape (2 x 2 waves)

// Wide-region kernel: the product shape that carries almost all of a
// factorisation's flops.  WMW x 2 waves own a (64 WMW) x 128 tile; each wave
// computes a 64 x 64 part of it: 16 MFMA blocks fed by 8 LDS fragment reads per
// 4-deep K step, with the fragments of the next step read while the current
// step's MFMAs run.  Stages of BK columns are double-buffered in LDS and staged
// through registers one stage ahead; loads past K return zeros (the buffer
// record count ends at column K), so only the final stage needs depth guards.
//   WMW = 2: 256 threads, 64 KB of LDS, two workgroups per CU (two waves per
//     SIMD from different workgroups, so one workgroup's barrier waits and
//     write-back are covered by the other's MFMAs);
//   WMW = 4: 512 threads, 96 KB of LDS, so at most one workgroup fits a CU: a
//     grid of C - R workgroups leaves R whole CUs free for kernels on another
//     stream (the lookahead panel work).
// The grid may be smaller than the tile count; each workgroup then walks the
// slots grid-stride.
// K depth of one LDS stage (double-buffered).  The one-workgroup-per-CU shape
// has the LDS for 24-deep binary64 stages (144 KB), which cuts its stage
// barriers, where both waves of a SIMD stall together, by a third.
template <typename T, int WMW> struct wide_depth { static constexpr int BK = 16; };
template <> struct wide_depth<double, 4> { static constexpr int BK = 24; };
template <int WMW> struct wide_depth<float, WMW> { static constexpr int BK = 32; };

template <typename T, int WW, int WMW>
struct wide_cfg {
    static constexpr int TM = WW * WMW, TN = 2 * WW;
    static constexpr int BK = wide_depth<T, WMW>::BK;
};

// One output tile (bi, bj) of C -= X Y^T: the whole K loop and the fused
// write-back.  Shared by the single-region and the grouped kernels; ends with a
// barrier so the caller may start another tile on the same LDS buffers.
template <typename T, int WW, int WMW, bool YROWS, bool LOWER>
__device__ __forceinline__ void wide_tile(int M, int N, int K, T* __restrict__ C, int64_t ldc,
                                          const T* __restrict__ X, int64_t ldx, const T* __restrict__ Y,
                                          int64_t ldy, int shift, int bi, int bj,
                                          T (&As)[2][wide_cfg<T, WW, WMW>::BK][wide_cfg<T, WW, WMW>::TM],
                                          T (&Bs)[2][wide_cfg<T, WW, WMW>::BK][wide_cfg<T, WW, WMW>::TN])
{
    constexpr int TM = WW * WMW, TN = 2 * WW;
    constexpr int NTH = 128 * WMW;
    constexpr int BK = wide_depth<T, WMW>::BK;
    constexpr int SZ = sizeof(T);
    constexpr int NLX = BK * TM / NTH;            // staged X elements per thread per stage
    constexpr int NLY = BK * TN / NTH;            // staged Y elements per thread per stage
    constexpr int XSTEP = NTH / TM, YSTEP = NTH / TN;
    static_assert(TM % 64 == 0 && TN % 64 == 0 && NLX * XSTEP == BK && NLY * YSTEP == BK, "staging map");
    constexpr int NB = WW / 16;                   // MFMA blocks per wave edge
    typedef acc_traits<T> AT;
    typedef typename AT::vec V;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave % WMW, wc = wave / WMW;
    // X staging (and Y when YROWS): thread owns one row and K positions k0 + step*q
    const int sxr = tid % TM, sxk = wave * 64 / TM;      // tid / TM, uniform per wave (TM % 64 == 0)
    const int syr = tid % TN, syk = wave * 64 / TN;      // tid / TN, uniform per wave (TN % 64 == 0)
    // Y staging when K runs down the columns: thread owns column yc, K positions yk0 + e
    const int yc = tid / YSTEP;
    const int yk0 = (tid % YSTEP) * NLY;
    const int nk = (K + BK - 1) / BK;
    const int xs = (int)ldx * SZ, ys = (int)ldy * SZ;

    const int row0 = bi * TM, col0 = bj * TN;
    const int mrem = M - row0, nrem = N - col0;
    const bool active = !LOWER || (row0 + WW * wr + WW - 1) - (col0 + WW * wc) >= shift;
    const int vx = sxr < mrem ? sxr * SZ : BUF_OOB;
    const int vy = YROWS ? (syr < nrem ? syr * SZ : BUF_OOB) : (yc < nrem ? yc * ys : BUF_OOB);
    const T* Xt = X + row0;
    const T* Yt = YROWS ? Y + col0 : Y + (int64_t)col0 * ldy;

    // Stage kt: a resource starting at K column kt*BK whose record count ends
    // at column K, so K columns past the end read zero; rows past M read zero
    // through vx / vy.
    T xa[NLX], ya[NLY];
    auto load = [&](int kt) {
        const int k0 = kt * BK;
        const int kv = K - k0 > 0 ? K - k0 : 0;
        const rsrc_t rx = make_rsrc_n(Xt + (int64_t)k0 * ldx, kv * xs);
#pragma unroll
        for (int q = 0; q < NLX; ++q) xa[q] = buf_load<T>(rx, vx, (sxk + XSTEP * q) * xs);
        if (YROWS) {
            const rsrc_t ry = make_rsrc_n(Yt + (int64_t)k0 * ldy, kv * ys);
#pragma unroll
            for (int q = 0; q < NLY; ++q) ya[q] = buf_load<T>(ry, vy, (syk + YSTEP * q) * ys);
        } else {
            const rsrc_t ry = make_rsrc(Yt + k0);
#pragma unroll
            for (int e = 0; e < NLY; ++e) ya[e] = buf_load<T>(ry, yk0 + e < kv ? vy + (yk0 + e) * SZ : BUF_OOB, 0);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < NLX; ++q) As[buf][sxk + XSTEP * q][sxr] = xa[q];
        if (YROWS) {
#pragma unroll
            for (int q = 0; q < NLY; ++q) Bs[buf][syk + YSTEP * q][syr] = ya[q];
        } else {
#pragma unroll
            for (int e = 0; e < NLY; ++e) Bs[buf][yk0 + e][yc] = ya[e];
        }
    };

    V acc[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = zero_vec<V>();

    // fa: column-operand fragments (the MFMA A input), fb: row-operand
    // fragments; the product tile is the transposed one (lanes along rows).
    auto frags = [&](int buf, int k4, T (&fa)[NB], T (&fb)[NB]) {
        const int kk = 4 * k4 + (lane >> 4);
#pragma unroll
        for (int b = 0; b < NB; ++b) fa[b] = Bs[buf][kk][WW * wc + 16 * b + (lane & 15)];
#pragma unroll
        for (int b = 0; b < NB; ++b) fb[b] = As[buf][kk][WW * wr + 16 * b + (lane & 15)];
    };
    auto mma = [&](const T (&fa)[NB], const T (&fb)[NB]) {
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
#pragma unroll
            for (int r4 = 0; r4 < NB; ++r4) acc[cb][r4] = AT::mfma(fa[cb], fb[r4], acc[cb][r4]);
    };
    auto compute_full = [&](int buf) {
        T fa0[NB], fb0[NB], fa1[NB], fb1[NB];
        // Two workgroups share each SIMD in the 2-wave-per-SIMD shapes: raising
        // the priority of a wave's MFMA phase lets it keep the matrix pipe busy
        // while the other workgroup's wave stages operands (measured +3..6%).
        // With one workgroup per CU both waves of a SIMD reach the MFMAs
        // together and the raise costs a little, so it is not used there.
        if (WMW == 2) __builtin_amdgcn_s_setprio(1);
        frags(buf, 0, fa0, fb0);
#pragma unroll
        for (int k4 = 0; k4 < BK / 4; k4 += 2) {
            frags(buf, k4 + 1, fa1, fb1);
            mma(fa0, fb0);
            if (k4 + 2 < BK / 4) frags(buf, k4 + 2, fa0, fb0);
            mma(fa1, fb1);
        }
        if (WMW == 2) __builtin_amdgcn_s_setprio(0);
    };
    auto compute_tail = [&](int buf, int nk4) {
#pragma unroll
        for (int k4 = 0; k4 < BK / 4; ++k4) {
            if (k4 < nk4) {
                T fa[NB], fb[NB];
                frags(buf, k4, fa, fb);
                mma(fa, fb);
            }
        }
    };

    load(0);
    store(0);
    __syncthreads();
    // No branch around the MFMAs: a conditional compute lets the compiler sink
    // the next stage's loads below it, next to their LDS stores, which exposes
    // the full load latency every stage.  Waves wholly outside the written
    // region (diagonal tiles only) compute and discard.
    for (int kt = 0; kt + 1 < nk; ++kt) {
        load(kt + 1);
        compute_full(kt & 1);
        store((kt + 1) & 1);
        __syncthreads();
    }
    // Write-back C - S.  Lane part of the offset in a register, the block column
    // in the scalar offset, the block row in the immediate.  Whole tiles read C
    // in column-block groups, each group's loads issued before the previous
    // group's stores and the first group's before the last stage's MFMAs, so
    // one memory latency per tile is exposed at most.  Tiles on an edge or
    // crossing the written region's boundary mask each entry.
    const rsrc_t rc = make_rsrc(C + row0 + (int64_t)col0 * ldc);
    const int li0 = WW * wr + (lane & 15);
    const int lj0 = WW * wc + AT::col_lane(lane);
    const int cs = (int)ldc * SZ;
    const int cbase = (li0 + lj0 * (int)ldc) * SZ;
    const bool full = mrem >= TM && nrem >= TN && (!LOWER || row0 - (col0 + TN - 1) >= shift);
    const int pbase = active && full ? cbase : BUF_OOB;
    T cv[2][NB][4];
    auto cload = [&](int cb, T (&d)[NB][4]) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int r4 = 0; r4 < NB; ++r4)
                d[r4][r] = bufop<T, AUX_NT>::load(rc, pbase == BUF_OOB ? BUF_OOB : pbase + 16 * r4 * SZ,
                                                  (16 * cb + AT::col_reg(r)) * cs);
    };
    cload(0, cv[0]);
    compute_tail((nk - 1) & 1, (K - (nk - 1) * BK + 3) / 4);

    if (active) {
        if (full) {
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) {
                if (cb + 1 < NB) cload(cb + 1, cv[(cb + 1) & 1]);
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int r4 = 0; r4 < NB; ++r4)
                        bufop<T, AUX_NT>::store(rc, cbase + 16 * r4 * SZ, cv[cb & 1][r4][r] - acc[cb][r4][r],
                                                (16 * cb + AT::col_reg(r)) * cs);
            }
        } else {
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) {
                T cv[NB][4];
                int off[NB][4];
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int r4 = 0; r4 < NB; ++r4) {
                        const int li = li0 + 16 * r4;
                        const int lj = lj0 + 16 * cb + AT::col_reg(r);
                        const bool ok = li < mrem && lj < nrem && (!LOWER || (row0 + li) - (col0 + lj) >= shift);
                        off[r4][r] = ok ? cbase + (16 * r4 + (16 * cb + AT::col_reg(r)) * (int)ldc) * SZ : BUF_OOB;
                        cv[r4][r] = bufop<T, AUX_NT>::load(rc, off[r4][r], 0);
                    }
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int r4 = 0; r4 < NB; ++r4)
                        bufop<T, AUX_NT>::store(rc, off[r4][r], cv[r4][r] - acc[cb][r4][r], 0);
            }
        }
    }
    __syncthreads();   // the next tile's first stage reuses buffer 0
}

// A persistent workgroup's walk over its tiles.
template <typename T, int WW, int WMW, bool YROWS, bool LOWER>
__device__ __forceinline__ void wide_walk(int M, int N, int K, T* __restrict__ C, int64_t ldc,
                                          const T* __restrict__ X, int64_t ldx, const T* __restrict__ Y, int64_t ldy,
                                          const Grid& g)
{
    typedef wide_cfg<T, WW, WMW> CF;
    __shared__ T As[2][CF::BK][CF::TM];   // row operand X(row0 + r, k)    stored [k][r]
    __shared__ T Bs[2][CF::BK][CF::TN];   // column operand Y(col0 + c, k) stored [k][c]
    int it0, it1, itd;
    tile_walk(g, it0, it1, itd);
    for (int it = it0; it < it1; it += itd) {
        int bi, bj;
        if (g.balanced) tile_of_index(g, LOWER, it, bi, bj);
        else if (!tile_of_slot(g, it, LOWER, bi, bj)) continue;
        wide_tile<T, WW, WMW, YROWS, LOWER>(M, N, K, C, ldc, X, ldx, Y, ldy, g.shift, bi, bj, As, Bs);
    }
}

template <typename T, int WW, int WMW, bool YROWS, bool LOWER>
__global__ __launch_bounds__(128 * WMW, 4 / WMW)
void update_wide_kernel(int M, int N, int K, T* __restrict__ C, int64_t ldc, const T* __restrict__ X, int64_t ldx,
                        const T* __restrict__ Y, int64_t ldy, Grid g, const int* __restrict__ info)
{
    if (info && *info != 0) return;
    wide_walk<T, WW, WMW, YROWS, LOWER>(M, N, K, C, ldc, X, ldx, Y, ldy, g);
}

// The same update over the last tiles of a split tile order, launched on the
// stream that owns the CUs kept free for panel work once that work is done (a
// separate entry point so that traces tell it from the main part).
template <typename T, int WW, int WMW, bool YROWS, bool LOWER>
__global__ __launch_bounds__(128 * WMW, 4 / WMW)
void update_wide_tail_kernel(int M, int N, int K, T* __restrict__ C, int64_t ldc, const T* __restrict__ X,
                             int64_t ldx, const T* __restrict__ Y, int64_t ldy, Grid g, const int* __restrict__ info)
{
    if (info && *info != 0) return;
    wide_walk<T, WW, WMW, YROWS, LOWER>(M, N, K, C, ldc, X, ldx, Y, ldy, g);
}

// Grouped trailing updates (many independent matrices, serving): the lower
// 128 x 128 tiles of every job form one flat queue; a workgroup finds its job by
// binary search over the tile offsets and runs the same tile body.
template <typename S>
__global__ __launch_bounds__(256, 2)
void update_grouped_kernel(const GroupUpd* __restrict__ jobs, int njobs, int ntiles)
{
    typedef wide_cfg<S, 64, 2> CF;
    __shared__ S As[2][CF::BK][CF::TM];
    __shared__ S Bs[2][CF::BK][CF::TN];
    for (int slot = blockIdx.x; slot < ntiles; slot += gridDim.x) {
        int lo = 0, hi = njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].tiles_begin <= slot) lo = mid;
            else hi = mid - 1;
        }
        const GroupUpd jb = jobs[lo];
        if (jb.info && *jb.info != 0) continue;
        const int t = slot - jb.tiles_begin;
        const int bi = tri_row(t), bj = t - bi * (bi + 1) / 2;
        wide_tile<S, 64, 2, true, true>(jb.m, jb.m, jb.w, static_cast<S*>(jb.c), jb.ld, static_cast<const S*>(jb.p),
                                        jb.ld, static_cast<const S*>(jb.p), jb.ld, 0, bi, bj, As, Bs);
    }
}

// bfloat16-operand variant (YROWS form, optional LOWER, persistent 128 tiles);
// binary32 storage and accumulation.  Operand tiles are stored row-major
// [row][k] with a 40-element row pitch (80 bytes) so the 16-byte fragment reads
// of a lane group hit distinct LDS banks.
constexpr int BF_BK = 32;
constexpr int BF_PITCH = 40;
constexpr int BF_TILE = 128;

template <bool LOWER>
__global__ __launch_bounds__(NT, 1)
void update_bf16_kernel(int M, int N, int K, float* __restrict__ C, int64_t ldc,
                        const float* __restrict__ X, int64_t ldx, const float* __restrict__ Y, int64_t ldy,
                        Grid g, const int* __restrict__ info)
{
    if (info && *info != 0) return;
    __shared__ __attribute__((aligned(16))) __bf16 As[2][BF_TILE][BF_PITCH];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[2][BF_TILE][BF_PITCH];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave & 1, wc = wave >> 1;
    const int sr = tid % BF_TILE, sh = tid / BF_TILE;   // staging: row, k-half
    const int nk = (K + BF_BK - 1) / BF_BK;

    int it0, it1, itd;
    tile_walk(g, it0, it1, itd);
    for (int it = it0; it < it1; it += itd) {
        int bi, bj;
        if (g.balanced) tile_of_index(g, LOWER, it, bi, bj);
        else if (!tile_of_slot(g, it, LOWER, bi, bj)) continue;
        const int row0 = bi * BF_TILE, col0 = bj * BF_TILE;
        const int mrem = M - row0, nrem = N - col0;
        const bool active = !LOWER || (row0 + 64 * wr + 63) - (col0 + 64 * wc) >= g.shift;
        const rsrc_t rx = make_rsrc(X + row0);
        const rsrc_t ry = make_rsrc(Y + col0);
        const rsrc_t rc = make_rsrc(C + row0 + (int64_t)col0 * ldc);

        float ra[16], rb[16];
        auto load = [&](int kt) {
            const int k0 = kt * BF_BK + 16 * sh;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int gk = k0 + e;
                ra[e] = buf_load<float>(rx, (sr < mrem && gk < K) ? (sr + gk * (int)ldx) * 4 : BUF_OOB);
                rb[e] = buf_load<float>(ry, (sr < nrem && gk < K) ? (sr + gk * (int)ldy) * 4 : BUF_OOB);
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
        auto c_off = [&](int cb, int r4, int r) -> int {
            const int li = 64 * wr + 16 * r4 + (lane & 15);
            const int lj = 64 * wc + 16 * cb + acc_traits<float>::col(lane, r);
            const bool ok = active && li < mrem && lj < nrem && (!LOWER || (row0 + li) - (col0 + lj) >= g.shift);
            return ok ? (li + lj * (int)ldc) * 4 : BUF_OOB;
        };

        f4_t acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = zero_vec<f4_t>();
        load(0);
        float cv[4][4][4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4)
#pragma unroll
                for (int r = 0; r < 4; ++r) cv[cb][r4][r] = buf_load<float>(rc, c_off(cb, r4, r));
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
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    buf_store<float>(rc, c_off(cb, r4, r), cv[cb][r4][r] - acc[cb][r4][r]);
    }
}

// bfloat16-operand update from a transposed bfloat16 copy of the panel (the
// form the factorisations use).  The copy is made once per step:
//     Pt[r * wp + k] = bf16(P[r + k * ldp])  for k < w,   0 for w <= k < wp,
// wp = w rounded up to BT_BK, so a row's K values are contiguous and zero-padded:
// a stage is four 16-byte loads per thread and operand with no K guard and no
// conversion in the K loop (the float-operand kernel above makes 32 scalar
// 4-byte loads per thread and stage and converts them).  64-deep stages (two
// 32-deep MFMA steps) and two workgroups per CU hide the load latency behind
// MFMA work.  Every output takes the same MFMAs in the same K order as the
// float-operand kernel on the same rounded operands, so the results agree bit
// for bit.
constexpr int BT_BK = 64;
constexpr int BT_PITCH = 72;     // bfloat16 per LDS row: 144 B, 16-byte aligned rows

__global__ __launch_bounds__(256)
void panel_bf16t_kernel(int m, int w, int wp, const float* __restrict__ P, int64_t ldp, __bf16* __restrict__ Pt)
{
    __shared__ __attribute__((aligned(16))) __bf16 t[64][BT_PITCH];
    const int r0 = blockIdx.x * 64, k0 = blockIdx.y * 64;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int r = e & 63, k = e >> 6;
        const float v = (r0 + r < m && k0 + k < w) ? P[r0 + r + (int64_t)(k0 + k) * ldp] : 0.0f;
        t[r][k] = to_bf16(v);
    }
    __syncthreads();
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    for (int c = threadIdx.x; c < 64 * 8; c += 256) {
        const int r = c >> 3, q = c & 7;
        if (r0 + r < m)
            *reinterpret_cast<u4*>(Pt + (int64_t)(r0 + r) * wp + k0 + 8 * q) = *reinterpret_cast<const u4*>(&t[r][8 * q]);
    }
}

template <bool LOWER>
__global__ __launch_bounds__(NT, 2)
void update_bf16t_kernel(int M, int N, int wp, float* __restrict__ C, int64_t ldc, const __bf16* __restrict__ Xt,
                         const __bf16* __restrict__ Yt, Grid g, const int* __restrict__ info)
{
    if (info && *info != 0) return;
    __shared__ __attribute__((aligned(16))) __bf16 As[2][BF_TILE][BT_PITCH];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[2][BF_TILE][BT_PITCH];
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave & 1, wc = wave >> 1;
    const int sr = tid >> 1, kh = 32 * (tid & 1);       // staging: row, 32-value half of the stage
    const int nk = wp / BT_BK;

    int it0, it1, itd;
    tile_walk(g, it0, it1, itd);
    for (int it = it0; it < it1; it += itd) {
        int bi, bj;
        if (g.balanced) tile_of_index(g, LOWER, it, bi, bj);
        else if (!tile_of_slot(g, it, LOWER, bi, bj)) continue;
        const int row0 = bi * BF_TILE, col0 = bj * BF_TILE;
        const int mrem = M - row0, nrem = N - col0;
        const bool active = !LOWER || (row0 + 64 * wr + 63) - (col0 + 64 * wc) >= g.shift;
        const rsrc_t rx = make_rsrc(Xt + (int64_t)row0 * wp);
        const rsrc_t ry = make_rsrc(Yt + (int64_t)col0 * wp);
        const rsrc_t rc = make_rsrc(C + row0 + (int64_t)col0 * ldc);
        const int ox = sr < mrem ? (sr * wp + kh) * 2 : BUF_OOB;
        const int oy = sr < nrem ? (sr * wp + kh) * 2 : BUF_OOB;

        u4 ra[4], rb[4];
        auto load = [&](int kt) {
            const int kb = kt * BT_BK * 2;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                ra[q] = __builtin_amdgcn_raw_buffer_load_b128(rx, ox == BUF_OOB ? BUF_OOB : ox + kb + 16 * q, 0, 0);
                rb[q] = __builtin_amdgcn_raw_buffer_load_b128(ry, oy == BUF_OOB ? BUF_OOB : oy + kb + 16 * q, 0, 0);
            }
        };
        auto store = [&](int buf) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                *reinterpret_cast<u4*>(&As[buf][sr][kh + 8 * q]) = ra[q];
                *reinterpret_cast<u4*>(&Bs[buf][sr][kh + 8 * q]) = rb[q];
            }
        };
        f4_t acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = zero_vec<f4_t>();
        load(0);
        store(0);
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            const int buf = kt & 1;
            if (kt + 1 < nk) load(kt + 1);
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int ks = 0; ks < BT_BK / 32; ++ks) {
                bf8_t fa[4], fb[4];
                const int ko = 32 * ks + 8 * (lane >> 4);
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
            __builtin_amdgcn_s_setprio(0);
            if (kt + 1 < nk) store(buf ^ 1);
            __syncthreads();
        }
        // write-back C - S, one 16-column block group at a time (the other
        // workgroup on the CU covers the load latency); whole tiles use the
        // lane's base offset, the column in the scalar offset and the row block
        // in the immediate; edge and diagonal tiles mask each entry
        const bool full = mrem >= BF_TILE && nrem >= BF_TILE && (!LOWER || row0 - (col0 + BF_TILE - 1) >= g.shift);
        const int li0 = 64 * wr + (lane & 15);
        const int lj0 = 64 * wc + 4 * (lane >> 4);
        const int cs = (int)ldc * 4;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            float cv[4][4];
            if (full) {
                const int base = active ? (li0 + lj0 * (int)ldc) * 4 : BUF_OOB;
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int r4 = 0; r4 < 4; ++r4)
                        cv[r4][r] = buf_load<float>(rc, base == BUF_OOB ? BUF_OOB : base + 64 * r4, (16 * cb + r) * cs);
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int r4 = 0; r4 < 4; ++r4)
                        buf_store<float>(rc, base == BUF_OOB ? BUF_OOB : base + 64 * r4, cv[r4][r] - acc[cb][r4][r],
                                         (16 * cb + r) * cs);
            } else {
                int off[4][4];
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int r4 = 0; r4 < 4; ++r4) {
                        const int li = li0 + 16 * r4, lj = lj0 + 16 * cb + r;
                        const bool ok =
                            active && li < mrem && lj < nrem && (!LOWER || (row0 + li) - (col0 + lj) >= g.shift);
                        off[r4][r] = ok ? (li + lj * (int)ldc) * 4 : BUF_OOB;
                        cv[r4][r] = buf_load<float>(rc, off[r4][r]);
                    }
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int r4 = 0; r4 < 4; ++r4) buf_store<float>(rc, off[r4][r], cv[r4][r] - acc[cb][r4][r]);
            }
        }
    }
}

// Largest K for which every in-range operand byte offset of one tile stays below
// BUF_RECORDS; longer products are applied in K chunks (chunks in increasing k).
inline int max_k_chunk(int64_t ldx, int64_t ldy, bool yrows, size_t sz) {
    const int64_t lim = (int64_t)BUF_RECORDS / (int64_t)sz - 2 * 128;
    const int64_t kx = lim / (ldx > 0 ? ldx : 1);
    const int64_t ky = yrows ? lim / (ldy > 0 ? ldy : 1) : lim - 128 * ldy;
    const int64_t k = kx < ky ? kx : ky;
    return (int)(k > (1 << 30) ? (1 << 30) : k);
}

template <typename T, int WW, int WMW>
hipError_t launch_wide(int M, int N, int Kc, T* C, int64_t ldc, const T* X, int64_t ldx, const T* Y, int64_t ldy,
                       bool yrows, bool lower, const Grid& g, int nwg, const int* info, hipStream_t st,
                       bool tail = false) {
#define FF_WIDE_LAUNCH(YR, LO)                                                                                       \
    if (tail)                                                                                                        \
        hipLaunchKernelGGL((update_wide_tail_kernel<T, WW, WMW, YR, LO>), dim3(nwg), dim3(128 * WMW), 0, st, M, N,   \
                           Kc, C, ldc, X, ldx, Y, ldy, g, info);                                                     \
    else                                                                                                             \
        hipLaunchKernelGGL((update_wide_kernel<T, WW, WMW, YR, LO>), dim3(nwg), dim3(128 * WMW), 0, st, M, N, Kc, C,  \
                           ldc, X, ldx, Y, ldy, g, info)
    if (yrows) {
        if (lower) FF_WIDE_LAUNCH(true, true);
        else FF_WIDE_LAUNCH(true, false);
    } else {
        if (lower) FF_WIDE_LAUNCH(false, true);
        else FF_WIDE_LAUNCH(false, false);
    }
#undef FF_WIDE_LAUNCH
    return hipGetLastError();
}

}  // namespace

int update_workers(int reserve_cus) {
    const int cus = cu_count();
    int w = cus - (reserve_cus > 0 ? reserve_cus : 0);
    w = (w / N_XCD) * N_XCD;
    return w < N_XCD ? N_XCD : w;
}

double update_range_entries(int M, int N, bool lower, int shift, int reserve_cus, double f0, double f1) {
    const int shape = update_shape(M, N, reserve_cus);
    Grid g = shape == FF_UPD_SHAPE_256x128 ? make_grid(256, 128, 4, 8, M, N, lower, shift)
           : shape == FF_UPD_SHAPE_128     ? make_grid(128, M, N, lower, shift)
                                           : make_grid(64, M, N, lower, shift);
    if (!grid_set_range(g, f0, f1)) return -1.0;
    double n = 0;
    for (int t = g.tfirst; t < g.tlast; ++t) {
        int bi, bj;
        tile_of_index(g, lower, t, bi, bj);
        const int64_t r0 = (int64_t)bi * g.tm, r1 = std::min<int64_t>(r0 + g.tm, M);
        const int64_t c0 = (int64_t)bj * g.tn, c1 = std::min<int64_t>(c0 + g.tn, N);
        for (int64_t j = c0; j < c1; ++j) {
            const int64_t lo = lower ? std::max<int64_t>(r0, j + shift) : r0;
            if (r1 > lo) n += (double)(r1 - lo);
        }
    }
    return n;
}

int update_order_tiles(int M, int N, bool lower, int shift, int reserve_cus) {
    const int shape = update_shape(M, N, reserve_cus);
    if (shape == FF_UPD_SHAPE_64) return 0;
    Grid g = shape == FF_UPD_SHAPE_256x128 ? make_grid(256, 128, 4, 8, M, N, lower, shift)
                                           : make_grid(128, M, N, lower, shift);
    return g.balanced ? g.ntiles : 0;
}

bool update_splittable(int M, int N, bool lower, int shift, int reserve_cus) {
    const int shape = update_shape(M, N, reserve_cus);
    if (shape == FF_UPD_SHAPE_64) return false;
    Grid g = shape == FF_UPD_SHAPE_256x128 ? make_grid(256, 128, 4, 8, M, N, lower, shift)
                                           : make_grid(128, M, N, lower, shift);
    return g.balanced != 0;
}

int update_shape(int M, int N, int reserve_cus) {
    // narrow regions (fewer 128-wide tiles than half the CUs) use 64 tiles
    const bool narrow = (M < 2 * 128 || N < 2 * 128) ||
                        ((int64_t)((M + 127) / 128) * ((N + 127) / 128) < (int64_t)cu_count() / 2);
    if (narrow) return FF_UPD_SHAPE_64;
    return reserve_cus > 0 ? FF_UPD_SHAPE_256x128 : FF_UPD_SHAPE_128;
}

template <typename T>
hipError_t launch_update(int M, int N, int K, T* C, int64_t ldc, const T* X, int64_t ldx, const T* Y, int64_t ldy,
                         bool yrows, bool lower, int shift, const int* info, hipStream_t st, int reserve_cus,
                         int max_cus, double f0, double f1) {
    if (M <= 0 || N <= 0 || K <= 0 || f1 <= f0) return hipSuccess;
    const bool part = f0 > 0.0 || f1 < 1.0;
    if (!ld_fits(ldc, sizeof(T)) || (!yrows && !ld_fits(ldy, sizeof(T)))) return hipErrorInvalidValue;
    const int kc = max_k_chunk(ldx, ldy, yrows, sizeof(T));
    if (kc < 1) return hipErrorInvalidValue;
    const int shape = update_shape(M, N, reserve_cus);
    const bool narrow = shape == FF_UPD_SHAPE_64;
    for (int k0 = 0; k0 < K; k0 += kc) {
        const int Kc = (K - k0 < kc) ? K - k0 : kc;
        const T* Xk = X + (int64_t)k0 * ldx;
        const T* Yk = yrows ? Y + (int64_t)k0 * ldy : Y + k0;
        hipError_t e;
        if (narrow) {
            // 64 x 64 tiles of 32 x 32 wave parts, one tile per workgroup
            Grid g = make_grid(64, M, N, lower, shift);
            if (part && !grid_set_range(g, f0, f1)) return hipErrorInvalidValue;
            int nwg = g.nslots;
            if (g.balanced) nwg = persistent_grid(g, g.tlast - g.tfirst);   // one tile per workgroup
            if (max_cus > 0 && nwg > 4 * max_cus) nwg = persistent_grid(g, 4 * max_cus);   // four fit a CU
            e = launch_wide<T, 32, 2>(M, N, Kc, C, ldc, Xk, ldx, Yk, ldy, yrows, lower, g, nwg, info, st);
        } else if (shape == FF_UPD_SHAPE_256x128) {
            // one workgroup per CU on all but reserve_cus CUs
            Grid g = make_grid(256, 128, 4, 8, M, N, lower, shift);
            if (part && !grid_set_range(g, f0, f1)) return hipErrorInvalidValue;
            if (g.tlast == g.tfirst && g.balanced) return hipSuccess;
            const int nwg = persistent_grid(g, max_cus > 0 ? max_cus : update_workers(reserve_cus));
            e = launch_wide<T, 64, 4>(M, N, Kc, C, ldc, Xk, ldx, Yk, ldy, yrows, lower, g, nwg, info, st, f0 > 0.0);
        } else {
            // two workgroups per CU
            Grid g = make_grid(128, M, N, lower, shift);
            if (part && !grid_set_range(g, f0, f1)) return hipErrorInvalidValue;
            if (g.tlast == g.tfirst && g.balanced) return hipSuccess;
            const int nwg = persistent_grid(g, max_cus > 0 ? 2 * max_cus : 2 * update_workers(0));
            e = launch_wide<T, 64, 2>(M, N, Kc, C, ldc, Xk, ldx, Yk, ldy, yrows, lower, g, nwg, info, st, f0 > 0.0);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int grouped_update_tile() { return 128; }

template <typename S>
hipError_t launch_update_grouped(int njobs, int total_tiles, const GroupUpd* d_jobs, hipStream_t st) {
    if (njobs <= 0 || total_tiles <= 0) return hipSuccess;
    int nwg = 2 * update_workers(0);
    if (nwg > total_tiles) nwg = total_tiles;
    hipLaunchKernelGGL((update_grouped_kernel<S>), dim3(nwg), dim3(256), 0, st, d_jobs, njobs, total_tiles);
    return hipGetLastError();
}
template hipError_t launch_update_grouped<double>(int, int, const GroupUpd*, hipStream_t);
template hipError_t launch_update_grouped<float>(int, int, const GroupUpd*, hipStream_t);

hipError_t launch_update_bf16(int M, int N, int K, float* C, int64_t ldc, const float* X, int64_t ldx,
                              const float* Y, int64_t ldy, bool lower, int shift, const int* info, hipStream_t st,
                              int reserve_cus) {
    if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
    if (!ld_fits(ldc, sizeof(float))) return hipErrorInvalidValue;
    const int kc = max_k_chunk(ldx, ldy, true, sizeof(float));
    if (kc < 1) return hipErrorInvalidValue;
    Grid g = make_grid(BF_TILE, M, N, lower, shift);
    const int nwg = persistent_grid(g, update_workers(reserve_cus));
    for (int k0 = 0; k0 < K; k0 += kc) {
        const int Kc = (K - k0 < kc) ? K - k0 : kc;
        const float* Xk = X + (int64_t)k0 * ldx;
        const float* Yk = Y + (int64_t)k0 * ldy;
        if (lower)
            hipLaunchKernelGGL(update_bf16_kernel<true>, dim3(nwg), dim3(NT), 0, st, M, N, Kc, C, ldc, Xk, ldx, Yk,
                               ldy, g, info);
        else
            hipLaunchKernelGGL(update_bf16_kernel<false>, dim3(nwg), dim3(NT), 0, st, M, N, Kc, C, ldc, Xk, ldx, Yk,
                               ldy, g, info);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int bf16t_width(int w) { return (w + BT_BK - 1) / BT_BK * BT_BK; }

hipError_t launch_panel_bf16t(int m, int w, const float* P, int64_t ldp, __bf16* Pt, hipStream_t st) {
    if (m <= 0 || w <= 0) return hipSuccess;
    const int wp = bf16t_width(w);
    hipLaunchKernelGGL(panel_bf16t_kernel, dim3((m + 63) / 64, wp / 64), dim3(256), 0, st, m, w, wp, P, ldp, Pt);
    return hipGetLastError();
}

hipError_t launch_update_bf16t(int M, int N, int w, float* C, int64_t ldc, const __bf16* Xt, const __bf16* Yt,
                               bool lower, int shift, const int* info, hipStream_t st, int reserve_cus) {
    if (M <= 0 || N <= 0 || w <= 0) return hipSuccess;
    if (!ld_fits(ldc, sizeof(float))) return hipErrorInvalidValue;
    const int wp = bf16t_width(w);
    if ((int64_t)BF_TILE * wp * 2 >= (int64_t)BUF_RECORDS / 2) return hipErrorInvalidValue;
    Grid g = make_grid(BF_TILE, M, N, lower, shift);
    const int nwg = persistent_grid(g, 2 * update_workers(reserve_cus));
    if (lower)
        hipLaunchKernelGGL(update_bf16t_kernel<true>, dim3(nwg), dim3(NT), 0, st, M, N, wp, C, ldc, Xt, Yt, g, info);
    else
        hipLaunchKernelGGL(update_bf16t_kernel<false>, dim3(nwg), dim3(NT), 0, st, M, N, wp, C, ldc, Xt, Yt, g, info);
    return hipGetLastError();
}

template hipError_t launch_update<double>(int, int, int, double*, int64_t, const double*, int64_t, const double*,
                                          int64_t, bool, bool, int, const int*, hipStream_t, int, int, double, double);
template hipError_t launch_update<float>(int, int, int, float*, int64_t, const float*, int64_t, const float*,
                                         int64_t, bool, bool, int, const int*, hipStream_t, int, int, double, double);

}  // namespace ff
