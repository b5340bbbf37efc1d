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
// Two shapes:
//   TILE 128, persistent: one 8-wave workgroup per CU (two waves per SIMD),
//     looping over tiles.  Each wave owns a 64 x 32 part of the tile (8 MFMA
//     blocks).  The tile's C is loaded into registers at the start of the tile
//     so its HBM traffic overlaps the K loop; the write-back is then a subtract
//     and a store.  The grid can be made smaller than the CU count, which leaves
//     whole CUs free for other streams.
//   TILE 64: one tile per 4-wave workgroup (32 x 32 per wave), several
//     workgroups per CU; for narrow regions where 128-wide tiles would leave most
//     of the chip idle.
//
// Element types: double (v_mfma_f64_16x16x4f64), float (v_mfma_f32_16x16x4f32),
// and bf16 operands (binary32 storage, operands rounded to bfloat16 while staged
// into LDS, binary32 accumulation, v_mfma_f32_16x16x32_bf16; YROWS only).
#include "common.hpp"
#include "internal.hpp"

namespace ff {

namespace {

constexpr int NT = 256;    // threads of the 64-tile and bfloat16 shapes (2 x 2 waves)

// Wave arrangement of a shape: WAVES_M x WAVES_N waves over a TILE x TILE tile.
template <int TILE, bool PERSIST> struct shape {
    static constexpr int WAVES_M = 2;
    static constexpr int WAVES_N = PERSIST ? 4 : 2;
    static constexpr int THREADS = 64 * WAVES_M * WAVES_N;
    static constexpr int WM = TILE / WAVES_M;     // rows per wave
    static constexpr int WN = TILE / WAVES_N;     // columns per wave
};

struct Grid {
    int tile;          // output tile edge
    int nbm, nbn;      // tiles along M and N
    int nsm, nsn;      // super-tiles along M and N
    int tri;           // 1: square lower region enumerated as a triangle of super-tiles
    int shift;         // LOWER: write only i - j >= shift
    int nslots;        // flat slots covering every super-tile
};

// Map a flat slot to an output tile (bi, bj).  Returns false when the slot is
// empty.  Workgroups are dealt to the 8 XCDs round-robin, so slot % 8 is the XCD;
// each XCD works through whole 8 x 8 super-tiles and the 16 operand blocks of a
// super-tile stay in that XCD's L2.
__device__ __forceinline__ bool tile_of_slot(const Grid& g, int slot, bool lower, int& bi, int& bj) {
    const int xcd = slot % N_XCD;
    const int k = slot / N_XCD;
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
    if (lower && (bi * g.tile + g.tile - 1) - bj * g.tile < g.shift) return false;   // wholly above the line
    return true;
}

// K depth of one LDS stage.  The binary64 persistent shape keeps 16 so that the
// accumulators, the prefetched C tile and the next stage fit in the register file.
template <typename T, bool PERSIST> struct stage_depth { static constexpr int BK = 32; };
template <> struct stage_depth<double, true> { static constexpr int BK = 16; };

template <typename T, int TILE, bool YROWS, bool LOWER, bool PERSIST>
__global__ __launch_bounds__((shape<TILE, PERSIST>::THREADS), (PERSIST ? 1 : 2))
void update_kernel(int M, int N, int K, T* __restrict__ C, int64_t ldc,
                   const T* __restrict__ X, int64_t ldx,
                   const T* __restrict__ Y, int64_t ldy, Grid g, const int* __restrict__ info)
{
    if (info && *info != 0) return;
    typedef shape<TILE, PERSIST> SH;
    constexpr int NTH = SH::THREADS;
    constexpr int BK = stage_depth<T, PERSIST>::BK;
    constexpr int WM = SH::WM, WN = SH::WN;
    constexpr int NBR = WM / 16, NBC = WN / 16;   // MFMA blocks per wave along rows / columns
    constexpr int NLD = BK * TILE / NTH;          // operand elements each thread stages per K step
    constexpr int SZ = sizeof(T);
    typedef acc_traits<T> AT;
    typedef typename AT::vec V;

    __shared__ T As[2][BK][TILE];   // row operand X[row0 + r, k]   stored [k][r]
    __shared__ T Bs[2][BK][TILE];   // column operand               stored [k][c ^ (k % 16)]

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave % SH::WAVES_M, wc = wave / SH::WAVES_M;
    const int nk = (K + BK - 1) / BK;

    for (int slot = blockIdx.x; slot < g.nslots; slot += (PERSIST ? gridDim.x : g.nslots)) {
        int bi, bj;
        if (!tile_of_slot(g, slot, LOWER, bi, bj)) continue;
        const int row0 = bi * TILE, col0 = bj * TILE;
        const int mrem = M - row0, nrem = N - col0;
        // a wave whose part lies wholly above the line computes nothing
        const bool active = !LOWER || (row0 + WM * wr + WM - 1) - (col0 + WN * wc) >= g.shift;

        const rsrc_t rx = make_rsrc(X + row0);
        const rsrc_t ry = YROWS ? make_rsrc(Y + col0) : make_rsrc(Y + (int64_t)col0 * ldy);
        const rsrc_t rc = make_rsrc(C + row0 + (int64_t)col0 * ldc);

        T ra[NLD], rb[NLD];
        auto load = [&](int kt) {
            const int k0 = kt * BK;
#pragma unroll
            for (int q = 0; q < NLD; ++q) {
                const int idx = tid + NTH * q;
                const int kk = idx / TILE, r = idx % TILE;
                const int gk = k0 + kk;
                ra[q] = buf_load<T>(rx, (r < mrem && gk < K) ? (r + gk * (int)ldx) * SZ : BUF_OOB);
            }
#pragma unroll
            for (int q = 0; q < NLD; ++q) {
                const int idx = tid + NTH * q;
                if (YROWS) {
                    const int kk = idx / TILE, c = idx % TILE;
                    const int gk = k0 + kk;
                    rb[q] = buf_load<T>(ry, (c < nrem && gk < K) ? (c + gk * (int)ldy) * SZ : BUF_OOB);
                } else {
                    const int kk = idx % BK, c = idx / BK;
                    const int gk = k0 + kk;
                    rb[q] = buf_load<T>(ry, (c < nrem && gk < K) ? (gk + c * (int)ldy) * SZ : BUF_OOB);
                }
            }
        };
        auto store = [&](int buf) {
#pragma unroll
            for (int q = 0; q < NLD; ++q) {
                const int idx = tid + NTH * q;
                As[buf][idx / TILE][idx % TILE] = ra[q];
            }
#pragma unroll
            for (int q = 0; q < NLD; ++q) {
                const int idx = tid + NTH * q;
                int kk, c;
                if (YROWS) { kk = idx / TILE; c = idx % TILE; }
                else { kk = idx % BK; c = idx / BK; }
                Bs[buf][kk][c ^ (kk & 15)] = rb[q];
            }
        };
        auto c_off = [&](int cb, int r4, int r) -> int {
            const int li = WM * wr + 16 * r4 + (lane & 15);
            const int lj = WN * wc + 16 * cb + AT::col(lane, r);
            const bool ok = active && li < mrem && lj < nrem && (!LOWER || (row0 + li) - (col0 + lj) >= g.shift);
            return ok ? (li + lj * (int)ldc) * SZ : BUF_OOB;
        };

        V acc[NBC][NBR];
#pragma unroll
        for (int a = 0; a < NBC; ++a)
#pragma unroll
            for (int b = 0; b < NBR; ++b) acc[a][b] = zero_vec<V>();

        load(0);
        // C of this tile, in flight during the K loop (PERSIST shape only)
        T cv[PERSIST ? NBC : 1][PERSIST ? NBR : 1][4];
        if constexpr (PERSIST) {
#pragma unroll
            for (int cb = 0; cb < NBC; ++cb)
#pragma unroll
                for (int r4 = 0; r4 < NBR; ++r4)
#pragma unroll
                    for (int r = 0; r < 4; ++r) cv[cb][r4][r] = buf_load<T>(rc, c_off(cb, r4, r));
        }
        store(0);
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            const int buf = kt & 1;
            if (kt + 1 < nk) load(kt + 1);
            if (active) {
                const int k0 = kt * BK;
#pragma unroll
                for (int k4 = 0; k4 < BK / 4; ++k4) {
                    if (k0 + 4 * k4 < K) {
                        const int kk = 4 * k4 + (lane >> 4);
                        T fa[NBC], fb[NBR];
#pragma unroll
                        for (int cb = 0; cb < NBC; ++cb)
                            fa[cb] = Bs[buf][kk][(WN * wc + 16 * cb + (lane & 15)) ^ (kk & 15)];
#pragma unroll
                        for (int r4 = 0; r4 < NBR; ++r4)
                            fb[r4] = As[buf][kk][WM * wr + 16 * r4 + (lane & 15)];
#pragma unroll
                        for (int cb = 0; cb < NBC; ++cb)
#pragma unroll
                            for (int r4 = 0; r4 < NBR; ++r4)
                                acc[cb][r4] = AT::mfma(fa[cb], fb[r4], acc[cb][r4]);
                    }
                }
            }
            if (kt + 1 < nk) store(buf ^ 1);
            __syncthreads();
        }

        // Fused write-back: C[i, j] -= S[i, j]; out-of-region entries are neither
        // read nor written (their offsets lie past the buffer's records).
        if constexpr (PERSIST) {
#pragma unroll
            for (int cb = 0; cb < NBC; ++cb)
#pragma unroll
                for (int r4 = 0; r4 < NBR; ++r4)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        buf_store<T>(rc, c_off(cb, r4, r), cv[cb][r4][r] - acc[cb][r4][r]);
        } else {
#pragma unroll
            for (int cb = 0; cb < NBC; ++cb) {
                T cw[NBR][4];
#pragma unroll
                for (int r4 = 0; r4 < NBR; ++r4)
#pragma unroll
                    for (int r = 0; r < 4; ++r) cw[r4][r] = buf_load<T>(rc, c_off(cb, r4, r));
#pragma unroll
                for (int r4 = 0; r4 < NBR; ++r4)
#pragma unroll
                    for (int r = 0; r < 4; ++r) buf_store<T>(rc, c_off(cb, r4, r), cw[r4][r] - acc[cb][r4][r]);
            }
        }
    }
}

// Persistent YROWS kernel for the wide regions that dominate a factorisation.
// One 8-wave workgroup per CU walks 128 x 128 tiles; each wave owns a 64 x 32
// part (8 MFMA blocks).  Operand stages are staged through registers two deep
// (the loads of stage k+2 are in flight while stage k is multiplied and stage
// k+1 is written to LDS), and the per-lane row offsets are computed once per
// tile: the K position of a load travels in the scalar offset.  The tile's C is
// loaded into registers at the start of the tile and written back as C - S at
// its end.
constexpr int PT_TILE = 128;
constexpr int PT_THREADS = 512;
constexpr int PT_WM = 64, PT_WN = 32;

template <typename T> struct pers_depth { static constexpr int BK = 16; };
template <> struct pers_depth<float> { static constexpr int BK = 32; };

template <typename T, bool LOWER>
__global__ __launch_bounds__(PT_THREADS, 1)
void update_rows_kernel(int M, int N, int K, T* __restrict__ C, int64_t ldc, const T* __restrict__ X, int64_t ldx,
                        const T* __restrict__ Y, int64_t ldy, Grid g, const int* __restrict__ info)
{
    if (info && *info != 0) return;
    constexpr int BK = pers_depth<T>::BK;
    constexpr int SZ = sizeof(T);
    constexpr int NLD = BK * PT_TILE / PT_THREADS;          // elements per thread per operand per stage
    constexpr int NBR = PT_WM / 16, NBC = PT_WN / 16;
    typedef acc_traits<T> AT;
    typedef typename AT::vec V;

    __shared__ T As[2][BK][PT_TILE];
    __shared__ T Bs[2][BK][PT_TILE];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave % 2, wc = wave / 2;
    const int sr = tid % PT_TILE;                 // staging row of this thread
    const int skk = wave / 2;                     // first staging K index (uniform per wave)
    const int nk = (K + BK - 1) / BK;
    const int xs = (int)ldx * SZ, ys = (int)ldy * SZ;

    for (int slot = blockIdx.x; slot < g.nslots; slot += gridDim.x) {
        int bi, bj;
        if (!tile_of_slot(g, slot, LOWER, bi, bj)) continue;
        const int row0 = bi * PT_TILE, col0 = bj * PT_TILE;
        const int mrem = M - row0, nrem = N - col0;
        const bool active = !LOWER || (row0 + PT_WM * wr + PT_WM - 1) - (col0 + PT_WN * wc) >= g.shift;
        const rsrc_t rx = make_rsrc(X + row0);
        const rsrc_t ry = make_rsrc(Y + col0);
        const rsrc_t rc = make_rsrc(C + row0 + (int64_t)col0 * ldc);
        const int vx = sr < mrem ? sr * SZ : BUF_OOB;
        const int vy = sr < nrem ? sr * SZ : BUF_OOB;

        T xa0[NLD], ya0[NLD], xa1[NLD], ya1[NLD];
        // K columns past the end get an offset at or beyond the records (the OR with
        // BUF_OOB), written without a select so every load issues unconditionally.
        auto load = [&](int kt, T (&xa)[NLD], T (&ya)[NLD]) {
#pragma unroll
            for (int q = 0; q < NLD; ++q) {
                const int gk = kt * BK + skk + 4 * q;
                const int past = (K - 1 - gk) >> 31;            // all ones when gk >= K
                xa[q] = buf_load<T>(rx, vx, (gk * xs) | (past & BUF_OOB));
                ya[q] = buf_load<T>(ry, vy, (gk * ys) | (past & BUF_OOB));
            }
        };
        auto store = [&](int buf, const T (&xa)[NLD], const T (&ya)[NLD]) {
#pragma unroll
            for (int q = 0; q < NLD; ++q) {
                As[buf][skk + 4 * q][sr] = xa[q];
                Bs[buf][skk + 4 * q][sr] = ya[q];
            }
        };

        V acc[NBC][NBR];
#pragma unroll
        for (int a = 0; a < NBC; ++a)
#pragma unroll
            for (int b = 0; b < NBR; ++b) acc[a][b] = zero_vec<V>();
        auto compute = [&](int kt, int buf) {
            if (!active) return;
            const int k0 = kt * BK;
#pragma unroll
            for (int k4 = 0; k4 < BK / 4; ++k4) {
                if (k0 + 4 * k4 < K) {
                    const int kk = 4 * k4 + (lane >> 4);
                    T fa[NBC], fb[NBR];
#pragma unroll
                    for (int cb = 0; cb < NBC; ++cb) fa[cb] = Bs[buf][kk][PT_WN * wc + 16 * cb + (lane & 15)];
#pragma unroll
                    for (int r4 = 0; r4 < NBR; ++r4) fb[r4] = As[buf][kk][PT_WM * wr + 16 * r4 + (lane & 15)];
#pragma unroll
                    for (int cb = 0; cb < NBC; ++cb)
#pragma unroll
                        for (int r4 = 0; r4 < NBR; ++r4) acc[cb][r4] = AT::mfma(fa[cb], fb[r4], acc[cb][r4]);
                }
            }
        };

        // C offsets: interior tiles take a per-lane base plus uniform column steps;
        // tiles on an edge or on the diagonal mask each entry.
        const bool full = mrem >= PT_TILE && nrem >= PT_TILE &&
                          (!LOWER || row0 - (col0 + PT_TILE - 1) >= g.shift);
        const int li0 = PT_WM * wr + (lane & 15);
        auto c_off = [&](int cb, int r4, int r) -> int {
            const int li = li0 + 16 * r4;
            const int lj = PT_WN * wc + 16 * cb + AT::col(lane, r);
            if (full) return (li + lj * (int)ldc) * SZ;
            const bool ok = active && li < mrem && lj < nrem && (!LOWER || (row0 + li) - (col0 + lj) >= g.shift);
            return ok ? (li + lj * (int)ldc) * SZ : BUF_OOB;
        };

        load(0, xa0, ya0);
        load(1, xa1, ya1);
        store(0, xa0, ya0);
        __syncthreads();
        T cv[NBC][NBR][4];
#pragma unroll
        for (int cb = 0; cb < NBC; ++cb)
#pragma unroll
            for (int r4 = 0; r4 < NBR; ++r4)
#pragma unroll
                for (int r = 0; r < 4; ++r) cv[cb][r4][r] = bufop<T, AUX_NT>::load(rc, c_off(cb, r4, r), 0);

        // The prefetch is issued unconditionally (stages past the end load zeros
        // without touching memory) so the compiler's wait before the LDS store
        // only covers the stage being stored.
        for (int kt = 0; kt < nk;) {
            // even step: registers 0 free, registers 1 hold stage kt+1
            load(kt + 2, xa0, ya0);
            compute(kt, 0);
            if (kt + 1 < nk) store(1, xa1, ya1);
            __syncthreads();
            if (++kt >= nk) break;
            // odd step: registers 1 free, registers 0 hold stage kt+1
            load(kt + 2, xa1, ya1);
            compute(kt, 1);
            if (kt + 1 < nk) store(0, xa0, ya0);
            __syncthreads();
            ++kt;
        }

        if (active) {
#pragma unroll
            for (int cb = 0; cb < NBC; ++cb)
#pragma unroll
                for (int r4 = 0; r4 < NBR; ++r4)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        bufop<T, AUX_NT>::store(rc, c_off(cb, r4, r), cv[cb][r4][r] - acc[cb][r4][r], 0);
        }
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

    for (int slot = blockIdx.x; slot < g.nslots; slot += gridDim.x) {
        int bi, bj;
        if (!tile_of_slot(g, slot, LOWER, bi, bj)) continue;
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

Grid make_grid(int tile, int M, int N, bool lower, int shift) {
    Grid g;
    g.tile = tile;
    g.nbm = (M + tile - 1) / tile;
    g.nbn = (N + tile - 1) / tile;
    g.nsm = (g.nbm + UPD_GROUP - 1) / UPD_GROUP;
    g.nsn = (g.nbn + UPD_GROUP - 1) / UPD_GROUP;
    g.tri = (lower && M == N && shift == 0) ? 1 : 0;
    g.shift = shift;
    const int nsup = g.tri ? g.nsm * (g.nsm + 1) / 2 : g.nsm * g.nsn;
    g.nslots = ((nsup + N_XCD - 1) / N_XCD) * N_XCD * UPD_WG_PER_SUPER;
    return g;
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
inline bool ld_fits(int64_t ld, size_t sz) { return (128 + 128 * ld) * (int64_t)sz < (int64_t)BUF_RECORDS; }

int cu_count() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cached[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        cached[dev] = v;
    }
    return cached[dev];
}

template <typename T, int TILE, bool PERSIST>
hipError_t launch_shape(int M, int N, int Kc, T* C, int64_t ldc, const T* X, int64_t ldx, const T* Y, int64_t ldy,
                        bool yrows, bool lower, const Grid& g, int nwg, const int* info, hipStream_t st) {
#define FF_UPD_LAUNCH(YR, LO)                                                                                     \
    hipLaunchKernelGGL((update_kernel<T, TILE, YR, LO, PERSIST>), dim3(nwg), dim3(shape<TILE, PERSIST>::THREADS), 0, \
                       st, M, N, Kc, C, ldc, X, \
                       ldx, Y, ldy, g, info)
    if (yrows) {
        if (lower) FF_UPD_LAUNCH(true, true);
        else FF_UPD_LAUNCH(true, false);
    } else {
        if (lower) FF_UPD_LAUNCH(false, true);
        else FF_UPD_LAUNCH(false, false);
    }
#undef FF_UPD_LAUNCH
    return hipGetLastError();
}

}  // namespace

int update_workers(int reserve_cus) {
    const int cus = cu_count();
    int w = cus - (reserve_cus > 0 ? reserve_cus : 0);
    w = (w / N_XCD) * N_XCD;
    return w < N_XCD ? N_XCD : w;
}

template <typename T>
hipError_t launch_update(int M, int N, int K, T* C, int64_t ldc, const T* X, int64_t ldx, const T* Y, int64_t ldy,
                         bool yrows, bool lower, int shift, const int* info, hipStream_t st, int reserve_cus) {
    if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
    if (!ld_fits(ldc, sizeof(T)) || (!yrows && !ld_fits(ldy, sizeof(T)))) return hipErrorInvalidValue;
    const int kc = max_k_chunk(ldx, ldy, yrows, sizeof(T));
    if (kc < 1) return hipErrorInvalidValue;
    // narrow regions (fewer 128-wide tiles than half the CUs) use 64 tiles
    const bool narrow = (M < 2 * 128 || N < 2 * 128) ||
                        ((int64_t)((M + 127) / 128) * ((N + 127) / 128) < (int64_t)cu_count() / 2);
    for (int k0 = 0; k0 < K; k0 += kc) {
        const int Kc = (K - k0 < kc) ? K - k0 : kc;
        const T* Xk = X + (int64_t)k0 * ldx;
        const T* Yk = yrows ? Y + (int64_t)k0 * ldy : Y + k0;
        hipError_t e;
        if (narrow) {
            const Grid g = make_grid(64, M, N, lower, shift);
            e = launch_shape<T, 64, false>(M, N, Kc, C, ldc, Xk, ldx, Yk, ldy, yrows, lower, g, g.nslots, info, st);
        } else if (yrows) {
            const Grid g = make_grid(PT_TILE, M, N, lower, shift);
            int nwg = update_workers(reserve_cus);
            if (nwg > g.nslots) nwg = g.nslots;
            if (lower)
                hipLaunchKernelGGL((update_rows_kernel<T, true>), dim3(nwg), dim3(PT_THREADS), 0, st, M, N, Kc, C, ldc,
                                   Xk, ldx, Yk, ldy, g, info);
            else
                hipLaunchKernelGGL((update_rows_kernel<T, false>), dim3(nwg), dim3(PT_THREADS), 0, st, M, N, Kc, C,
                                   ldc, Xk, ldx, Yk, ldy, g, info);
            e = hipGetLastError();
        } else {
            const Grid g = make_grid(128, M, N, lower, shift);
            int nwg = update_workers(reserve_cus);
            if (nwg > g.nslots) nwg = g.nslots;
            e = launch_shape<T, 128, true>(M, N, Kc, C, ldc, Xk, ldx, Yk, ldy, yrows, lower, g, nwg, info, st);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_update_bf16(int M, int N, int K, float* C, int64_t ldc, const float* X, int64_t ldx,
                              const float* Y, int64_t ldy, bool lower, int shift, const int* info, hipStream_t st,
                              int reserve_cus) {
    if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
    if (!ld_fits(ldc, sizeof(float))) return hipErrorInvalidValue;
    const int kc = max_k_chunk(ldx, ldy, true, sizeof(float));
    if (kc < 1) return hipErrorInvalidValue;
    const Grid g = make_grid(BF_TILE, M, N, lower, shift);
    int nwg = update_workers(reserve_cus);
    if (nwg > g.nslots) nwg = g.nslots;
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

template hipError_t launch_update<double>(int, int, int, double*, int64_t, const double*, int64_t, const double*,
                                          int64_t, bool, bool, int, const int*, hipStream_t, int);
template hipError_t launch_update<float>(int, int, int, float*, int64_t, const float*, int64_t, const float*,
                                         int64_t, bool, bool, int, const int*, hipStream_t, int);

}  // namespace ff
