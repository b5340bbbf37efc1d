// solve.hip -- solves with a computed factor and the binary64 refinement pieces.
//
// Solving A x = b from A = L L^T (Introduction of arXiv 1812.02056) needs two
// triangular solves.  Refinement (binary64 residual r = b - A x, correction
// from the low-precision factor, x += d) is how the mixed-precision factor wins
// back binary64 accuracy.
//
// Triangular solves: the n rows are cut into 64-row blocks, solved in order
// (forward sweep L y = b, then backward sweep L^T x = y).  Block j needs
// b_j - sum_i L(j, i) x_i over the blocks solved before it.  One persistent
// workgroup (the solver) walks the blocks: it keeps the newest TRI_F solutions
// in LDS, folds their tiles (held in registers, loaded one block ahead)
// itself, adds the partial sum of all older blocks, and applies the
// precomputed inverse of the diagonal block.  The older blocks are folded by
// one helper workgroup per block, which takes each solved block as it appears
// and hands its partial sum over when done.  The chain from one block to the
// next therefore stays inside one workgroup; the helpers have TRI_F blocks of
// the solver's time to deliver.
//
// Hand-over between workgroups goes through values, not flags: solved blocks
// and partial sums are written with relaxed agent-scope atomic stores into an
// area filled beforehand with a sentinel bit pattern (a NaN that is never
// stored: NaN results are stored as the canonical quiet NaN), and a reader
// polls each value with relaxed atomic loads until it is no longer the
// sentinel.  Each value is its own flag, so no release fence is needed.  Every
// wait is bounded: past the spin limit, or once another workgroup has recorded
// an expired wait, the workgroup records the error and leaves.
//
// The binary64 residual R = B - A X reads tril(A) once per use of symmetry:
// workgroups own (row block, chunk of column blocks) pairs and write partial
// products, which a second kernel adds in a fixed order.
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace ff {

namespace {

constexpr int TB = TRI_TB;      // row block of the triangular solves
constexpr int RHS_CHUNK = 16;   // right-hand sides per residual launch
constexpr int RC = TRI_RC;      // right-hand sides per triangular sweep
constexpr int NQ = RC / 4;      // columns a thread owns in the sweep's reductions (at most)
constexpr int SPIN_LIMIT = 1 << 20;

template <typename S>
__global__ void copy_lower_kernel(int n, const double* __restrict__ A, int64_t lda, S* __restrict__ W, int64_t ldw) {
    const int j = blockIdx.y;
    for (int i = j + blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        W[i + (int64_t)j * ldw] = (S)A[i + (int64_t)j * lda];
}

template <typename S>
__global__ void convert_kernel(int n, const double* __restrict__ B, int64_t ldb, S* __restrict__ X, int64_t ldx) {
    const int j = blockIdx.y;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        X[i + (int64_t)j * ldx] = (S)B[i + (int64_t)j * ldb];
}

// Per-factor data of the triangular solves: 64 x 64 tiles stored in the order
// the solving workgroup's threads read them ("thread-major"): element (r, k)
// at ((k / 16) * 64 + r) * 16 + k % 16, so thread (r, g) = (lane, wave) finds
// row r, columns 16g..16g+15 as 16 contiguous values.  Tile index:
//   [0, nblk)                       inverse of diagonal block j
//   [nblk, 2 nblk)                  its transpose
//   2 nblk + j F + f - 1            L(j, j - f)          (forward sweep), j >= f
//   2 nblk + nblk F + j F + f - 1   L(j + f, j)^T        (backward sweep), j + f < nblk
// with F = TRI_F, rows or columns past n zero.
__device__ __forceinline__ int tm_index(int r, int k) { return ((k >> 4) * TB + r) * 16 + (k & 15); }

// Inverses of the 64 x 64 lower-triangular diagonal blocks of L, computed in
// binary64 by column-wise forward substitution and rounded to S (zero above
// the diagonal and outside a short last block).
template <typename S>
__global__ __launch_bounds__(64)
void inv_diag_kernel(int n, const S* __restrict__ L, int64_t ldl, S* __restrict__ fac) {
    __shared__ double x[TB][TB + 1];    // x[i][c]
    __shared__ double l[TB][TB + 1];    // l[i][k]
    const int nblk = (n + TB - 1) / TB;
    const int b = blockIdx.x;
    const int r0 = b * TB;
    const int nb = min(TB, n - r0);
    const int c = threadIdx.x;
    for (int k = 0; k < TB; ++k)
        l[c][k] = (c < nb && k < nb && k <= c) ? (double)L[(int64_t)(r0 + c) + (int64_t)(r0 + k) * ldl] : 0.0;
    __syncthreads();
    // column c of the inverse: solve L x = e_c
    for (int i = 0; i < TB; ++i) {
        double v = 0.0;
        if (c < nb && i < nb && i >= c) {
            v = (i == c) ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) v -= l[i][k] * x[k][c];
            v = v / l[i][i];
        }
        x[i][c] = v;
    }
    __syncthreads();
    S* inv = fac + (size_t)b * TB * TB;
    S* invt = fac + ((size_t)nblk + b) * TB * TB;
    for (int e = c; e < TB * TB; e += 64) {
        const int tm = e >> 4, r = tm & (TB - 1), k = ((tm >> 6) << 4) | (e & 15);
        inv[e] = (S)x[r][k];
        invt[e] = (S)x[k][r];
    }
}

// The tiles the solving workgroup folds itself (blockIdx.z = 0: L(j, j - f) of
// the forward sweep; 1: L(j + f, j)^T of the backward sweep), f = blockIdx.y + 1.
template <typename S>
__global__ __launch_bounds__(256)
void near_tiles_kernel(int n, const S* __restrict__ L, int64_t ldl, S* __restrict__ fac) {
    __shared__ S t[TB][TB + 1];
    const int nblk = (n + TB - 1) / TB;
    const int j = blockIdx.x, f = blockIdx.y + 1;
    const bool back = blockIdx.z == 1;
    const int i = back ? j + f : j - f;
    if (i < 0 || i >= nblk) return;
    // the tile's rows belong to block rb (possibly short), its columns to block cb (whole)
    const int rb = back ? i : j, cb = back ? j : i;
    const int r0 = rb * TB, c0 = cb * TB, nbr = min(TB, n - r0);
    for (int e = threadIdx.x; e < TB * TB; e += 256) {
        const int a = e % TB, c = e / TB;
        t[a][c] = a < nbr ? L[(int64_t)(r0 + a) + (int64_t)(c0 + c) * ldl] : S(0);
    }
    __syncthreads();
    S* out = fac + ((size_t)2 * nblk + (back ? (size_t)nblk * TRI_F : 0) + (size_t)j * TRI_F + f - 1) * TB * TB;
    for (int e = threadIdx.x; e < TB * TB; e += 256) {
        const int tm = e >> 4, r = tm & (TB - 1), k = ((tm >> 6) << 4) | (e & 15);
        out[e] = back ? t[k][r] : t[r][k];
    }
}

// 16 contiguous values of a thread-major tile (16-byte aligned), as vector loads.
template <typename S>
__device__ __forceinline__ void load16(const S* __restrict__ p, S (&v)[16]) {
    if constexpr (sizeof(S) == 4) {
        const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float4 w = q[u];
            v[4 * u] = w.x; v[4 * u + 1] = w.y; v[4 * u + 2] = w.z; v[4 * u + 3] = w.w;
        }
    } else {
        const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double2 w = q[u];
            v[2 * u] = w.x; v[2 * u + 1] = w.y;
        }
    }
}

// Bit patterns of the hand-off area: SENT marks "not written yet"; a NaN
// result is stored as QNAN so that no stored value equals SENT.
template <typename S> struct PubBits;
template <> struct PubBits<float> {
    typedef unsigned int U;
    static constexpr U SENT = 0xFFFFFFFFu;
    static constexpr U QNAN = 0x7FC00000u;
    static __device__ __forceinline__ U bits(float v) { return __float_as_uint(v); }
    static __device__ __forceinline__ float val(U b) { return __uint_as_float(b); }
};
template <> struct PubBits<double> {
    typedef unsigned long long U;
    static constexpr U SENT = 0xFFFFFFFFFFFFFFFFull;
    static constexpr U QNAN = 0x7FF8000000000000ull;
    static __device__ __forceinline__ U bits(double v) { return (U)__double_as_longlong(v); }
    static __device__ __forceinline__ double val(U b) { return __longlong_as_double((long long)b); }
};

template <typename S>
__device__ __forceinline__ void pub_put(S* p, S v) {
    using B = PubBits<S>;
    typename B::U b = B::bits(v);
    if (b == B::SENT) b = B::QNAN;
    __hip_atomic_store(reinterpret_cast<typename B::U*>(p), b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename S>
__device__ __forceinline__ typename PubBits<S>::U pub_peek(const S* p) {
    using U = typename PubBits<S>::U;
    return __hip_atomic_load(reinterpret_cast<U*>(const_cast<S*>(p)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Poll *p until it holds a published value; b holds the value last read.
// False when the wait expired or another workgroup recorded an error.
template <typename S>
__device__ __forceinline__ bool pub_wait(const S* p, typename PubBits<S>::U& b, const int* err) {
    int spins = 0;
    while (b == PubBits<S>::SENT) {
        if (++spins > SPIN_LIMIT) return false;
        if ((spins & 127) == 0 &&
            __hip_atomic_load(const_cast<int*>(err), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
            return false;
        __builtin_amdgcn_s_sleep(1);
        b = pub_peek(p);
    }
    return true;
}

__device__ __forceinline__ void record_error(int* err, int* sh_bad) {
    *sh_bad = 1;
    __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// LDS of the sweep kernel, shared by the two roles (elements of S):
//   solver: ring[TRI_F][TB][RC] (newest solutions), red[4][TB][RC + 1], ys[TB][RC]
//   helper: xs[2][TB][RC] (solved block), red[4][TB][RC + 1], stg[4][16][68]
constexpr int RED_ELEMS = 4 * TB * (RC + 1);
constexpr int SOLVER_ELEMS = TRI_F * TB * RC + RED_ELEMS + TB * RC;
constexpr int HELPER_ELEMS = 2 * TB * RC + RED_ELEMS + 4 * 16 * 68;
constexpr int SWEEP_LDS_ELEMS = SOLVER_ELEMS > HELPER_ELEMS ? SOLVER_ELEMS : HELPER_ELEMS;

// The solving workgroup of a sweep (forward: L y = b; TRANS: L^T x = y), all
// blocks in sweep order jj (block j = jj, or nblk - 1 - jj backward).  Thread
// (r, g) = (lane, wave) owns row r of a block and the quarter g of its inner
// index (columns 16g..16g+15 of a tile); in the reductions it owns the
// right-hand-side columns c = g + 4q.  NRC >= nr columns are computed.
template <typename S, bool TRANS, int NRC>
__device__ void tri_solver(int n, int nr, const S* __restrict__ L, int64_t ldl, const S* __restrict__ fac, S* X,
                           int64_t ldx, S* xpub, const S* part, int* err, S* smem, int* sh_bad) {
    constexpr int F = TRI_F;
    constexpr int QN = (NRC + 3) / 4;   // column slots c = g + 4q that can hold a column
    using U = typename PubBits<S>::U;
    const int nblk = (n + TB - 1) / TB;
    const int tid = threadIdx.x, r = tid & (TB - 1), g = tid >> 6;
    S (*ring)[TB][RC] = reinterpret_cast<S (*)[TB][RC]>(smem);
    S (*red)[TB][RC + 1] = reinterpret_cast<S (*)[TB][RC + 1]>(smem + F * TB * RC);
    S (*ys)[RC] = reinterpret_cast<S (*)[RC]>(smem + F * TB * RC + RED_ELEMS);
    const S* inv = fac + (TRANS ? (size_t)nblk * TB * TB : 0);
    const S* nearb = fac + ((size_t)2 * nblk + (TRANS ? (size_t)nblk * TRI_F : 0)) * TB * TB;

    S T[F][16];     // fold tiles of the current block: distance f + 1, row r, inner quarter g
    S V[16];        // inverse of the current diagonal block: row r, inner quarter g
    S bq[QN];       // right-hand side (r, g + 4q) of the current block, as loaded
    U pq[QN];       // older blocks' partial sum (r, g + 4q) of the current block, as loaded (SENT: not yet seen)

    // Prefetches for block jj.  Each issues the same loads whatever jj, nr and
    // the block's height (addresses clamped into the buffers), and keeps the
    // raw values: masks are applied where the values are used, so the number of
    // loads in flight does not depend on the path, nothing waits at issue, and
    // each wait covers only the loads it needs.
    auto load_fold = [&](int jj) {
        const int jc = min(jj, nblk - 1);
        const int j = TRANS ? nblk - 1 - jc : jc;
#pragma unroll
        for (int f = 0; f < F; ++f) load16(nearb + ((size_t)j * F + f) * TB * TB + tid * 16, T[f]);
    };
    auto load_inv = [&](int jj) {
        const int jc = min(jj, nblk - 1);
        const int j = TRANS ? nblk - 1 - jc : jc;
        load16(inv + (size_t)j * TB * TB + tid * 16, V);
    };
    auto load_rhs = [&](int jj) {
        const int jc = min(jj, nblk - 1);
        const int j = TRANS ? nblk - 1 - jc : jc;
        const int j0 = j * TB, nbr = min(TB, n - j0);
        const int rr = r < nbr ? r : 0;
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            const int cc = g + 4 * q < nr ? g + 4 * q : 0;
            bq[q] = X[(int64_t)(j0 + rr) + (int64_t)cc * ldx];
            pq[q] = pub_peek(part + ((size_t)jc * TB + r) * RC + cc);
        }
    };

    // Each of the next block's prefetches is issued after the last use of its
    // registers in this block: fold tiles after the fold, the inverse after the
    // inverse, right-hand side and partial sum after the publish (by then the
    // helper has had TRI_F - 1 blocks of time since its last source appeared).
    load_fold(0);
    load_inv(0);
    load_rhs(0);
    for (int jj = 0; jj < nblk; ++jj) {
        const int j = TRANS ? nblk - 1 - jj : jj;
        const int j0 = j * TB, nbr = min(TB, n - j0);
        // 1. fold the newest solved blocks over this thread's inner quarter (one
        //    column: four interleaved partial sums, added in a fixed order)
        {
            constexpr int NS = NRC == 1 ? 4 : 1;
            S s[NS][NRC];
#pragma unroll
            for (int u = 0; u < NS; ++u)
#pragma unroll
                for (int c = 0; c < NRC; ++c) s[u][c] = S(0);
#pragma unroll
            for (int f = 0; f < F; ++f) {
                if (f < jj) {
                    const int slot = (jj - 1 - f) % F;
#pragma unroll
                    for (int t = 0; t < 16; ++t) {
                        const S tv = T[f][t];
                        const S* xr = ring[slot][16 * g + t];
#pragma unroll
                        for (int c = 0; c < NRC; ++c) s[t % NS][c] += tv * xr[c];
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < NRC; ++c) {
                S v = s[0][c];
                if constexpr (NS == 4) v = (s[0][c] + s[1][c]) + (s[2][c] + s[3][c]);
                red[g][r][c] = v;
            }
        }
        load_fold(jj + 1);
        __syncthreads();
        // 2. y = b - (older blocks) - (newest blocks) for the columns this thread owns
        bool ok = true;
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            const int c = g + 4 * q;
            if (c < NRC) {
                S p = S(0);
                if (jj > F && c < nr) {
                    ok &= pub_wait(part + ((size_t)jj * TB + r) * RC + c, pq[q], err);
                    p = PubBits<S>::val(pq[q]);
                }
                const S b = (c < nr && r < nbr) ? bq[q] : S(0);
                ys[r][c] = b - p - ((red[0][r][c] + red[1][r][c]) + (red[2][r][c] + red[3][r][c]));
            }
        }
        if (!ok) record_error(err, sh_bad);
        __syncthreads();
        if (*sh_bad) return;
        // 3. x = (inverse of the diagonal block) y, over this thread's inner quarter
        {
            constexpr int NS = NRC == 1 ? 4 : 1;
            S u[NS][NRC];
#pragma unroll
            for (int v = 0; v < NS; ++v)
#pragma unroll
                for (int c = 0; c < NRC; ++c) u[v][c] = S(0);
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const S* yr = ys[16 * g + t];
#pragma unroll
                for (int c = 0; c < NRC; ++c) u[t % NS][c] += V[t] * yr[c];
            }
#pragma unroll
            for (int c = 0; c < NRC; ++c) {
                S v = u[0][c];
                if constexpr (NS == 4) v = (u[0][c] + u[1][c]) + (u[2][c] + u[3][c]);
                red[g][r][c] = v;
            }
        }
        load_inv(jj + 1);
        __syncthreads();
        // 4. publish the solved block (the next block's right-hand side and
        //    partial sum are requested first)
        load_rhs(jj + 1);
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            const int c = g + 4 * q;
            if (c < NRC) {
                const S x = (red[0][r][c] + red[1][r][c]) + (red[2][r][c] + red[3][r][c]);
                ring[jj % F][r][c] = x;
                if (c < nr) {
                    if (r < nbr) X[(int64_t)(j0 + r) + (int64_t)c * ldx] = x;
                    pub_put(xpub + ((size_t)jj * TB + r) * RC + c, x);
                }
            }
        }
        __syncthreads();
    }
}

// A helper workgroup: the partial sum over the blocks at distance > TRI_F from
// block jj (sweep order), taken oldest first as they are published.
template <typename S, bool TRANS, int NRC>
__device__ void tri_helper(int jj, int n, int nr, const S* __restrict__ L, int64_t ldl, const S* xpub, S* part,
                           int* err, S* smem, int* sh_bad) {
    constexpr int F = TRI_F;
    constexpr int QN = (NRC + 3) / 4;
    using U = typename PubBits<S>::U;
    const int nblk = (n + TB - 1) / TB;
    const int tid = threadIdx.x, r = tid & (TB - 1), g = tid >> 6;
    S (*xs)[TB][RC] = reinterpret_cast<S (*)[TB][RC]>(smem);
    S (*red)[TB][RC + 1] = reinterpret_cast<S (*)[TB][RC + 1]>(smem + 2 * TB * RC);
    S (*stg)[16][68] = reinterpret_cast<S (*)[16][68]>(smem + 2 * TB * RC + RED_ELEMS);
    const int j = TRANS ? nblk - 1 - jj : jj;
    const int j0 = j * TB, nbr = min(TB, n - j0);
    const int nsrc = jj - F;        // sources ii = 0 .. nsrc - 1
    S acc[NRC];
#pragma unroll
    for (int c = 0; c < NRC; ++c) acc[c] = S(0);
    S Tn[16], Tc[16];
    // Tile of source ii as loaded: (r, g) layout forward; backward a 16-row slab
    // of L(i, j) per wave, lane (a, cb) = (r & 15, r >> 4) holding row a and
    // columns cb + 4u, turned into (r, g) layout through the wave's own LDS.
    auto load_tile = [&](int ii) {
        if (!TRANS) {
            const int i0 = ii * TB;
            const S* src = L + (int64_t)(j0 + (r < nbr ? r : 0)) + (int64_t)(i0 + 16 * g) * ldl;
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const S v = src[(int64_t)t * ldl];
                Tn[t] = r < nbr ? v : S(0);
            }
        } else {
            const int i = nblk - 1 - ii, i0 = i * TB, nbi = min(TB, n - i0);
            const int a = r & 15, cb = r >> 4;
            const bool in = 16 * g + a < nbi;
            const S* src = L + (int64_t)(i0 + (in ? 16 * g + a : 0)) + (int64_t)(j0 + cb) * ldl;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const S v = src[(int64_t)(4 * u) * ldl];
                Tn[u] = in ? v : S(0);
            }
        }
    };
    auto settle_tile = [&]() {
        if (!TRANS) {
#pragma unroll
            for (int t = 0; t < 16; ++t) Tc[t] = Tn[t];
        } else {
            const int a = r & 15, cb = r >> 4;
#pragma unroll
            for (int u = 0; u < 16; ++u) stg[g][a][cb + 4 * u] = Tn[u];
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int t = 0; t < 16; ++t) Tc[t] = stg[g][t][r];
            __builtin_amdgcn_wave_barrier();
        }
    };
    load_tile(0);
    for (int ii = 0; ii < nsrc; ++ii) {
        settle_tile();
        if (ii + 1 < nsrc) load_tile(ii + 1);
        S (*xb)[RC] = xs[ii & 1];
        bool ok = true;
        U b[QN];
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            const int c = g + 4 * q;
            b[q] = (c < NRC && c < nr) ? pub_peek(xpub + ((size_t)ii * TB + r) * RC + c) : PubBits<S>::bits(S(0));
        }
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            const int c = g + 4 * q;
            if (c < NRC) {
                if (c < nr) ok &= pub_wait(xpub + ((size_t)ii * TB + r) * RC + c, b[q], err);
                xb[r][c] = PubBits<S>::val(b[q]);
            }
        }
        if (!ok) record_error(err, sh_bad);
        __syncthreads();
        if (*sh_bad) return;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const S tv = Tc[t];
            const S* xr = xb[16 * g + t];
#pragma unroll
            for (int c = 0; c < NRC; ++c) acc[c] += tv * xr[c];
        }
    }
#pragma unroll
    for (int c = 0; c < NRC; ++c) red[g][r][c] = acc[c];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QN; ++q) {
        const int c = g + 4 * q;
        if (c < NRC && c < nr)
            pub_put(part + ((size_t)jj * TB + r) * RC + c,
                    (red[0][r][c] + red[1][r][c]) + (red[2][r][c] + red[3][r][c]));
    }
}

// One sweep over nr <= RC right-hand sides (X in place).  Workgroup tickets in
// start order: ticket 0 is the solver, ticket t >= 1 the helper of block
// TRI_F + t.  pub: solved blocks (nblk*64 x RC) then partial sums (nblk*64 x
// RC), all SENT on entry.
template <typename S, bool TRANS, int NRC>
__global__ __launch_bounds__(256)
void trisolve_kernel(int n, int nr_all, int groups, const S* __restrict__ L, int64_t ldl, const S* __restrict__ fac,
                     S* X, int64_t ldx, S* pub, int* err, int* ticket)
{
    __shared__ S smem[SWEEP_LDS_ELEMS];
    __shared__ int sh_ticket, sh_bad;
    // workgroup b serves chain b % groups (columns [c0, c0 + NRC)); within a
    // chain the first workgroup to start is the solver
    const int grp = blockIdx.x % groups;
    if (threadIdx.x == 0) {
        sh_ticket = atomicAdd(ticket + grp, 1);
        sh_bad = 0;
    }
    __syncthreads();
    const int nblk = (n + TB - 1) / TB;
    const int c0 = grp * NRC;
    const int nr = min(NRC, nr_all - c0);
    X += (int64_t)c0 * ldx;
    S* xpub = pub + c0;
    S* part = pub + (size_t)nblk * TB * RC + c0;
    if (sh_ticket == 0)
        tri_solver<S, TRANS, NRC>(n, nr, L, ldl, fac, X, ldx, xpub, part, err, smem, &sh_bad);
    else
        tri_helper<S, TRANS, NRC>(TRI_F + sh_ticket, n, nr, L, ldl, xpub, part, err, smem, &sh_bad);
}

// Fill the hand-off area with SENT and clear the sweeps' tickets.
template <typename S>
__global__ void pub_reset_kernel(S* pub, size_t count, int* tickets) {
    using U = typename PubBits<S>::U;
    U* q = reinterpret_cast<U*>(pub);
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        q[i] = PubBits<S>::SENT;
    if (blockIdx.x == 0 && threadIdx.x < 2 * TRI_GROUPS) tickets[threadIdx.x] = 0;
}

template <typename S, bool TRANS>
hipError_t launch_sweep(int n, int nr, const S* L, int64_t ldl, const S* fac, S* X, int64_t ldx, S* pub, int* err,
                        int* ticket, hipStream_t st) {
    const int nblk = (n + TB - 1) / TB;
    const int per_chain = 1 + std::max(0, nblk - TRI_F - 1);
    // chain width measured at n = 16384 (ms per solve pair, binary32 / binary64):
    // 2 columns 1.32 / 2.54 (4 rhs), 1.65 / 3.09 (8), 2.12 / 4.96 (16); 4 columns
    // 1.67 / 2.86, 1.95 / 3.11, 2.35 / 3.69; 1 and 8 columns slower throughout
    if (nr == 1) {
        hipLaunchKernelGGL((trisolve_kernel<S, TRANS, 1>), dim3(per_chain), dim3(256), 0, st, n, nr, 1, L, ldl, fac,
                           X, ldx, pub, err, ticket);
    } else if (sizeof(S) == 4 || nr <= 8) {
        const int groups = (nr + TRI_GC - 1) / TRI_GC;
        hipLaunchKernelGGL((trisolve_kernel<S, TRANS, TRI_GC>), dim3(per_chain * groups), dim3(256), 0, st, n, nr,
                           groups, L, ldl, fac, X, ldx, pub, err, ticket);
    } else {
        const int groups = (nr + TRI_GC_WIDE - 1) / TRI_GC_WIDE;
        hipLaunchKernelGGL((trisolve_kernel<S, TRANS, TRI_GC_WIDE>), dim3(per_chain * groups), dim3(256), 0, st, n,
                           nr, groups, L, ldl, fac, X, ldx, pub, err, ticket);
    }
    return hipGetLastError();
}

// Partial products of R = B - A X in binary64 with A symmetric, only tril(A)
// read, each stored tile once.  The 64 x 64 tiles of the lower triangle are
// grouped into segments of RS_G x RS_G tiles; workgroup (J, I), J >= I, takes
// the tiles (j, i), j in row segment J, i in column segment I, j >= i, column
// block by column block, and uses each twice:
//   A(j, i) x_i     for row block j: summed over i (ascending) into
//                    part[D, I] (rows of segment J);
//   A(j, i)^T x_j   for row block i (j > i): summed over j (ascending) into
//                    part[T, J] (rows of segment I).
// A diagonal tile (j = i) is made symmetric in LDS and taken once, as a row
// product.  The products run on v_mfma_f64_16x16x4f64, one 16-row slice of the
// tile per wave over all 16 right-hand sides.  With rsum the absolute row sums are formed the same way (column
// RHS_CHUNK of each part).  residual_reduce_kernel adds, for a row of segment
// K, part[D, I] for I = 0..K and then part[T, J] for J = K..nseg-1: a fixed
// order, so results do not depend on scheduling.
// Layout: part[D, I] holds rows [I SR, n) (SR = 64 RS_G rows), part[T, J] rows
// [0, min(n, (J+1) SR)), each as RS_COLS columns of that length; all D parts
// first, then all T parts: 17 (nseg + 1) n doubles in all.
constexpr int RS_G = RESIDUAL_SEG;
constexpr int RS_COLS = RHS_CHUNK + 1;
constexpr int RS_SR = RS_G * TB;
__device__ __forceinline__ int64_t rs_d_off(int n, int I) {
    return (int64_t)RS_COLS * ((int64_t)I * n - (int64_t)RS_SR * I * (I - 1) / 2);
}
__device__ __forceinline__ int64_t rs_t_off(int n, int nseg, int J) {
    return rs_d_off(n, nseg) + (int64_t)RS_COLS * RS_SR * ((int64_t)J * (J + 1) / 2);
}
static_assert(RHS_CHUNK == 16 && TB == 64, "one 16 x 16 MFMA tile per wave: 16 right-hand sides, 64-row blocks");

__global__ __launch_bounds__(256, 2)
void residual_part_kernel(int n, int nr, int nseg, const double* __restrict__ A, int64_t lda,
                          const double* __restrict__ X, int64_t ldx, double* __restrict__ part, int with_rsum)
{
    __shared__ double T[TB][TB + 1];           // T[k][r] = A(j0 + r, i0 + k)
    __shared__ double xi[TB][RHS_CHUNK];       // x of column block i
    __shared__ double xj[TB][RHS_CHUNK];       // x of row block j
    const int J = tri_row((int)blockIdx.x);
    const int I = (int)blockIdx.x - J * (J + 1) / 2;
    const int nblk = (n + TB - 1) / TB;
    const int jb0 = J * RS_G, jb1 = min(nblk, jb0 + RS_G);
    const int ib0 = I * RS_G, ib1 = min(nblk, ib0 + RS_G);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // part[D, I] (rows from I SR) and part[T, J] (rows from 0), column stride ldD / ldT
    const int64_t ldD = n - (int64_t)I * RS_SR, ldT = min((int64_t)n, (int64_t)(J + 1) * RS_SR);
    double* partD = part + rs_d_off(n, I) - (int64_t)I * RS_SR;
    double* partT = part + rs_t_off(n, nseg, J);
    constexpr int NE = TB * TB / 256;
    // wave wv owns rows 16 wv .. 16 wv + 15 of a row block (and columns
    // 16 wv .. of a column block) for all 16 right-hand sides; wave 0 also the
    // row sums (lane = row)
    d4_t yD[RS_G];
    double rD[RS_G];
#pragma unroll
    for (int u = 0; u < RS_G; ++u) {
        rD[u] = 0.0;
        yD[u] = zero_vec<d4_t>();
    }
    double tv[NE], xv[4];
    auto load = [&](int j, int i) {
        const int i0 = i * TB, j0 = j * TB;
        const int nbi = min(TB, n - i0), nbj = min(TB, n - j0);
#pragma unroll
        for (int u = 0; u < NE; ++u) {
            const int e = tid + 256 * u;
            const int a = e % TB, bcol = e / TB;    // row a of block j, column bcol of block i
            const bool in = a < nbj && bcol < nbi && (j != i || a >= bcol);
            const double v = A[in ? (int64_t)(j0 + a) + (int64_t)(i0 + bcol) * lda : 0];
            tv[u] = in ? v : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + 256 * u;
            const int a = e % TB, c = e / TB;
            xv[u] = (a < nbj && c < nr) ? X[(int64_t)(j0 + a) + (int64_t)c * ldx] : 0.0;
        }
    };
    for (int i = ib0; i < ib1; ++i) {
        const int i0 = i * TB, nbi = min(TB, n - i0);
        const int jst = J == I ? i : jb0;
        __syncthreads();   // the previous column block is done with xi
        for (int e = tid; e < TB * RHS_CHUNK; e += 256) {
            const int a = e % TB, c = e / TB;
            xi[a][c] = (a < nbi && c < nr) ? X[(int64_t)(i0 + a) + (int64_t)c * ldx] : 0.0;
        }
        d4_t yT = zero_vec<d4_t>();
        double rT = 0.0;
        if (jst < jb1) load(jst, i);
        for (int j = jst; j < jb1; ++j) {
#pragma unroll
            for (int u = 0; u < NE; ++u) {
                const int e = tid + 256 * u;
                T[e / TB][e % TB] = tv[u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = tid + 256 * u;
                xj[e % TB][e / TB] = xv[u];
            }
            if (j + 1 < jb1) load(j + 1, i);
            __syncthreads();
            if (j == i) {
                // the diagonal tile: fill the upper part from the lower
                for (int e = tid; e < TB * TB; e += 256) {
                    const int r = e % TB, k = e / TB;
                    if (r < k) T[k][r] = T[r][k];
                }
                __syncthreads();
            }
            const int jj = j - jb0;
            // row products of block j, rows 16 wv .. 16 wv + 15 of this wave, as
            // the transposed MFMA tile: D'[c][r] = sum_k x_i(k, c) A(r, k), lane
            // r + 16 (c % 4) holding column c = 4 g + lane / 16 in register g
            {
                d4_t acc = zero_vec<d4_t>();
#pragma unroll 4
                for (int k = 0; k < TB; k += 4) {
                    const int kk = k + (lane >> 4);
                    acc = mfma_f64(xi[kk][lane & 15], T[kk][16 * wv + (lane & 15)], acc);
                }
#pragma unroll
                for (int u = 0; u < RS_G; ++u)
                    if (u == jj) yD[u] += acc;
                if (with_rsum && wv == 0) {
                    double ra = 0.0;
                    for (int k = 0; k < TB; ++k) ra += fabs(T[k][lane]);
#pragma unroll
                    for (int u = 0; u < RS_G; ++u)
                        if (u == jj) rD[u] += ra;
                }
            }
            // column products of block i (j > i), columns 16 wv .. 16 wv + 15 of
            // the tile: D'[c][k] = sum_r x_j(r, c) A(r, k)
            if (j > i) {
                d4_t acc = zero_vec<d4_t>();
#pragma unroll 4
                for (int r = 0; r < TB; r += 4) {
                    const int rr = r + (lane >> 4);
                    acc = mfma_f64(xj[rr][lane & 15], T[16 * wv + (lane & 15)][rr], acc);
                }
                yT += acc;
                if (with_rsum && wv == 0) {
                    double ra = 0.0;
                    for (int r = 0; r < TB; ++r) ra += fabs(T[lane][r]);
                    rT += ra;
                }
            }
            __syncthreads();   // T and xj are free
        }
        // column products of block i from this row segment
        {
            const int k = 16 * wv + (lane & 15);
            if (k < nbi) {
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int c = 4 * g + (lane >> 4);
                    if (c < nr) partT[(int64_t)c * ldT + i0 + k] = yT[g];
                }
            }
            if (with_rsum && wv == 0 && lane < nbi) partT[(int64_t)RHS_CHUNK * ldT + i0 + lane] = rT;
        }
    }
    // row products of the row segment from this column segment
#pragma unroll
    for (int u = 0; u < RS_G; ++u) {
        const int j0 = (jb0 + u) * TB;
        if (jb0 + u < jb1) {
            const int r = j0 + 16 * wv + (lane & 15);
            if (r < n) {
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int c = 4 * g + (lane >> 4);
                    if (c < nr) partD[(int64_t)c * ldD + r] = yD[u][g];
                }
            }
            if (with_rsum && wv == 0 && j0 + lane < n) partD[(int64_t)RHS_CHUNK * ldD + j0 + lane] = rD[u];
        }
    }
}

// R = B - (sum over I <= K of part[D, I] + sum over J >= K of part[T, J]) for a
// row of segment K, in that order; rowsum likewise from the row-sum column.
__global__ void residual_reduce_kernel(int n, int nr, int nseg, const double* __restrict__ part,
                                       const double* __restrict__ B, int64_t ldb, double* __restrict__ R, int64_t ldr,
                                       double* __restrict__ rowsum)
{
    const int cc = blockIdx.y;
    const int col = cc < nr ? cc : RHS_CHUNK;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int K = i / RS_SR;
        double s = 0.0;
        for (int I = 0; I <= K; ++I)
            s += part[rs_d_off(n, I) + (int64_t)col * (n - (int64_t)I * RS_SR) + (i - (int64_t)I * RS_SR)];
        for (int Jx = K; Jx < nseg; ++Jx)
            s += part[rs_t_off(n, nseg, Jx) + (int64_t)col * min((int64_t)n, (int64_t)(Jx + 1) * RS_SR) + i];
        if (cc < nr) R[i + (int64_t)cc * ldr] = B[i + (int64_t)cc * ldb] - s;
        else rowsum[i] = s;
    }
}

template <typename S>
__global__ void axpy_kernel(int n, const S* __restrict__ D, int64_t ldd, double* __restrict__ X, int64_t ldx) {
    const int j = blockIdx.y;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        X[i + (int64_t)j * ldx] += (double)D[i + (int64_t)j * ldd];
}

// out[0] = max|D|, out[1] = max|X|, out[2] = max_i rowsum[i] (if rowsum),
// out[3 + 3c + {0,1,2}] = max|R[:,c]|, max|X[:,c]|, max|B[:,c]| (NaN entries
// count as 0).  Workgroup (x, y) takes rows [x NR_ROWS, (x+1) NR_ROWS) of column
// y (y = nrhs: the row sums) and folds its maxima into out with atomic maxima of
// the bit patterns, which order like the values for non-negative doubles; out
// must hold zeros first.  A maximum does not depend on the order of its terms.
constexpr int NR_ROWS = 2048;

__device__ __forceinline__ double abs_or_zero(double v) {
    const double a = fabs(v);
    return a == a ? a : 0.0;
}
__device__ __forceinline__ double block_max(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    const double r = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    return r;
}
__device__ __forceinline__ void atomic_max_nonneg(double* p, double v) {
    atomicMax(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v));
}

__global__ __launch_bounds__(256)
void norms_kernel(int n, int nrhs, const double* rowsum, const double* X, int64_t ldx, const double* D,
                  int64_t ldd, const double* R, int64_t ldr, const double* B, int64_t ldb, double* out)
{
    __shared__ double red[4];
    const int c = blockIdx.y;
    const int i0 = blockIdx.x * NR_ROWS, i1 = min(n, i0 + NR_ROWS);
    if (c == nrhs) {
        double ma = 0.0;
        if (rowsum)
            for (int i = i0 + threadIdx.x; i < i1; i += 256) ma = fmax(ma, abs_or_zero(rowsum[i]));
        ma = block_max(ma, red);
        if (threadIdx.x == 0) atomic_max_nonneg(out + 2, ma);
        return;
    }
    double vd = 0.0, vr = 0.0, vx = 0.0, vb = 0.0;
    for (int i = i0 + threadIdx.x; i < i1; i += 256) {
        if (D) vd = fmax(vd, abs_or_zero(D[i + (int64_t)c * ldd]));
        if (R) vr = fmax(vr, abs_or_zero(R[i + (int64_t)c * ldr]));
        vx = fmax(vx, abs_or_zero(X[i + (int64_t)c * ldx]));
        if (B) vb = fmax(vb, abs_or_zero(B[i + (int64_t)c * ldb]));
    }
    vd = block_max(vd, red);
    vr = block_max(vr, red);
    vx = block_max(vx, red);
    vb = block_max(vb, red);
    if (threadIdx.x == 0) {
        atomic_max_nonneg(out + 0, vd);
        atomic_max_nonneg(out + 1, vx);
        atomic_max_nonneg(out + 3 + 3 * c, vr);
        atomic_max_nonneg(out + 4 + 3 * c, vx);
        atomic_max_nonneg(out + 5 + 3 * c, vb);
    }
}

// Widen / narrow the lower triangle of a w x w block between binary32 storage
// and a binary64 work copy.
template <typename S>
__global__ void widen_lower_kernel(int w, const S* __restrict__ a, int64_t lda, double* __restrict__ d, int64_t ldd) {
    const int j = blockIdx.y;
    for (int i = j + blockIdx.x * blockDim.x + threadIdx.x; i < w; i += gridDim.x * blockDim.x)
        d[i + (int64_t)j * ldd] = (double)a[i + (int64_t)j * lda];
}
template <typename S>
__global__ void narrow_lower_kernel(int w, const double* __restrict__ d, int64_t ldd, S* __restrict__ a, int64_t lda) {
    const int j = blockIdx.y;
    for (int i = j + blockIdx.x * blockDim.x + threadIdx.x; i < w; i += gridDim.x * blockDim.x)
        a[i + (int64_t)j * lda] = (S)d[i + (int64_t)j * ldd];
}
template <typename S>
__global__ void widen_kernel(int n, const S* __restrict__ D, int64_t ldd, double* __restrict__ X, int64_t ldx) {
    const int j = blockIdx.y;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        X[i + (int64_t)j * ldx] = (double)D[i + (int64_t)j * ldd];
}
__global__ void zero2_kernel(double* p) { if (threadIdx.x < 2) p[threadIdx.x] = 0.0; }

// X += D (binary64), and out[0] = max|D|, out[1] = max|X| over all entries.
// Non-negative binary64 values order like their bit patterns, so the maxima are
// exact and independent of the order in which workgroups arrive.
template <typename S>
__global__ __launch_bounds__(256)
void axpy_max_kernel(int n, const S* __restrict__ D, int64_t ldd, double* __restrict__ X, int64_t ldx,
                     double* __restrict__ out, int os) {
    __shared__ unsigned long long md[256], mx[256];
    const int j = blockIdx.y;
    unsigned long long a = 0, b = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double d = (double)D[i + (int64_t)j * ldd];
        const double x = X[i + (int64_t)j * ldx] + d;
        X[i + (int64_t)j * ldx] = x;
        const unsigned long long bd = (unsigned long long)__double_as_longlong(fabs(d));
        const unsigned long long bx = (unsigned long long)__double_as_longlong(fabs(x));
        a = a > bd ? a : bd;
        b = b > bx ? b : bx;
    }
    md[threadIdx.x] = a;
    mx[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            md[threadIdx.x] = md[threadIdx.x] > md[threadIdx.x + s] ? md[threadIdx.x] : md[threadIdx.x + s];
            mx[threadIdx.x] = mx[threadIdx.x] > mx[threadIdx.x + s] ? mx[threadIdx.x] : mx[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax(reinterpret_cast<unsigned long long*>(&out[j * os]), md[0]);
        atomicMax(reinterpret_cast<unsigned long long*>(&out[j * os + 1]), mx[0]);
    }
}

// ---------------------------------------------------------------- GMRES pieces
// Batched over the columns of a multi-column solve: column c (blockIdx.y) has
// its own Krylov basis V + c*vs (n x k, column-major, ld = ldv) and vectors at
// w + c*ws.  Sums are taken in a fixed order (per-workgroup partials over row
// chunks, then the partials in workgroup order), so results do not depend on
// scheduling.
constexpr int KV_MAX = 32;          // basis vectors one launch handles
constexpr int KV_WG = 256;          // threads per workgroup
constexpr int KV_ROWS = 2048;       // rows per workgroup

// part[c][g * KV_MAX + i] = sum over the rows of workgroup g of V_c[:, i] w_c.
__global__ __launch_bounds__(KV_WG)
void multidot_part_kernel(int n, int k, const double* __restrict__ V, int64_t ldv, int64_t vs,
                          const double* __restrict__ w, int64_t ws, double* __restrict__ part, int64_t ps) {
    __shared__ double red[KV_WG];
    const int c = blockIdx.y;
    V += c * vs;
    w += c * ws;
    part += c * ps;
    const int r0 = blockIdx.x * KV_ROWS;
    const int r1 = min(n, r0 + KV_ROWS);
    for (int i = 0; i < k; ++i) {
        double acc = 0.0;
        for (int r = r0 + threadIdx.x; r < r1; r += KV_WG) acc += V[r + (int64_t)i * ldv] * w[r];
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int s = KV_WG / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[blockIdx.x * KV_MAX + i] = red[0];
        __syncthreads();
    }
}

// out[c][i] = sum_g part[c][g * KV_MAX + i] (g ascending), i < k.
__global__ void multidot_reduce_kernel(int k, int ngroups, const double* __restrict__ part, int64_t ps,
                                       double* __restrict__ out, int64_t os) {
    const int i = threadIdx.x, c = blockIdx.x;
    if (i >= k) return;
    double s = 0.0;
    for (int g = 0; g < ngroups; ++g) s += part[c * ps + g * KV_MAX + i];
    out[c * os + i] = s;
}

// w_c += alpha * V_c h_c (h_c: k values on the device).
__global__ void gemv_add_kernel(int n, int k, const double* __restrict__ V, int64_t ldv, int64_t vs,
                                const double* __restrict__ h, int64_t hs_, double alpha, double* __restrict__ w,
                                int64_t ws) {
    __shared__ double hs[KV_MAX];
    const int c = blockIdx.y;
    V += c * vs;
    w += c * ws;
    if (threadIdx.x < k) hs[threadIdx.x] = h[c * hs_ + threadIdx.x];
    __syncthreads();
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int i = 0; i < k; ++i) s += V[r + (int64_t)i * ldv] * hs[i];
        w[r] += alpha * s;
    }
}

// y_c = x_c / sqrt(sq_c) where sq_c > 0 (a squared norm), else unchanged; y may alias x.
__global__ void normalize_kernel(int n, const double* x, int64_t xs, const double* __restrict__ sq, int64_t ss,
                                 double* y, int64_t ys) {
    const int c = blockIdx.y;
    const double q = sq[c * ss];
    if (!(q > 0.0)) return;
    const double inv = 1.0 / sqrt(q);
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
        y[c * ys + r] = x[c * xs + r] * inv;
}

__global__ void fill_double_kernel(int n, double* __restrict__ y, double v) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) y[r] = v;
}

// y_c = -x_c (y may alias x).
__global__ void negate_kernel(int n, const double* x, int64_t xs, double* y, int64_t ys) {
    const int c = blockIdx.y;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
        y[c * ys + r] = -x[c * xs + r];
}

}  // namespace

template <typename S>
hipError_t launch_copy_lower_from_f64(int n, const double* A, int64_t lda, S* W, int64_t ldw, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((copy_lower_kernel<S>), dim3((n + 255) / 256, n), dim3(256), 0, st, n, A, lda, W, ldw);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_convert_from_f64(int n, int nrhs, const double* B, int64_t ldb, S* X, int64_t ldx, hipStream_t st) {
    if (n <= 0 || nrhs <= 0) return hipSuccess;
    hipLaunchKernelGGL((convert_kernel<S>), dim3((n + 255) / 256, nrhs), dim3(256), 0, st, n, B, ldb, X, ldx);
    return hipGetLastError();
}

template <typename S>
hipError_t trisolve_impl(int n, int nrhs, const S* L, int64_t ldl, S* X, int64_t ldx, const TriWs<S>& w,
                         bool make_fac, hipStream_t st) {
    if (n <= 0 || nrhs <= 0) return hipSuccess;
    const int nblk = trisolve_nblk(n);
    if (make_fac) {
        hipLaunchKernelGGL((inv_diag_kernel<S>), dim3(nblk), dim3(64), 0, st, n, L, ldl, w.fac);
        if (nblk > 1)
            hipLaunchKernelGGL((near_tiles_kernel<S>), dim3(nblk, TRI_F, 2), dim3(256), 0, st, n, L, ldl, w.fac);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const size_t all = trisolve_pub_elems(n);
    const size_t sweep = all / 2;
    const int rgrid = (int)std::min<size_t>(1024, (all + 255) / 256);
    for (int c0 = 0; c0 < nrhs; c0 += RC) {
        const int nr = std::min(RC, nrhs - c0);
        S* Xc = X + (int64_t)c0 * ldx;
        hipLaunchKernelGGL((pub_reset_kernel<S>), dim3(rgrid), dim3(256), 0, st, w.pub, all, w.ctl + 1);
        hipError_t e = launch_sweep<S, false>(n, nr, L, ldl, w.fac, Xc, ldx, w.pub, w.ctl, w.ctl + 1, st);
        if (e == hipSuccess)
            e = launch_sweep<S, true>(n, nr, L, ldl, w.fac, Xc, ldx, w.pub + sweep, w.ctl, w.ctl + 1 + TRI_GROUPS, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template hipError_t trisolve_impl<double>(int, int, const double*, int64_t, double*, int64_t, const TriWs<double>&,
                                          bool, hipStream_t);
template hipError_t trisolve_impl<float>(int, int, const float*, int64_t, float*, int64_t, const TriWs<float>&, bool,
                                         hipStream_t);

hipError_t launch_residual_f64(int n, int nrhs, const double* A, int64_t lda, const double* X, int64_t ldx,
                               const double* B, int64_t ldb, double* R, int64_t ldr, double* rowsum, double* part,
                               hipStream_t st) {
    if (n <= 0 || nrhs <= 0) return hipSuccess;
    const int nseg = residual_segments(n);
    const int nwg = nseg * (nseg + 1) / 2;
    for (int c0 = 0; c0 < nrhs; c0 += RHS_CHUNK) {
        const int nr = std::min(RHS_CHUNK, nrhs - c0);
        const bool rs = c0 == 0 && rowsum;
        hipLaunchKernelGGL(residual_part_kernel, dim3(nwg), dim3(256), 0, st, n, nr, nseg, A, lda,
                           X + (int64_t)c0 * ldx, ldx, part, rs ? 1 : 0);
        hipLaunchKernelGGL(residual_reduce_kernel, dim3(std::min(1024, (n + 255) / 256), nr + (rs ? 1 : 0)), dim3(256),
                           0, st, n, nr, nseg, part, B + (int64_t)c0 * ldb, ldb, R + (int64_t)c0 * ldr, ldr,
                           rs ? rowsum : nullptr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename S>
hipError_t launch_axpy_update(int n, int nrhs, const S* D, int64_t ldd, double* X, int64_t ldx, hipStream_t st) {
    if (n <= 0 || nrhs <= 0) return hipSuccess;
    hipLaunchKernelGGL((axpy_kernel<S>), dim3((n + 255) / 256, nrhs), dim3(256), 0, st, n, D, ldd, X, ldx);
    return hipGetLastError();
}

hipError_t launch_norms(int n, int nrhs, const double* rowsum, const double* X, int64_t ldx, const double* D,
                        int64_t ldd, const double* R, int64_t ldr, const double* B, int64_t ldb, double* out,
                        hipStream_t st) {
    const int nout = 3 + 3 * nrhs;
    hipLaunchKernelGGL(fill_double_kernel, dim3((nout + 255) / 256), dim3(256), 0, st, nout, out, 0.0);
    if (n <= 0 || nrhs <= 0) return hipGetLastError();
    hipLaunchKernelGGL(norms_kernel, dim3((n + NR_ROWS - 1) / NR_ROWS, nrhs + 1), dim3(256), 0, st, n, nrhs, rowsum,
                       X, ldx, D, ldd, R, ldr, B, ldb, out);
    return hipGetLastError();
}

template hipError_t launch_copy_lower_from_f64<double>(int, const double*, int64_t, double*, int64_t, hipStream_t);
template hipError_t launch_copy_lower_from_f64<float>(int, const double*, int64_t, float*, int64_t, hipStream_t);
template hipError_t launch_convert_from_f64<double>(int, int, const double*, int64_t, double*, int64_t, hipStream_t);
template hipError_t launch_convert_from_f64<float>(int, int, const double*, int64_t, float*, int64_t, hipStream_t);
template hipError_t launch_axpy_update<double>(int, int, const double*, int64_t, double*, int64_t, hipStream_t);
template hipError_t launch_axpy_update<float>(int, int, const float*, int64_t, double*, int64_t, hipStream_t);

template <typename S>
hipError_t launch_widen_lower(int w, const S* a, int64_t lda, double* d, int64_t ldd, hipStream_t st) {
    if (w <= 0) return hipSuccess;
    hipLaunchKernelGGL((widen_lower_kernel<S>), dim3((w + 255) / 256, w), dim3(256), 0, st, w, a, lda, d, ldd);
    return hipGetLastError();
}
template <typename S>
hipError_t launch_narrow_lower(int w, const double* d, int64_t ldd, S* a, int64_t lda, hipStream_t st) {
    if (w <= 0) return hipSuccess;
    hipLaunchKernelGGL((narrow_lower_kernel<S>), dim3((w + 255) / 256, w), dim3(256), 0, st, w, d, ldd, a, lda);
    return hipGetLastError();
}
template <typename S>
hipError_t launch_widen(int n, int nrhs, const S* D, int64_t ldd, double* X, int64_t ldx, hipStream_t st) {
    if (n <= 0 || nrhs <= 0) return hipSuccess;
    hipLaunchKernelGGL((widen_kernel<S>), dim3((n + 255) / 256, nrhs), dim3(256), 0, st, n, D, ldd, X, ldx);
    return hipGetLastError();
}
template <typename S>
hipError_t launch_axpy_max(int n, int nrhs, const S* D, int64_t ldd, double* X, int64_t ldx, double* out,
                           hipStream_t st) {
    hipLaunchKernelGGL(zero2_kernel, dim3(1), dim3(64), 0, st, out);
    if (n <= 0 || nrhs <= 0) return hipGetLastError();
    const int gx = std::min((n + 255) / 256, 1024);
    hipLaunchKernelGGL((axpy_max_kernel<S>), dim3(gx, nrhs), dim3(256), 0, st, n, D, ldd, X, ldx, out, 0);
    return hipGetLastError();
}

// X += D, out[2j] = max|D_j|, out[2j + 1] = max|X_j| per column.
template <typename S>
hipError_t launch_axpy_max_cols(int n, int nrhs, const S* D, int64_t ldd, double* X, int64_t ldx, double* out,
                                hipStream_t st) {
    if (nrhs <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_double_kernel, dim3(1), dim3(256), 0, st, 2 * nrhs, out, 0.0);
    if (n <= 0) return hipGetLastError();
    const int gx = std::min((n + 255) / 256, 1024);
    hipLaunchKernelGGL((axpy_max_kernel<S>), dim3(gx, nrhs), dim3(256), 0, st, n, D, ldd, X, ldx, out, 2);
    return hipGetLastError();
}
template hipError_t launch_axpy_max_cols<double>(int, int, const double*, int64_t, double*, int64_t, double*,
                                                 hipStream_t);
template hipError_t launch_widen_lower<float>(int, const float*, int64_t, double*, int64_t, hipStream_t);
template hipError_t launch_narrow_lower<float>(int, const double*, int64_t, float*, int64_t, hipStream_t);
template hipError_t launch_widen<double>(int, int, const double*, int64_t, double*, int64_t, hipStream_t);
template hipError_t launch_widen<float>(int, int, const float*, int64_t, double*, int64_t, hipStream_t);
template hipError_t launch_axpy_max<double>(int, int, const double*, int64_t, double*, int64_t, double*, hipStream_t);
template hipError_t launch_axpy_max<float>(int, int, const float*, int64_t, double*, int64_t, double*, hipStream_t);

size_t multidot_part_doubles(int n) { return (size_t)((n + KV_ROWS - 1) / KV_ROWS) * KV_MAX; }

hipError_t launch_multidot(int n, int nc, int k, const double* V, int64_t ldv, int64_t vs, const double* w, int64_t ws,
                           double* part, double* out, int64_t os, hipStream_t st) {
    if (k <= 0 || nc <= 0) return hipSuccess;
    if (k > KV_MAX) return hipErrorInvalidValue;
    const int ng = (n + KV_ROWS - 1) / KV_ROWS;
    const int64_t ps = (int64_t)multidot_part_doubles(n);
    if (ng > 0)
        hipLaunchKernelGGL(multidot_part_kernel, dim3(ng, nc), dim3(KV_WG), 0, st, n, k, V, ldv, vs, w, ws, part, ps);
    hipLaunchKernelGGL(multidot_reduce_kernel, dim3(nc), dim3(KV_MAX), 0, st, k, ng, part, ps, out, os);
    return hipGetLastError();
}

hipError_t launch_gemv_add(int n, int nc, int k, const double* V, int64_t ldv, int64_t vs, const double* h,
                           int64_t hs, double alpha, double* w, int64_t ws, hipStream_t st) {
    if (k <= 0 || n <= 0 || nc <= 0) return hipSuccess;
    if (k > KV_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gemv_add_kernel, dim3(std::min(1024, (n + 255) / 256), nc), dim3(256), 0, st, n, k, V, ldv, vs,
                       h, hs, alpha, w, ws);
    return hipGetLastError();
}

hipError_t launch_normalize(int n, int nc, const double* x, int64_t xs, const double* sq, int64_t ss, double* y,
                            int64_t ys, hipStream_t st) {
    if (n <= 0 || nc <= 0) return hipSuccess;
    hipLaunchKernelGGL(normalize_kernel, dim3(std::min(1024, (n + 255) / 256), nc), dim3(256), 0, st, n, x, xs, sq, ss,
                       y, ys);
    return hipGetLastError();
}

hipError_t launch_fill_double(int n, double* y, double v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_double_kernel, dim3(std::min(1024, (n + 255) / 256)), dim3(256), 0, st, n, y, v);
    return hipGetLastError();
}

hipError_t launch_negate(int n, int nc, const double* x, int64_t xs, double* y, int64_t ys, hipStream_t st) {
    if (n <= 0 || nc <= 0) return hipSuccess;
    hipLaunchKernelGGL(negate_kernel, dim3(std::min(1024, (n + 255) / 256), nc), dim3(256), 0, st, n, x, xs, y, ys);
    return hipGetLastError();
}

}  // namespace ff
