// solve.hip -- solves with a computed factor and the binary64 refinement pieces.
//
// Solving A x = b from A = L L^T (Introduction of arXiv 1812.02056) needs two
// triangular solves.  Refinement (binary64 residual r = b - A x, correction
// from the low-precision factor, x += d) is how the mixed-precision factor wins
// back binary64 accuracy.
//
// Triangular solves: the n rows are cut into 64-row blocks, and each block gets
// TP workgroups that take tickets from an atomic counter in block order.  The
// first TP - 1 fold disjoint sets of already-solved blocks into partial sums as
// those blocks' flags appear (streaming their tiles of L, the next tile loaded
// while the current one is applied); the last one folds the newest solved block,
// adds the partial sums in a fixed order, applies the precomputed inverse of the
// 64 x 64 diagonal block and publishes the block.  Every wait is on a workgroup
// with a smaller ticket, so every wait ends; each is also bounded: past the spin
// limit the workgroup records an error and exits.
//
// The binary64 residual R = B - A X reads tril(A) once per use of symmetry:
// workgroups own (row block, chunk of column blocks) pairs and write partial
// products, which a second kernel adds in a fixed order.
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace ff {

namespace {

constexpr int TB = 64;          // row block of the triangular solves
constexpr int RHS_CHUNK = 16;   // right-hand sides per launch
constexpr int TP = TRISOLVE_TP; // workgroups per row block of a triangular solve
constexpr int RCB = RESIDUAL_CB;// column blocks per residual workgroup
constexpr int SPIN_LIMIT = 1 << 24;

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

// Inverse of the 64 x 64 lower-triangular diagonal blocks of L, computed in
// binary64 by column-wise forward substitution, stored in S (block b at
// Linv + b*64*64, column-major, ld 64; entries above the diagonal are zero).
template <typename S>
__global__ __launch_bounds__(64)
void inv_diag_kernel(int n, const S* __restrict__ L, int64_t ldl, S* __restrict__ Linv) {
    __shared__ double x[TB][TB + 1];    // x[i][c]
    __shared__ double l[TB][TB + 1];    // l[i][k]
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
    for (int i = 0; i < TB; ++i) Linv[(int64_t)b * TB * TB + i + (int64_t)c * TB] = (S)x[i][c];
}

// Spin on a relaxed load (an acquire load would invalidate the caches on every
// iteration); callers issue one acquire fence after the flag is seen.
__device__ __forceinline__ bool wait_flag(const int* f) {
    int spins = 0;
    while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
        if (++spins > SPIN_LIMIT) return false;
        __builtin_amdgcn_s_sleep(2);
    }
    return true;
}

// Make this workgroup's global writes visible at agent scope, then set *f.  The
// barrier orders every wave's writes before thread 0's release fence (which is
// cumulative over them), so one fence, one L2 write-back, serves the
// workgroup; the flag store after it may then be relaxed.
__device__ __forceinline__ void publish(int* f) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Row r of the 64 x 64 LDS tile t (column r of it for TRANS) times the columns
// c = g + 4q of xv.  With nr <= 4 a thread has one live column (q = 0), whose
// dependent chain is on the critical path of a block: it is summed as four
// interleaved partial sums added in a fixed order.  With more columns each is a
// plain sum over k, the columns giving the thread independent chains.  (So a
// column's rounding depends on whether nr <= 4; results are deterministic for
// a given nr.)
template <bool TRANS, typename S>
__device__ __forceinline__ void dots64(const S (&t)[TB][TB + 1], const S (&xv)[TB][RHS_CHUNK], int r, int g, int nr,
                                       S (&out)[RHS_CHUNK / 4]) {
    constexpr int NQ = RHS_CHUNK / 4;
    if (nr <= 4) {
        S s0 = S(0), s1 = S(0), s2 = S(0), s3 = S(0);
#pragma unroll 4
        for (int k = 0; k < TB; k += 4) {
            if (!TRANS) {
                s0 += t[r][k] * xv[k][g];
                s1 += t[r][k + 1] * xv[k + 1][g];
                s2 += t[r][k + 2] * xv[k + 2][g];
                s3 += t[r][k + 3] * xv[k + 3][g];
            } else {
                s0 += t[k][r] * xv[k][g];
                s1 += t[k + 1][r] * xv[k + 1][g];
                s2 += t[k + 2][r] * xv[k + 2][g];
                s3 += t[k + 3][r] * xv[k + 3][g];
            }
        }
        out[0] = (s0 + s1) + (s2 + s3);
#pragma unroll
        for (int q = 1; q < NQ; ++q) out[q] = S(0);
        return;
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int c = g + 4 * q;
        S sum = S(0);
        if (!TRANS) { for (int k = 0; k < TB; ++k) sum += t[r][k] * xv[k][c]; }
        else        { for (int k = 0; k < TB; ++k) sum += t[k][r] * xv[k][c]; }
        out[q] = sum;
    }
}

// Forward (TRANS = false: L y = b) or backward (TRANS = true: L^T x = y)
// substitution on nr <= 16 columns of X in place.  fl: [0] ticket, [1] error
// word, [2, 2 + nblk) block flags, then nblk * TP partial flags; all start at
// zero.  parts: (TP - 1) partial sums of 64 x 16 per block.
template <typename S, bool TRANS>
__global__ __launch_bounds__(256)
void trisolve_kernel(int n, int nr, const S* __restrict__ L, int64_t ldl, const S* __restrict__ Linv,
                     S* X, int64_t ldx, int* fl, S* __restrict__ parts)
{
    __shared__ S tile[TB][TB + 1];
    __shared__ S xv[TB][RHS_CHUNK];
    __shared__ int sh_ticket, bad;
    const int nblk = (n + TB - 1) / TB;
    int* const err = fl + 1;
    int* const bflag = fl + 2;
    int* const pflag = fl + 2 + nblk;
    const int tid = threadIdx.x;
    if (tid == 0) {
        sh_ticket = atomicAdd(&fl[0], 1);
        bad = 0;
    }
    __syncthreads();
    const int jj = sh_ticket / TP, p = sh_ticket % TP;   // jj blocks are solved before this one
    const int j = TRANS ? (nblk - 1 - jj) : jj;
    const int r0 = j * TB;
    const int nbr = min(TB, n - r0);
    const int r = tid % TB, g = tid / TB;
    const bool fin = p == TP - 1;
    S acc[RHS_CHUNK / 4];
#pragma unroll
    for (int q = 0; q < RHS_CHUNK / 4; ++q) {
        const int c = g + 4 * q;
        acc[q] = (fin && r < nbr && c < nr) ? X[(int64_t)(r0 + r) + (int64_t)c * ldx] : S(0);
    }
    // Blocks folded here, by distance d from block j: the finisher takes d = 1,
    // workgroup p < TP - 1 takes d = p + 2, p + 2 + (TP - 1), ... and walks them
    // oldest first, so it works through the blocks already solved while the newer
    // ones are still being solved.
    const int dlo = fin ? 1 : p + 2;
    const int d0 = fin ? 1 : (jj >= dlo ? dlo + (jj - dlo) / (TP - 1) * (TP - 1) : 0);
    const int dstep = fin ? -(jj + 1) : -(TP - 1);
    constexpr int NE = TB * TB / 256;
    S tv[NE];
    auto load_tile = [&](int d) {
        const int i = TRANS ? j + d : j - d;
        const int i0 = i * TB, nbi = min(TB, n - i0);
#pragma unroll
        for (int u = 0; u < NE; ++u) {
            const int e = tid + 256 * u;
            const int a = e % TB, b = e / TB;    // a: row within the tile (contiguous), b: column
            const bool in = !TRANS ? (a < nbr && b < nbi) : (a < nbi && b < nbr);
            const int64_t off = !TRANS ? (int64_t)(r0 + a) + (int64_t)(i0 + b) * ldl
                                       : (int64_t)(i0 + a) + (int64_t)(r0 + b) * ldl;
            const S v = L[in ? off : 0];
            tv[u] = in ? v : S(0);
        }
    };
    S* const mine = parts + ((int64_t)j * (TP - 1)) * TB * RHS_CHUNK;
    S lv[NE];                                    // the finisher's inverse diagonal block, loaded early
    if (fin) {
        // partial sums first (their blocks were solved earlier), all flags at once
        if (tid < TP - 1 && !wait_flag(&pflag[j * TP + tid])) bad = 1;
        if (tid < 64) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __syncthreads();
        if (bad) {
            if (tid == 0) atomicExch(err, 1);
            return;
        }
#pragma unroll
        for (int pp = 0; pp < TP - 1; ++pp)
#pragma unroll
            for (int q = 0; q < RHS_CHUNK / 4; ++q) acc[q] += mine[(int64_t)pp * TB * RHS_CHUNK + r * RHS_CHUNK + g + 4 * q];
#pragma unroll
        for (int u = 0; u < NE; ++u) lv[u] = Linv[(int64_t)j * TB * TB + tid + 256 * u];
    }
    if (d0 >= dlo && d0 <= jj) load_tile(d0);
    for (int d = d0; d >= dlo && d <= jj; d += dstep) {
        const int i = TRANS ? j + d : j - d;
        const int i0 = i * TB, nbi = min(TB, n - i0);
#pragma unroll
        for (int u = 0; u < NE; ++u) {
            const int e = tid + 256 * u;
            tile[e % TB][e / TB] = tv[u];
        }
        if (d + dstep >= dlo) load_tile(d + dstep);      // next tile in flight during this one
        // one wave takes the acquire (the invalidation acts for the whole CU)
        if (tid == 0 && !wait_flag(&bflag[i])) bad = 1;
        if (tid < 64) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __syncthreads();
        if (bad) {
            if (tid == 0) atomicExch(err, 1);
            return;
        }
        for (int e = tid; e < TB * RHS_CHUNK; e += 256) {
            const int a = e % TB, c = e / TB;
            xv[a][c] = (a < nbi && c < nr) ? X[(int64_t)(i0 + a) + (int64_t)c * ldx] : S(0);
        }
        __syncthreads();
        {
            S sum[RHS_CHUNK / 4];
            dots64<TRANS>(tile, xv, r, g, nr, sum);
#pragma unroll
            for (int q = 0; q < RHS_CHUNK / 4; ++q)
                if (g + 4 * q < nr) acc[q] -= sum[q];
        }
        __syncthreads();
    }
    if (!fin) {
#pragma unroll
        for (int q = 0; q < RHS_CHUNK / 4; ++q) mine[(int64_t)p * TB * RHS_CHUNK + r * RHS_CHUNK + g + 4 * q] = acc[q];
        publish(&pflag[j * TP + p]);
        return;
    }
    // apply the inverse diagonal block (column-major, ld 64)
#pragma unroll
    for (int u = 0; u < NE; ++u) {
        const int e = tid + 256 * u;
        tile[e % TB][e / TB] = lv[u];
    }
#pragma unroll
    for (int q = 0; q < RHS_CHUNK / 4; ++q) xv[r][g + 4 * q] = acc[q];
    __syncthreads();
    {
        S sum[RHS_CHUNK / 4];
        dots64<TRANS>(tile, xv, r, g, nr, sum);
#pragma unroll
        for (int q = 0; q < RHS_CHUNK / 4; ++q) {
            const int c = g + 4 * q;
            if (c < nr && r < nbr) X[(int64_t)(r0 + r) + (int64_t)c * ldx] = sum[q];
        }
    }
    publish(&bflag[j]);
}

__global__ void fill_int_kernel(int* p, int count, int v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = v;
}

// Partial products of R = B - A X in binary64 with A symmetric, only tril(A)
// read: workgroup (j, c) takes the 64-row block j against column blocks
// i in [c*RCB, (c+1)*RCB): A[j-block, i-block] for i < j, A[i-block, j-block]^T
// for i > j, the symmetric diagonal block for i = j.  part[c] receives A X of
// those columns (n x nr, ld n) and, when rsum is non-null, the absolute row sums.
__global__ __launch_bounds__(256)
void residual_part_kernel(int n, int nr, const double* __restrict__ A, int64_t lda, const double* __restrict__ X,
                          int64_t ldx, double* __restrict__ part, int64_t pstride, double* __restrict__ rsum)
{
    __shared__ double tile[TB][TB + 1];
    __shared__ double xv[TB][RHS_CHUNK];
    const int j = blockIdx.x, c = blockIdx.y;
    const int r0 = j * TB;
    const int nbr = min(TB, n - r0);
    const int nblk = (n + TB - 1) / TB;
    const int tid = threadIdx.x, r = tid % TB, g = tid / TB;
    const int ib = c * RCB, ie = min(nblk, ib + RCB);
    double acc[RHS_CHUNK / 4];
    double asum = 0.0;
#pragma unroll
    for (int q = 0; q < RHS_CHUNK / 4; ++q) acc[q] = 0.0;
    constexpr int NE = TB * TB / 256;
    double tv[NE];
    auto load_tile = [&](int i) {
        const int i0 = i * TB, nbi = min(TB, n - i0);
#pragma unroll
        for (int u = 0; u < NE; ++u) {
            const int e = tid + 256 * u;
            const int a = e % TB, b = e / TB;
            bool in;
            int64_t off;
            if (i < j) { in = a < nbr && b < nbi; off = (int64_t)(r0 + a) + (int64_t)(i0 + b) * lda; }
            else if (i > j) { in = a < nbi && b < nbr; off = (int64_t)(i0 + a) + (int64_t)(r0 + b) * lda; }
            else { in = a < nbr && b < nbr && a >= b; off = (int64_t)(r0 + a) + (int64_t)(r0 + b) * lda; }
            const double v = A[in ? off : 0];
            tv[u] = in ? v : 0.0;
        }
    };
    if (ib < ie) load_tile(ib);
    for (int i = ib; i < ie; ++i) {
        const int i0 = i * TB, nbi = min(TB, n - i0);
#pragma unroll
        for (int u = 0; u < NE; ++u) {
            const int e = tid + 256 * u;
            tile[e % TB][e / TB] = tv[u];
        }
        for (int e = tid; e < TB * RHS_CHUNK; e += 256) {
            const int a = e % TB, cc = e / TB;
            xv[a][cc] = (a < nbi && cc < nr) ? X[(int64_t)(i0 + a) + (int64_t)cc * ldx] : 0.0;
        }
        if (i + 1 < ie) load_tile(i + 1);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < RHS_CHUNK / 4; ++q) {
            const int cc = g + 4 * q;
            if (cc < nr) {
                double sum = 0.0;
                if (i < j) { for (int k = 0; k < TB; ++k) sum += tile[r][k] * xv[k][cc]; }
                else if (i > j) { for (int k = 0; k < TB; ++k) sum += tile[k][r] * xv[k][cc]; }
                else { for (int k = 0; k < TB; ++k) sum += (r >= k ? tile[r][k] : tile[k][r]) * xv[k][cc]; }
                acc[q] += sum;
            }
        }
        if (rsum && g == 0) {
            double sum = 0.0;
            if (i < j) { for (int k = 0; k < TB; ++k) sum += fabs(tile[r][k]); }
            else if (i > j) { for (int k = 0; k < TB; ++k) sum += fabs(tile[k][r]); }
            else { for (int k = 0; k < TB; ++k) sum += fabs(r >= k ? tile[r][k] : tile[k][r]); }
            asum += sum;
        }
        __syncthreads();
    }
    double* pc = part + (int64_t)c * pstride;
#pragma unroll
    for (int q = 0; q < RHS_CHUNK / 4; ++q) {
        const int cc = g + 4 * q;
        if (cc < nr && r < nbr) pc[(int64_t)(r0 + r) + (int64_t)cc * n] = acc[q];
    }
    if (rsum && g == 0 && r < nbr) rsum[(int64_t)c * n + r0 + r] = asum;
}

// R = B - sum_c part[c] (c ascending), rowsum = sum_c rsum[c].
__global__ void residual_reduce_kernel(int n, int nr, int nch, const double* __restrict__ part, int64_t pstride,
                                       const double* __restrict__ B, int64_t ldb, double* __restrict__ R, int64_t ldr,
                                       const double* __restrict__ rsum, double* __restrict__ rowsum)
{
    const int cc = blockIdx.y;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < nch; ++c) s += part[(int64_t)c * pstride + i + (int64_t)cc * n];
        R[i + (int64_t)cc * ldr] = B[i + (int64_t)cc * ldb] - s;
        if (rowsum && cc == 0) {
            double t = 0.0;
            for (int c = 0; c < nch; ++c) t += rsum[(int64_t)c * n + i];
            rowsum[i] = t;
        }
    }
}

template <typename S>
__global__ void axpy_kernel(int n, const S* __restrict__ D, int64_t ldd, double* __restrict__ X, int64_t ldx) {
    const int j = blockIdx.y;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        X[i + (int64_t)j * ldx] += (double)D[i + (int64_t)j * ldd];
}

// out[0] = max|D|, out[1] = max|X|, out[2] = max_i rowsum[i] (if rowsum),
// out[3 + 3c + {0,1,2}] = max|R[:,c]|, max|X[:,c]|, max|B[:,c]|.
__global__ __launch_bounds__(256)
void norms_kernel(int n, int nrhs, const double* rowsum, const double* X, int64_t ldx, const double* D,
                  int64_t ldd, const double* R, int64_t ldr, const double* B, int64_t ldb, double* out)
{
    __shared__ double red[256];
    const int tid = threadIdx.x;
    auto reduce = [&](double v) -> double {
        red[tid] = v;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
            __syncthreads();
        }
        const double res = red[0];
        __syncthreads();
        return res;
    };
    double md = 0.0, mx = 0.0, ma = 0.0;
    for (int c = 0; c < nrhs; ++c)
        for (int i = tid; i < n; i += 256) {
            if (D) md = fmax(md, fabs(D[i + (int64_t)c * ldd]));
            mx = fmax(mx, fabs(X[i + (int64_t)c * ldx]));
        }
    if (rowsum)
        for (int i = tid; i < n; i += 256) ma = fmax(ma, rowsum[i]);
    md = reduce(md);
    mx = reduce(mx);
    ma = reduce(ma);
    if (tid == 0) { out[0] = md; out[1] = mx; out[2] = ma; }
    for (int c = 0; c < nrhs; ++c) {
        double vr = 0.0, vx = 0.0, vb = 0.0;
        for (int i = tid; i < n; i += 256) {
            if (R) vr = fmax(vr, fabs(R[i + (int64_t)c * ldr]));
            vx = fmax(vx, fabs(X[i + (int64_t)c * ldx]));
            if (B) vb = fmax(vb, fabs(B[i + (int64_t)c * ldb]));
        }
        vr = reduce(vr);
        vx = reduce(vx);
        vb = reduce(vb);
        if (tid == 0) { out[3 + 3 * c] = vr; out[4 + 3 * c] = vx; out[5 + 3 * c] = vb; }
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
                     double* __restrict__ out) {
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
        atomicMax(reinterpret_cast<unsigned long long*>(&out[0]), md[0]);
        atomicMax(reinterpret_cast<unsigned long long*>(&out[1]), mx[0]);
    }
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
hipError_t trisolve_impl(int n, int nrhs, const S* L, int64_t ldl, S* X, int64_t ldx, S* Linv, int* flags,
                         S* parts, bool make_inverses, hipStream_t st) {
    if (n <= 0 || nrhs <= 0) return hipSuccess;
    const int nblk = (n + TB - 1) / TB;
    if (make_inverses) {
        hipLaunchKernelGGL((inv_diag_kernel<S>), dim3(nblk), dim3(64), 0, st, n, L, ldl, Linv);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int per = (int)trisolve_sweep_ints(n);
    for (int c0 = 0; c0 < nrhs; c0 += RHS_CHUNK) {
        const int nr = (nrhs - c0 < RHS_CHUNK) ? nrhs - c0 : RHS_CHUNK;
        S* Xc = X + (int64_t)c0 * ldx;
        hipLaunchKernelGGL(fill_int_kernel, dim3(std::min(64, (2 * per + 255) / 256)), dim3(256), 0, st, flags,
                           2 * per, 0);
        hipLaunchKernelGGL((trisolve_kernel<S, false>), dim3(nblk * TP), dim3(256), 0, st, n, nr, L, ldl, Linv, Xc,
                           ldx, flags, parts);
        hipLaunchKernelGGL((trisolve_kernel<S, true>), dim3(nblk * TP), dim3(256), 0, st, n, nr, L, ldl, Linv, Xc,
                           ldx, flags + per, parts);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template hipError_t trisolve_impl<double>(int, int, const double*, int64_t, double*, int64_t, double*, int*, double*, bool,
                                          hipStream_t);
template hipError_t trisolve_impl<float>(int, int, const float*, int64_t, float*, int64_t, float*, int*, float*, bool,
                                         hipStream_t);

hipError_t launch_residual_f64(int n, int nrhs, const double* A, int64_t lda, const double* X, int64_t ldx,
                               const double* B, int64_t ldb, double* R, int64_t ldr, double* rowsum, double* part,
                               hipStream_t st) {
    if (n <= 0 || nrhs <= 0) return hipSuccess;
    const int nblk = (n + TB - 1) / TB;
    const int nch = (nblk + RCB - 1) / RCB;
    const int64_t pstride = (int64_t)n * RHS_CHUNK;
    double* rsum = part + (int64_t)nch * pstride;
    for (int c0 = 0; c0 < nrhs; c0 += RHS_CHUNK) {
        const int nr = std::min(RHS_CHUNK, nrhs - c0);
        double* rs = (c0 == 0 && rowsum) ? rsum : nullptr;
        hipLaunchKernelGGL(residual_part_kernel, dim3(nblk, nch), dim3(256), 0, st, n, nr, A, lda,
                           X + (int64_t)c0 * ldx, ldx, part, pstride, rs);
        hipLaunchKernelGGL(residual_reduce_kernel, dim3(std::min(1024, (n + 255) / 256), nr), dim3(256), 0, st, n, nr,
                           nch, part, pstride, B + (int64_t)c0 * ldb, ldb, R + (int64_t)c0 * ldr, ldr, rs,
                           c0 == 0 ? rowsum : nullptr);
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
    hipLaunchKernelGGL(norms_kernel, dim3(1), dim3(256), 0, st, n, nrhs, rowsum, X, ldx, D, ldd, R, ldr, B, ldb, out);
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
    hipLaunchKernelGGL((axpy_max_kernel<S>), dim3(gx, nrhs), dim3(256), 0, st, n, D, ldd, X, ldx, out);
    return hipGetLastError();
}
template hipError_t launch_widen_lower<float>(int, const float*, int64_t, double*, int64_t, hipStream_t);
template hipError_t launch_narrow_lower<float>(int, const double*, int64_t, float*, int64_t, hipStream_t);
template hipError_t launch_widen<double>(int, int, const double*, int64_t, double*, int64_t, hipStream_t);
template hipError_t launch_widen<float>(int, int, const float*, int64_t, double*, int64_t, hipStream_t);
template hipError_t launch_axpy_max<double>(int, int, const double*, int64_t, double*, int64_t, double*, hipStream_t);
template hipError_t launch_axpy_max<float>(int, int, const float*, int64_t, double*, int64_t, double*, hipStream_t);

}  // namespace ff
