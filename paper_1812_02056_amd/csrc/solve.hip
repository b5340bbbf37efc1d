// solve.hip -- solves with a computed factor and the binary64 refinement pieces.
//
// Solving A x = b from A = L L^T (Introduction of arXiv 1812.02056) needs two
// triangular solves.  Refinement (binary64 residual r = b - A x, correction
// from the low-precision factor, x += d) is how the mixed-precision factor wins
// back binary64 accuracy.
//
// Triangular solves: the n rows are cut into 64-row blocks.  One workgroup per
// block takes a ticket from an atomic counter, so a workgroup only ever waits for
// blocks whose workgroups already started; it streams its row of L against the
// solved blocks as their flags appear, then applies the precomputed inverse of
// its 64 x 64 diagonal block and publishes its result.  Every wait is bounded:
// past the spin limit the workgroup records an error and exits.
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace ff {

namespace {

constexpr int TB = 64;          // row block of the triangular solves
constexpr int RHS_CHUNK = 16;   // right-hand sides per launch
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

__device__ __forceinline__ bool wait_flag(const int* f) {
    int spins = 0;
    while (__hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0) {
        if (++spins > SPIN_LIMIT) return false;
        __builtin_amdgcn_s_sleep(2);
    }
    return true;
}

// Forward (TRANS = false: L y = b) or backward (TRANS = true: L^T x = y)
// substitution on nrhs <= 16 columns of X in place.  flags[0..nblk-1] are the
// per-block "published" flags, flags[nblk] the ticket counter, flags[nblk+1]
// the error word; all start at zero.
template <typename S, bool TRANS>
__global__ __launch_bounds__(256)
void trisolve_kernel(int n, int nrhs, const S* __restrict__ L, int64_t ldl, const S* __restrict__ Linv,
                     S* X, int64_t ldx, int* flags)
{
    __shared__ S tile[TB][TB + 1];
    __shared__ S yv[TB][RHS_CHUNK];
    __shared__ S acc[TB][RHS_CHUNK];
    __shared__ int ticket, bad;
    const int nblk = (n + TB - 1) / TB;
    const int tid = threadIdx.x;
    if (tid == 0) {
        ticket = atomicAdd(&flags[nblk], 1);
        bad = 0;
    }
    __syncthreads();
    const int j = TRANS ? (nblk - 1 - ticket) : ticket;
    const int r0 = j * TB;
    const int nbr = min(TB, n - r0);
    const int r = tid % TB, g = tid / TB;

    for (int c = g; c < RHS_CHUNK; c += 4)
        acc[r][c] = (r < nbr && c < nrhs) ? X[(int64_t)(r0 + r) + (int64_t)c * ldx] : S(0);

    for (int t = 0; t < nblk - 1; ++t) {
        const int i = TRANS ? (nblk - 1 - t) : t;     // solved block to fold in
        if (TRANS ? (i <= j) : (i >= j)) break;
        const int i0 = i * TB;
        const int nbi = min(TB, n - i0);
        // tile = L[j-block, i-block] (forward) or L[i-block, j-block] (backward), both below the diagonal
        for (int e = tid; e < TB * TB; e += 256) {
            const int a = e % TB, b = e / TB;      // a: row within tile (contiguous), b: column
            S v = S(0);
            if (!TRANS) { if (a < nbr && b < nbi) v = L[(int64_t)(r0 + a) + (int64_t)(i0 + b) * ldl]; }
            else        { if (a < nbi && b < nbr) v = L[(int64_t)(i0 + a) + (int64_t)(r0 + b) * ldl]; }
            tile[a][b] = v;
        }
        if (tid == 0 && !wait_flag(&flags[i])) bad = 1;
        __syncthreads();
        if (bad) {
            if (tid == 0) atomicExch(&flags[nblk + 1], 1);
            return;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        for (int e = tid; e < TB * RHS_CHUNK; e += 256) {
            const int a = e % TB, c = e / TB;
            yv[a][c] = (a < nbi && c < nrhs) ? X[(int64_t)(i0 + a) + (int64_t)c * ldx] : S(0);
        }
        __syncthreads();
        for (int c = g; c < nrhs; c += 4) {
            S s = S(0);
            if (!TRANS) { for (int k = 0; k < TB; ++k) s += tile[r][k] * yv[k][c]; }
            else        { for (int k = 0; k < TB; ++k) s += tile[k][r] * yv[k][c]; }
            acc[r][c] -= s;
        }
        __syncthreads();
    }
    // apply the inverse diagonal block
    for (int e = tid; e < TB * TB; e += 256) {
        const int a = e % TB, b = e / TB;
        tile[a][b] = Linv[(int64_t)j * TB * TB + a + (int64_t)b * TB];
    }
    __syncthreads();
    for (int c = g; c < nrhs; c += 4) {
        S s = S(0);
        if (!TRANS) { for (int k = 0; k < TB; ++k) s += tile[r][k] * acc[k][c]; }
        else        { for (int k = 0; k < TB; ++k) s += tile[k][r] * acc[k][c]; }
        if (r < nbr) X[(int64_t)(r0 + r) + (int64_t)c * ldx] = s;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0) __hip_atomic_store(&flags[j], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void fill_int_kernel(int* p, int count, int v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = v;
}

// R = B - A X in binary64 with A symmetric, only tril(A) read: the 64-row block j
// takes A[j-block, i-block] for i <= j and A[i-block, j-block]^T for i > j.  Also
// writes the absolute row sums of A (for ||A||_inf) into rowsum when non-null.
__global__ __launch_bounds__(256)
void residual_kernel(int n, int nrhs, const double* __restrict__ A, int64_t lda, const double* __restrict__ X,
                     int64_t ldx, const double* __restrict__ B, int64_t ldb, double* __restrict__ R, int64_t ldr,
                     double* __restrict__ rowsum)
{
    __shared__ double tile[TB][TB + 1];
    __shared__ double xv[TB][RHS_CHUNK];
    const int j = blockIdx.x;
    const int chunk0 = blockIdx.y * RHS_CHUNK;
    const int nr = min(RHS_CHUNK, nrhs - chunk0);
    const int r0 = j * TB;
    const int nbr = min(TB, n - r0);
    const int nblk = (n + TB - 1) / TB;
    const int tid = threadIdx.x, r = tid % TB, g = tid / TB;
    double acc[RHS_CHUNK / 4];
    double asum = 0.0;
#pragma unroll
    for (int q = 0; q < RHS_CHUNK / 4; ++q) acc[q] = 0.0;
    for (int i = 0; i < nblk; ++i) {
        const int i0 = i * TB;
        const int nbi = min(TB, n - i0);
        for (int e = tid; e < TB * TB; e += 256) {
            const int a = e % TB, b = e / TB;
            double v = 0.0;
            if (i < j) { if (a < nbr && b < nbi) v = A[(int64_t)(r0 + a) + (int64_t)(i0 + b) * lda]; }
            else if (i > j) { if (a < nbi && b < nbr) v = A[(int64_t)(i0 + a) + (int64_t)(r0 + b) * lda]; }
            else { if (a < nbr && b < nbr && a >= b) v = A[(int64_t)(r0 + a) + (int64_t)(r0 + b) * lda]; }
            tile[a][b] = v;
        }
        for (int e = tid; e < TB * RHS_CHUNK; e += 256) {
            const int a = e % TB, c = e / TB;
            xv[a][c] = (a < nbi && c < nr) ? X[(int64_t)(i0 + a) + (int64_t)(chunk0 + c) * ldx] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < RHS_CHUNK / 4; ++q) {
            const int c = g + 4 * q;
            if (c < nr) {
                double s = 0.0;
                if (i < j) { for (int k = 0; k < TB; ++k) s += tile[r][k] * xv[k][c]; }
                else if (i > j) { for (int k = 0; k < TB; ++k) s += tile[k][r] * xv[k][c]; }
                else { for (int k = 0; k < TB; ++k) s += (r >= k ? tile[r][k] : tile[k][r]) * xv[k][c]; }
                acc[q] += s;
            }
        }
        if (rowsum && g == 0 && blockIdx.y == 0) {
            double s = 0.0;
            if (i < j) { for (int k = 0; k < TB; ++k) s += fabs(tile[r][k]); }
            else if (i > j) { for (int k = 0; k < TB; ++k) s += fabs(tile[k][r]); }
            else { for (int k = 0; k < TB; ++k) s += fabs(r >= k ? tile[r][k] : tile[k][r]); }
            asum += s;
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < RHS_CHUNK / 4; ++q) {
        const int c = g + 4 * q;
        if (c < nr && r < nbr)
            R[(int64_t)(r0 + r) + (int64_t)(chunk0 + c) * ldr] = B[(int64_t)(r0 + r) + (int64_t)(chunk0 + c) * ldb] - acc[q];
    }
    if (rowsum && g == 0 && blockIdx.y == 0 && r < nbr) rowsum[r0 + r] = asum;
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
                         bool make_inverses, hipStream_t st) {
    if (n <= 0 || nrhs <= 0) return hipSuccess;
    const int nblk = (n + TB - 1) / TB;
    if (make_inverses) {
        hipLaunchKernelGGL((inv_diag_kernel<S>), dim3(nblk), dim3(64), 0, st, n, L, ldl, Linv);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    for (int c0 = 0; c0 < nrhs; c0 += RHS_CHUNK) {
        const int nr = (nrhs - c0 < RHS_CHUNK) ? nrhs - c0 : RHS_CHUNK;
        S* Xc = X + (int64_t)c0 * ldx;
        hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(256), 0, st, flags, 2 * (nblk + 2), 0);
        hipLaunchKernelGGL((trisolve_kernel<S, false>), dim3(nblk), dim3(256), 0, st, n, nr, L, ldl, Linv, Xc, ldx,
                           flags);
        hipLaunchKernelGGL((trisolve_kernel<S, true>), dim3(nblk), dim3(256), 0, st, n, nr, L, ldl, Linv, Xc, ldx,
                           flags + (nblk + 2));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template hipError_t trisolve_impl<double>(int, int, const double*, int64_t, double*, int64_t, double*, int*, bool, hipStream_t);
template hipError_t trisolve_impl<float>(int, int, const float*, int64_t, float*, int64_t, float*, int*, bool, hipStream_t);

hipError_t launch_residual_f64(int n, int nrhs, const double* A, int64_t lda, const double* X, int64_t ldx,
                               const double* B, int64_t ldb, double* R, int64_t ldr, double* rowsum, hipStream_t st) {
    if (n <= 0 || nrhs <= 0) return hipSuccess;
    const int nblk = (n + TB - 1) / TB;
    const int nchunk = (nrhs + RHS_CHUNK - 1) / RHS_CHUNK;
    hipLaunchKernelGGL(residual_kernel, dim3(nblk, nchunk), dim3(256), 0, st, n, nrhs, A, lda, X, ldx, B, ldb, R, ldr,
                       rowsum);
    return hipGetLastError();
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
