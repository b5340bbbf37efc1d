// driver.hip -- host side of libfastfact: argument checks, the block schedule of
// Algorithms 1 and 2 (Sec. 2 of arXiv 1812.02056), workspace carving and the
// refinement loop of chol_solve.  Implements include/fastfact.h.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <utility>
#include <vector>

#include "fastfact.h"
#include "grid.hpp"
#include "internal.hpp"

// Device scratch of the allocation-free entry point (see noalloc_scratch).
static __device__ __align__(256) unsigned char scratch[FF_NOALLOC_SCRATCH_BYTES];

namespace ff {
namespace {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// Inner step used when a diagonal block is larger than the single-workgroup
// diagonal kernels take: the block is itself factored by the same delayed-update
// schedule with this step.

struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* p) : base(static_cast<char*>(p)) {}
    template <typename T> T* take(size_t count) {
        T* p = reinterpret_cast<T*>(base + off);
        off += align_up(count * sizeof(T));
        return p;
    }
};

// Workspace of a float-storage factorisation: the w x w binary64 diagonal block
// (widened, factored, rounded back), then for FF_BF16 the transposed bfloat16
// copy of the panel the update reads (n rows of bf16t_width(w) values).
size_t diag_ws_bytes(int64_t n, int64_t s, int dtype) {
    if (dtype == FF_F64 || n <= 0) return 0;
    const int64_t w = std::min<int64_t>(s, n);
    size_t b = align_up((size_t)w * (size_t)w * sizeof(double));
    if (dtype == FF_BF16) b += align_up((size_t)n * (size_t)bf16t_width((int)w) * 2);
    return b;
}
__bf16* bf16_panel_ws(double* ws64, int64_t n, int64_t s) {
    const int64_t w = std::min<int64_t>(s, n);
    return reinterpret_cast<__bf16*>(reinterpret_cast<char*>(ws64) + align_up((size_t)w * (size_t)w * sizeof(double)));
}

#define FF_TRY(expr)                                  \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return FF_ERR_HIP;      \
    } while (0)

// ---------------------------------------------------------------- side streams
// Lookahead runs the diagonal factorisation and panel solve of block k+1 on a
// second stream while the rest of update k runs on the caller's stream.  Side
// streams (default priority, non-blocking) are created once per device and
// pooled; ordering between the two streams is carried by events created per
// call, so concurrent calls stay correct even when they share a side stream.
struct SidePool {
    std::mutex mu;
    std::vector<std::pair<int, hipStream_t>> free_list;
};
SidePool& side_pool() {
    static SidePool p;
    return p;
}
hipStream_t acquire_side(int dev) {
    SidePool& p = side_pool();
    {
        std::lock_guard<std::mutex> lk(p.mu);
        for (size_t i = 0; i < p.free_list.size(); ++i)
            if (p.free_list[i].first == dev) {
                hipStream_t s = p.free_list[i].second;
                p.free_list.erase(p.free_list.begin() + i);
                return s;
            }
    }
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    return s;
}
void release_side(int dev, hipStream_t s) {
    SidePool& p = side_pool();
    std::lock_guard<std::mutex> lk(p.mu);
    p.free_list.emplace_back(dev, s);
}

struct Events {
    std::vector<hipEvent_t> ev;
    ~Events() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
    hipEvent_t make() {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        ev.push_back(e);
        return e;
    }
};

// ---------------------------------------------------------------- update profile
// Measurement aid behind ff_update_profile_*: event pairs around the trailing
// updates of chol_factor, tallied per kernel shape.
struct UpdProfile {
    std::mutex mu;
    bool on = false;
    struct Rec {
        hipEvent_t e0, e1;
        double flops, bytes;
        int shape;
    };
    std::vector<Rec> recs;
    ff_kernel_profile tally[FF_UPD_NSHAPES];
};
UpdProfile& upd_profile() {
    static UpdProfile p;
    return p;
}

// Entries (i, j), i < M, j < N, with i - j >= shift.
double region_entries(int M, int N, int shift) {
    double c = 0;
    for (int j = 0; j < N; ++j) {
        const int lo = std::max(0, j + shift);
        if (lo < M) c += (double)(M - lo);
    }
    return c;
}

struct UpdTimer {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double flops = 0, bytes = 0;
    int shape = 0;
    hipStream_t st = nullptr;
    // shape_of < 0: the binary64 kernel shape launch_update picks; else that tally
    // (FF_UPD_SHAPE_F32 / FF_UPD_SHAPE_BF16).  elem: bytes per stored element.
    UpdTimer(int M, int N, int K, int shift, int reserve, hipStream_t s, double f0 = 0.0, double f1 = 1.0,
             int shape_of = -1, int elem = 8) : st(s) {
        // the tail part of a split update runs concurrently on another stream and
        // is not recorded (the profile covers the launches on the caller's stream)
        if (f0 > 0.0) return;
        UpdProfile& p = upd_profile();
        {
            std::lock_guard<std::mutex> lk(p.mu);
            if (!p.on) return;
        }
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            if (e0) (void)hipEventDestroy(e0);
            e0 = e1 = nullptr;
            return;
        }
        const double part = f1 < 1.0 ? update_range_entries(M, N, true, shift, reserve, f0, f1) : -1.0;
        const double entries = part >= 0.0 ? part : region_entries(M, N, shift);
        flops = 2.0 * (double)K * entries;
        // C entries read and written once, the region's panel rows (its columns
        // are rows of the same panel) read once
        bytes = (double)elem * (2.0 * entries + (double)M * (double)K);
        shape = shape_of >= 0 ? shape_of : update_shape(M, N, reserve);
        (void)hipEventRecord(e0, st);
    }
    void stop() {
        if (!e0) return;
        (void)hipEventRecord(e1, st);
        UpdProfile& p = upd_profile();
        std::lock_guard<std::mutex> lk(p.mu);
        p.recs.push_back({e0, e1, flops, bytes, shape});
        e0 = e1 = nullptr;
    }
};

// ---------------------------------------------------------------- panel solves
// X T = B for the m x w panel, T upper triangular (see launch_trsm), solved in
// column chunks of TRSM_MAX when w is wider: chunk [c0, c1) first subtracts the
// solved columns, X[:, c0:c1] -= X[:, 0:c0] T[0:c0, c0:c1], then is solved with
// the diagonal block T[c0:c1, c0:c1].  xcol: X column-major (xi = 1, xj = ldx);
// otherwise X(i, j) = x[j + i*ldx] (rows of X are columns of x).
template <typename T>
int trsm_blocked(int m, int w, T* x, int64_t ldx, bool xcol, const T* t, int64_t ldt, bool t_is_rows, int unit,
                 const int* info, hipStream_t st, int max_wg = 0) {
    // t_is_rows: T(k, j) = t[j + k*ldt] (T = L^T of a lower factor); else T(k, j) = t[k + j*ldt]
    const int64_t tk = t_is_rows ? ldt : 1, tj = t_is_rows ? 1 : ldt;
    const int64_t xi = xcol ? 1 : ldx, xj = xcol ? ldx : 1;
    for (int c0 = 0; c0 < w; c0 += TRSM_MAX) {
        const int c1 = std::min(w, c0 + TRSM_MAX);
        const int wc = c1 - c0;
        if (c0 > 0) {
            if (xcol) {
                // C = X[:, c0:c1] (m x wc), K = c0, Y(j, k) = T(k, c0 + j)
                const T* ybase = t_is_rows ? t + c0 : t + (int64_t)c0 * ldt;
                FF_TRY(launch_update<T>(m, wc, c0, x + (int64_t)c0 * ldx, ldx, x, ldx, ybase, ldt, t_is_rows, false,
                                        0, info, st, 0, max_wg));
            } else {
                // transposed form on the stored matrix x (rows [c0, c1) of x, all m columns):
                // x[c0 + i', j'] -= sum_k T(k, c0 + i') x[k, j'];  X operand (i', k) = T(k, c0 + i')
                if (!t_is_rows) return FF_ERR_UNSUPPORTED;
                FF_TRY(launch_update<T>(wc, m, c0, x + c0, ldx, t + c0, ldt, x, ldx, false, false, 0, info, st));
            }
        }
        T* xc = xcol ? x + (int64_t)c0 * ldx : x + c0;
        const T* tc = t + (int64_t)c0 * tk + (int64_t)c0 * tj;
        FF_TRY(launch_trsm<T>(m, wc, xc, xi, xj, tc, tk, tj, unit, info, st, max_wg));
    }
    return 0;
}

// ---------------------------------------------------------------- Cholesky
// Algorithm 1 as a block schedule: block k covers columns c0 = k*s .. c0+w-1;
// the diagonal factorisation and the panel solve form those columns from the
// matrix as updated so far, then the deferred product of the w new columns is
// subtracted from the trailing square (the update of the paper's conditional,
// which fires floor((n-1)/s) times).
template <typename S>
int chol_diag(int w, S* A11, int64_t lda, int dtype, double* ws64, int* info, int col_base, hipStream_t st);

template <typename S>
int chol_panel(int n, int c0, int w, S* A, int64_t lda, int dtype, double* ws64, int* info, int col_base,
               hipStream_t st, int max_wg = 0) {
    S* A11 = A + (int64_t)c0 + (int64_t)c0 * lda;
    int rc = chol_diag<S>(w, A11, lda, dtype, ws64, info, col_base + c0, st);
    if (rc) return rc;
    const int m = n - c0 - w;
    if (m > 0) {
        S* A21 = A + (int64_t)(c0 + w) + (int64_t)c0 * lda;
        // L21 = A21 L11^-T: x T = b with T(k, j) = L11(j, k)
        rc = trsm_blocked<S>(m, w, A21, lda, true, A11, lda, true, 0, info, st, max_wg);
    }
    return rc;
}

// A22 region update: C(i, j) -= sum_k P(i, k) P(j, k) over rows [r0, m) and
// columns [q0, q1) of the m x m trailing matrix, lower part only.
// [f0, f1): the part of the region's tile order to apply (see launch_update);
// max_cus > 0 sizes the launch for a stream that owns only that many CUs.
// pt (FF_BF16): the transposed bfloat16 panel copy; the call whose region starts
// at row and column 0 (the first of a step) writes it, later calls of the step
// on the same stream read it.
template <typename S>
int chol_update(int m, int w, S* A22, int64_t lda, const S* P, int r0, int q0, int q1, int dtype, unsigned flags,
                const int* info, hipStream_t st, int reserve = 0, double f0 = 0.0, double f1 = 1.0,
                int max_cus = 0, __bf16* pt = nullptr) {
    const int M = m - r0, N = q1 - q0;
    if (M <= 0 || N <= 0) return 0;
    S* C = A22 + (int64_t)r0 + (int64_t)q0 * lda;
    const int shift = q0 - r0;     // global i >= j  <=>  local i' - j' >= q0 - r0
    if constexpr (sizeof(S) == sizeof(double)) {
        if ((flags & FF_FLAG_STRASSEN1) && M == N && shift == 0) {
            FF_TRY(launch_update_syrk_strassen_f64(M, w, reinterpret_cast<double*>(C), lda,
                                                   reinterpret_cast<const double*>(P + r0), lda, info, st, reserve));
            return 0;
        }
        UpdTimer tm(M, N, w, shift, reserve, st, f0, f1);
        FF_TRY(launch_update<double>(M, N, w, reinterpret_cast<double*>(C), lda,
                                     reinterpret_cast<const double*>(P + r0), lda,
                                     reinterpret_cast<const double*>(P + q0), lda, true, true, shift, info, st,
                                     reserve, max_cus, f0, f1));
        tm.stop();
    } else {
        UpdTimer tm(M, N, w, shift, reserve, st, f0, f1, dtype == FF_BF16 ? FF_UPD_SHAPE_BF16 : FF_UPD_SHAPE_F32,
                    (int)sizeof(float));
        if (dtype == FF_BF16 && pt) {
            const int wp = bf16t_width(w);
            if (r0 == 0 && q0 == 0) FF_TRY(launch_panel_bf16t(m, w, P, lda, pt, st));
            FF_TRY(launch_update_bf16t(M, N, w, C, lda, pt + (int64_t)r0 * wp, pt + (int64_t)q0 * wp, true, shift,
                                       info, st, reserve));
        } else if (dtype == FF_BF16)
            FF_TRY(launch_update_bf16(M, N, w, C, lda, P + r0, lda, P + q0, lda, true, shift, info, st, reserve));
        else
            FF_TRY(launch_update<float>(M, N, w, C, lda, P + r0, lda, P + q0, lda, true, true, shift, info, st,
                                        reserve, max_cus, f0, f1));
        tm.stop();
    }
    return 0;
}

// CUs to keep free for the next block's diagonal factorisation and panel solve
// while the rest of the update runs: 32 if the panel estimate fits under the
// update's estimate there, else the one of 32/64 that minimises the longer of
// the two.  Model: the diagonal block costs diag_us, the panel solve trsm_us.
// *tail: the fraction of the update's tiles (its last ones) that the reserved
// CUs can take after the panel work and still finish with the rest, which runs
// on the other CUs: (U - P) / (U (1 + (C - R) / R)) for update and panel
// estimates U and P, less a margin (0 when the panel is the longer).
// upd_factor: update flops per mr^2 w (1 for the lower-triangle product, 2 for
// LU's full product); n_solves: panel solves per step (1 Cholesky, 2 LU);
// diag_us: the next block's diagonal factorisation (chol_diag_us, lu_diag_us).
//
// The estimates are fitted to kernel traces on MI355X (binary64):
//  - a panel-solve round: one workgroup of four waves solves 64 rows of a chunk
//    of up to TRSM_MAX columns, ~7 us of staging and tile inverses plus ~16 us of
//    MFMA solve at 12 tiles, growing with the tile pairs;
//  - chunks after the first subtract the solved columns first (an update on the
//    same CUs) and launch a second solve.
double trsm_us(int mr, int wn, int r, int cus, size_t sz, double rate) {
    double t = 0.0;
    for (int c0 = 0; c0 < wn; c0 += TRSM_MAX) {
        const int wc = std::min(TRSM_MAX, wn - c0);
        const int tiles = (wc + 15) / 16;
        const double round = 7.0 + 16.0 * tiles * (tiles + 1) / 156.0 * (sz == sizeof(double) ? 1.0 : 0.5);
        t += std::ceil((double)mr / (64.0 * r)) * round;
        // the chunk's columns less the solved ones: mr x wc x c0
        if (c0 > 0) t += 2.0 * mr * (double)wc * c0 / (rate * r / cus) * 1e6 + 5.0;
    }
    return t;
}
// Cholesky diagonal block: one LDS kernel up to LDS_DIAG_MAX (68 us at 192
// columns), else LDS_DIAG_MAX-wide blocks with a solve and an update between.
double chol_diag_us(int wn) {
    auto one = [](int w) { return 10.0 + 0.3 * w; };
    if (wn <= LDS_DIAG_MAX) return one(wn);
    double t = 0.0;
    for (int c0 = 0; c0 < wn; c0 += LDS_DIAG_MAX) t += one(std::min(LDS_DIAG_MAX, wn - c0)) + (c0 > 0 ? 45.0 : 0.0);
    return t;
}
// LU diagonal block: one LDS kernel up to LU_LDS_MAX (62 us at 128 columns), else
// LU_LDS_MAX-wide blocks with two solves and an update between.
double lu_diag_us(int wn) {
    double t = 0.0;
    for (int c0 = 0; c0 < wn; c0 += LU_LDS_MAX) t += 6.0 + 0.44 * std::min(LU_LDS_MAX, wn - c0) + (c0 > 0 ? 60.0 : 0.0);
    return t;
}
int lookahead_reserve(int mr, int w, int wn, size_t sz, double diag_us, double* tail, double upd_factor = 1.0,
                      int n_solves = 1, double* upd_est = nullptr, double* pan_est = nullptr) {
    const double rate = (sz == sizeof(double) ? 50e12 : 90e12);
    const int cus = update_workers(0);
    // At least 4 free CUs per XCD: with fewer, the side stream's workgroups are
    // often placed behind the update's (the free CUs of an XCD are not all
    // reachable) and the panel solve waits for the whole update to drain.
    int best = 32;
    double best_t = 1e30, best_u = 0, best_p = 0;
    for (int r : {32, 64}) {
        const double upd_us = upd_factor * (double)mr * (double)mr * (double)w / (rate * (double)(cus - r) / cus) * 1e6;
        const double pan_us = diag_us + n_solves * trsm_us(mr, wn, r, cus, sz, rate);
        const double t = std::max(upd_us, pan_us);
        if (t < best_t) { best_t = t; best = r; best_u = upd_us; best_p = pan_us; }
        if (pan_us <= upd_us) break;
    }
    if (tail) {
        const double f = best_u > best_p ? (best_u - best_p) / (best_u * (1.0 + (double)(cus - best) / best)) : 0.0;
        *tail = 0.9 * f;
    }
    if (upd_est) *upd_est = best_u;
    if (pan_est) *pan_est = best_p;
    return best;
}

// The update's main part runs in rounds of one tile per workgroup, so a part
// that ends a few tiles into a round leaves most of the workgroups idle for that
// round.  Given the tile order's T tiles, the main part's nwg workgroups, the r
// reserved CUs and the model's update (u, all T tiles on the main CUs) and panel
// (p) estimates, moves the split to the whole round nearest it when that shortens
// the longer of the main part and the panel plus the tail.
double round_aligned_tail(int T, int nwg, int r, double f, double u, double p) {
    if (T <= 0 || nwg <= 0 || r <= 0 || f <= 0.0) return f;
    const double tau = u * nwg / T;      // one round of the main part
    auto cost = [&](int nmain) {
        const double main = std::ceil((double)nmain / nwg) * tau;
        const double rest = T > nmain ? p + std::ceil((double)(T - nmain) / r) * tau : 0.0;
        return std::max(main, rest);
    };
    const int n0 = std::min(T, std::max(0, (int)((1.0 - f) * T + 0.5)));
    int best = n0;
    double bc = cost(n0);
    for (int k = n0 / nwg - 1; k <= n0 / nwg + 1; ++k) {
        const int nm = std::min(T, k * nwg);
        if (nm <= 0) continue;
        const double c = cost(nm);
        if (c < bc) { bc = c; best = nm; }
    }
    return 1.0 - (double)best / T;
}

// Width of the Cholesky block starting at column c0 for step size s (the closing
// remarks of Sec. 2 allow s to change during the run).  The first
// block, and every block over the last CHOL_TAIL_COLS columns, is cut to
// LDS_DIAG_MAX when s is wider: nothing overlaps the first block's factorisation,
// and near the end the trailing update is small and the next block's
// factorisation sets the pace; a block that fits one workgroup's LDS is factored
// by one kernel instead of a recursive chain of four or more (measured at
// n = 16384, s = 320 and 512: the time is flat for thresholds 4608 to 8192).
constexpr int CHOL_TAIL_COLS = 6144;
// Columns (at most a quarter of the matrix) after which the lookahead schedule
// finishes in order on one stream (measured at n = 16384, s = 768: 0.25 ms
// faster than lookahead to the end, flat for thresholds 1152 to 2304).
constexpr int CHOL_INORDER_COLS = 1536;
inline int chol_block_width(int s, int c0, int n, unsigned flags) {
    const bool edge = c0 == 0 || n - c0 <= CHOL_TAIL_COLS;
    const int w = (s > LDS_DIAG_MAX && edge && !(flags & FF_FLAG_FIXED_STEP)) ? LDS_DIAG_MAX : s;
    return std::min(w, n - c0);
}

template <typename S>
int chol_blocked(int n, int s, S* A, int64_t lda, int dtype, unsigned flags, double* ws64, int* info,
                 int col_base, hipStream_t st, bool lookahead) {
    if (n <= 0) return 0;
    __bf16* pt = (dtype == FF_BF16 && ws64) ? bf16_panel_ws(ws64, n, s) : nullptr;
    hipStream_t side = nullptr;
    int dev = 0;
    Events evs;
    if (lookahead && n > s) {
        if (hipGetDevice(&dev) != hipSuccess) return FF_ERR_HIP;
        side = acquire_side(dev);
        if (!side) return FF_ERR_HIP;
    }
    // blocks from column c_start on, in order on `st`
    auto in_order = [&](int c_start) {
        int rc = 0;
        for (int c0 = c_start, w = 0; c0 < n && !rc; c0 += w) {
            w = chol_block_width(s, c0, n, flags);
            const int m = n - c0 - w;
            rc = chol_panel<S>(n, c0, w, A, lda, dtype, ws64, info, col_base, st);
            if (rc || m <= 0) break;
            S* A21 = A + (int64_t)(c0 + w) + (int64_t)c0 * lda;
            S* A22 = A + (int64_t)(c0 + w) + (int64_t)(c0 + w) * lda;
            rc = chol_update<S>(m, w, A22, lda, A21, 0, 0, m, dtype, flags, info, st, 0, 0.0, 1.0, 0, pt);
        }
        return rc;
    };
    int rc = 0;
    if (!side) return in_order(0);
    const int last_in_order = std::min(CHOL_INORDER_COLS, n / 4);
    // lookahead schedule
    hipEvent_t e0 = evs.make();
    if (!e0) { release_side(dev, side); return FF_ERR_HIP; }
    auto fail = [&](int code) { release_side(dev, side); return code; };
    if (hipEventRecord(e0, st) != hipSuccess || hipStreamWaitEvent(side, e0, 0) != hipSuccess) return fail(FF_ERR_HIP);
    rc = chol_panel<S>(n, 0, chol_block_width(s, 0, n, flags), A, lda, dtype, ws64, info, col_base, side);
    if (rc) return fail(rc);
    hipEvent_t ep = evs.make();
    if (!ep || hipEventRecord(ep, side) != hipSuccess || hipStreamWaitEvent(st, ep, 0) != hipSuccess)
        return fail(FF_ERR_HIP);
    for (int c0 = 0, w = 0; c0 < n; c0 += w) {
        w = chol_block_width(s, c0, n, flags);
        const int m = n - c0 - w;
        if (m <= 0) break;
        S* A21 = A + (int64_t)(c0 + w) + (int64_t)c0 * lda;
        S* A22 = A + (int64_t)(c0 + w) + (int64_t)(c0 + w) * lda;
        if (m <= last_in_order) {
            // the last steps in order on `st`: there the whole update is shorter
            // than the two hand-overs between the streams a lookahead step makes
            rc = chol_update<S>(m, w, A22, lda, A21, 0, 0, m, dtype, flags, info, st, 0, 0.0, 1.0, 0, pt);
            release_side(dev, side);
            return rc ? rc : in_order(c0 + w);
        }
        const int wn = chol_block_width(s, c0 + w, n, flags);    // width of the next block
        // 1) the next block's columns of the update, then hand them to the side stream
        rc = chol_update<S>(m, w, A22, lda, A21, 0, 0, wn, dtype, flags & ~FF_FLAG_STRASSEN1, info, st, 0, 0.0, 1.0,
                            0, pt);
        if (rc) return fail(rc);
        hipEvent_t en = evs.make();
        if (!en || hipEventRecord(en, st) != hipSuccess || hipStreamWaitEvent(side, en, 0) != hipSuccess)
            return fail(FF_ERR_HIP);
        // 2) the rest of the update, concurrently with the next panel, on all but
        //    `reserve` CUs; the panel solve's grid is sized to those free CUs,
        //    which then take the last `tail` of the update's tile order
        double tail = 0.0, u_est = 0.0, p_est = 0.0;
        const int reserve = lookahead_reserve(m - wn, w, wn, sizeof(S), chol_diag_us(wn), &tail, 1.0, 1, &u_est, &p_est);
        if ((flags & FF_FLAG_STRASSEN1) || dtype == FF_BF16 || tail < 0.01 ||
            !update_splittable(m - wn, m - wn, true, 0, reserve))
            tail = 0.0;
        else
            tail = round_aligned_tail(update_order_tiles(m - wn, m - wn, true, 0, reserve), update_workers(reserve),
                                      reserve, tail, u_est, p_est);
        rc = chol_panel<S>(n, c0 + w, wn, A, lda, dtype, ws64, info, col_base, side, reserve);
        if (rc) return fail(rc);
        if (tail > 0.0) {
            rc = chol_update<S>(m, w, A22, lda, A21, wn, wn, m, dtype, flags, info, side, reserve, 1.0 - tail, 1.0,
                                reserve);
            if (rc) return fail(rc);
        }
        hipEvent_t ep2 = evs.make();
        if (!ep2 || hipEventRecord(ep2, side) != hipSuccess) return fail(FF_ERR_HIP);
        rc = chol_update<S>(m, w, A22, lda, A21, wn, wn, m, dtype, flags, info, st, reserve, 0.0, 1.0 - tail, 0, pt);
        if (rc) return fail(rc);
        if (hipStreamWaitEvent(st, ep2, 0) != hipSuccess) return fail(FF_ERR_HIP);
    }
    release_side(dev, side);
    return 0;
}

template <typename S>
int chol_diag(int w, S* A11, int64_t lda, int dtype, double* ws64, int* info, int col_base, hipStream_t st) {
    if (w <= LDS_DIAG_MAX) {
        FF_TRY(launch_potrf_diag<S>(w, A11, lda, info, col_base, st));
        return 0;
    }
    if constexpr (sizeof(S) == sizeof(double)) {
        return chol_blocked<double>(w, LDS_DIAG_MAX, reinterpret_cast<double*>(A11), lda, FF_F64, 0, nullptr, info,
                                    col_base, st, false);
    } else {
        // widen the block, factor it in binary64, round it back
        FF_TRY(launch_widen_lower<float>(w, A11, lda, ws64, w, st));
        int rc = chol_blocked<double>(w, LDS_DIAG_MAX, ws64, w, FF_F64, 0, nullptr, info, col_base, st, false);
        if (rc) return rc;
        FF_TRY(launch_narrow_lower<float>(w, ws64, w, A11, lda, st));
        return 0;
    }
}

// ---------------------------------------------------------------- LU
// Algorithm 2 as a block schedule (Doolittle packing): diagonal GETRF, then
// L21 = A21 U11^-1 and U12 = L11^-1 A12, then A22 -= L21 U12.
// LU panel of block [c0, c0 + w): GETRF-nopiv of the diagonal block, then
// L21 = A21 U11^-1 and U12 = L11^-1 A12; max_wg caps the panel solves' grids.
// Width of the LU block starting at column c0 for step size s: as for Cholesky,
// the first block and the blocks of the last LU_TAIL_COLS columns are cut to
// LU_LDS_MAX when s is wider (one LDS kernel each), unless FF_FLAG_FIXED_STEP
// (measured at n = 16384, s = 512 and 768: best at 4096, within 0.2 ms at 6144).
constexpr int LU_TAIL_COLS = 4096;
// Columns (at most a quarter of the matrix) after which the lookahead schedule
// finishes in order on one stream (measured at n = 16384, s = 768: 0.4 ms
// faster than lookahead to the end, flat for thresholds 1024 to 3072).
constexpr int LU_INORDER_COLS = 1536;
inline int lu_block_width(int s, int c0, int n, unsigned flags) {
    const bool edge = c0 == 0 || n - c0 <= LU_TAIL_COLS;
    const int w = (s > LU_LDS_MAX && edge && !(flags & FF_FLAG_FIXED_STEP)) ? LU_LDS_MAX : s;
    return std::min(w, n - c0);
}
int lu_blocked(int n, int s, double* A, int64_t lda, unsigned flags, int* info, int col_base, hipStream_t st,
               double* s2ws = nullptr);
// A22 -= X Y for the LU: classical, one Strassen level, or two (FF_FLAG_STRASSEN2,
// scratch s2ws); reserve CUs are left to the side stream.
hipError_t lu_product(int m, int w, double* C, int64_t lda, const double* X, const double* Y, unsigned flags,
                      double* s2ws, const int* info, hipStream_t st, int reserve = 0) {
    if (flags & FF_FLAG_STRASSEN2)
        return launch_update_gemm_strassen2_f64(m, w, C, lda, X, lda, Y, lda, s2ws, info, st, reserve);
    if (flags & FF_FLAG_STRASSEN1)
        return launch_update_gemm_strassen_f64(m, w, C, lda, X, lda, Y, lda, info, st, reserve);
    return launch_update<double>(m, m, w, C, lda, X, lda, Y, lda, false, false, 0, info, st, reserve);
}
// GETRF-nopiv of the w x w diagonal block: one LDS kernel up to LU_LDS_MAX,
// blocks of LU_LDS_MAX (in order) when wider.
int lu_diag(int w, double* A11, int64_t lda, int* info, int col_base, hipStream_t st) {
    if (w <= LU_LDS_MAX) {
        FF_TRY(launch_getrf_lds(w, A11, lda, info, col_base, st));
        return 0;
    }
    return lu_blocked(w, LU_LDS_MAX, A11, lda, FF_FLAG_NO_LOOKAHEAD, info, col_base, st);
}
int lu_panel(int n, int c0, int w, double* A, int64_t lda, int* info, int col_base, hipStream_t st, int max_wg = 0) {
    double* A11 = A + (int64_t)c0 + (int64_t)c0 * lda;
    {
        int rc = lu_diag(w, A11, lda, info, col_base + c0, st);
        if (rc) return rc;
    }
    const int m = n - c0 - w;
    if (m <= 0) return 0;
    double* A21 = A + (int64_t)(c0 + w) + (int64_t)c0 * lda;
    double* A12 = A + (int64_t)c0 + (int64_t)(c0 + w) * lda;
    // L21 U11 = A21: T(k, j) = U11(k, j) = A11[k + j*lda]
    int rc = trsm_blocked<double>(m, w, A21, lda, true, A11, lda, false, 0, info, st, max_wg);
    if (rc) return rc;
    // L11 U12 = A12  <=>  U12^T L11^T = A12^T: rows of X are columns of A12,
    // T(k, j) = L11(j, k) with unit diagonal
    return trsm_blocked<double>(m, w, A12, lda, false, A11, lda, true, 1, info, st, max_wg);
}

// Blocks from column c_start on, in order on `st`.
int lu_in_order(int n, int s, double* A, int64_t lda, unsigned flags, int* info, int col_base, hipStream_t st,
                int c_start, double* s2ws = nullptr) {
    for (int c0 = c_start, w = 0; c0 < n; c0 += w) {
        w = lu_block_width(s, c0, n, flags);
        const int m = n - c0 - w;
        double* A11 = A + (int64_t)c0 + (int64_t)c0 * lda;
        {
            int rc = lu_diag(w, A11, lda, info, col_base + c0, st);
            if (rc) return rc;
        }
        if (m <= 0) break;
        double* A21 = A + (int64_t)(c0 + w) + (int64_t)c0 * lda;
        double* A12 = A + (int64_t)c0 + (int64_t)(c0 + w) * lda;
        double* A22 = A + (int64_t)(c0 + w) + (int64_t)(c0 + w) * lda;
        // L21 U11 = A21: T(k, j) = U11(k, j) = A11[k + j*lda]
        int rc = trsm_blocked<double>(m, w, A21, lda, true, A11, lda, false, 0, info, st);
        if (rc) return rc;
        // L11 U12 = A12  <=>  U12^T L11^T = A12^T: rows of X are columns of A12,
        // T(k, j) = L11(j, k) with unit diagonal
        rc = trsm_blocked<double>(m, w, A12, lda, false, A11, lda, true, 1, info, st);
        if (rc) return rc;
        FF_TRY(lu_product(m, w, A22, lda, A21, A12, flags, s2ws, info, st));
    }
    return 0;
}

// Lookahead schedule of the LU (as for Cholesky): while the rest of update k
// runs on `st` on all but `reserve` CUs, the side stream factors block k + 1
// (whose column and row strips were updated first) and then takes the tail of
// update k's tile order.
int lu_lookahead(int n, int s, double* A, int64_t lda, unsigned flags, int* info, int col_base, hipStream_t st,
                 double* s2ws) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return FF_ERR_HIP;
    hipStream_t side = acquire_side(dev);
    if (!side) return FF_ERR_HIP;
    Events evs;
    auto fail = [&](int code) { release_side(dev, side); return code; };
    hipEvent_t e0 = evs.make();
    if (!e0 || hipEventRecord(e0, st) != hipSuccess || hipStreamWaitEvent(side, e0, 0) != hipSuccess)
        return fail(FF_ERR_HIP);
    const int last_in_order = std::min(LU_INORDER_COLS, n / 4);
    int rc = lu_panel(n, 0, lu_block_width(s, 0, n, flags), A, lda, info, col_base, side);
    if (rc) return fail(rc);
    hipEvent_t ep = evs.make();
    if (!ep || hipEventRecord(ep, side) != hipSuccess || hipStreamWaitEvent(st, ep, 0) != hipSuccess)
        return fail(FF_ERR_HIP);
    for (int c0 = 0, w = 0; c0 < n; c0 += w) {
        w = lu_block_width(s, c0, n, flags);
        const int m = n - c0 - w;
        if (m <= 0) break;
        double* A21 = A + (int64_t)(c0 + w) + (int64_t)c0 * lda;
        double* A12 = A + (int64_t)c0 + (int64_t)(c0 + w) * lda;
        double* A22 = A + (int64_t)(c0 + w) + (int64_t)(c0 + w) * lda;
        if (m <= last_in_order) {
            // the last steps in order on `st`: there the whole update is shorter
            // than the two hand-overs between the streams a lookahead step makes
            hipError_t e = lu_product(m, w, A22, lda, A21, A12, flags, s2ws, info, st);
            release_side(dev, side);
            return e != hipSuccess ? FF_ERR_HIP : lu_in_order(n, s, A, lda, flags, info, col_base, st, c0 + w, s2ws);
        }
        const int wn = lu_block_width(s, c0 + w, n, flags);
        const int mr = m - wn;
        // 1) the next block's column strip (all rows) and row strip
        hipError_t e = launch_update<double>(m, wn, w, A22, lda, A21, lda, A12, lda, false, false, 0, info, st);
        if (e == hipSuccess && mr > 0)
            e = launch_update<double>(wn, mr, w, A22 + (int64_t)wn * lda, lda, A21, lda, A12 + (int64_t)wn * lda, lda,
                                      false, false, 0, info, st);
        if (e != hipSuccess) return fail(FF_ERR_HIP);
        hipEvent_t en = evs.make();
        if (!en || hipEventRecord(en, st) != hipSuccess || hipStreamWaitEvent(side, en, 0) != hipSuccess)
            return fail(FF_ERR_HIP);
        // 2) the next panel on the side stream, sized to the reserved CUs; the
        //    rest of the update on the others, its tail on the reserved CUs after
        //    the panel
        double tail = 0.0, u_est = 0.0, p_est = 0.0;
        const int reserve = lookahead_reserve(mr, w, wn, sizeof(double), lu_diag_us(wn), &tail, 2.0, 2, &u_est, &p_est);
        const bool strassen = (flags & (FF_FLAG_STRASSEN1 | FF_FLAG_STRASSEN2)) != 0;
        if (strassen || tail < 0.01 || mr <= 0 || !update_splittable(mr, mr, false, 0, reserve))
            tail = 0.0;
        else
            tail = round_aligned_tail(update_order_tiles(mr, mr, false, 0, reserve), update_workers(reserve), reserve,
                                      tail, u_est, p_est);
        rc = lu_panel(n, c0 + w, wn, A, lda, info, col_base, side, reserve);
        if (rc) return fail(rc);
        double* C2 = A22 + wn + (int64_t)wn * lda;
        double* X2 = A21 + wn;
        double* Y2 = A12 + (int64_t)wn * lda;
        if (tail > 0.0 &&
            launch_update<double>(mr, mr, w, C2, lda, X2, lda, Y2, lda, false, false, 0, info, side, reserve, reserve,
                                  1.0 - tail, 1.0) != hipSuccess)
            return fail(FF_ERR_HIP);
        hipEvent_t ep2 = evs.make();
        if (!ep2 || hipEventRecord(ep2, side) != hipSuccess) return fail(FF_ERR_HIP);
        if (mr > 0) {
            if (strassen)
                e = lu_product(mr, w, C2, lda, X2, Y2, flags, s2ws, info, st, reserve);
            else
                e = launch_update<double>(mr, mr, w, C2, lda, X2, lda, Y2, lda, false, false, 0, info, st, reserve, 0,
                                          0.0, 1.0 - tail);
            if (e != hipSuccess) return fail(FF_ERR_HIP);
        }
        if (hipStreamWaitEvent(st, ep2, 0) != hipSuccess) return fail(FF_ERR_HIP);
    }
    release_side(dev, side);
    return 0;
}

int lu_blocked(int n, int s, double* A, int64_t lda, unsigned flags, int* info, int col_base, hipStream_t st,
               double* s2ws) {
    if (n > s && !(flags & FF_FLAG_NO_LOOKAHEAD)) return lu_lookahead(n, s, A, lda, flags, info, col_base, st, s2ws);
    return lu_in_order(n, s, A, lda, flags, info, col_base, st, 0, s2ws);
}

int check_common(int64_t n, int64_t s, const void* A, int64_t lda, int dtype, unsigned flags) {
    if (n < 0 || n > (int64_t)INT32_MAX / 2) return -1;
    if (s < 1) return -2;
    if (n > 0 && A == nullptr) return -3;
    if (lda < std::max<int64_t>(1, n)) return -4;
    if (dtype != FF_F64 && dtype != FF_F32 && dtype != FF_BF16) return -5;
    if (flags & ~(unsigned)(FF_FLAG_STRASSEN1 | FF_FLAG_STRASSEN2 | FF_FLAG_NO_LOOKAHEAD | FF_FLAG_FIXED_STEP))
        return -6;
    return 0;
}

// GMRES-IR: restart length (the basis has GM_RESTART + 1 columns, at most the
// 32 the multi-dot kernels take) and the inner tolerance on the preconditioned
// residual relative to its starting norm.
constexpr int GM_RESTART = 30;
constexpr double GM_INNER_TOL = 1e-8;
constexpr int GM_SCAL = 4 * 32;     // device scalars per column: squared norm, h1, h2, y

template <typename S>
struct SolveWs {
    TriWs<S> tri;
    double* diag64;
    int* d_info;
    double* rpart;
    double* R;
    S* D;
    double* rowsum;
    double* norms;
    // GMRES-IR: Krylov basis (n x GM_RESTART + 1), two vectors, partial sums, scalars
    double* V;
    double* t;
    double* d;
    double* mpart;
    double* scal;
    size_t bytes;
};

// Triangular-solve workspace: the control words first, so that the error word
// is the first int32 of the workspace.
template <typename S>
TriWs<S> carve_tri(Carver& cv, int64_t n) {
    TriWs<S> t;
    t.ctl = cv.take<int>(TRI_CTL);
    t.fac = cv.take<S>(trisolve_fac_elems((int)n));
    t.pub = cv.take<S>(trisolve_pub_elems((int)n));
    return t;
}

template <typename S>
SolveWs<S> carve_solve(void* base, int64_t n, int64_t s, int64_t nrhs, int dtype) {
    Carver cv(base);
    SolveWs<S> w;
    w.tri = carve_tri<S>(cv, n);
    w.diag64 = cv.take<double>(diag_ws_bytes(n, s, dtype) / sizeof(double));
    w.d_info = cv.take<int>(1);
    w.rpart = cv.take<double>(residual_part_doubles((int)n));
    w.R = cv.take<double>((size_t)n * (size_t)nrhs);
    w.D = cv.take<S>((size_t)n * (size_t)nrhs);
    w.rowsum = cv.take<double>((size_t)n);
    w.norms = cv.take<double>(3 + 3 * (size_t)nrhs);
    w.V = cv.take<double>((size_t)n * (GM_RESTART + 1) * (size_t)nrhs);
    w.t = cv.take<double>((size_t)n * (size_t)nrhs);
    w.d = cv.take<double>((size_t)n * (size_t)nrhs);
    w.mpart = cv.take<double>(multidot_part_doubles((int)n) * (size_t)nrhs);
    w.scal = cv.take<double>((size_t)GM_SCAL * (size_t)nrhs);
    w.bytes = cv.off;
    return w;
}

// Correction of the active columns of X by left-preconditioned GMRES in binary64:
// per column, solve M^-1 A d = M^-1 r with M = W W^T (the factor in its storage
// precision, applied by the two triangular solves) and r = b - A x, then x += d.
// The columns run in lockstep: one residual, one pair of triangular solves and
// one set of multi-dot launches per Arnoldi step serve all of them, while each
// keeps its own basis, Hessenberg matrix and Givens rotations (on the host) and
// its own stop.  Classical Gram-Schmidt applied twice orthogonalises each new
// vector.  Inactive columns get d = 0.  On return norms[2c], norms[2c + 1] hold
// max|d_c|, max|x_c| (device) and k_used[c] the Krylov steps column c took.
template <typename S>
int gmres_correct(int n, int nr, const double* A64, int64_t lda, const S* W, int64_t ldw, const double* B,
                  int64_t ldb, double* X, int64_t ldx, const SolveWs<S>& w, hipStream_t st, const char* active,
                  int* k_used) {
    const int m = GM_RESTART;
    const int64_t vs = (int64_t)n * (m + 1);      // one column's basis
    const int64_t ps = (int64_t)multidot_part_doubles(n);
    double* V = w.V;
    double* zero_rhs = w.d;                       // n x nr zeros: the matvec is a residual with b = 0
    FF_TRY(launch_fill_double(n * nr, zero_rhs, 0.0, st));
    auto precond = [&](const double* in, int64_t ldi, double* out, int64_t ldo) -> hipError_t {
        // out = W^-T W^-1 in, in the factor's precision, all columns
        hipError_t e = launch_convert_from_f64<S>(n, nr, in, ldi, w.D, n, st);
        if (e == hipSuccess) e = trisolve_impl<S>(n, nr, W, ldw, w.D, n, w.tri, false, st);
        if (e == hipSuccess) e = launch_widen<S>(n, nr, w.D, n, out, ldo, st);
        return e;
    };
    double* sq = w.scal;                          // column c: [c*GM_SCAL] squared norm, +32 h1, +64 h2, +96 y
    double* h1 = w.scal + 32;
    double* h2 = w.scal + 64;
    double* ydev = w.scal + 96;
    // r = b - A x, z = M^-1 r into V_c[:, 0], beta_c^2 = z.z
    FF_TRY(launch_residual_f64(n, nr, A64, lda, X, ldx, B, ldb, w.R, n, nullptr, w.rpart, st));
    FF_TRY(precond(w.R, n, V, vs));
    FF_TRY(launch_multidot(n, nr, 1, V, n, vs, V, vs, w.mpart, sq, GM_SCAL, st));
    std::vector<double> hostv((size_t)nr * GM_SCAL);
    FF_TRY(hipMemcpyAsync(hostv.data(), w.scal, hostv.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    FF_TRY(hipStreamSynchronize(st));
    std::vector<double> beta(nr), H((size_t)nr * (m + 1) * m, 0.0), cs((size_t)nr * m), sn((size_t)nr * m),
        g((size_t)nr * (m + 1), 0.0);
    std::vector<char> done(nr, 1);
    int running = 0;
    for (int c = 0; c < nr; ++c) {
        k_used[c] = 0;
        const double b2 = hostv[(size_t)c * GM_SCAL];
        if (active[c] && b2 > 0.0) {               // else nothing to correct (or an unusable value)
            beta[c] = std::sqrt(b2);
            g[(size_t)c * (m + 1)] = beta[c];
            done[c] = 0;
            ++running;
        }
    }
    FF_TRY(launch_normalize(n, nr, V, vs, sq, GM_SCAL, V, vs, st));
    for (int k = 0; k < m && running > 0; ++k) {
        double* vk = V + (int64_t)k * n;
        double* vn = V + (int64_t)(k + 1) * n;
        // t = -A v_k (a residual with b = 0), vn = M^-1 (-A v_k), then negated
        FF_TRY(launch_residual_f64(n, nr, A64, lda, vk, vs, zero_rhs, n, w.t, n, nullptr, w.rpart, st));
        FF_TRY(precond(w.t, n, vn, vs));
        FF_TRY(launch_negate(n, nr, vn, vs, vn, vs, st));
        FF_TRY(launch_multidot(n, nr, k + 1, V, n, vs, vn, vs, w.mpart, h1, GM_SCAL, st));
        FF_TRY(launch_gemv_add(n, nr, k + 1, V, n, vs, h1, GM_SCAL, -1.0, vn, vs, st));
        FF_TRY(launch_multidot(n, nr, k + 1, V, n, vs, vn, vs, w.mpart, h2, GM_SCAL, st));
        FF_TRY(launch_gemv_add(n, nr, k + 1, V, n, vs, h2, GM_SCAL, -1.0, vn, vs, st));
        FF_TRY(launch_multidot(n, nr, 1, vn, n, vs, vn, vs, w.mpart, sq, GM_SCAL, st));
        FF_TRY(hipMemcpyAsync(hostv.data(), w.scal, hostv.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        FF_TRY(hipStreamSynchronize(st));
        for (int c = 0; c < nr; ++c) {
            if (done[c]) continue;
            const double* hc = &hostv[(size_t)c * GM_SCAL];
            double* col = &H[((size_t)c * m + k) * (m + 1)];   // column k of column c's H, rows 0..k+1
            for (int i = 0; i <= k; ++i) col[i] = hc[32 + i] + hc[64 + i];
            const double hn = std::sqrt(std::max(hc[0], 0.0));
            col[k + 1] = hn;
            double* csc = &cs[(size_t)c * m];
            double* snc = &sn[(size_t)c * m];
            double* gc = &g[(size_t)c * (m + 1)];
            // apply the earlier rotations, then a new one that zeroes col[k + 1]
            for (int i = 0; i < k; ++i) {
                const double a = col[i], b = col[i + 1];
                col[i] = csc[i] * a + snc[i] * b;
                col[i + 1] = -snc[i] * a + csc[i] * b;
            }
            const double rr = std::hypot(col[k], col[k + 1]);
            csc[k] = rr > 0.0 ? col[k] / rr : 1.0;
            snc[k] = rr > 0.0 ? col[k + 1] / rr : 0.0;
            col[k] = rr;
            col[k + 1] = 0.0;
            gc[k + 1] = -snc[k] * gc[k];
            gc[k] = csc[k] * gc[k];
            k_used[c] = k + 1;
            if (std::fabs(gc[k + 1]) <= GM_INNER_TOL * beta[c] || !(hn > 0.0) || !(rr > 0.0)) {
                done[c] = 1;
                --running;
            }
        }
        // columns still running normalise their new vector (a zero norm leaves it as is)
        FF_TRY(launch_normalize(n, nr, vn, vs, sq, GM_SCAL, vn, vs, st));
    }
    // y_c = R_c^-1 g_c (upper triangular k_c x k_c), d_c = V_c y_c, x_c += d_c
    int kmax = 0;
    for (int c = 0; c < nr; ++c) {
        const int kc = k_used[c];
        kmax = std::max(kmax, kc);
        double* yc = &hostv[(size_t)c * GM_SCAL + 96];
        for (int i = 0; i < 32; ++i) yc[i] = 0.0;
        const double* gc = &g[(size_t)c * (m + 1)];
        for (int i = kc - 1; i >= 0; --i) {
            double v = gc[i];
            for (int j = i + 1; j < kc; ++j) v -= H[((size_t)c * m + j) * (m + 1) + i] * yc[j];
            const double dii = H[((size_t)c * m + i) * (m + 1) + i];
            yc[i] = dii != 0.0 ? v / dii : 0.0;
        }
    }
    FF_TRY(hipMemcpyAsync(w.scal, hostv.data(), hostv.size() * sizeof(double), hipMemcpyHostToDevice, st));
    FF_TRY(launch_fill_double(n * nr, w.t, 0.0, st));
    FF_TRY(launch_gemv_add(n, nr, kmax, V, n, vs, ydev, GM_SCAL, 1.0, w.t, n, st));
    FF_TRY(launch_axpy_max_cols<double>(n, nr, w.t, n, X, ldx, w.norms, st));
    FF_TRY(hipStreamSynchronize(st));             // the host copy of y is done before hostv goes
    return 0;
}

template <typename S>
int solve_impl(int n, int s, int nrhs, const double* A64, int64_t lda, S* W, int64_t ldw, int dtype,
               unsigned flags, int w_is_factored, const double* B, int64_t ldb, double* X, int64_t ldx,
               double tol, int max_iter, void* ws, hipStream_t st, ff_solve_info* out) {
    SolveWs<S> w = carve_solve<S>(ws, n, s, nrhs, dtype);
    FF_TRY(launch_set_int(w.tri.ctl, 0, st));
    out->info = 0;
    out->iters = 0;
    out->converged = 0;
    out->dtype_used = dtype;
    out->last_correction = 0.0;
    out->backward_err = 0.0;
    out->krylov_iters = 0;
    if (!w_is_factored) {
        FF_TRY(launch_copy_lower_from_f64<S>(n, A64, lda, W, ldw, st));
        FF_TRY(launch_set_int(w.d_info, 0, st));
        int rc = chol_blocked<S>(n, s, W, ldw, dtype, flags & ~(unsigned)FF_FLAG_GMRES_IR, w.diag64, w.d_info, 0,
                                 st, !(flags & FF_FLAG_NO_LOOKAHEAD));
        if (rc) return rc;
        int info = 0;
        FF_TRY(hipMemcpyAsync(&info, w.d_info, sizeof(int), hipMemcpyDeviceToHost, st));
        FF_TRY(hipStreamSynchronize(st));
        if (info != 0) {
            out->info = info;
            return 0;
        }
    }
    // iteration 0: X = W^-T W^-1 B in the factor's precision
    FF_TRY(launch_convert_from_f64<S>(n, nrhs, B, ldb, w.D, n, st));
    FF_TRY(trisolve_impl<S>(n, nrhs, W, ldw, w.D, n, w.tri, true, st));
    FF_TRY(launch_widen<S>(n, nrhs, w.D, n, X, ldx, st));
    double prev = -1.0;
    double host[2];
    int bad_wait = 0;
    if (flags & FF_FLAG_GMRES_IR) {
        // outer refinement steps, each solving the correction equations of the
        // active columns by preconditioned GMRES; a column leaves on its own stop
        // rule; iters reports the most outer steps of a column
        std::vector<char> active(nrhs, 1);
        std::vector<int> kused(nrhs, 0), its(nrhs, 0);
        std::vector<double> pc(nrhs, -1.0), hn(2 * (size_t)nrhs);
        std::vector<char> conv(nrhs, 0);
        int left = nrhs;
        for (int it = 1; it <= max_iter && left > 0; ++it) {
            int rc = gmres_correct<S>(n, nrhs, A64, lda, W, ldw, B, ldb, X, ldx, w, st, active.data(), kused.data());
            if (rc) return rc;
            FF_TRY(hipMemcpyAsync(hn.data(), w.norms, hn.size() * sizeof(double), hipMemcpyDeviceToHost, st));
            FF_TRY(hipStreamSynchronize(st));
            for (int c = 0; c < nrhs; ++c) {
                if (!active[c]) continue;
                out->krylov_iters += kused[c];
                its[c] = it;
                const double corr = (hn[2 * c + 1] > 0.0) ? hn[2 * c] / hn[2 * c + 1] : hn[2 * c];
                out->last_correction = std::max(out->last_correction, corr);
                if (corr <= tol) {
                    conv[c] = 1;
                    active[c] = 0;
                } else if (!(corr == corr) || (pc[c] >= 0.0 && corr > 0.5 * pc[c])) {
                    active[c] = 0;
                }
                pc[c] = corr;
                if (!active[c]) --left;
            }
        }
        int all_conv = 1, max_it = 0;
        for (int c = 0; c < nrhs; ++c) {
            all_conv &= conv[c];
            max_it = std::max(max_it, its[c]);
        }
        out->iters = max_it;
        out->converged = all_conv;
    }
    for (int it = 1; it <= max_iter && !(flags & FF_FLAG_GMRES_IR); ++it) {
        FF_TRY(launch_residual_f64(n, nrhs, A64, lda, X, ldx, B, ldb, w.R, n, nullptr, w.rpart, st));
        FF_TRY(launch_convert_from_f64<S>(n, nrhs, w.R, n, w.D, n, st));
        FF_TRY(trisolve_impl<S>(n, nrhs, W, ldw, w.D, n, w.tri, false, st));
        FF_TRY(launch_axpy_max<S>(n, nrhs, w.D, n, X, ldx, w.norms, st));
        FF_TRY(hipMemcpyAsync(host, w.norms, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        FF_TRY(hipStreamSynchronize(st));
        out->iters = it;
        const double corr = (host[1] > 0.0) ? host[0] / host[1] : host[0];
        out->last_correction = corr;
        if (corr <= tol) {
            out->converged = 1;
            break;
        }
        if (prev >= 0.0 && corr > 0.5 * prev) break;   // stagnation
        prev = corr;
    }
    // backward error of the returned X
    FF_TRY(launch_residual_f64(n, nrhs, A64, lda, X, ldx, B, ldb, w.R, n, w.rowsum, w.rpart, st));
    FF_TRY(launch_norms(n, nrhs, w.rowsum, X, ldx, nullptr, 0, w.R, n, B, ldb, w.norms, st));
    std::vector<double> nh(3 + 3 * (size_t)nrhs);
    FF_TRY(hipMemcpyAsync(nh.data(), w.norms, nh.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    FF_TRY(hipMemcpyAsync(&bad_wait, w.tri.ctl, sizeof(int), hipMemcpyDeviceToHost, st));
    FF_TRY(hipStreamSynchronize(st));
    if (bad_wait) return FF_ERR_HIP;
    const double anorm = nh[2];
    double be = 0.0;
    for (int c = 0; c < nrhs; ++c) {
        const double den = anorm * nh[4 + 3 * c] + nh[5 + 3 * c];
        const double v = den > 0.0 ? nh[3 + 3 * c] / den : nh[3 + 3 * c];
        be = std::max(be, v);
    }
    out->backward_err = be;
    if (max_iter == 0) out->converged = 0;
    return 0;
}

// Solve with the triangular-solve workspace already carved; clears the error word first.
int trisolve_entry(int64_t n, int64_t nrhs, const void* L, int64_t ldl, int dtype, void* X, int64_t ldx, void* ws,
                   hipStream_t st) {
    Carver cv(ws);
    hipError_t e;
    if (dtype == FF_F64) {
        TriWs<double> t = carve_tri<double>(cv, n);
        e = launch_set_int(t.ctl, 0, st);
        if (e == hipSuccess)
            e = trisolve_impl<double>((int)n, (int)nrhs, static_cast<const double*>(L), ldl, static_cast<double*>(X),
                                      ldx, t, true, st);
    } else {
        TriWs<float> t = carve_tri<float>(cv, n);
        e = launch_set_int(t.ctl, 0, st);
        if (e == hipSuccess)
            e = trisolve_impl<float>((int)n, (int)nrhs, static_cast<const float*>(L), ldl, static_cast<float*>(X), ldx,
                                     t, true, st);
    }
    return e == hipSuccess ? 0 : FF_ERR_HIP;
}

// Scratch of chol_trisolve_noalloc: a file-scope device array (one copy per
// device, held until the process ends).  Host code never passes `scratch`
// itself to a kernel: its device address is taken once per device with
// hipGetSymbolAddress and kept in noalloc_scratch_ptr.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)FF_NOALLOC_SCRATCH_BYTES;
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex noalloc_mu;
void* noalloc_scratch_ptr[NOALLOC_MAX_DEVICES];

int noalloc_scratch(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return FF_ERR_HIP;
    std::lock_guard<std::mutex> lk(noalloc_mu);
    if (noalloc_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return FF_ERR_HIP;
        noalloc_scratch_ptr[dev] = p;
    }
    *out = noalloc_scratch_ptr[dev];
    return 0;
}

// ---------------------------------------------------------------- QR (Algorithm 3)
// Workspace of qr_factor: the panel workgroups' hand-off slots,
// the block product C = B_Q^T M[:, c..] and the split-K partial products.
struct QrWs {
    double* part;
    double* C;
    double* tp;
    size_t bytes;
};

int qr_step(int64_t m, int64_t n, int64_t s) {
    return (int)std::min<int64_t>(std::min<int64_t>(s, n), qr_panel_max_width(m));
}

QrWs carve_qr(void* base, int64_t m, int64_t n, int64_t s) {
    Carver cv(base);
    QrWs w;
    const int ws = qr_step(m, n, s);
    size_t tp = tn_gemm_part_elems((int)n, (int)n, (int)m, true);
    for (int64_t z = 0; z < n; z += ws) {
        const int wb = (int)std::min<int64_t>(ws, n - z);
        const int64_t N = n - z - wb;
        if (N > 0) tp = std::max(tp, tn_gemm_part_elems(wb, (int)N, (int)m, false));
    }
    w.part = cv.take<double>(qr_panel_part_elems(m, ws));
    w.C = cv.take<double>((size_t)ws * (size_t)n);
    w.tp = cv.take<double>(tp);
    w.bytes = cv.off;
    return w;
}

// K rows of one R slab: about what the idle CUs finish, one tile each, while
// a panel of w columns runs (measured at n = 16384: 48 K rows per panel column
// gives the shortest factorisation, against 24 / 32 / 40 / 56).
int qr_slab_k(int m, int w) {
    const int k = std::max(512, (48 * w + 15) / 16 * 16);
    return std::min(k, m);
}

// Algorithm 3 with step ws: Q := A (Q holds M), then per block the in-block
// Gram-Schmidt, the block product C = B_Q^T M[:, c..] and M[:, c..] -= B_Q C;
// finally R = Q^T A.  Every kernel does nothing once *d_info != 0.
//
// R's tile rows need only finished columns of Q, and the in-block Gram-Schmidt
// holds one workgroup on each of P CUs and leaves the rest idle, so R is formed
// by slabs beside the panels: when a panel starts, a side stream takes a group
// of finished tiles (at most one per idle CU) over the next K chunk, stored for
// the first chunk and added for the later ones, in K order; a group is done when
// its chunks cover all m rows.  A slab is sized to end with the panel, so it
// leaves the projections the whole chip.  After the last panel the open group's
// remaining K range and all tiles not yet started are formed on both streams,
// which then join; R's strict lower triangle is cleared last.
int qr_blocked(int m, int n, int ws, const double* A, int64_t lda, double* Q, int64_t ldq, double* R, int64_t ldr,
               const QrWs& w, int* d_info, hipStream_t st) {
    FF_TRY(hipMemcpy2DAsync(Q, (size_t)ldq * sizeof(double), A, (size_t)lda * sizeof(double),
                            (size_t)m * sizeof(double), (size_t)n, hipMemcpyDeviceToDevice, st));
    FF_TRY(launch_qr_part_clear(m, w.part, st));
    const int side_wg = cu_count() - qr_panel_workgroups(m);
    int dev = 0;
    hipStream_t side = nullptr;
    if (n > ws && side_wg >= 32) {
        if (hipGetDevice(&dev) != hipSuccess) return FF_ERR_HIP;
        side = acquire_side(dev);
    }
    Events evs;
    auto fail = [&](int code) {
        if (side) release_side(dev, side);
        return code;
    };
    const int rt = r_slab_tile();
    const int kc = qr_slab_k(m, ws);
    int64_t g0 = 0, g1 = 0;   // the open group of R tiles
    int kpos = 0;             // its next K row
    for (int z = 0; z < n; z += ws) {
        const int wb = std::min(ws, n - z);
        double* Bq = Q + (int64_t)z * ldq;
        if (side && z > 0) {
            bool open = g1 > g0 && kpos < m;
            if (!open) {
                const int64_t avail = r_slab_tiles_before(n, z / rt);
                if (avail > g1) {
                    g0 = g1;
                    g1 = std::min<int64_t>(avail, g0 + side_wg);
                    kpos = 0;
                    open = true;
                }
            }
            if (open) {
                hipEvent_t e = evs.make();
                if (!e || hipEventRecord(e, st) != hipSuccess || hipStreamWaitEvent(side, e, 0) != hipSuccess)
                    return fail(FF_ERR_HIP);
                const int k1 = std::min(m, kpos + kc);
                if (launch_r_slab(n, g0, g1, kpos, k1, Q, ldq, A, lda, R, ldr, d_info, side, side_wg) != hipSuccess)
                    return fail(FF_ERR_HIP);
                kpos = k1;
            }
        }
        if (launch_qr_panel(m, wb, z, Bq, ldq, w.part, d_info, st) != hipSuccess) return fail(FF_ERR_HIP);
        const int N = n - z - wb;
        if (N <= 0) break;
        double* Bm = Q + (int64_t)(z + wb) * ldq;
        if (launch_tn_gemm(wb, N, m, Bq, ldq, Bm, ldq, w.C, wb, false, w.tp, d_info, st) != hipSuccess ||
            launch_update<double>(m, N, wb, Bm, ldq, Bq, ldq, w.C, wb, false, false, 0, d_info, st, 0, 0, 0.0,
                                  1.0) != hipSuccess)
            return fail(FF_ERR_HIP);
    }
    if (!side) {
        FF_TRY(launch_tn_gemm(n, n, m, Q, ldq, A, lda, R, ldr, true, w.tp, d_info, st));
        return 0;
    }
    // Every column of Q is final: the open group's remaining K range on the side
    // stream (after its earlier chunks), the tiles not yet started on the caller's.
    hipEvent_t ef = evs.make();
    if (!ef || hipEventRecord(ef, st) != hipSuccess || hipStreamWaitEvent(side, ef, 0) != hipSuccess)
        return fail(FF_ERR_HIP);
    if (g1 > g0 && kpos < m &&
        launch_r_slab(n, g0, g1, kpos, m, Q, ldq, A, lda, R, ldr, d_info, side, side_wg) != hipSuccess)
        return fail(FF_ERR_HIP);
    if (launch_r_slab(n, g1, r_slab_tiles_before(n, n), 0, m, Q, ldq, A, lda, R, ldr, d_info, st, 0) != hipSuccess)
        return fail(FF_ERR_HIP);
    hipEvent_t ej = evs.make();
    if (!ej || hipEventRecord(ej, side) != hipSuccess || hipStreamWaitEvent(st, ej, 0) != hipSuccess)
        return fail(FF_ERR_HIP);
    release_side(dev, side);
    FF_TRY(launch_zero_strict_lower(n, R, ldr, d_info, st));
    return 0;
}
}  // namespace
}  // namespace ff

using namespace ff;

extern "C" {

const char* ff_status_string(int code) {
    switch (code) {
        case 0: return "success";
        case FF_ERR_HIP: return "HIP runtime error";
        case FF_ERR_WORKSPACE: return "workspace too small";
        case FF_ERR_UNSUPPORTED: return "unsupported argument combination";
        case FF_ERR_SCRATCH: return "problem larger than the static scratch of the allocation-free entry point";
        default: break;
    }
    if (code < 0 && code > -100) return "invalid argument (index = -code)";
    return "unknown status";
}

const char* ff_version(void) { return "fastfact 0.1 gfx950"; }

size_t ff_chol_workspace_size(int64_t n, int64_t s, int dtype, unsigned flags) {
    (void)flags;
    if (n <= 0 || s < 1) return 0;
    return diag_ws_bytes(n, s, dtype);
}

int chol_factor(int64_t n, int64_t s, void* A, int64_t lda, int dtype, unsigned flags, void* ws, size_t ws_bytes,
                int32_t* d_info, void* stream) {
    int rc = check_common(n, s, A, lda, dtype, flags);
    if (rc) return rc;
    if (d_info == nullptr) return -9;
    if ((flags & FF_FLAG_STRASSEN1) && dtype != FF_F64) return FF_ERR_UNSUPPORTED;
    if (flags & FF_FLAG_STRASSEN2) return FF_ERR_UNSUPPORTED;
    const size_t need = ff_chol_workspace_size(n, s, dtype, flags);
    if (need > 0 && (ws == nullptr || ws_bytes < need)) return FF_ERR_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (launch_set_int(d_info, 0, st) != hipSuccess) return FF_ERR_HIP;
    if (n == 0) return 0;
    const int si = (int)std::min<int64_t>(s, n);
    const bool la = !(flags & FF_FLAG_NO_LOOKAHEAD);
    if (dtype == FF_F64)
        return chol_blocked<double>((int)n, si, static_cast<double*>(A), lda, dtype, flags, nullptr, d_info, 0, st,
                                    la);
    return chol_blocked<float>((int)n, si, static_cast<float*>(A), lda, dtype, flags, static_cast<double*>(ws), d_info,
                               0, st, la);
}

size_t ff_lu_workspace_size(int64_t n, int64_t s, int dtype, unsigned flags) {
    if (n <= 0 || s < 1 || dtype != FF_F64 || !(flags & FF_FLAG_STRASSEN2)) return 0;
    return strassen2_ws_doubles((int)n, (int)std::min<int64_t>(s, n)) * sizeof(double);
}
int lu_nopiv_factor(int64_t n, int64_t s, void* A, int64_t lda, int dtype, unsigned flags, void* ws, size_t ws_bytes,
                    int32_t* d_info, void* stream) {
    int rc = check_common(n, s, A, lda, dtype, flags);
    if (rc) return rc;
    if (d_info == nullptr) return -9;
    if (dtype != FF_F64) return FF_ERR_UNSUPPORTED;
    if ((flags & FF_FLAG_STRASSEN1) && (flags & FF_FLAG_STRASSEN2)) return -6;
    const size_t need = ff_lu_workspace_size(n, s, dtype, flags);
    if (need > 0 && (ws == nullptr || ws_bytes < need)) return FF_ERR_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (launch_set_int(d_info, 0, st) != hipSuccess) return FF_ERR_HIP;
    if (n == 0) return 0;
    const int si = (int)std::min<int64_t>(s, n);
    return lu_blocked((int)n, si, static_cast<double*>(A), lda, flags, d_info, 0, st,
                      (flags & FF_FLAG_STRASSEN2) ? static_cast<double*>(ws) : nullptr);
}

size_t ff_qr_workspace_size(int64_t m, int64_t n, int64_t s, int dtype, unsigned flags) {
    (void)dtype; (void)flags;
    if (n <= 0 || m < n || s < 1 || qr_panel_rows(m) == 0) return 0;
    return carve_qr(nullptr, m, n, s).bytes;
}

int qr_factor(int64_t m, int64_t n, int64_t s, const void* A, int64_t lda, void* Q, int64_t ldq, void* R, int64_t ldr,
              int dtype, unsigned flags, void* ws, size_t ws_bytes, int32_t* d_info, void* stream) {
    if (n < 0 || n > (int64_t)INT32_MAX / 2) return -2;
    if (m < n || m > (int64_t)INT32_MAX / 2) return -1;
    if (s < 1) return -3;
    if (n > 0 && A == nullptr) return -4;
    if (lda < std::max<int64_t>(1, m)) return -5;
    if (n > 0 && Q == nullptr) return -6;
    if (ldq < std::max<int64_t>(1, m)) return -7;
    if (n > 0 && R == nullptr) return -8;
    if (ldr < std::max<int64_t>(1, n)) return -9;
    if (dtype != FF_F64 && dtype != FF_F32 && dtype != FF_BF16) return -10;
    if (flags != 0) return -11;
    if (d_info == nullptr) return -14;
    if (dtype != FF_F64) return FF_ERR_UNSUPPORTED;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (launch_set_int(d_info, 0, st) != hipSuccess) return FF_ERR_HIP;
    if (n == 0) return 0;
    if (qr_panel_rows(m) == 0 || !tn_gemm_fits(m, ldq, std::max(ldq, lda)) || !ld_fits(ldq, sizeof(double)) ||
        !ld_fits(ldr, sizeof(double)))
        return FF_ERR_UNSUPPORTED;
    const size_t need = ff_qr_workspace_size(m, n, s, dtype, flags);
    if (ws == nullptr || ws_bytes < need) return FF_ERR_WORKSPACE;
    const QrWs w = carve_qr(ws, m, n, s);
    return qr_blocked((int)m, (int)n, qr_step(m, n, s), static_cast<const double*>(A), lda, static_cast<double*>(Q),
                      ldq, static_cast<double*>(R), ldr, w, d_info, st);
}

int ff_qr_step(int64_t m, int64_t n, int64_t s) {
    if (n <= 0 || m < n || s < 1) return 0;
    return qr_step(m, n, s);
}

size_t ff_solve_workspace_size(int64_t n, int64_t s, int64_t nrhs, int dtype, unsigned flags) {
    if (n <= 0 || nrhs <= 0 || s < 1) return 0;
    if (dtype == FF_F64) return carve_solve<double>(nullptr, n, s, nrhs, dtype).bytes;
    size_t bytes = carve_solve<float>(nullptr, n, s, nrhs, dtype).bytes;
    if (flags & FF_FLAG_ESCALATE)
        bytes += align_up((size_t)n * (size_t)n * sizeof(double)) +
                 carve_solve<double>(nullptr, n, s, nrhs, FF_F64).bytes;
    return bytes;
}

int chol_solve(int64_t n, int64_t s, int64_t nrhs, const double* A64, int64_t lda, void* W, int64_t ldw, int dtype,
               unsigned flags, int w_is_factored, const double* B, int64_t ldb, double* X, int64_t ldx, double tol,
               int max_iter, void* ws, size_t ws_bytes, void* stream, ff_solve_info* out) {
    if (n < 0 || n > (int64_t)INT32_MAX / 2) return -1;
    if (s < 1) return -2;
    if (nrhs < 0) return -3;
    if (n > 0 && A64 == nullptr) return -4;
    if (lda < std::max<int64_t>(1, n)) return -5;
    if (n > 0 && W == nullptr) return -6;
    if (ldw < std::max<int64_t>(1, n)) return -7;
    if (dtype != FF_F64 && dtype != FF_F32 && dtype != FF_BF16) return -8;
    if (flags & ~(unsigned)(FF_FLAG_STRASSEN1 | FF_FLAG_NO_LOOKAHEAD | FF_FLAG_FIXED_STEP | FF_FLAG_ESCALATE |
                             FF_FLAG_GMRES_IR))
        return -9;
    if (n > 0 && nrhs > 0 && B == nullptr) return -11;
    if (ldb < std::max<int64_t>(1, n)) return -12;
    if (n > 0 && nrhs > 0 && X == nullptr) return -13;
    if (ldx < std::max<int64_t>(1, n)) return -14;
    if (!(tol >= 0.0)) return -15;
    if (max_iter < 0) return -16;
    if (out == nullptr) return -20;
    if ((flags & FF_FLAG_STRASSEN1) && dtype != FF_F64) return FF_ERR_UNSUPPORTED;
    memset(out, 0, sizeof(*out));
    out->dtype_used = dtype;
    out->escalated_to = -1;
    if (n == 0 || nrhs == 0) return 0;
    const size_t need = ff_solve_workspace_size(n, s, nrhs, dtype, flags);
    if (ws == nullptr || ws_bytes < need) return FF_ERR_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int si = (int)std::min<int64_t>(s, n);
    const unsigned fflags = flags & ~(unsigned)FF_FLAG_ESCALATE;   // what the factorisations see
    int rc;
    if (dtype == FF_F64)
        rc = solve_impl<double>((int)n, si, (int)nrhs, A64, lda, static_cast<double*>(W), ldw, dtype, fflags,
                                w_is_factored, B, ldb, X, ldx, tol, max_iter, ws, st, out);
    else
        rc = solve_impl<float>((int)n, si, (int)nrhs, A64, lda, static_cast<float*>(W), ldw, dtype, fflags,
                               w_is_factored, B, ldb, X, ldx, tol, max_iter, ws, st, out);
    out->first_info = out->info;
    out->total_iters = out->iters;
    out->escalated_to = -1;
    if (rc != 0 || !(flags & FF_FLAG_ESCALATE) || dtype == FF_F64) return rc;
    auto accepted = [&](const ff_solve_info& o) { return o.info == 0 && (o.converged || o.backward_err <= tol); };
    auto take = [&](const ff_solve_info& o, int to) {
        const int first = out->first_info, total = out->total_iters + o.iters, esc = out->escalations + 1;
        const int kry = out->krylov_iters + o.krylov_iters;
        *out = o;
        out->first_info = first;
        out->total_iters = total;
        out->escalations = esc;
        out->escalated_to = to;
        out->krylov_iters = kry;
    };
    if (accepted(*out)) return 0;
    ff_solve_info o{};
    if (dtype == FF_BF16) {
        rc = solve_impl<float>((int)n, si, (int)nrhs, A64, lda, static_cast<float*>(W), ldw, FF_F32, fflags, 0, B, ldb,
                               X, ldx, tol, max_iter, ws, st, &o);
        if (rc != 0) return rc;
        take(o, FF_F32);
        if (accepted(*out)) return 0;
    }
    Carver cv(static_cast<char*>(ws) + carve_solve<float>(nullptr, n, s, nrhs, dtype).bytes);
    double* W64 = cv.take<double>((size_t)n * (size_t)n);
    void* ws64 = cv.base + cv.off;
    o = ff_solve_info{};
    rc = solve_impl<double>((int)n, si, (int)nrhs, A64, lda, W64, n, FF_F64, fflags, 0, B, ldb, X, ldx, tol, max_iter,
                            ws64, st, &o);
    if (rc != 0) return rc;
    take(o, FF_F64);
    return 0;
}

size_t ff_trisolve_workspace_size(int64_t n, int dtype) {
    if (n <= 0) return 0;
    Carver cv(nullptr);
    if (dtype == FF_F64) (void)carve_tri<double>(cv, n);
    else (void)carve_tri<float>(cv, n);
    return cv.off;
}

int chol_trisolve(int64_t n, int64_t nrhs, const void* L, int64_t ldl, int dtype, void* X, int64_t ldx, void* ws,
                  size_t ws_bytes, void* stream) {
    if (n < 0 || n > (int64_t)INT32_MAX / 2) return -1;
    if (nrhs < 0) return -2;
    if (n > 0 && L == nullptr) return -3;
    if (ldl < std::max<int64_t>(1, n)) return -4;
    if (dtype != FF_F64 && dtype != FF_F32 && dtype != FF_BF16) return -5;
    if (n > 0 && nrhs > 0 && X == nullptr) return -6;
    if (ldx < std::max<int64_t>(1, n)) return -7;
    if (n == 0 || nrhs == 0) return 0;
    if (ws == nullptr || ws_bytes < ff_trisolve_workspace_size(n, dtype)) return FF_ERR_WORKSPACE;
    return trisolve_entry(n, nrhs, L, ldl, dtype, X, ldx, ws, static_cast<hipStream_t>(stream));
}

int chol_trisolve_noalloc(int64_t n, int64_t nrhs, const void* L, int64_t ldl, int dtype, void* X, int64_t ldx,
                          int32_t* d_status, void* stream) {
    if (n < 0 || n > (int64_t)INT32_MAX / 2) return -1;
    if (nrhs < 0) return -2;
    if (n > 0 && L == nullptr) return -3;
    if (ldl < std::max<int64_t>(1, n)) return -4;
    if (dtype != FF_F64 && dtype != FF_F32 && dtype != FF_BF16) return -5;
    if (n > 0 && nrhs > 0 && X == nullptr) return -6;
    if (ldx < std::max<int64_t>(1, n)) return -7;
    if (ff_trisolve_workspace_size(n, dtype) > NOALLOC_SCRATCH_BYTES) return FF_ERR_SCRATCH;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (n == 0 || nrhs == 0) {
        if (d_status != nullptr && launch_set_int(d_status, 0, st) != hipSuccess) return FF_ERR_HIP;
        return 0;
    }
    void* ws = nullptr;
    int rc = noalloc_scratch(&ws);
    if (rc) return rc;
    rc = trisolve_entry(n, nrhs, L, ldl, dtype, X, ldx, ws, st);
    if (rc == 0 && d_status != nullptr && launch_copy_int(static_cast<const int*>(ws), d_status, st) != hipSuccess)
        return FF_ERR_HIP;
    return rc;
}

int ff_update_syrk(int64_t m, int64_t w, void* C, int64_t ldc, const void* P, int64_t ldp, int dtype, unsigned flags,
                   void* stream) {
    if (m < 0 || m > (int64_t)INT32_MAX / 2) return -1;
    if (w < 0 || w > (int64_t)INT32_MAX / 2) return -2;
    if (m > 0 && C == nullptr) return -3;
    if (ldc < std::max<int64_t>(1, m)) return -4;
    if (m > 0 && w > 0 && P == nullptr) return -5;
    if (ldp < std::max<int64_t>(1, m)) return -6;
    if (dtype != FF_F64 && dtype != FF_F32 && dtype != FF_BF16) return -7;
    if (flags & ~(unsigned)(FF_FLAG_STRASSEN1 | FF_FLAG_NO_LOOKAHEAD | FF_FLAG_FIXED_STEP)) return -8;
    if ((flags & FF_FLAG_STRASSEN1) && dtype != FF_F64) return FF_ERR_UNSUPPORTED;
    if (m == 0 || w == 0) return 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e;
    const int mi = (int)m, wi = (int)w;
    if (dtype == FF_F64) {
        const double* Pd = static_cast<const double*>(P);
        if (flags & FF_FLAG_STRASSEN1)
            e = launch_update_syrk_strassen_f64(mi, wi, static_cast<double*>(C), ldc, Pd, ldp, nullptr, st);
        else
            e = launch_update<double>(mi, mi, wi, static_cast<double*>(C), ldc, Pd, ldp, Pd, ldp, true, true, 0,
                                      nullptr, st);
    } else if (dtype == FF_F32) {
        const float* Pf = static_cast<const float*>(P);
        e = launch_update<float>(mi, mi, wi, static_cast<float*>(C), ldc, Pf, ldp, Pf, ldp, true, true, 0, nullptr,
                                 st);
    } else {
        const float* Pf = static_cast<const float*>(P);
        e = launch_update_bf16(mi, mi, wi, static_cast<float*>(C), ldc, Pf, ldp, Pf, ldp, true, 0, nullptr, st);
    }
    return e == hipSuccess ? 0 : FF_ERR_HIP;
}

int ff_update_gemm(int64_t m, int64_t w, void* C, int64_t ldc, const void* X, int64_t ldx, const void* Y, int64_t ldy,
                   int dtype, unsigned flags, void* stream) {
    if (m < 0 || m > (int64_t)INT32_MAX / 2) return -1;
    if (w < 0 || w > (int64_t)INT32_MAX / 2) return -2;
    if (m > 0 && C == nullptr) return -3;
    if (ldc < std::max<int64_t>(1, m)) return -4;
    if (m > 0 && w > 0 && X == nullptr) return -5;
    if (ldx < std::max<int64_t>(1, m)) return -6;
    if (m > 0 && w > 0 && Y == nullptr) return -7;
    if (ldy < std::max<int64_t>(1, w)) return -8;
    if (dtype != FF_F64 && dtype != FF_F32 && dtype != FF_BF16) return -9;
    if (flags & ~(unsigned)(FF_FLAG_STRASSEN1 | FF_FLAG_NO_LOOKAHEAD | FF_FLAG_FIXED_STEP)) return -10;
    if (dtype == FF_BF16) return FF_ERR_UNSUPPORTED;
    if ((flags & FF_FLAG_STRASSEN1) && dtype != FF_F64) return FF_ERR_UNSUPPORTED;
    if (m == 0 || w == 0) return 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (dtype == FF_F64) {
        if (flags & FF_FLAG_STRASSEN1)
            e = launch_update_gemm_strassen_f64((int)m, (int)w, static_cast<double*>(C), ldc,
                                                static_cast<const double*>(X), ldx, static_cast<const double*>(Y), ldy,
                                                nullptr, st);
        else
            e = launch_update<double>((int)m, (int)m, (int)w, static_cast<double*>(C), ldc,
                                      static_cast<const double*>(X), ldx, static_cast<const double*>(Y), ldy, false,
                                      false, 0, nullptr, st);
    } else {
        e = launch_update<float>((int)m, (int)m, (int)w, static_cast<float*>(C), ldc, static_cast<const float*>(X), ldx,
                                 static_cast<const float*>(Y), ldy, false, false, 0, nullptr, st);
    }
    return e == hipSuccess ? 0 : FF_ERR_HIP;
}

int ff_update_profile_enable(int enable) {
    UpdProfile& p = upd_profile();
    std::lock_guard<std::mutex> lk(p.mu);
    if (enable) {
        for (auto& r : p.recs) {
            (void)hipEventDestroy(r.e0);
            (void)hipEventDestroy(r.e1);
        }
        p.recs.clear();
        for (auto& t : p.tally) t = ff_kernel_profile{0, 0.0, 0.0, 0.0};
    }
    p.on = enable != 0;
    return 0;
}

int ff_update_profile_read(ff_kernel_profile out[FF_UPD_NSHAPES]) {
    UpdProfile& p = upd_profile();
    std::lock_guard<std::mutex> lk(p.mu);
    int rc = 0;
    for (auto& r : p.recs) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.e1) != hipSuccess || hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess) rc = FF_ERR_HIP;
        ff_kernel_profile& t = p.tally[r.shape];
        t.launches += 1;
        t.total_ms += ms;
        t.total_flops += r.flops;
        t.total_bytes += r.bytes;
        (void)hipEventDestroy(r.e0);
        (void)hipEventDestroy(r.e1);
    }
    p.recs.clear();
    if (out)
        for (int i = 0; i < FF_UPD_NSHAPES; ++i) out[i] = p.tally[i];
    return rc;
}

}  // extern "C"
