// serve.hip -- continuous batching of many independent SPD solves.
//
// Each request is Algorithm 1 of arXiv 1812.02056 (Sec. 2) on its own matrix,
// followed by the two triangular solves (solving linear systems being the
// use of the factorisation, Introduction).  The scheduling (arena, resident
// factors, admission, the stage of every request) is serve_core.hpp; this file
// is its device side: one scheduler iteration advances every admitted
// factorisation by one block with three grouped launches (diagonal blocks,
// panel solves, trailing updates of all active matrices) and runs the solves.
//
// Two precisions:
//   FF_F64  factors in binary64, one forward and one backward solve;
//   FF_F32  factors stored in binary32 (diagonal blocks factored in binary64,
//           panel solves and updates in binary32), solves refined in binary64
//           against the request's A: each iteration computes R = B - A X,
//           solves with the factor, adds the correction and copies
//           ||dX||_inf / ||X||_inf to the host, where the scheduler decides on
//           the next iteration at a later scheduler iteration, without waiting.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "fastfact.h"
#include "internal.hpp"
#include "serve_core.hpp"

namespace ff {
namespace {

using ffserve::align_up;

constexpr int MAX_ACTIVE = 512;      // admitted requests (job-table capacity, host slots)
constexpr int MAX_FACTORS = 8192;    // live factors (info words)
constexpr int RING = 4;              // job-table slots in flight
constexpr size_t TAB_BYTES = MAX_ACTIVE * (sizeof(GroupDiag) + sizeof(GroupTrsm) + sizeof(GroupUpd)) + 3 * 256;

// Pinned host slot of an admitted request: the last refinement check and the
// triangular solves' error word.
struct HostSlot {
    double norms[2];     // max |dX|, max |X|
    int err;
    int pad;
};

struct Handles {
    hipEvent_t t_arrive = nullptr, t_done = nullptr, t_check = nullptr;
};

// Workspace of a request's solve, carved from its arena block.
struct SolveWs {
    int* ctl;            // triangular-solve control words (ctl[0]: error word)
    void* fac;
    void* pub;
    double* R;           // n x nrhs residual (binary32 mode)
    float* D;            // n x nrhs correction in the factor's precision
    double* rpart;       // residual partial sums
    double* norms;       // 2 doubles
    size_t bytes;
};

SolveWs carve(char* base, int n, int nrhs, int dtype) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += align_up(bytes ? bytes : 1);
        return p;
    };
    const size_t es = dtype == FF_F64 ? sizeof(double) : sizeof(float);
    SolveWs w{};
    w.ctl = reinterpret_cast<int*>(take(TRI_CTL * sizeof(int)));
    w.fac = take(trisolve_fac_elems(n) * es);
    w.pub = take(trisolve_pub_elems(n) * es);
    if (dtype != FF_F64) {
        w.R = reinterpret_cast<double*>(take((size_t)n * nrhs * sizeof(double)));
        w.D = reinterpret_cast<float*>(take((size_t)n * nrhs * sizeof(float)));
        w.rpart = reinterpret_cast<double*>(take(residual_part_doubles(n) * sizeof(double)));
        w.norms = reinterpret_cast<double*>(take(4 * sizeof(double)));
    }
    w.bytes = off;
    return w;
}

class HipExecutor : public ffserve::Executor {
public:
    hipStream_t st = nullptr;      // all server work
    hipStream_t clock = nullptr;   // idle stream: arrival stamps
    char* base = nullptr;
    int dtype = FF_F64;
    int* d_info = nullptr;
    int* h_info = nullptr;
    HostSlot* h_slot = nullptr;
    void* h_tab[RING] = {};
    void* d_tab[RING] = {};
    hipEvent_t tab_ev[RING] = {};

    int init(void* arena, void* stream, int dt) {
        st = static_cast<hipStream_t>(stream);
        base = static_cast<char*>(arena);
        dtype = dt;
        if (hipStreamCreateWithFlags(&clock, hipStreamNonBlocking) != hipSuccess ||
            hipMalloc(&d_info, MAX_FACTORS * sizeof(int)) != hipSuccess ||
            hipHostMalloc(&h_info, MAX_FACTORS * sizeof(int)) != hipSuccess ||
            hipHostMalloc(&h_slot, MAX_ACTIVE * sizeof(HostSlot)) != hipSuccess)
            return FF_ERR_HIP;
        for (int i = 0; i < RING; ++i)
            if (hipHostMalloc(&h_tab[i], TAB_BYTES) != hipSuccess || hipMalloc(&d_tab[i], TAB_BYTES) != hipSuccess ||
                hipEventCreateWithFlags(&tab_ev[i], hipEventDisableTiming) != hipSuccess)
                return FF_ERR_HIP;
        memset(h_slot, 0, MAX_ACTIVE * sizeof(HostSlot));
        return 0;
    }
    ~HipExecutor() override {
        if (st) (void)hipStreamSynchronize(st);
        for (int i = 0; i < RING; ++i) {
            if (h_tab[i]) (void)hipHostFree(h_tab[i]);
            if (d_tab[i]) (void)hipFree(d_tab[i]);
            if (tab_ev[i]) (void)hipEventDestroy(tab_ev[i]);
        }
        if (d_info) (void)hipFree(d_info);
        if (h_info) (void)hipHostFree(h_info);
        if (h_slot) (void)hipHostFree(h_slot);
        if (clock) (void)hipStreamDestroy(clock);
    }

    size_t es() const { return dtype == FF_F64 ? sizeof(double) : sizeof(float); }
    size_t factor_bytes(int n) const override { return (size_t)n * (size_t)n * es(); }
    size_t solve_bytes(int n, int nrhs) const override { return carve(nullptr, n, nrhs, dtype).bytes; }
    char* factor_ptr(const ffserve::Factor* f) const { return base + f->off; }

    int arrive(ffserve::Request* r) override {
        Handles* h = new (std::nothrow) Handles();
        if (!h) return FF_ERR_HIP;
        r->dev = h;
        if (hipEventCreate(&h->t_arrive) != hipSuccess || hipEventCreate(&h->t_done) != hipSuccess ||
            hipEventCreateWithFlags(&h->t_check, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(h->t_arrive, clock) != hipSuccess)
            return FF_ERR_HIP;
        return 0;
    }

    int start_factor(ffserve::Request* r) override {
        const ffserve::Factor* f = r->f;
        if (dtype == FF_F64) {
            // the factor starts as a copy of A (lower triangle read)
            if (hipMemcpy2DAsync(factor_ptr(f), (size_t)r->n * sizeof(double), r->A, (size_t)r->lda * sizeof(double),
                                 (size_t)r->n * sizeof(double), r->n, hipMemcpyDeviceToDevice, st) != hipSuccess)
                return FF_ERR_HIP;
        } else if (launch_copy_lower_from_f64<float>(r->n, r->A, r->lda, reinterpret_cast<float*>(factor_ptr(f)), r->n,
                                                     st) != hipSuccess) {
            return FF_ERR_HIP;
        }
        return launch_set_int(d_info + f->info_slot, 0, st) == hipSuccess ? 0 : FF_ERR_HIP;
    }

    template <typename S>
    int step_typed(const std::vector<ffserve::Request*>& rs, int slot) {
        char* h = static_cast<char*>(h_tab[slot]);
        char* d = static_cast<char*>(d_tab[slot]);
        const size_t o1 = align_up(MAX_ACTIVE * sizeof(GroupDiag));
        const size_t o2 = o1 + align_up(MAX_ACTIVE * sizeof(GroupTrsm));
        GroupDiag* hd = reinterpret_cast<GroupDiag*>(h);
        GroupTrsm* ht = reinterpret_cast<GroupTrsm*>(h + o1);
        GroupUpd* hu = reinterpret_cast<GroupUpd*>(h + o2);
        int nd = 0, nt = 0, nu = 0, wg = 0, tiles = 0;
        const int rows_wg = trsm_rows_per_wg(), ut = grouped_update_tile();
        for (ffserve::Request* r : rs) {
            const int n = r->n, c0 = r->c0, w = std::min(r->s, n - c0), m = n - c0 - w;
            S* L = reinterpret_cast<S*>(factor_ptr(r->f));
            int* info = d_info + r->f->info_slot;
            S* A11 = L + c0 + (int64_t)c0 * n;
            hd[nd++] = GroupDiag{A11, n, w, c0, info};
            if (m > 0) {
                S* A21 = L + (c0 + w) + (int64_t)c0 * n;
                const int nwg = std::min((m + rows_wg - 1) / rows_wg, 64);
                ht[nt++] = GroupTrsm{A21, A11, n, m, w, wg, nwg, info};
                wg += nwg;
                const int nb = (m + ut - 1) / ut;
                hu[nu++] = GroupUpd{L + (c0 + w) + (int64_t)(c0 + w) * n, A21, n, m, w, tiles, info};
                tiles += nb * (nb + 1) / 2;
            }
        }
        if (nd == 0) return 0;
        if (hipMemcpyAsync(d, h, TAB_BYTES, hipMemcpyHostToDevice, st) != hipSuccess) return FF_ERR_HIP;
        if (launch_potrf_grouped<S>(nd, reinterpret_cast<const GroupDiag*>(d), st) != hipSuccess ||
            launch_trsm_grouped<S>(nt, wg, reinterpret_cast<const GroupTrsm*>(d + o1), st) != hipSuccess ||
            launch_update_grouped<S>(nu, tiles, reinterpret_cast<const GroupUpd*>(d + o2), st) != hipSuccess)
            return FF_ERR_HIP;
        return 0;
    }
    int step(const std::vector<ffserve::Request*>& rs, int slot) override {
        return dtype == FF_F64 ? step_typed<double>(rs, slot) : step_typed<float>(rs, slot);
    }

    int factor_done(ffserve::Request* r) override {
        const int k = r->f->info_slot;
        return hipMemcpyAsync(h_info + k, d_info + k, sizeof(int), hipMemcpyDeviceToHost, st) == hipSuccess ? 0
                                                                                                          : FF_ERR_HIP;
    }

    SolveWs ws_of(const ffserve::Request* r) const { return carve(base + r->ws_off, r->n, r->nrhs, dtype); }

    int solve(ffserve::Request* r) override {
        const int n = r->n, nrhs = r->nrhs;
        if (dtype == FF_F64) {
            const double* L = reinterpret_cast<const double*>(factor_ptr(r->f));
            if (hipMemcpy2DAsync(r->X, (size_t)r->ldx * sizeof(double), r->B, (size_t)r->ldb * sizeof(double),
                                 (size_t)n * sizeof(double), nrhs, hipMemcpyDeviceToDevice, st) != hipSuccess)
                return FF_ERR_HIP;
            return chol_trisolve(n, nrhs, L, n, FF_F64, r->X, r->ldx, base + r->ws_off, r->ws_bytes, st);
        }
        const SolveWs w = ws_of(r);
        const float* W = reinterpret_cast<const float*>(factor_ptr(r->f));
        const TriWs<float> tri{w.ctl, static_cast<float*>(w.fac), static_cast<float*>(w.pub)};
        if (launch_set_int(w.ctl, 0, st) != hipSuccess ||
            launch_convert_from_f64<float>(n, nrhs, r->B, r->ldb, w.D, n, st) != hipSuccess ||
            trisolve_impl<float>(n, nrhs, W, n, w.D, n, tri, true, st) != hipSuccess ||
            launch_widen<float>(n, nrhs, w.D, n, r->X, r->ldx, st) != hipSuccess)
            return FF_ERR_HIP;
        return refine(r);
    }

    // One binary64 refinement iteration, then its correction norms to the host.
    int refine(ffserve::Request* r) override {
        const int n = r->n, nrhs = r->nrhs;
        const SolveWs w = ws_of(r);
        const float* W = reinterpret_cast<const float*>(factor_ptr(r->f));
        const TriWs<float> tri{w.ctl, static_cast<float*>(w.fac), static_cast<float*>(w.pub)};
        Handles* h = static_cast<Handles*>(r->dev);
        if (launch_residual_f64(n, nrhs, r->A, r->lda, r->X, r->ldx, r->B, r->ldb, w.R, n, nullptr, w.rpart, st) !=
                hipSuccess ||
            launch_convert_from_f64<float>(n, nrhs, w.R, n, w.D, n, st) != hipSuccess ||
            trisolve_impl<float>(n, nrhs, W, n, w.D, n, tri, false, st) != hipSuccess ||
            launch_axpy_max<float>(n, nrhs, w.D, n, r->X, r->ldx, w.norms, st) != hipSuccess ||
            hipMemcpyAsync(h_slot[r->slot].norms, w.norms, 2 * sizeof(double), hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipEventRecord(h->t_check, st) != hipSuccess)
            return FF_ERR_HIP;
        return 0;
    }

    int refine_poll(ffserve::Request* r, bool* ready, double* corr) override {
        Handles* h = static_cast<Handles*>(r->dev);
        const hipError_t e = hipEventQuery(h->t_check);
        if (e == hipErrorNotReady) {
            *ready = false;
            return 0;
        }
        if (e != hipSuccess) return FF_ERR_HIP;
        const HostSlot& hs = h_slot[r->slot];
        *ready = true;
        *corr = hs.norms[1] > 0.0 ? hs.norms[0] / hs.norms[1] : hs.norms[0];
        return 0;
    }

    int finish(ffserve::Request* r) override {
        Handles* h = static_cast<Handles*>(r->dev);
        const int* err = dtype == FF_F64 ? reinterpret_cast<const int*>(base + r->ws_off) : ws_of(r).ctl;
        if (hipMemcpyAsync(&h_slot[r->slot].err, err, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipEventRecord(h->t_done, st) != hipSuccess)
            return FF_ERR_HIP;
        return 0;
    }

    bool finished(ffserve::Request* r) override {
        return hipEventQuery(static_cast<Handles*>(r->dev)->t_done) == hipSuccess;
    }

    int info(const ffserve::Factor* f, const ffserve::Request* r) override {
        if (h_slot[r->slot].err != 0) return FF_ERR_HIP;
        return h_info[f->info_slot];
    }

    double latency_ms(ffserve::Request* r) override {
        Handles* h = static_cast<Handles*>(r->dev);
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, h->t_arrive, h->t_done);
        return (double)ms;
    }

    void release(ffserve::Request* r) override {
        Handles* h = static_cast<Handles*>(r->dev);
        if (!h) return;
        if (h->t_arrive) (void)hipEventDestroy(h->t_arrive);
        if (h->t_done) (void)hipEventDestroy(h->t_done);
        if (h->t_check) (void)hipEventDestroy(h->t_check);
        delete h;
        r->dev = nullptr;
    }

    int slot_wait(int slot) override { return hipEventSynchronize(tab_ev[slot]) == hipSuccess ? 0 : FF_ERR_HIP; }
    int slot_done(int slot) override { return hipEventRecord(tab_ev[slot], st) == hipSuccess ? 0 : FF_ERR_HIP; }
};

}  // namespace
}  // namespace ff

using namespace ff;

struct ff_server {
    HipExecutor ex;
    ffserve::Scheduler* sched = nullptr;
};

extern "C" {

ff_server* ff_server_create(void* arena, size_t arena_bytes, int dtype, void* stream, int* status) {
    int rc = 0;
    if (arena_bytes > 0 && arena == nullptr) rc = -1;
    if (!rc && dtype != FF_F64 && dtype != FF_F32) rc = dtype == FF_BF16 ? FF_ERR_UNSUPPORTED : -3;
    ff_server* s = nullptr;
    if (!rc) {
        s = new (std::nothrow) ff_server();
        if (!s) rc = FF_ERR_HIP;
    }
    if (!rc) rc = s->ex.init(arena, stream, dtype);
    if (!rc) {
        ffserve::Config cfg;
        cfg.max_active = MAX_ACTIVE;
        cfg.max_factors = MAX_FACTORS;
        cfg.ring = RING;
        cfg.step_cols = LDS_DIAG_MAX;
        cfg.refine = dtype != FF_F64;
        cfg.tol = 1e-12;
        cfg.max_iter = 30;
        s->sched = new (std::nothrow) ffserve::Scheduler(&s->ex, arena_bytes, cfg);
        if (!s->sched) rc = FF_ERR_HIP;
    }
    if (status) *status = rc;
    if (rc && s) {
        ff_server_destroy(s);
        return nullptr;
    }
    return s;
}

int ff_server_destroy(ff_server* s) {
    if (!s) return 0;
    if (s->ex.st) (void)hipStreamSynchronize(s->ex.st);
    delete s->sched;
    delete s;
    return 0;
}

int ff_server_submit(ff_server* s, uint64_t key, int64_t n, const double* A, int64_t lda, const double* B,
                     int64_t nrhs, int64_t ldb, double* X, int64_t ldx, int64_t* req_id) {
    if (!s) return -1;
    if (n < 1 || n > 65536) return -3;
    if (!A) return -4;
    if (lda < n) return -5;
    if (!B) return -6;
    if (nrhs < 1 || nrhs > 65536) return -7;
    if (ldb < n) return -8;
    if (!X) return -9;
    if (ldx < n) return -10;
    return s->sched->submit(key, (int)n, A, lda, B, (int)nrhs, ldb, X, ldx, req_id);
}

int ff_server_step(ff_server* s) {
    if (!s) return -1;
    return s->sched->step();
}

int ff_server_poll(ff_server* s, ff_server_result* out, int max_out, int* n_out) {
    if (!s) return -1;
    if (max_out < 0 || (max_out > 0 && !out)) return -2;
    std::vector<ffserve::Result> res((size_t)max_out);
    int k = 0;
    const int rc = s->sched->poll(res.data(), max_out, &k);
    for (int i = 0; i < k; ++i)
        out[i] = ff_server_result{res[i].id, res[i].info, res[i].cache_hit, res[i].latency_ms, res[i].iters,
                                  res[i].converged};
    if (n_out) *n_out = k;
    return rc;
}

int ff_server_get_stats(ff_server* s, ff_server_stats* out) {
    if (!s || !out) return -1;
    const ffserve::Stats& st = s->sched->stats();
    out->submitted = st.submitted;
    out->completed = st.completed;
    out->steps = st.steps;
    out->grouped_launches = st.grouped_launches;
    out->cache_hits = st.cache_hits;
    out->evictions = st.evictions;
    out->arena_free = (int64_t)s->sched->arena_free();
    out->resident_factors = (int64_t)s->sched->resident_count();
    out->queued = (int64_t)s->sched->queued_count();
    out->active = (int64_t)s->sched->active_count();
    return 0;
}

}  // extern "C"
