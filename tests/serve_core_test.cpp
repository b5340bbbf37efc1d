// Host-only tests of the serving scheduler (paper_1812_02056_amd/csrc/serve_core.hpp)
// with a fake executor and a fake clock: no device, every "launch" completes a
// fixed number of scheduler iterations after it was enqueued.  Built with
// -fsanitize=address,undefined by tests/test_serve_core_cpu.py.
#include <cassert>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <set>
#include <vector>

#include "serve_core.hpp"

using namespace ffserve;

static int failures = 0;
#define CHECK(c)                                                                 \
    do {                                                                         \
        if (!(c)) {                                                              \
            std::fprintf(stderr, "%s:%d: CHECK failed: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                                          \
        }                                                                        \
    } while (0)

// Fake device: a clock that advances by one per scheduler iteration; work
// enqueued at time t completes at t + latency.  Factor info and refinement
// corrections are scripted per matrix key / request.
struct FakeExec : Executor {
    int64_t now = 0;
    int latency = 2;
    size_t fbytes_per_elem = 8;
    std::map<uint64_t, int> fail_info;        // key -> info of its factorisation
    std::map<int64_t, std::vector<double>> corr_script;   // request id -> corrections per check
    std::map<int64_t, int64_t> check_at, done_at;         // request id -> completion time of the latest check / of the request
    std::map<int64_t, int> checks;            // request id -> checks enqueued
    std::map<int, int> info_mirror;           // info slot -> value
    std::map<int, int64_t> info_ready_at;
    std::set<int64_t> live;                   // requests with handles
    std::vector<uint64_t> factor_order;       // keys in the order their factorisations started
    int64_t arrived = 0, released = 0, steps_launched = 0, solves = 0, refines = 0;
    std::map<int, int> slot_busy_until;

    size_t factor_bytes(int n) const override { return (size_t)n * n * fbytes_per_elem; }
    size_t solve_bytes(int n, int nrhs) const override { return (size_t)n * 64 + (size_t)n * nrhs * 16; }
    int arrive(Request* r) override { live.insert(r->id); ++arrived; r->dev = this; return 0; }
    int start_factor(Request* r) override {
        factor_order.push_back(r->key);
        info_mirror[r->f->info_slot] = 0;
        return 0;
    }
    int step(const std::vector<Request*>& rs, int slot) override {
        CHECK(!rs.empty());
        for (Request* r : rs) CHECK(r->st == FACTOR && r->c0 < r->n);
        ++steps_launched;
        (void)slot;
        return 0;
    }
    int factor_done(Request* r) override {
        auto it = fail_info.find(r->key);
        info_mirror[r->f->info_slot] = it == fail_info.end() ? 0 : it->second;
        info_ready_at[r->f->info_slot] = now + latency;
        return 0;
    }
    int solve(Request* r) override {
        ++solves;
        CHECK(r->f->ready);
        checks[r->id] = 1;
        check_at[r->id] = now + latency;
        return 0;
    }
    int refine_poll(Request* r, bool* ready, double* corr) override {
        *ready = now >= check_at[r->id];
        if (*ready) {
            const std::vector<double>& s = corr_script[r->id];
            const int k = checks[r->id] - 1;
            *corr = s.empty() ? 0.0 : s[std::min<size_t>((size_t)k, s.size() - 1)];
        }
        return 0;
    }
    int refine(Request* r) override {
        ++refines;
        checks[r->id]++;
        check_at[r->id] = now + latency;
        return 0;
    }
    int finish(Request* r) override { done_at[r->id] = now + latency; return 0; }
    bool finished(Request* r) override { return done_at.count(r->id) && now >= done_at[r->id]; }
    int info(const Factor* f, const Request* r) override {
        CHECK(now >= info_ready_at[f->info_slot] || r->hit);
        return info_mirror[f->info_slot];
    }
    double latency_ms(Request* r) override { return (double)(done_at[r->id]); }
    void release(Request* r) override {
        if (r->dev) { live.erase(r->id); ++released; r->dev = nullptr; }
    }
    int slot_wait(int slot) override { CHECK(now >= slot_busy_until[slot] - 1); return 0; }
    int slot_done(int slot) override { slot_busy_until[slot] = now + 1; return 0; }
};

struct Driver {
    FakeExec ex;
    Scheduler sched;
    std::vector<Result> results;
    Driver(size_t arena, const Config& cfg) : sched(&ex, arena, cfg) {}
    int run(int max_steps = 100000) {
        int rc = 0;
        for (int i = 0; i < max_steps; ++i) {
            rc = sched.step();
            if (rc < 0) return rc;
            Result out[64];
            int k = 0;
            do {
                CHECK(sched.poll(out, 64, &k) == 0);
                for (int j = 0; j < k; ++j) results.push_back(out[j]);
            } while (k == 64);
            ex.now++;
            if (rc == 0 && sched.active_count() == 0) return 0;
        }
        return 1;   // did not drain
    }
};

static const double DUMMY[1] = {0.0};
static double XOUT[1];

static int64_t submit(Driver& d, uint64_t key, int n, int nrhs = 1) {
    int64_t id = -1;
    const int rc = d.sched.submit(key, n, DUMMY, n, DUMMY, nrhs, n, XOUT, n, &id);
    CHECK(rc == 0);
    return id;
}

static void test_fifo_cache_and_accounting() {
    Config cfg;
    cfg.step_cols = 64;
    Driver d(1 << 24, cfg);
    const int64_t a = submit(d, 1, 300);
    const int64_t b = submit(d, 2, 200);
    const int64_t c = submit(d, 1, 300);     // repeat of a while a is still factoring
    CHECK(d.run() == 0);
    CHECK(d.results.size() == 3);
    std::map<int64_t, Result> by;
    for (const Result& r : d.results) by[r.id] = r;
    CHECK(by[a].cache_hit == 0 && by[b].cache_hit == 0 && by[c].cache_hit == 1);
    CHECK(by[a].info == 0 && by[c].info == 0);
    CHECK(d.ex.factor_order == (std::vector<uint64_t>{1, 2}));   // one factorisation per key, in arrival order
    CHECK(d.sched.stats().cache_hits == 1);
    CHECK(d.sched.stats().completed == 3);
    // both keyed factors stay resident; everything else returned to the arena
    CHECK(d.sched.resident_count() == 2);
    CHECK(d.sched.arena_free() == d.sched.arena_size() - align_up(300 * 300 * 8) - align_up(200 * 200 * 8));
    CHECK(d.ex.live.empty() && d.ex.arrived == d.ex.released);
}

static void test_lru_eviction_and_in_use_factors() {
    Config cfg;
    cfg.step_cols = 64;
    // room for two 256-factors and their workspaces, not three
    FakeExec probe;
    const size_t one = align_up(probe.factor_bytes(256)) + align_up(probe.solve_bytes(256, 1));
    Driver d(2 * one + one / 2, cfg);
    submit(d, 10, 256);
    submit(d, 11, 256);
    CHECK(d.run() == 0);
    CHECK(d.sched.resident_count() == 2);
    submit(d, 10, 256);                       // touch 10: 11 becomes least recently used
    CHECK(d.run() == 0);
    submit(d, 12, 256);                       // needs room: evicts 11, not 10
    CHECK(d.run() == 0);
    CHECK(d.sched.stats().evictions >= 1);
    std::set<uint64_t> keys;
    for (Factor* f : d.sched.resident()) keys.insert(f->key);
    CHECK(keys.count(10) == 1 && keys.count(12) == 1 && keys.count(11) == 0);
    // a request for the evicted key is factored again
    const size_t before = d.ex.factor_order.size();
    submit(d, 11, 256);
    CHECK(d.run() == 0);
    CHECK(d.ex.factor_order.size() == before + 1);
}

static void test_failed_factor_is_not_served_again() {
    Config cfg;
    cfg.step_cols = 64;
    Driver d(1 << 24, cfg);
    d.ex.fail_info[7] = 13;
    const int64_t a = submit(d, 7, 128);
    CHECK(d.run() == 0);
    CHECK(d.results.size() == 1 && d.results[0].id == a && d.results[0].info == 13);
    CHECK(d.sched.resident_count() == 0 && d.sched.live_factors() == 0);
    CHECK(d.sched.arena_free() == d.sched.arena_size());
    d.ex.fail_info.erase(7);
    submit(d, 7, 128);                        // factored again, not a cache hit
    CHECK(d.run() == 0);
    CHECK(d.results.size() == 2 && d.results[1].cache_hit == 0 && d.results[1].info == 0);
}

static void test_refinement_stops() {
    Config cfg;
    cfg.step_cols = 64;
    cfg.refine = true;
    cfg.tol = 1e-12;
    cfg.max_iter = 6;
    Driver d(1 << 24, cfg);
    const int64_t conv = submit(d, 0, 100);
    const int64_t stag = submit(d, 0, 100);
    const int64_t lim = submit(d, 0, 100);
    const int64_t nan = submit(d, 0, 100);
    d.ex.corr_script[conv] = {1e-6, 1e-9, 1e-13};
    d.ex.corr_script[stag] = {1e-6, 1e-9, 0.9e-9};              // shrank by less than half
    d.ex.corr_script[lim] = {1e-1, 4e-2, 1.6e-2, 6.4e-3, 2.5e-3, 1e-3, 4e-4};
    d.ex.corr_script[nan] = {std::nan("")};
    CHECK(d.run() == 0);
    std::map<int64_t, Result> by;
    for (const Result& r : d.results) by[r.id] = r;
    CHECK(by[conv].converged == 1 && by[conv].iters == 3);
    CHECK(by[stag].converged == 0 && by[stag].iters == 3);
    CHECK(by[lim].converged == 0 && by[lim].iters == 6);
    CHECK(by[nan].converged == 0 && by[nan].iters == 1);
    CHECK(d.ex.solves == 4);
}

static void test_tight_arena_drains_without_livelock() {
    Config cfg;
    cfg.step_cols = 32;
    FakeExec probe;
    const size_t big = align_up(probe.factor_bytes(512)) + align_up(probe.solve_bytes(512, 8));
    Driver d(big + 4096, cfg);                // exactly one of the largest request at a time
    srand(5);
    std::vector<int64_t> ids;
    for (int i = 0; i < 200; ++i) {
        const int n = 16 + rand() % 497;
        const uint64_t key = (rand() % 3 == 0 && i > 0) ? (uint64_t)(1 + rand() % (i + 1)) : (uint64_t)(i + 1);
        ids.push_back(submit(d, key, n, 1 + rand() % 8));
    }
    CHECK(d.run(200000) == 0);
    CHECK(d.results.size() == ids.size());
    // admission is first come, first served: results of new factorisations come in order
    CHECK(d.sched.stats().completed == (int64_t)ids.size());
    CHECK(d.ex.live.empty());
    size_t resident_bytes = 0;
    for (Factor* f : d.sched.resident()) resident_bytes += align_up(f->bytes);
    CHECK(d.sched.arena_free() == d.sched.arena_size() - resident_bytes);
}

static void test_never_fits_is_rejected_at_submit() {
    Config cfg;
    Driver d(1 << 20, cfg);
    int64_t id = -1;
    CHECK(d.sched.submit(1, 4096, DUMMY, 4096, DUMMY, 1, 4096, XOUT, 4096, &id) == ERR_WORKSPACE);
    CHECK(d.sched.queued_count() == 0);
}

static void test_max_active_respected() {
    Config cfg;
    cfg.max_active = 3;
    cfg.step_cols = 16;
    Driver d(1 << 26, cfg);
    for (int i = 0; i < 20; ++i) submit(d, (uint64_t)(i + 1), 64);
    int max_seen = 0;
    for (int i = 0; i < 10000 && d.sched.stats().completed < 20; ++i) {
        CHECK(d.sched.step() >= 0);
        max_seen = std::max(max_seen, (int)d.sched.active_count());
        Result out[8];
        int k = 0;
        d.sched.poll(out, 8, &k);
        d.ex.now++;
    }
    CHECK(d.sched.stats().completed == 20);
    CHECK(max_seen <= 3);
}

int main() {
    test_fifo_cache_and_accounting();
    test_lru_eviction_and_in_use_factors();
    test_failed_factor_is_not_served_again();
    test_refinement_stops();
    test_tight_arena_drains_without_livelock();
    test_never_fits_is_rejected_at_submit();
    test_max_active_respected();
    if (failures) {
        std::fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("serve_core: all checks passed\n");
    return 0;
}
