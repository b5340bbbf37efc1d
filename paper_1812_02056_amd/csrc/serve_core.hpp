// serve_core.hpp -- host-side scheduler of the serving interface.
//
// Many independent SPD systems A_i X_i = B_i, each factored by Algorithm 1 of
// arXiv 1812.02056 (Sec. 2) and solved with its factor.  This header holds the
// scheduling only, with no device code: the arena (first-fit with coalescing,
// the HBM budget), the resident-factor cache (least recently used first out
// when space is needed), admission in arrival order, and the stage of each
// request (queued, factoring one block per scheduler iteration, waiting on a
// factor another request computes, solving, refining, done).  Device work goes
// through an Executor; serve.hip implements it with HIP, and the CPU tests
// drive the same code with a fake executor and clock.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <iterator>
#include <list>
#include <map>
#include <new>
#include <vector>

namespace ffserve {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// Status codes (the library's FF_ERR_* values).
constexpr int ERR_HIP = -100;
constexpr int ERR_WORKSPACE = -101;

// First-fit allocator over [0, size) with coalescing on free.
struct Arena {
    size_t size = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    void init(size_t n) {
        size = n;
        free_.clear();
        if (n) free_[0] = n;
    }
    bool alloc(size_t n, size_t& off) {
        n = align_up(n ? n : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                off = it->first;
                const size_t rest = it->second - n;
                free_.erase(it);
                if (rest) free_[off + n] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = align_up(n ? n : 1);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t free_bytes() const {
        size_t s = 0;
        for (auto& kv : free_) s += kv.second;
        return s;
    }
};

struct Factor {            // a factor buffer in the arena
    uint64_t key = 0;
    int n = 0;
    size_t off = 0, bytes = 0;
    int users = 0;         // requests that read or write it
    bool ready = false;    // factorisation finished (enqueued)
    bool dead = false;     // failed or unkeyed: freed when the last user is done
    int info_slot = -1;
};

enum Stage { QUEUED, FACTOR, WAIT_FACTOR, SOLVE, REFINE, DONE };

struct Request {
    int64_t id = 0;
    uint64_t key = 0;
    int n = 0, nrhs = 0;
    const double* A = nullptr;
    int64_t lda = 0;
    const double* B = nullptr;
    int64_t ldb = 0;
    double* X = nullptr;
    int64_t ldx = 0;
    Stage st = QUEUED;
    Factor* f = nullptr;
    bool owner = false;    // this request computes f
    int s = 0, c0 = 0;     // step and next column of the factorisation
    size_t ws_off = 0, ws_bytes = 0;
    int slot = -1;         // per-request host slot of the executor
    bool hit = false;
    int iters = 0;         // refinement iterations enqueued
    double prev_corr = -1.0;
    bool converged = false;
    void* dev = nullptr;   // executor's handles
};

struct Result {
    int64_t id;
    int info;              // factorisation info; < 0: a device error (ERR_HIP)
    int cache_hit;
    int iters;
    int converged;
    double latency_ms;
};

struct Stats {
    int64_t submitted = 0, completed = 0, steps = 0, grouped_launches = 0, cache_hits = 0, evictions = 0;
};

struct Config {
    int max_active = 512;      // admitted requests at once (job tables, host slots)
    int max_factors = 8192;    // live factors (info words)
    int ring = 4;              // job tables in flight
    int step_cols = 192;       // columns per factorisation step
    bool refine = false;       // solves are refined (binary32 factors)
    double tol = 1e-12;        // refinement stop: ||dX|| <= tol ||X||
    int max_iter = 30;
};

// What the scheduler asks of the device.  Every call only enqueues work,
// except the non-blocking queries and slot_wait.
class Executor {
public:
    virtual ~Executor() {}
    virtual size_t factor_bytes(int n) const = 0;              // arena bytes of a factor of order n
    virtual size_t solve_bytes(int n, int nrhs) const = 0;     // arena bytes of a solve's workspace
    virtual int arrive(Request* r) = 0;                        // stamp the arrival, create handles
    virtual int start_factor(Request* r) = 0;                  // factor buffer := A, info := 0
    virtual int step(const std::vector<Request*>& rs, int slot) = 0;  // one block step of each (grouped)
    virtual int factor_done(Request* r) = 0;                   // copy the factor's info to the host
    virtual int solve(Request* r) = 0;                         // the solve (and, refining, its first check)
    virtual int refine_poll(Request* r, bool* ready, double* corr) = 0;   // latest check, non-blocking
    virtual int refine(Request* r) = 0;                        // one more iteration and check
    virtual int finish(Request* r) = 0;                        // mark the request's end on the device
    virtual bool finished(Request* r) = 0;                     // device done with it (non-blocking)
    virtual int info(const Factor* f, const Request* r) = 0;   // host mirror of info (or ERR_HIP)
    virtual double latency_ms(Request* r) = 0;
    virtual void release(Request* r) = 0;                      // destroy the request's handles
    virtual int slot_wait(int slot) = 0;                       // job table `slot` free again
    virtual int slot_done(int slot) = 0;                       // mark its use by this iteration
};

class Scheduler {
public:
    Scheduler(Executor* ex, size_t arena_bytes, const Config& cfg) : ex_(ex), cfg_(cfg) {
        arena_.init(arena_bytes);
        for (int i = cfg.max_factors - 1; i >= 0; --i) free_info_.push_back(i);
        for (int i = cfg.max_active - 1; i >= 0; --i) free_slot_.push_back(i);
        slot_used_.assign((size_t)std::max(1, cfg.ring), 0);
    }
    ~Scheduler() {
        for (Request* r : active_) { ex_->release(r); delete r; }
        for (Request* r : queue_) { ex_->release(r); delete r; }
        for (Factor* f : factors_) delete f;
    }
    Scheduler(const Scheduler&) = delete;
    Scheduler& operator=(const Scheduler&) = delete;

    // Bytes a request of order n needs while it runs (factor and workspace).
    size_t need(int n, int nrhs) const { return align_up(ex_->factor_bytes(n)) + align_up(ex_->solve_bytes(n, nrhs)); }

    int submit(uint64_t key, int n, const double* A, int64_t lda, const double* B, int nrhs, int64_t ldb,
               double* X, int64_t ldx, int64_t* id) {
        if (need(n, nrhs) > arena_.size) return ERR_WORKSPACE;
        Request* r = new (std::nothrow) Request();
        if (!r) return ERR_HIP;
        r->id = next_id_++;
        r->key = key;
        r->n = n;
        r->nrhs = nrhs;
        r->A = A; r->lda = lda; r->B = B; r->ldb = ldb; r->X = X; r->ldx = ldx;
        if (ex_->arrive(r) != 0) {
            ex_->release(r);
            delete r;
            return ERR_HIP;
        }
        queue_.push_back(r);
        stats_.submitted++;
        if (id) *id = r->id;
        return 0;
    }

    // One scheduler iteration.  Returns the number of requests not finished
    // (>= 0) or an error.
    int step() {
        const int slot = (int)(stats_.steps % (int64_t)slot_used_.size());
        if (slot_used_[slot] && ex_->slot_wait(slot) != 0) return ERR_HIP;
        int rc = admit();
        if (rc) return rc;
        // nothing running and the oldest request still not admitted: it cannot be
        // (with nothing active every resident factor is evictable), so this is a
        // broken invariant, reported instead of spinning
        if (active_.empty() && !queue_.empty()) return ERR_WORKSPACE;
        for (Request* r : active_)
            if (r->st == WAIT_FACTOR && r->f->ready) r->st = SOLVE;
        std::vector<Request*> stepping;
        for (Request* r : active_)
            if (r->st == FACTOR) stepping.push_back(r);
        if (!stepping.empty()) {
            if (ex_->step(stepping, slot) != 0) return ERR_HIP;
            stats_.grouped_launches += 3;
        }
        for (Request* r : stepping) {
            r->c0 += std::min(r->s, r->n - r->c0);
            if (r->c0 >= r->n) {
                if (ex_->factor_done(r) != 0) return ERR_HIP;
                r->f->ready = true;
                if (r->f->key) resident_.push_front(r->f);
                else r->f->dead = true;
                r->st = SOLVE;
            }
        }
        for (Request* r : active_) {
            if (r->st == SOLVE) {
                if (ex_->solve(r) != 0) return ERR_HIP;
                if (cfg_.refine && cfg_.max_iter > 0) {
                    r->iters = 1;
                    r->st = REFINE;
                } else {
                    if (ex_->finish(r) != 0) return ERR_HIP;
                    r->st = DONE;
                }
            } else if (r->st == REFINE) {
                bool ready = false;
                double corr = 0.0;
                if (ex_->refine_poll(r, &ready, &corr) != 0) return ERR_HIP;
                if (!ready) continue;
                bool stop;
                if (corr <= cfg_.tol) {                                   // converged
                    r->converged = true;
                    stop = true;
                } else {
                    // stagnation (the correction shrank by less than half), an
                    // unusable value, or the iteration limit
                    stop = !(corr == corr) || (r->prev_corr >= 0.0 && corr > 0.5 * r->prev_corr) ||
                           r->iters >= cfg_.max_iter;
                }
                r->prev_corr = corr;
                if (stop) {
                    if (ex_->finish(r) != 0) return ERR_HIP;
                    r->st = DONE;
                } else {
                    if (ex_->refine(r) != 0) return ERR_HIP;
                    r->iters++;
                }
            }
        }
        if (ex_->slot_done(slot) != 0) return ERR_HIP;
        slot_used_[slot] = 1;
        stats_.steps++;
        int inflight = 0;
        for (Request* r : active_) inflight += r->st != DONE;
        return inflight + (int)queue_.size();
    }

    // Up to max_out requests whose device work has completed.
    int poll(Result* out, int max_out, int* n_out) {
        int k = 0;
        for (size_t i = 0; i < active_.size() && k < max_out;) {
            Request* r = active_[i];
            if (r->st != DONE || !ex_->finished(r)) { ++i; continue; }
            Factor* f = r->f;
            const int info = ex_->info(f, r);
            out[k++] = Result{r->id, info, r->hit ? 1 : 0, r->iters, r->converged ? 1 : 0, ex_->latency_ms(r)};
            arena_.release(r->ws_off, r->ws_bytes);
            free_slot_.push_back(r->slot);
            f->users--;
            if (info != 0 && !f->dead) {
                // a failed factor is never served again
                f->dead = true;
                resident_.remove(f);
                auto it = by_key_.find(f->key);
                if (it != by_key_.end() && it->second == f) by_key_.erase(it);
            }
            if (f->dead && f->users == 0) drop_factor(f);
            ex_->release(r);
            delete r;
            active_.erase(active_.begin() + (std::ptrdiff_t)i);
            stats_.completed++;
        }
        if (n_out) *n_out = k;
        return 0;
    }

    const Stats& stats() const { return stats_; }
    size_t arena_size() const { return arena_.size; }
    size_t arena_free() const { return arena_.free_bytes(); }
    size_t resident_count() const { return resident_.size(); }
    size_t queued_count() const { return queue_.size(); }
    size_t active_count() const { return active_.size(); }
    size_t live_factors() const { return factors_.size(); }
    const std::list<Factor*>& resident() const { return resident_; }
    const std::vector<Request*>& active() const { return active_; }

private:
    void drop_factor(Factor* f) {
        arena_.release(f->off, f->bytes);
        if (f->info_slot >= 0) free_info_.push_back(f->info_slot);
        if (f->key) {
            auto it = by_key_.find(f->key);
            if (it != by_key_.end() && it->second == f) by_key_.erase(it);
        }
        resident_.remove(f);
        factors_.erase(std::remove(factors_.begin(), factors_.end(), f), factors_.end());
        delete f;
    }

    // Drop the least recently used resident factor no request is using.
    bool evict_one() {
        Factor* victim = nullptr;
        for (auto it = resident_.rbegin(); it != resident_.rend(); ++it)
            if ((*it)->users == 0) { victim = *it; break; }
        if (!victim) return false;
        drop_factor(victim);
        stats_.evictions++;
        return true;
    }

    bool make_room(size_t bytes, size_t& off) {
        while (!arena_.alloc(bytes, off))
            if (!evict_one()) return false;
        return true;
    }

    // Admit queued requests in arrival order while space allows.
    int admit() {
        while (!queue_.empty() && (int)active_.size() < cfg_.max_active && !free_slot_.empty()) {
            Request* r = queue_.front();
            const size_t ws = ex_->solve_bytes(r->n, r->nrhs);
            Factor* f = nullptr;
            bool owner = false;
            auto it = r->key ? by_key_.find(r->key) : by_key_.end();
            if (it != by_key_.end() && it->second->n == r->n) {
                f = it->second;
            } else {
                if (free_info_.empty() && !evict_one()) break;
                f = new (std::nothrow) Factor();
                if (!f) return ERR_HIP;
                f->key = r->key;
                f->n = r->n;
                f->bytes = ex_->factor_bytes(r->n);
                owner = true;
            }
            size_t ws_off = 0, f_off = 0;
            f->users++;                       // keep it from being evicted below
            if (owner && !make_room(f->bytes, f_off)) {
                f->users--;
                delete f;
                break;
            }
            if (owner) {
                f->off = f_off;
                factors_.push_back(f);
            }
            if (!make_room(ws, ws_off)) {
                f->users--;
                if (owner) {
                    arena_.release(f->off, f->bytes);
                    factors_.pop_back();
                    delete f;
                }
                break;
            }
            queue_.pop_front();
            r->f = f;
            r->owner = owner;
            r->ws_off = ws_off;
            r->ws_bytes = ws;
            r->slot = free_slot_.back();
            free_slot_.pop_back();
            if (owner) {
                f->info_slot = free_info_.back();
                free_info_.pop_back();
                if (f->key) by_key_[f->key] = f;
                if (ex_->start_factor(r) != 0) return ERR_HIP;
                r->st = FACTOR;
                r->s = std::max(1, std::min(r->n, cfg_.step_cols));
                r->c0 = 0;
            } else {
                r->hit = true;
                r->st = f->ready ? SOLVE : WAIT_FACTOR;
                if (f->ready) {
                    resident_.remove(f);
                    resident_.push_front(f);
                }
                stats_.cache_hits++;
            }
            active_.push_back(r);
        }
        return 0;
    }

    Executor* ex_;
    Config cfg_;
    Arena arena_;
    std::list<Request*> queue_;     // not yet admitted
    std::vector<Request*> active_;
    std::list<Factor*> resident_;   // ready keyed factors, front = most recently used
    std::map<uint64_t, Factor*> by_key_;
    std::vector<Factor*> factors_;  // every live factor
    std::vector<int> free_info_, free_slot_;
    std::vector<int> slot_used_;
    int64_t next_id_ = 1;
    Stats stats_;
};

}  // namespace ffserve
