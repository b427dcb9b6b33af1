// Request server with continuous batching (a systems layer on top of the
// paper's method: the plans it runs are those of Section 4).
//
// A scheduler thread owns the launches:
//   admit  -- pending requests whose plan is ready, in arrival order, while
//             each fits the budget (output + scratch + descriptor image from
//             an arena carved out of one reservation) and fewer than
//             max_inflight are admitted; the first that does not fit blocks
//             the ones behind it;
//   launch -- everything admitted since the last launch becomes one batch
//             (build_batch_layout) whose descriptor image is copied to the
//             arena and launched on the next of n_streams streams, after the
//             requests' input events; an event marks its end;
//   retire -- finished launches (event queries) complete their requests,
//             return scratch and descriptors to the arena and wake waiters.
// A planner thread makes the plans of requests whose problem is not cached,
// meanwhile the scheduler keeps going.  Cached plans keep their tables in the
// arena (inside the budget); plans no request holds are evicted, least
// recently used first, when memory is short.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch.h"

namespace mfft {

const char *last_error_text();

// Failures inside the scheduler thread are reported per request through
// mfft_server_wait; MFFT_LOG=1 also prints their text to stderr.
static void log_failure(const char *what, int rc)
{
    static const bool on = getenv("MFFT_LOG") && atoi(getenv("MFFT_LOG")) > 0;
    if (on) fprintf(stderr, "mfft server: %s failed (%d): %s\n", what, rc, last_error_text());
}

static double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// First-fit arena over one device reservation, 256-byte granules, coalescing.
// Thread safe (the planner thread allocates plan tables from it).
class Arena {
  public:
    bool init(size_t bytes, const mfft_allocator *alloc)
    {
        size_ = bytes / 256 * 256;
        if (alloc && alloc->alloc) {
            alloc_ = *alloc;
            has_alloc_ = true;
            base_ = alloc_.alloc(size_, nullptr, alloc_.ctx);
        } else if (hipMalloc(&base_, size_) != hipSuccess) {
            (void)hipGetLastError();
            base_ = nullptr;
        }
        if (!base_) return false;
        free_[0] = size_;
        return true;
    }
    ~Arena()
    {
        if (!base_) return;
        if (has_alloc_) {
            if (alloc_.free) alloc_.free(base_, nullptr, alloc_.ctx);
        } else {
            (void)hipFree(base_);
        }
    }
    void *alloc(size_t n)
    {
        std::lock_guard<std::mutex> lk(m_);
        n = std::max<size_t>(256, (n + 255) / 256 * 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                const size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > n) free_[off + n] = len - n;
                used_ += n;
                peak_ = std::max(peak_, used_);
                sizes_[off] = n;
                return (char *)base_ + off;
            }
        }
        return nullptr;
    }
    void release(void *p)
    {
        if (!p) return;
        std::lock_guard<std::mutex> lk(m_);
        const size_t off = (char *)p - (char *)base_;
        auto s = sizes_.find(off);
        if (s == sizes_.end()) return;
        size_t n = s->second;
        sizes_.erase(s);
        used_ -= n;
        size_t start = off;
        auto next = free_.lower_bound(off);
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                start = prev->first;
                n += prev->second;
                free_.erase(prev);
            }
        }
        next = free_.lower_bound(start + n);
        if (next != free_.end() && next->first == start + n) {
            n += next->second;
            free_.erase(next);
        }
        free_[start] = n;
    }
    size_t size() const { return size_; }
    size_t used()
    {
        std::lock_guard<std::mutex> lk(m_);
        return used_;
    }
    size_t peak()
    {
        std::lock_guard<std::mutex> lk(m_);
        return peak_;
    }

  private:
    std::mutex m_;
    void *base_ = nullptr;
    size_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
    std::unordered_map<size_t, size_t> sizes_;
    mfft_allocator alloc_{};
    bool has_alloc_ = false;
};

struct Req {
    uint64_t id = 0;
    mfft_request r{};
    std::string key;                // canonical problem (plan cache key)
    hipEvent_t ready = nullptr;     // recorded on r.in_stream at submission
    int state = MFFT_REQ_PENDING;   // or DONE (0) or a negative error
    mfft_plan plan = nullptr;       // held (counted in the cache entry's users)
    void *out = nullptr;
    bool own_out = false;
    void *scratch = nullptr;
    size_t out_bytes = 0;
    double t_arrival = 0, t_done = 0;
    double flops = 0, bytes = 0;
    bool cancelled = false;
};

struct CachedPlan {
    mfft_plan plan = nullptr;
    int users = 0;             // requests holding the plan (pending or admitted)
    uint64_t last_use = 0;
    size_t bytes = 0;          // its tables in the arena
};

struct PlanJob {
    std::string key;
    mfft_request r{};
};

struct Launch {
    std::vector<std::shared_ptr<Req>> reqs;
    hipEvent_t done = nullptr;
    size_t desc_reserved = 0;
    void *desc = nullptr;
    BatchLayout layout;
    double t_start = 0;
};

}  // namespace mfft

struct mfft_server_s {
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_plan;
    std::thread worker, planner;
    bool stop = false;
    mfft::Arena arena;   // request outputs and scratch, plan tables
    mfft::Arena descs;   // launch descriptor images (part of the budget)
    int max_inflight = 1;
    std::vector<hipStream_t> streams;
    size_t next_stream = 0;
    uint64_t next_id = 1;
    uint64_t gen = 0;   // bumped by every event that may let a request be admitted
    std::deque<std::shared_ptr<mfft::Req>> pending;
    std::unordered_map<uint64_t, std::shared_ptr<mfft::Req>> reqs;
    std::deque<mfft::Launch> inflight;
    int admitted_open = 0;   // admitted, not yet finished
    std::map<std::string, mfft::CachedPlan> plans;
    std::deque<mfft::PlanJob> plan_jobs;
    std::set<std::string> planning;   // keys queued for or in the planner
    uint64_t use_clock = 0;
    mfft_allocator plan_alloc{};      // plan tables from the arena
    hipStream_t plan_stream = nullptr;
    int device = 0;
    // stats
    uint64_t submitted = 0, admitted = 0, completed = 0, rejected = 0, failed = 0, cancelled = 0,
             launches = 0;
    std::vector<double> lat_ms;
    double busy_s = 0, busy_since = -1, flops = 0, bytes = 0;
    size_t plan_bytes = 0;
    int max_inflight_seen = 0, plans_evicted = 0;
};

namespace mfft {

// Output span (elements) of a request; its minimum offset must be 0 for a
// server-allocated output.
static bool out_span(const mfft_request &r, int64_t *lo, int64_t *hi)
{
    int64_t l = 0, h = 0;
    for (int i = 0; i < r.rank + r.howmany_rank; ++i) {
        const mfft_iodim &d = i < r.rank ? r.dims[i] : r.howmany_dims[i - r.rank];
        if (d.n <= 0) {
            *lo = 0;
            *hi = -1;
            return true;
        }
        const int64_t e = (d.n - 1) * d.os;
        if (e < 0) l += e;
        else h += e;
    }
    *lo = l;
    *hi = h;
    return true;
}

// ------------------------------------------------------------ plan cache
// (all with S->mu held)

static void *arena_alloc_cb(size_t bytes, void *, void *ctx)
{
    return ((mfft_server_s *)ctx)->arena.alloc(bytes);
}

static void arena_free_cb(void *ptr, void *, void *ctx) { ((mfft_server_s *)ctx)->arena.release(ptr); }

// Take a reference to the cached plan of q's problem, if there is one.
static bool attach_plan(mfft_server_s *S, Req *q)
{
    if (q->plan) return true;
    auto it = S->plans.find(q->key);
    if (it == S->plans.end()) return false;
    q->plan = it->second.plan;
    it->second.users++;
    it->second.last_use = ++S->use_clock;
    return true;
}

static void drop_plan(mfft_server_s *S, Req *q)
{
    if (!q->plan) return;
    auto it = S->plans.find(q->key);
    if (it != S->plans.end() && it->second.plan == q->plan) {
        it->second.users--;
        it->second.last_use = ++S->use_clock;
    }
    q->plan = nullptr;
}

// Destroy the least recently used plan no request holds (its tables return
// to the arena); false if there is none.
static bool evict_one(mfft_server_s *S)
{
    auto victim = S->plans.end();
    for (auto it = S->plans.begin(); it != S->plans.end(); ++it)
        if (it->second.users == 0 && (victim == S->plans.end() || it->second.last_use < victim->second.last_use))
            victim = it;
    if (victim == S->plans.end()) return false;
    mfft_plan_destroy(victim->second.plan);
    S->plan_bytes -= victim->second.bytes;
    S->plans.erase(victim);
    S->plans_evicted++;
    return true;
}

static void finish_request(mfft_server_s *S, Req *q)
{
    drop_plan(S, q);
    if (q->ready) {
        (void)hipEventDestroy(q->ready);
        q->ready = nullptr;
    }
}

static void wake(mfft_server_s *S)
{
    S->gen++;
    S->cv_work.notify_one();
    S->cv_plan.notify_one();
}

// Planner thread: plans the problems of pending requests that are not
// cached, one at a time, with the plan tables in the arena; the scheduler
// admits and retires other requests meanwhile.
static void planner_loop(mfft_server_s *S)
{
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_plan.wait(lk, [&] { return S->stop || !S->plan_jobs.empty(); });
        if (S->stop) break;
        PlanJob job = S->plan_jobs.front();
        S->plan_jobs.pop_front();
        bool needed = false;
        for (auto &q : S->pending)
            if (q->key == job.key && !q->cancelled && q->state == MFFT_REQ_PENDING) needed = true;
        if (!needed) {
            S->planning.erase(job.key);
            continue;
        }
        const mfft_request &r = job.r;
        mfft_plan pl = nullptr;
        lk.unlock();
        int rc = plan_dft_locked(&pl, r.rank, r.dims, r.howmany_rank, r.howmany_dims,
                                 r.in == r.out ? 1 : 0, r.sign, (int)r.prec,
                                 MFFT_ESTIMATE | kPlanNoOwnScratch, &S->plan_alloc, S->plan_stream);
        lk.lock();
        if (rc == MFFT_ENOMEM) {
            // make room: unused cached plans first, else wait for memory that
            // requests still hold, unless none is held
            bool evicted = false;
            while (evict_one(S)) evicted = true;
            if (evicted) {
                S->plan_jobs.push_front(job);
                continue;
            }
            // memory that requests hold (outputs, scratch, plans in use) comes
            // back as they finish or are released
            bool held = S->admitted_open > 0 || S->arena.used() > S->plan_bytes;
            for (auto &kv : S->plans) held = held || kv.second.users > 0;
            if (held && !S->stop) {
                const uint64_t g = S->gen;
                S->cv_plan.wait(lk, [&] { return S->stop || S->gen != g; });
                S->plan_jobs.push_front(job);
                continue;
            }
            rc = fail(MFFT_EBUDGET, "plan tables do not fit the server's HBM budget");
        }
        S->planning.erase(job.key);
        if (rc) {
            log_failure("planning", rc);
            for (auto &q : S->pending)
                if (q->key == job.key && !q->cancelled && q->state == MFFT_REQ_PENDING) {
                    q->state = rc;
                    if (rc == MFFT_EBUDGET) S->rejected++;
                    else S->failed++;
                }
            S->cv_done.notify_all();
            wake(S);
            continue;
        }
        CachedPlan cp;
        cp.plan = pl;
        for (const DeviceAlloc &t : pl->impl.tables) cp.bytes += std::max<size_t>(256, (t.bytes + 255) / 256 * 256);
        cp.last_use = ++S->use_clock;
        S->plans[job.key] = cp;
        S->plan_bytes += cp.bytes;
        for (auto &q : S->pending)
            if (q->key == job.key && !q->cancelled && q->state == MFFT_REQ_PENDING) attach_plan(S, q.get());
        wake(S);
    }
}

// Scheduler thread.
static void server_loop(mfft_server_s *S)
{
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        // ---- retire finished launches (in order per stream is not required)
        bool progressed = false;
        for (auto it = S->inflight.begin(); it != S->inflight.end();) {
            if (hipEventQuery(it->done) == hipSuccess) {
                const double t = now_s();
                for (auto &q : it->reqs) {
                    q->state = MFFT_REQ_DONE;
                    q->t_done = t;
                    S->arena.release(q->scratch);
                    q->scratch = nullptr;
                    finish_request(S, q.get());
                    S->completed++;
                    S->lat_ms.push_back((t - q->t_arrival) * 1e3);
                    S->flops += q->flops;
                    S->bytes += q->bytes;
                    S->admitted_open--;
                }
                S->descs.release(it->desc);
                (void)hipEventDestroy(it->done);
                it = S->inflight.erase(it);
                progressed = true;
            } else {
                ++it;
            }
        }
        if (S->inflight.empty() && S->busy_since >= 0) {
            S->busy_s += now_s() - S->busy_since;
            S->busy_since = -1;
        }
        if (progressed) {
            S->cv_done.notify_all();
            S->gen++;
            S->cv_plan.notify_one();   // a planner waiting for memory may retry
        }

        // ---- on shutdown, requests not yet admitted are cancelled
        if (S->stop && !S->pending.empty()) {
            for (auto &q : S->pending) {
                if (q->state == MFFT_REQ_PENDING) {
                    q->state = MFFT_ECANCELED;
                    S->cancelled++;
                }
                finish_request(S, q.get());
            }
            S->pending.clear();
            S->cv_done.notify_all();
        }

        // ---- admit: requests whose plan is ready, in arrival order
        const uint64_t gen = S->gen;
        std::vector<std::shared_ptr<Req>> tick;
        size_t desc_need = 512;   // upper bound of the tick's descriptor image
        for (auto it = S->pending.begin();
             it != S->pending.end() && S->admitted_open < S->max_inflight;) {
            std::shared_ptr<Req> q = *it;
            if (q->cancelled || q->state != MFFT_REQ_PENDING) {   // cancelled or failed planning
                finish_request(S, q.get());
                it = S->pending.erase(it);
                continue;
            }
            if (!attach_plan(S, q.get())) {   // being planned: the ones behind may go first
                ++it;
                continue;
            }
            const PlanImpl *p = &q->plan->impl;
            // descriptor image bound: per pass one descriptor, a prefix entry and
            // (at worst) its own group's alignment padding
            const size_t dneed = p->passes.size() * (sizeof(PassArgs) + 8 + 520) + 64;
            if (desc_need + dneed > S->descs.size() - S->descs.used()) {
                if (tick.empty() && S->inflight.empty()) {
                    q->state = fail(MFFT_EBUDGET, "plan has too many passes for the descriptor area");
                    log_failure("admission", q->state);
                    finish_request(S, q.get());
                    it = S->pending.erase(it);
                    S->rejected++;
                    S->cv_done.notify_all();
                    continue;
                }
                break;
            }
            const size_t tables = S->plans[q->key].bytes;
            if (q->out_bytes + p->scratch_bytes + tables + 4096 > S->arena.size()) {
                q->state = MFFT_EBUDGET;
                finish_request(S, q.get());
                it = S->pending.erase(it);
                S->rejected++;
                S->cv_done.notify_all();
                continue;
            }
            void *out = q->r.out;
            void *scratch = nullptr;
            bool got = false;
            for (;;) {
                if (!out && q->out_bytes) out = S->arena.alloc(q->out_bytes);
                if (out || !q->out_bytes) {
                    if (p->scratch_bytes) scratch = S->arena.alloc(p->scratch_bytes);
                    if (scratch || !p->scratch_bytes) {
                        got = true;
                        break;
                    }
                    if (!q->r.out) {
                        S->arena.release(out);
                        out = nullptr;
                    }
                }
                if (!evict_one(S)) break;   // room from plans no request holds
            }
            if (!got) break;   // wait for memory (the first ready request blocks the rest)
            desc_need += dneed;
            q->out = out;
            q->own_out = !q->r.out;
            q->scratch = scratch;
            q->state = MFFT_REQ_RUNNING;
            it = S->pending.erase(it);
            S->admitted++;
            S->admitted_open++;
            tick.push_back(q);
        }
        S->max_inflight_seen = std::max(S->max_inflight_seen, S->admitted_open);

        // ---- launch the tick as one batch
        if (!tick.empty()) {
            Launch L;
            std::vector<BatchItem> items;
            for (auto &q : tick)
                items.push_back({&q->plan->impl, q->r.in, q->out, q->scratch});
            int rc = build_batch_layout(items, &L.layout);
            if (rc == MFFT_OK) {
                L.desc = S->descs.alloc(std::max<size_t>(L.layout.bytes, 256));
                if (!L.desc) rc = fail(MFFT_ENOMEM, "descriptor image of " + std::to_string(L.layout.bytes) +
                                             " bytes does not fit (estimate " +
                                             std::to_string(desc_need) + ")");
            }
            hipStream_t s = S->streams[S->next_stream++ % S->streams.size()];
            // inputs produced on the callers' streams
            for (auto &q : tick)
                if (rc == MFFT_OK && q->ready && hipStreamWaitEvent(s, q->ready, 0) != hipSuccess)
                    rc = fail(MFFT_EHIP, "waiting for a request's input stream");
            if (rc == MFFT_OK &&
                hipMemcpyAsync(L.desc, L.layout.host.data(), L.layout.bytes,
                               hipMemcpyHostToDevice, s) != hipSuccess)
                rc = MFFT_EHIP;
            if (rc == MFFT_OK) rc = enqueue_batch_layout(L.layout, (char *)L.desc, s);
            if (rc == MFFT_OK && (hipEventCreateWithFlags(&L.done, hipEventDisableTiming) !=
                                      hipSuccess ||
                                  hipEventRecord(L.done, s) != hipSuccess))
                rc = MFFT_EHIP;
            if (rc != MFFT_OK) {
                log_failure("launch", rc);
                (void)hipStreamSynchronize(s);
                for (auto &q : tick) {
                    q->state = rc;
                    S->arena.release(q->scratch);
                    if (q->own_out) S->arena.release(q->out);
                    q->out = nullptr;
                    finish_request(S, q.get());
                    S->failed++;
                    S->admitted_open--;
                }
                S->descs.release(L.desc);
                if (L.done) (void)hipEventDestroy(L.done);
                S->cv_done.notify_all();
            } else {
                L.reqs = tick;
                L.t_start = now_s();
                if (S->busy_since < 0) S->busy_since = L.t_start;
                S->inflight.push_back(std::move(L));
                S->launches++;
            }
            continue;   // look for completions / more work right away
        }

        if (S->stop && S->pending.empty() && S->inflight.empty()) break;
        if (!S->inflight.empty()) {
            // poll finished launches without holding the lock
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        } else {
            // idle, waiting for plans, or the first ready request waits for
            // memory that only a client's release (or a cancel) can free:
            // sleep until something changes
            S->cv_work.wait(lk, [&] { return S->stop || S->gen != gen; });
        }
    }
}

}  // namespace mfft

using namespace mfft;

extern "C" {

int mfft_server_create(mfft_server *out, size_t hbm_budget_bytes, int max_inflight, int n_streams,
                       const mfft_allocator *alloc)
{
    if (!out || max_inflight < 1 || n_streams < 1 || n_streams > 64 || hbm_budget_bytes < 4096)
        return fail(MFFT_EINVAL, "bad server arguments");
    if (alloc && (!alloc->alloc || !alloc->free))
        return fail(MFFT_EINVAL, "allocator needs both alloc and free");
    *out = nullptr;
    mfft_server_s *S = new (std::nothrow) mfft_server_s();
    if (!S) return fail(MFFT_ENOMEM, "host allocation failed");
    (void)hipGetDevice(&S->device);
    // 1/16 of the budget (at most 16 MiB) holds launch descriptor images, in
    // the same reservation as the rest
    const size_t dbytes = std::min<size_t>((size_t)16 << 20, hbm_budget_bytes / 16) / 256 * 256;
    if (!S->descs.init(dbytes, alloc) || !S->arena.init(hbm_budget_bytes - dbytes, alloc)) {
        delete S;
        return fail(MFFT_ENOMEM, "could not reserve the HBM budget");
    }
    S->plan_alloc.alloc = arena_alloc_cb;
    S->plan_alloc.free = arena_free_cb;
    S->plan_alloc.ctx = S;
    S->max_inflight = max_inflight;
    for (int i = 0; i < n_streams + 1; ++i) {
        hipStream_t s;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t t : S->streams) (void)hipStreamDestroy(t);
            if (S->plan_stream) (void)hipStreamDestroy(S->plan_stream);
            delete S;
            return fail(MFFT_EHIP, "stream creation failed");
        }
        if (i == n_streams) S->plan_stream = s;
        else S->streams.push_back(s);
    }
    S->worker = std::thread(server_loop, S);
    S->planner = std::thread(planner_loop, S);
    *out = S;
    return MFFT_OK;
}

int mfft_server_submit(mfft_server S, const mfft_request *req, uint64_t *ticket)
{
    if (!S || !req || !ticket) return fail(MFFT_EINVAL, "NULL argument");
    const mfft_request &r = *req;
    Problem p;
    int rc = canonicalize(r.rank, r.dims, r.howmany_rank, r.howmany_dims, r.in == r.out ? 1 : 0,
                          r.sign, (int)r.prec, &p);
    if (rc) return rc;
    if (!p.empty && !r.in) return fail(MFFT_EINVAL, "NULL input");
    auto q = std::make_shared<Req>();
    q->r = r;
    q->key = problem_key(p);
    const size_t eb = r.prec == MFFT_C64 ? 16 : 8;
    if (!r.out && !p.empty) {
        int64_t lo, hi;
        out_span(r, &lo, &hi);
        if (lo < 0) return fail(MFFT_EINVAL, "server-allocated outputs need non-negative strides");
        q->out_bytes = (size_t)(hi + 1) * eb;
    }
    const double N = (double)p.n_total;
    q->flops = (p.empty || N < 2) ? 0.0 : 5.0 * N * std::log2(N) * (double)p.howmany;
    q->bytes = p.empty ? 0.0 : 2.0 * eb * N * (double)p.howmany;
    // a lower bound of what the request needs: its output
    if (q->out_bytes > S->arena.size()) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->rejected++;
        return fail(MFFT_EBUDGET, "request larger than the server's HBM budget");
    }
    if (r.in_stream && !p.empty) {
        if (hipEventCreateWithFlags(&q->ready, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(q->ready, (hipStream_t)r.in_stream) != hipSuccess) {
            if (q->ready) (void)hipEventDestroy(q->ready);
            return fail(MFFT_EHIP, "could not record an event on the input stream");
        }
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) {
        if (q->ready) (void)hipEventDestroy(q->ready);
        return fail(MFFT_ESTATE, "server is stopping");
    }
    q->id = S->next_id++;
    q->t_arrival = r.arrival > 0 ? r.arrival : now_s();
    S->reqs[q->id] = q;
    S->submitted++;
    if (p.empty) {
        q->state = MFFT_REQ_DONE;
        q->t_done = now_s();
        S->completed++;
        S->cv_done.notify_all();
    } else {
        if (!attach_plan(S, q.get()) && !S->planning.count(q->key)) {
            S->planning.insert(q->key);
            S->plan_jobs.push_back({q->key, r});
        }
        S->pending.push_back(q);
        wake(S);
    }
    *ticket = q->id;
    return MFFT_OK;
}

int mfft_server_wait(mfft_server S, uint64_t ticket, int timeout_ms, int *status)
{
    if (!S) return fail(MFFT_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(MFFT_ESTATE, "unknown ticket");
    std::shared_ptr<Req> q = it->second;
    auto finished = [&] { return q->state <= 0; };
    if (timeout_ms < 0) S->cv_done.wait(lk, finished);
    else S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), finished);
    if (status) *status = q->state;
    if (!finished()) return fail(MFFT_ETIMEOUT, "request still running");
    return MFFT_OK;
}

int mfft_server_output(mfft_server S, uint64_t ticket, void **out)
{
    if (!S || !out) return fail(MFFT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(MFFT_ESTATE, "unknown ticket");
    if (it->second->state != MFFT_REQ_DONE) return fail(MFFT_ESTATE, "request not finished");
    *out = it->second->out;
    return MFFT_OK;
}

int mfft_server_release(mfft_server S, uint64_t ticket)
{
    if (!S) return fail(MFFT_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(MFFT_ESTATE, "unknown ticket");
    std::shared_ptr<Req> q = it->second;
    if (q->state > 0) return fail(MFFT_ESTATE, "request not finished");
    if (q->own_out) S->arena.release(q->out);
    q->out = nullptr;
    S->reqs.erase(it);
    wake(S);   // memory may admit the next request
    return MFFT_OK;
}

int mfft_server_cancel(mfft_server S, uint64_t ticket)
{
    if (!S) return fail(MFFT_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(MFFT_ESTATE, "unknown ticket");
    std::shared_ptr<Req> q = it->second;
    if (q->state != MFFT_REQ_PENDING) return fail(MFFT_ESTATE, "request already admitted");
    // the scheduler admits only requests still pending under this lock, so a
    // cancelled request never runs (also when its plan is being made)
    q->cancelled = true;
    q->state = MFFT_ECANCELED;
    finish_request(S, q.get());
    S->cancelled++;
    wake(S);
    S->cv_done.notify_all();
    return MFFT_OK;
}

int mfft_server_stats(mfft_server S, mfft_server_stats_t *st)
{
    if (!S || !st) return fail(MFFT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    std::memset(st, 0, sizeof(*st));
    st->submitted = S->submitted;
    st->admitted = S->admitted;
    st->completed = S->completed;
    st->rejected = S->rejected;
    st->failed = S->failed;
    st->cancelled = S->cancelled;
    st->launches = S->launches;
    std::vector<double> l = S->lat_ms;
    if (!l.empty()) {
        std::sort(l.begin(), l.end());
        auto pct = [&](double q) {
            const double pos = q * (double)(l.size() - 1);
            const size_t i = (size_t)pos;
            const double f = pos - (double)i;
            return i + 1 < l.size() ? l[i] * (1 - f) + l[i + 1] * f : l[i];
        };
        st->p50_ms = pct(0.50);
        st->p99_ms = pct(0.99);
        double s = 0;
        for (double v : l) s += v;
        st->mean_ms = s / (double)l.size();
        st->max_ms = l.back();
    }
    st->busy_s = S->busy_s + (S->busy_since >= 0 ? now_s() - S->busy_since : 0.0);
    st->flops = S->flops;
    st->bytes = S->bytes;
    st->bytes_in_use = S->arena.used() + S->descs.used();
    st->peak_bytes = S->arena.peak() + S->descs.peak();
    st->plan_bytes = S->plan_bytes;
    st->plans_cached = (int)S->plans.size();
    st->max_inflight_seen = S->max_inflight_seen;
    st->plans_evicted = S->plans_evicted;
    return MFFT_OK;
}

int mfft_server_reset_stats(mfft_server S)
{
    if (!S) return fail(MFFT_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lk(S->mu);
    S->submitted = S->admitted = S->completed = S->rejected = S->failed = S->cancelled = 0;
    S->launches = 0;
    S->lat_ms.clear();
    S->busy_s = 0;
    if (S->busy_since >= 0) S->busy_since = now_s();
    S->flops = S->bytes = 0;
    S->max_inflight_seen = S->admitted_open;
    return MFFT_OK;
}

int mfft_server_destroy(mfft_server S)
{
    if (!S) return MFFT_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv_work.notify_all();
        S->cv_plan.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    if (S->planner.joinable()) S->planner.join();
    for (hipStream_t s : S->streams) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    if (S->plan_stream) (void)hipStreamDestroy(S->plan_stream);
    for (auto &kv : S->plans) mfft_plan_destroy(kv.second.plan);
    for (auto &kv : S->reqs)
        if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
    delete S;
    return MFFT_OK;
}

}  // extern "C"
