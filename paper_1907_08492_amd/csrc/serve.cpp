// Request loop for Poisson solves (sipg_submit / sipg_poll): continuous
// batching of multigrid solves on one GPU.
//
// Requests wait in a FIFO queue.  A pool of worker threads, each with its own
// HIP stream (default priority), takes the oldest request whose memory fits:
// a worker checks out an idle multigrid hierarchy of the request's problem
// from a cache (or builds one), assembles the right-hand side on the device,
// runs the FP64-CG / multigrid solve and returns the hierarchy to the cache.
// Queued requests of the same problem are taken along (batch_max_rhs,
// batch_max_dofs) and solved together by one sipg_mg_solve_many (one
// iteration loop for all of their right-hand sides).
// Solves of different requests therefore run concurrently on the device;
// requests that arrive while others run are admitted as soon as a worker and
// enough of the HBM budget are free.  The budget counts the cached
// hierarchies and the per-request vectors; idle hierarchies are evicted in
// least-recently-used order when a request needs the memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "setup.hpp"
#include "sipg_common.hpp"

using Clock = std::chrono::steady_clock;

namespace {

struct Key {
    int32_t n[3];
    double lo[3], hi[3], width[3], lin[9], a;
    int degree, basis, precision;
    double penalty;
    bool operator<(const Key& o) const { return std::memcmp(this, &o, sizeof(Key)) < 0; }
};

struct CacheEntry {
    sipg_mg* mg = nullptr;
    bool busy = false;
    int64_t bytes = 0;
    Clock::time_point last_used;
};

struct Job {
    uint64_t ticket = 0;
    sipg_request req{};
    Key key{};
    int64_t ndofs = 0;
    int64_t est_bytes = 0;           // hierarchy estimate + request vectors
    Clock::time_point t_submit, t_start, t_end;
    bool done = false;
    sipg_result res{};
    double* x_owned = nullptr;       // server-owned solution buffer
};

}  // namespace

struct sipg_server {
    sipg_server_opts opts{};
    sipg_allocator user_alloc{nullptr, nullptr, nullptr};
    sipg::DevAlloc mem;              // provider of hierarchies and result buffers
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Job*> queue;
    std::map<uint64_t, std::unique_ptr<Job>> jobs;
    std::multimap<Key, CacheEntry> cache;
    int64_t used_bytes = 0;          // cached hierarchies + running requests' vectors
    uint64_t next_ticket = 1;
    bool stop = false;
    std::vector<std::thread> workers;
    hipStream_t house = nullptr;     // stream for releasing result buffers
    std::vector<sipg_mg*> evicted;   // hierarchies to free outside the lock
    int64_t peak_bytes = 0;
    int64_t completed = 0;
    int64_t batched_solves = 0;      // solves over 2 or more requests
    int64_t batched_requests = 0;
    int running = 0;                 // admitted jobs not yet finished
};

namespace sipg {

static Key make_key(const sipg_request& r, int precision) {
    Key k;
    std::memset(&k, 0, sizeof(k));
    for (int d = 0; d < 3; ++d) {
        k.n[d] = r.mesh.n[d];
        k.lo[d] = r.mesh.lo[d];
        k.hi[d] = r.mesh.hi[d];
        k.width[d] = r.mesh.width[d];
    }
    for (int i = 0; i < 9; ++i) k.lin[i] = r.mesh.lin[i];
    k.a = r.mesh.deform_amp;
    k.degree = r.degree;
    k.basis = r.basis;
    k.precision = precision;
    k.penalty = r.penalty_factor;
    return k;
}

// Multigrid options of every solve of the server.
static sipg_mg_opts solver_opts(const sipg_server_opts& so) {
    sipg_mg_opts o;
    sipg_mg_default_opts(&o);
    o.precision = so.precision;
    o.smoother = so.smoother;
    o.p_coarsening = so.p_coarsening;
    o.coarse_reduction = so.coarse_reduction;
    o.graded_coarsening = so.graded_coarsening;
    o.coarse_direct_max_dofs = so.coarse_direct_max_dofs;
    return o;
}

// Upper estimate of a hierarchy's device memory before it exists (its level
// sequence, metric terms, diagonals and level vectors, plus the FP64 fine
// operator and CG vectors).
static int64_t estimate_hierarchy_bytes(const sipg_request& r, const sipg_server_opts& so) {
    return mg_estimate_bytes(r.mesh, r.degree, solver_opts(so));
}

static void finish_job(sipg_server* s, Job* j, int status) {
    j->t_end = Clock::now();
    j->res.status = status;
    j->res.queue_s = std::chrono::duration<double>(j->t_start - j->t_submit).count();
    j->res.solve_s = std::chrono::duration<double>(j->t_end - j->t_start).count();
    j->res.total_s = std::chrono::duration<double>(j->t_end - j->t_submit).count();
    j->res.ndofs = j->ndofs;
    j->done = true;
    s->completed++;
}

// A queued request that has waited this long is not overtaken by later,
// smaller ones any more: nothing else is admitted until it fits.
constexpr double kMaxOvertakeSeconds = 2.0;

// Pick the oldest queued job that fits the budget (evicting idle cached
// hierarchies if needed); called with the lock held.  A request that does not
// fit while no solve runs and nothing can be evicted (only results the client
// has not released hold the budget) is finished with SIPG_E_BUDGET instead
// of waiting for ever.
static Job* admit(sipg_server* s) {
    const Clock::time_point now = Clock::now();
    for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
        Job* j = *it;
        // an idle cached hierarchy of this problem?
        bool cached = false;
        auto range = s->cache.equal_range(j->key);
        for (auto c = range.first; c != range.second; ++c)
            if (!c->second.busy) { cached = true; break; }
        const int64_t vec_bytes = j->req.x_out ? 0 : 8 * j->ndofs;   // server-owned solution
        const int64_t need = vec_bytes + (cached ? 0 : estimate_hierarchy_bytes(j->req, s->opts));
        // evict idle hierarchies (least recently used first) until it fits
        while (s->used_bytes + need > s->opts.hbm_budget_bytes) {
            auto victim = s->cache.end();
            for (auto c = s->cache.begin(); c != s->cache.end(); ++c) {
                if (c->second.busy) continue;
                if (cached && !(c->first < j->key) && !(j->key < c->first)) continue;   // keep ours
                if (victim == s->cache.end() || c->second.last_used < victim->second.last_used) victim = c;
            }
            if (victim == s->cache.end()) break;
            // freed by the admitting worker after it releases the lock (a
            // device free waits for the whole device)
            s->evicted.push_back(victim->second.mg);
            s->used_bytes -= victim->second.bytes;
            s->cache.erase(victim);
        }
        if (s->used_bytes + need > s->opts.hbm_budget_bytes) {
            if (s->running == 0) {
                bool evictable = false;
                for (auto& c : s->cache) evictable = evictable || !c.second.busy;
                if (!evictable) {
                    set_error("request loop: unreleased results hold the memory budget");
                    j->t_start = now;
                    s->queue.erase(it);
                    finish_job(s, j, SIPG_E_BUDGET);
                    s->cv_done.notify_all();
                    return admit(s);
                }
            }
            // later, smaller requests may overtake it for a while
            if (std::chrono::duration<double>(now - j->t_submit).count() > kMaxOvertakeSeconds) return nullptr;
            continue;
        }
        j->est_bytes = need;
        s->running++;
        s->used_bytes += need;
        s->peak_bytes = std::max(s->peak_bytes, s->used_bytes);
        s->queue.erase(it);
        return j;
    }
    return nullptr;
}

// Queued requests of j's problem (same key, tolerance and iteration limit)
// that join j in one sipg_mg_solve_many, within the batch limits and the
// budget; called with the lock held right after admit(j), which charged j.
// Only the next 2 x workers queued requests are looked at, so that requests
// finish in about the order they arrived (a client that consumes results in
// order holds the finished ones' memory until then).  The group's workspace
// (its level and CG vectors, and the stacked b and x) is charged to j.
static std::vector<Job*> gather_batch(sipg_server* s, Job* j) {
    std::vector<Job*> group{j};
    const int maxr = s->opts.batch_max_rhs;
    if (maxr < 2) return group;
    std::vector<Job*> cand;   // in queue order
    int64_t dofs = j->ndofs;
    int seen = 0;
    for (Job* c : s->queue) {
        if (int(cand.size()) + 1 >= maxr || ++seen > 2 * s->opts.workers) break;
        if (c->key < j->key || j->key < c->key || c->req.rel_tol != j->req.rel_tol ||
            c->req.max_iter != j->req.max_iter || dofs + c->ndofs > s->opts.batch_max_dofs)
            continue;
        cand.push_back(c);
        dofs += c->ndofs;
    }
    // the largest group whose vectors and workspace fit the budget
    while (!cand.empty()) {
        const int k = int(cand.size()) + 1;
        int64_t vec_need = 0;
        for (Job* c : cand) vec_need += c->req.x_out ? 0 : 8 * c->ndofs;
        const int64_t ws = mg_many_estimate(j->req.mesh, j->req.degree, solver_opts(s->opts), k) +
                           2 * 8 * int64_t(k) * j->ndofs;
        if (s->used_bytes + vec_need + ws <= s->opts.hbm_budget_bytes) {
            j->est_bytes += ws;
            s->used_bytes += ws;
            break;
        }
        cand.pop_back();
    }
    if (cand.empty()) return group;
    for (Job* c : cand) {
        c->est_bytes = c->req.x_out ? 0 : 8 * c->ndofs;
        s->used_bytes += c->est_bytes;
        s->running++;
        group.push_back(c);
    }
    // take them out of the queue in one pass (an erase in the middle of a
    // deque invalidates its iterators)
    s->queue.erase(std::remove_if(s->queue.begin(), s->queue.end(),
                                  [&](Job* q) { return std::find(cand.begin(), cand.end(), q) != cand.end(); }),
                   s->queue.end());
    s->peak_bytes = std::max(s->peak_bytes, s->used_bytes);
    return group;
}

// Solves the requests of `group` (one problem) on hierarchy mg: one
// sipg_mg_solve alone, else one sipg_mg_solve_many over their stacked
// right-hand sides, the solutions then copied to each request's vector.
// Fills every request's result fields except status; returns the status of
// each in `status`.
static void solve_group(sipg_server* s, sipg_mg* mg, const std::vector<Job*>& group, std::vector<double*>& xs,
                        std::vector<int>& status, hipStream_t st) {
    const int k = int(group.size());
    const Job* j = group[0];
    const int64_t n = j->ndofs;
    sipg_op* fine = mg_fine_operator(mg);
    if (k == 1) {
        double* b = mg_rhs_buffer(mg);
        sipg_solve_info info{};
        int rc = launch_rhs_sines(fine, j->req.nmodes, j->req.amps, &j->req.waves[0][0], b, st);
        if (rc == SIPG_OK && hipMemsetAsync(xs[0], 0, sizeof(double) * size_t(n), st) != hipSuccess) rc = SIPG_E_HIP;
        if (rc == SIPG_OK) rc = sipg_mg_solve(mg, b, xs[0], j->req.rel_tol, j->req.max_iter, &info, st);
        double bn = 0.0;
        if (rc == SIPG_OK || rc == SIPG_E_NOCONV) bn = mg_last_rhs_norm(mg);
        group[0]->res.iterations = info.iterations;
        group[0]->res.true_residual = info.true_residual;
        group[0]->res.rel_residual = bn > 0.0 ? info.true_residual / bn : info.true_residual;
        status[0] = rc;
        return;
    }
    for (const Job* g : group) {
        if (g->ndofs != n) {   // one problem per group (gather_batch)
            set_error("request loop: requests of different sizes in one group");
            std::fill(status.begin(), status.end(), SIPG_E_ARG);
            return;
        }
    }
    // stacked right-hand sides and solutions (stream-ordered, or the caller's allocator)
    const size_t bytes = sizeof(double) * size_t(n) * k;
    void* q = nullptr;
    int rc = SIPG_OK;
    if (s->mem.a.alloc) rc = s->mem.alloc(&q, 2 * bytes, "request loop: stacked vectors");
    else if (hipMallocAsync(&q, 2 * bytes, st) != hipSuccess) { (void)hipGetLastError(); rc = SIPG_E_OOM; }
    double* bw = static_cast<double*>(q);
    double* xw = bw ? bw + size_t(n) * k : nullptr;
    for (int v = 0; v < k && rc == SIPG_OK; ++v)
        rc = launch_rhs_sines(fine, group[v]->req.nmodes, group[v]->req.amps, &group[v]->req.waves[0][0],
                              bw + size_t(v) * n, st);
    if (rc == SIPG_OK && hipMemsetAsync(xw, 0, bytes, st) != hipSuccess) rc = SIPG_E_HIP;
    std::vector<sipg_solve_info> info(k);
    std::vector<double> bn(k, 0.0);
    std::vector<int> conv(k, 0);
    if (rc == SIPG_OK)
        rc = mg_solve_many(mg, k, bw, xw, j->req.rel_tol, j->req.max_iter, info.data(), bn.data(), conv.data(), st);
    for (int v = 0; v < k; ++v) {
        int sv = rc == SIPG_OK || rc == SIPG_E_NOCONV ? (conv[v] ? SIPG_OK : SIPG_E_NOCONV) : rc;
        if ((rc == SIPG_OK || rc == SIPG_E_NOCONV) &&
            hipMemcpyAsync(xs[v], xw + size_t(v) * n, sizeof(double) * size_t(n), hipMemcpyDeviceToDevice, st) !=
                hipSuccess)
            sv = SIPG_E_HIP;
        group[v]->res.iterations = info[v].iterations;
        group[v]->res.true_residual = info[v].true_residual;
        group[v]->res.rel_residual = bn[v] > 0.0 ? info[v].true_residual / bn[v] : info[v].true_residual;
        status[v] = sv;
    }
    if (q) {
        if (s->mem.a.alloc) {
            (void)hipStreamSynchronize(st);
            s->mem.release(q);
        } else {
            (void)hipFreeAsync(q, st);
        }
    }
}

static void worker_main(sipg_server* s) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        Job* j = nullptr;
        s->cv_work.wait(lk, [&] { return s->stop || (j = admit(s)) != nullptr; });
        if (!j) break;   // stop requested and nothing admissible
        const std::vector<Job*> group = gather_batch(s, j);
        const int k = int(group.size());
        const Clock::time_point t0 = Clock::now();
        for (Job* g : group) g->t_start = t0;
        // check out a cached hierarchy
        sipg_mg* mg = nullptr;
        CacheEntry* ce = nullptr;
        auto range = s->cache.equal_range(j->key);
        for (auto c = range.first; c != range.second; ++c)
            if (!c->second.busy) { ce = &c->second; break; }
        if (ce) { ce->busy = true; mg = ce->mg; }
        std::vector<sipg_mg*> to_free;
        to_free.swap(s->evicted);
        lk.unlock();
        for (sipg_mg* e : to_free) sipg_mg_destroy(e);

        int status = SIPG_OK;
        int64_t built_bytes = 0;
        if (!mg) {
            const sipg_mg_opts o = solver_opts(s->opts);
            status = sipg_mg_setup(&j->req.mesh, j->req.degree, j->req.penalty_factor, j->req.basis, &o,
                                   &s->user_alloc, st, &mg);
            if (status == SIPG_OK) {
                sipg_mg_info info;
                sipg_mg_get_info(mg, &info);
                built_bytes = info.device_bytes;
            }
        }
        // result vectors: the request's own, or server-owned (stream-ordered:
        // no device-wide synchronisation between workers)
        std::vector<double*> xs(k, nullptr);
        std::vector<int> stat(k, status);
        for (int v = 0; v < k && status == SIPG_OK; ++v) {
            Job* g = group[v];
            xs[v] = g->req.x_out;
            if (xs[v]) continue;
            const size_t xb = sizeof(double) * size_t(g->ndofs);
            if (s->mem.a.alloc) {
                void* q = nullptr;
                status = s->mem.alloc(&q, xb, "request loop: solution buffer");
                g->x_owned = static_cast<double*>(q);
            } else if (hipMallocAsync(reinterpret_cast<void**>(&g->x_owned), xb, st) != hipSuccess) {
                g->x_owned = nullptr;
                status = SIPG_E_OOM;
            }
            xs[v] = g->x_owned;
        }
        if (status == SIPG_OK) {
            solve_group(s, mg, group, xs, stat, st);
            (void)hipStreamSynchronize(st);
        } else {
            std::fill(stat.begin(), stat.end(), status);
        }
        for (int v = 0; v < k; ++v) group[v]->res.x = xs[v];

        lk.lock();
        // return or insert the hierarchy into the cache, settle the budget;
        // a server-owned result buffer stays charged until it is released
        int64_t kept = 0;
        for (Job* g : group) {
            s->used_bytes -= g->est_bytes;
            s->running--;
            kept += g->x_owned ? 8 * g->ndofs : 0;
        }
        if (ce) {
            ce->busy = false;
            ce->last_used = Clock::now();
            s->used_bytes += kept;
        } else if (mg) {
            CacheEntry e;
            e.mg = mg;
            e.bytes = built_bytes;
            e.last_used = Clock::now();
            s->cache.emplace(j->key, e);
            s->used_bytes += built_bytes + kept;
        } else {
            s->used_bytes += kept;
        }
        s->peak_bytes = std::max(s->peak_bytes, s->used_bytes);
        if (k > 1) {
            s->batched_solves++;
            s->batched_requests += k;
        }
        for (int v = 0; v < k; ++v) finish_job(s, group[v], stat[v]);
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
    lk.unlock();
    (void)hipStreamDestroy(st);
}

}  // namespace sipg

using namespace sipg;

extern "C" {

int sipg_server_default_opts(sipg_server_opts* o) {
    if (!o) { set_error("sipg_server_default_opts: null"); return SIPG_E_ARG; }
    o->hbm_budget_bytes = int64_t(64) << 30;
    o->workers = 8;
    o->precision = 0;
    o->smoother = 1;
    o->p_coarsening = 1;
    o->coarse_reduction = 10.0;
    o->graded_coarsening = 0;
    o->coarse_direct_max_dofs = 256;
    o->batch_max_rhs = 8;
    o->batch_max_dofs = int64_t(1) << 20;
    return SIPG_OK;
}

int sipg_server_create(const sipg_server_opts* opts, const sipg_allocator* allocator, sipg_server** out) {
    if (!out) { set_error("sipg_server_create: null out"); return SIPG_E_ARG; }
    *out = nullptr;
    if (!allocator_valid(allocator)) { set_error("sipg_server_create: allocator needs both callbacks"); return SIPG_E_ARG; }
    sipg_server_opts o;
    sipg_server_default_opts(&o);
    if (opts) o = *opts;
    if (o.workers < 1 || o.workers > 16 || o.hbm_budget_bytes <= 0 || (o.precision != 0 && o.precision != 1) ||
        (o.smoother != 0 && o.smoother != 1) || o.p_coarsening < 0 || o.p_coarsening > 2 ||
        !(o.coarse_reduction > 1.0) || (o.graded_coarsening != 0 && o.graded_coarsening != 1) ||
        o.coarse_direct_max_dofs < 0 || o.coarse_direct_max_dofs > 1024 || o.batch_max_rhs < 1 ||
        o.batch_max_rhs > kMaxSolveRhs || o.batch_max_dofs < 0) {
        set_error("sipg_server_create: workers in [1,16], budget > 0, precision and smoother 0 or 1, p_coarsening 0..2, "
                  "coarse_reduction > 1, graded_coarsening 0 or 1, coarse_direct_max_dofs 0..1024, batch_max_rhs "
                  "1..16, batch_max_dofs >= 0");
        return SIPG_E_ARG;
    }
    sipg_server* s = new (std::nothrow) sipg_server();
    if (!s) { set_error("sipg_server_create: out of host memory"); return SIPG_E_OOM; }
    s->opts = o;
    if (allocator) s->user_alloc = *allocator;
    s->mem = DevAlloc(allocator);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { delete s; set_error("sipg_server_create: no device"); return SIPG_E_HIP; }
    if (hipStreamCreateWithFlags(&s->house, hipStreamNonBlocking) != hipSuccess) {
        delete s;
        set_error("sipg_server_create: stream creation failed");
        return SIPG_E_HIP;
    }
    for (int w = 0; w < o.workers; ++w)
        s->workers.emplace_back([s, dev] {
            (void)hipSetDevice(dev);
            worker_main(s);
        });
    *out = s;
    return SIPG_OK;
}

int sipg_submit(sipg_server* s, const sipg_request* r, uint64_t* ticket) {
    if (!s || !r || !ticket) { set_error("sipg_submit: null argument"); return SIPG_E_ARG; }
    if (r->degree < 1 || r->degree > 8 || r->nmodes < 1 || r->nmodes > 16 || !(r->rel_tol > 0.0) ||
        r->max_iter < 0 || !(r->penalty_factor > 0.0) || r->basis < 0 || r->basis > 2) {
        set_error("sipg_submit: invalid request");
        return SIPG_E_ARG;
    }
    for (int d = 0; d < 3; ++d)
        if (r->mesh.n[d] <= 0) { set_error("sipg_submit: cell counts must be positive"); return SIPG_E_ARG; }
    auto j = std::make_unique<Job>();
    j->req = *r;
    j->key = make_key(*r, s->opts.precision);
    const int n = r->degree + 1;
    j->ndofs = int64_t(r->mesh.n[0]) * r->mesh.n[1] * r->mesh.n[2] * n * n * n;
    const int64_t need = estimate_hierarchy_bytes(*r, s->opts) + 3 * 8 * j->ndofs;
    if (need > s->opts.hbm_budget_bytes) {
        set_error("sipg_submit: the request alone exceeds the memory budget");
        return SIPG_E_BUDGET;
    }
    j->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) { set_error("sipg_submit: server is shutting down"); return SIPG_E_ARG; }
    j->ticket = s->next_ticket++;
    *ticket = j->ticket;
    s->queue.push_back(j.get());
    s->jobs.emplace(j->ticket, std::move(j));
    s->cv_work.notify_one();
    return SIPG_OK;
}

int sipg_poll(sipg_server* s, uint64_t ticket, sipg_result* res) {
    if (!s || !res) { set_error("sipg_poll: null argument"); return SIPG_E_ARG; }
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) { set_error("sipg_poll: unknown ticket"); return SIPG_E_ARG; }
    if (!it->second->done) return SIPG_E_NOTREADY;
    *res = it->second->res;
    return SIPG_OK;
}

int sipg_wait(sipg_server* s, uint64_t ticket, sipg_result* res) {
    if (!s || !res) { set_error("sipg_wait: null argument"); return SIPG_E_ARG; }
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) { set_error("sipg_wait: unknown ticket"); return SIPG_E_ARG; }
    Job* j = it->second.get();
    s->cv_done.wait(lk, [&] { return j->done; });
    *res = j->res;
    return SIPG_OK;
}

// Frees a result buffer whose writer (the worker stream) has finished.
static void free_result(sipg_server* s, double* x) {
    if (s->mem.a.free) s->mem.release(x);
    else (void)hipFreeAsync(x, s->house);
}

int sipg_release(sipg_server* s, uint64_t ticket, void* stream) {
    if (!s) { set_error("sipg_release: null server"); return SIPG_E_ARG; }
    double* x = nullptr;
    int64_t bytes = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->jobs.find(ticket);
        if (it == s->jobs.end()) { set_error("sipg_release: unknown ticket"); return SIPG_E_ARG; }
        if (!it->second->done) { set_error("sipg_release: request still running"); return SIPG_E_NOTREADY; }
        x = it->second->x_owned;
        bytes = x ? 8 * it->second->ndofs : 0;
        s->jobs.erase(it);
    }
    if (x) {
        // the caller's queued reads of the solution (on `stream`) end first
        hipEvent_t ev = nullptr;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(ev, static_cast<hipStream_t>(stream)) != hipSuccess || hipEventSynchronize(ev) != hipSuccess) {
            if (ev) (void)hipEventDestroy(ev);
            set_error("sipg_release: could not wait for the caller's stream (buffer kept)");
            return SIPG_E_HIP;
        }
        (void)hipEventDestroy(ev);
        free_result(s, x);
        std::lock_guard<std::mutex> lk(s->mu);
        s->used_bytes -= bytes;
    }
    s->cv_work.notify_all();
    return SIPG_OK;
}

int sipg_server_stats(sipg_server* s, sipg_server_stats_t* st) {
    if (!s || !st) { set_error("sipg_server_stats: null argument"); return SIPG_E_ARG; }
    std::lock_guard<std::mutex> lk(s->mu);
    st->queued = int64_t(s->queue.size());
    st->completed = s->completed;
    st->cached_hierarchies = int64_t(s->cache.size());
    st->used_bytes = s->used_bytes;
    st->peak_bytes = s->peak_bytes;
    st->batched_solves = s->batched_solves;
    st->batched_requests = s->batched_requests;
    return SIPG_OK;
}

int sipg_server_destroy(sipg_server* s) {
    if (!s) return SIPG_OK;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        // finish everything queued, then stop the workers
        s->cv_done.wait(lk, [&] {
            for (auto& kv : s->jobs)
                if (!kv.second->done) return false;
            return true;
        });
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
    for (auto& kv : s->jobs)
        if (kv.second->x_owned) free_result(s, kv.second->x_owned);
    (void)hipStreamSynchronize(s->house);
    (void)hipStreamDestroy(s->house);
    for (auto& kv : s->cache) sipg_mg_destroy(kv.second.mg);
    for (sipg_mg* e : s->evicted) sipg_mg_destroy(e);
    delete s;
    return SIPG_OK;
}

}  // extern "C"
