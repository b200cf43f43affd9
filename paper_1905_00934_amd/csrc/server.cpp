// Continuous batching of slice reconstructions: requests are admitted into slots
// as slots and device memory free up, and every slot in flight advances in the
// same batched launches (one launch per kernel per shape group).
//
// The worker thread repeats one step:
//   admit queued requests in FIFO order while a slot is free and the footprint
//     fits the budget (copy counts, ingest, initialise);
//   regroup the slots if the set changed;
//   run g outer iterations of every slot, g = smallest distance of a slot to its
//     next check (so no slot runs past a check or past max_iters);
//   at each slot's check, read its last two log records and stop it on
//     convergence, at max_iters or on a non-finite value (copy x out, free slot).
// A slot's iterations and checks depend only on its own request, so its result
// is the one it would reach alone.
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <thread>

#include "common.h"
#include "kernels.h"
#include "runner.h"

namespace dect {
namespace {

using Clock = std::chrono::steady_clock;

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

// Device bytes of one request in flight: its state, measurements (m, w for both
// spectra) and counts.
struct Footprint {
    size_t state, meas, counts, total;
};
Footprint footprint(const dect_plan* p) {
    Footprint f;
    f.state = round256(p->layout.bytes);
    f.meas = round256((size_t)p->M * p->elem);
    f.counts = round256((size_t)p->M * p->elem);
    f.total = f.state + 4 * f.meas + 2 * f.counts;
    return f;
}

struct Request {
    uint64_t ticket = 0;
    dect_request req{};
    std::vector<char> ch, cl;  // host copies of the counts
    Clock::time_point t_submit, t_admit;
};

struct Slot {
    std::unique_ptr<Request> r;
    char* mem = nullptr;
    size_t bytes = 0;
    void* state = nullptr;
    void* meas[4] = {nullptr, nullptr, nullptr, nullptr};
    void* counts[2] = {nullptr, nullptr};
    int iters = 0, next_check = 0;
};

int64_t ns_between(Clock::time_point a, Clock::time_point b) {
    return (int64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(b - a).count();
}

}  // namespace
}  // namespace dect

using namespace dect;

struct dect_server {
    dect_server_config cfg{};
    int device = 0;
    hipStream_t stream = nullptr;
    double* host_log = nullptr;  // pinned: two log records per slot

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    dect_status fatal = DECT_OK;
    std::deque<std::unique_ptr<Request>> queue;
    std::set<uint64_t> pending;  // queued or in flight
    std::map<uint64_t, dect_result> done;
    uint64_t next_ticket = 1;
    size_t in_use = 0;           // footprints of admitted requests
    dect_server_stats stats{};

    // Worker-owned.
    std::thread worker;
    std::vector<Slot> slots;
    std::vector<std::pair<size_t, char*>> pool;  // free device blocks by size
    Runner<float> rf;
    Runner<double> rd;

    ~dect_server() {
        for (auto& s : slots)
            if (s.mem) (void)hipFree(s.mem);
        for (auto& b : pool) (void)hipFree(b.second);
        if (host_log) (void)hipHostFree(host_log);
        if (stream) (void)hipStreamDestroy(stream);
    }

    // A device block of `bytes`, from the cache if one fits exactly; cached blocks
    // of other sizes are released first when the budget would be exceeded.
    hipError_t take_block(size_t bytes, char** out) {
        for (size_t k = 0; k < pool.size(); ++k)
            if (pool[k].first == bytes) {
                *out = pool[k].second;
                pool.erase(pool.begin() + (long)k);
                return hipSuccess;
            }
        size_t held;
        {
            std::lock_guard<std::mutex> lk(mu);
            held = stats.hbm_held;
        }
        while (!pool.empty() && held + bytes > cfg.hbm_budget_bytes) {
            hipError_t e = hipFree(pool.back().second);
            held -= pool.back().first;
            pool.pop_back();
            if (e != hipSuccess) return e;
        }
        hipError_t e = hipMalloc(reinterpret_cast<void**>(out), bytes);
        if (e == hipSuccess) held += bytes;
        std::lock_guard<std::mutex> lk(mu);
        stats.hbm_held = held;
        return e;
    }

    void finish(Slot& s, const dect_result& res) {
        pool.emplace_back(s.bytes, s.mem);
        s.mem = nullptr;
        std::lock_guard<std::mutex> lk(mu);
        in_use -= s.bytes;
        pending.erase(s.r->ticket);
        done[s.r->ticket] = res;
        stats.completed++;
        // Counted out of flight in the same step that publishes the result, so a
        // caller that has every result sees none in flight.
        if (stats.in_flight > 0) stats.in_flight--;
        cv_done.notify_all();
    }

    // Every request still queued or in flight ends with status st.
    void fail_all(dect_status st) {
        std::lock_guard<std::mutex> lk(mu);
        fatal = st;
        dect_result res{};
        res.status = st;
        for (uint64_t t : pending) done[t] = res;
        pending.clear();
        queue.clear();
        cv_done.notify_all();
    }

    template <typename T>
    hipError_t admit(Slot& s) {
        const dect_request& q = s.r->req;
        const dect_plan* p = q.plan;
        const Footprint f = footprint(p);
        char* b = s.mem;
        s.state = b;
        b += f.state;
        for (auto& m : s.meas) {
            m = b;
            b += f.meas;
        }
        for (auto& c : s.counts) {
            c = b;
            b += f.counts;
        }
        const size_t cb = (size_t)p->M * p->elem;
        hipError_t e = hipMemcpyAsync(s.counts[0], s.r->ch.data(), cb, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(s.counts[1], s.r->cl.data(), cb, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = launch_ingest<T>(p, s.counts[0], s.counts[1], q.i0_h, q.i0_l, s.meas[0], s.meas[1],
                                 s.meas[2], s.meas[3], stream);
        if (e != hipSuccess) return e;
        if (dect_admm_init(p, s.meas[0], s.meas[1], s.meas[2], s.meas[3], s.state, &q.params,
                           stream) != DECT_OK)
            return hipErrorLaunchFailure;
        s.iters = 0;
        s.next_check = std::min(cfg.step_iters, q.max_iters);
        return hipSuccess;
    }

    hipError_t regroup() {
        std::vector<SliceJob<float>> jf;
        std::vector<SliceJob<double>> jd;
        for (const Slot& s : slots) {
            const dect_request& q = s.r->req;
            if (q.plan->dtype == DECT_F32)
                jf.push_back(make_job<float>(q.plan, s.meas[0], s.meas[1], s.meas[2], s.meas[3],
                                             s.state, &q.params));
            else
                jd.push_back(make_job<double>(q.plan, s.meas[0], s.meas[1], s.meas[2], s.meas[3],
                                              s.state, &q.params));
        }
        // The argument tables may still be read by the previous step's kernels.
        hipError_t e = hipStreamSynchronize(stream);
        if (e == hipSuccess) e = rf.set(jf);
        if (e == hipSuccess) e = rd.set(jd);
        return e;
    }

    void run() {
        if (hipSetDevice(device) != hipSuccess) {
            fail_all(DECT_E_DEVICE);
            return;
        }
        bool changed = false;
        for (;;) {
            std::vector<std::unique_ptr<Request>> admitted;
            {
                std::unique_lock<std::mutex> lk(mu);
                for (;;) {
                    if (stop) return;
                    while (!queue.empty() &&
                           (int)(slots.size() + admitted.size()) < cfg.max_slots) {
                        const size_t need = footprint(queue.front()->req.plan).total;
                        if (in_use + need > cfg.hbm_budget_bytes) break;
                        in_use += need;
                        queue.front()->t_admit = Clock::now();
                        admitted.push_back(std::move(queue.front()));
                        queue.pop_front();
                    }
                    if (!admitted.empty() || !slots.empty()) break;
                    cv_work.wait(lk);
                }
                stats.queued = (int64_t)queue.size();
            }
            hipError_t e = hipSuccess;
            for (auto& r : admitted) {
                Slot s;
                s.bytes = footprint(r->req.plan).total;
                s.r = std::move(r);
                e = take_block(s.bytes, &s.mem);
                if (e == hipSuccess)
                    e = s.r->req.plan->dtype == DECT_F32 ? admit<float>(s) : admit<double>(s);
                slots.push_back(std::move(s));
                if (e != hipSuccess) break;
                changed = true;
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                stats.in_flight = (int64_t)slots.size();
                stats.peak_in_flight = std::max(stats.peak_in_flight, stats.in_flight);
            }
            if (e == hipSuccess && changed) {
                e = regroup();
                changed = false;
            }
            if (slots.empty()) continue;
            int g = std::numeric_limits<int>::max();
            for (const Slot& s : slots) g = std::min(g, s.next_check - s.iters);
            for (int k = 0; k < g && e == hipSuccess; ++k) {
                e = rf.enqueue(stream);
                if (e == hipSuccess) e = rd.enqueue(stream);
            }
            for (size_t k = 0; k < slots.size() && e == hipSuccess; ++k) {
                Slot& s = slots[k];
                s.iters += g;
                if (s.iters != s.next_check) continue;
                const dect_plan* p = s.r->req.plan;
                const char* ring = static_cast<const char*>(s.state) + p->off_log;
                for (int back = 1; back <= 2 && back <= s.iters && e == hipSuccess; ++back) {
                    const size_t it = (size_t)(s.iters - back);
                    e = hipMemcpyAsync(host_log + (2 * k + back - 1) * kLogStride,
                                       ring + (it % kLogCap) * kLogStride * sizeof(double),
                                       kLogStride * sizeof(double), hipMemcpyDeviceToHost, stream);
                }
            }
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
            {
                std::lock_guard<std::mutex> lk(mu);
                stats.steps++;
            }
            if (e != hipSuccess) {
                set_error("server step failed: %s", hipGetErrorString(e));
                fail_all(DECT_E_DEVICE);
                return;
            }
            std::vector<Slot> keep;
            for (size_t k = 0; k < slots.size(); ++k) {
                Slot& s = slots[k];
                const dect_request& q = s.r->req;
                if (s.iters != s.next_check) {
                    keep.push_back(std::move(s));
                    continue;
                }
                const double* last = host_log + 2 * k * kLogStride;
                const double* prev = last + kLogStride;
                const double phi = last[8] + last[9];
                double rel = std::numeric_limits<double>::infinity();
                if (s.iters >= 2) {
                    const double prv = prev[8] + prev[9];
                    rel = phi != 0.0 ? std::fabs(phi - prv) / std::fabs(phi)
                                     : (prv == 0.0 ? 0.0 : rel);
                }
                const bool bad = last[1] != 0.0 || !std::isfinite(phi);
                if (!bad && rel > q.tol && s.iters < q.max_iters) {
                    s.next_check = std::min(s.iters + cfg.step_iters, q.max_iters);
                    keep.push_back(std::move(s));
                    continue;
                }
                const dect_plan* p = q.plan;
                e = hipMemcpyAsync(q.x_out, static_cast<const char*>(s.state) + p->layout.x,
                                   (size_t)p->N * 2 * p->elem, hipMemcpyDeviceToHost, stream);
                if (e == hipSuccess) e = hipStreamSynchronize(stream);
                dect_result res{};
                res.status = e != hipSuccess ? DECT_E_DEVICE : (bad ? DECT_E_NONFINITE : DECT_OK);
                res.iters = s.iters;
                res.objective = phi;
                res.rel_change = rel;
                const Clock::time_point now = Clock::now();
                res.queue_ns = ns_between(s.r->t_submit, s.r->t_admit);
                res.latency_ns = ns_between(s.r->t_submit, now);
                finish(s, res);
                changed = true;
                if (e != hipSuccess) {
                    set_error("server result copy failed: %s", hipGetErrorString(e));
                    slots.clear();
                    for (auto& r : keep) slots.push_back(std::move(r));
                    fail_all(DECT_E_DEVICE);
                    return;
                }
            }
            slots = std::move(keep);
            std::lock_guard<std::mutex> lk(mu);
            stats.in_flight = (int64_t)slots.size();
        }
    }
};

extern "C" {

size_t dect_serve_footprint(const dect_plan* plan) { return plan ? footprint(plan).total : 0; }

dect_status dect_server_create(const dect_server_config* cfg, dect_server** out) {
    if (!out || !cfg) return fail(DECT_E_ARG, "null argument");
    *out = nullptr;
    if (cfg->max_slots < 1 || cfg->step_iters < 1 || cfg->max_queue < 0)
        return fail(DECT_E_ARG, "max_slots and step_iters must be >= 1, max_queue >= 0");
    std::unique_ptr<dect_server> S(new (std::nothrow) dect_server());
    if (!S) return fail(DECT_E_NOMEM, "out of host memory");
    S->cfg = *cfg;
    DECT_HIP(hipGetDevice(&S->device));
    if (S->cfg.hbm_budget_bytes == 0) {
        size_t fr = 0, tot = 0;
        DECT_HIP(hipMemGetInfo(&fr, &tot));
        S->cfg.hbm_budget_bytes = fr / 2;
    }
    DECT_HIP(hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking));
    DECT_HIP(hipHostMalloc(reinterpret_cast<void**>(&S->host_log),
                           (size_t)S->cfg.max_slots * 2 * kLogStride * sizeof(double)));
    dect_server* raw = S.get();
    S->worker = std::thread([raw] { raw->run(); });
    *out = S.release();
    return DECT_OK;
}

dect_status dect_serve_submit(dect_server* S, const dect_request* req, uint64_t* ticket) {
    if (!S || !req || !ticket) return fail(DECT_E_ARG, "null argument");
    if (!req->plan || !req->counts_h || !req->counts_l || !req->x_out)
        return fail(DECT_E_ARG, "request needs a plan, both count arrays and x_out");
    if (!(req->i0_h > 0) || !(req->i0_l > 0)) return fail(DECT_E_ARG, "I0 must be positive");
    if (!(req->tol >= 0) || req->max_iters < 1)
        return fail(DECT_E_ARG, "tol must be >= 0 and max_iters >= 1");
    dect_status st = check_batch_params(&req->params);
    if (st) return st;
    if (req->params.precond && !req->plan->has_precond)
        return fail(DECT_E_SHAPE, "no preconditioner for this request's image size");
    const size_t need = footprint(req->plan).total;
    if (need > S->cfg.hbm_budget_bytes)
        return fail(DECT_E_CAPACITY, "request needs %zu device bytes; the budget is %zu", need,
                    S->cfg.hbm_budget_bytes);
    std::unique_ptr<Request> r(new (std::nothrow) Request());
    if (!r) return fail(DECT_E_NOMEM, "out of host memory");
    r->req = *req;
    r->req.params.rho_schedule = nullptr;
    r->req.params.rho_schedule_len = 0;
    const size_t cb = (size_t)req->plan->M * req->plan->elem;
    r->ch.assign(static_cast<const char*>(req->counts_h), static_cast<const char*>(req->counts_h) + cb);
    r->cl.assign(static_cast<const char*>(req->counts_l), static_cast<const char*>(req->counts_l) + cb);
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->fatal) return fail(S->fatal, "the server stopped after a device error");
    if (S->cfg.max_queue > 0 && (int64_t)S->queue.size() >= S->cfg.max_queue) {
        S->stats.rejected++;
        return fail(DECT_E_CAPACITY, "the queue holds its limit of %d requests", S->cfg.max_queue);
    }
    r->ticket = S->next_ticket++;
    *ticket = r->ticket;
    S->pending.insert(r->ticket);
    S->queue.push_back(std::move(r));
    S->stats.submitted++;
    S->stats.queued = (int64_t)S->queue.size();
    S->cv_work.notify_one();
    return DECT_OK;
}

dect_status dect_serve_wait(dect_server* S, uint64_t ticket, int64_t timeout_ms,
                            dect_result* out) {
    if (!S || !out) return fail(DECT_E_ARG, "null argument");
    std::unique_lock<std::mutex> lk(S->mu);
    auto ready = [&] { return S->done.count(ticket) > 0 || !S->pending.count(ticket); };
    if (timeout_ms < 0)
        S->cv_done.wait(lk, ready);
    else if (timeout_ms > 0)
        S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
    auto it = S->done.find(ticket);
    if (it != S->done.end()) {
        *out = it->second;
        S->done.erase(it);
        return DECT_OK;
    }
    if (S->pending.count(ticket)) return DECT_NOT_READY;
    return fail(DECT_E_ARG, "unknown or already collected ticket %llu", (unsigned long long)ticket);
}

dect_status dect_serve_poll(dect_server* S, uint64_t ticket, dect_result* out) {
    return dect_serve_wait(S, ticket, 0, out);
}

dect_status dect_server_get_stats(dect_server* S, dect_server_stats* out) {
    if (!S || !out) return fail(DECT_E_ARG, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->stats;
    out->queued = (int64_t)S->queue.size();
    return DECT_OK;
}

void dect_server_destroy(dect_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv_work.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    if (S->stream) (void)hipStreamSynchronize(S->stream);
    delete S;
}

}  // extern "C"
