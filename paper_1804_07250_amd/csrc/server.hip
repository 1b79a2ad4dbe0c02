// Served form: a request loop with continuous batching.  Sampling jobs of
// different sizes are queued by tl_server_submit; a scheduler thread admits
// them in arrival order while the device-memory budget and the slot count
// allow, keeps every admitted chain resident on the device, and advances each
// one by quanta of sweeps on its own stream, so jobs that arrive while others
// run start as soon as memory and a slot are free and share the GPU with them.
// A finished chain is hashed, its observable read, its memory released and the
// next queued job admitted.  Every draw is keyed by the job's own seed and
// sweep counter, so a job's result does not depend on what else is running.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "errors.hpp"
#include "internal.hpp"
#include "models.hpp"

namespace {

struct Job {
    uint64_t ticket = 0;
    tl_domain dom{};
    tl_weights w{};
    uint64_t seed = 0;
    uint64_t sweeps = 0;
    uint64_t done = 0;
    size_t bytes = 0;
    double t_submit = 0, t_start = 0, t_done = 0;
    tl_sampler *s = nullptr;
    hipEvent_t ev = nullptr;
    bool in_flight = false;
};

}  // namespace

struct tl_server {
    size_t budget = 0;
    int32_t max_slots = 0;
    uint32_t quantum = 250;
    uint32_t obs_bin = 1;
    int device = 0;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv;       // wakes the scheduler
    std::condition_variable done_cv;  // wakes waiters
    std::deque<Job> queue;
    std::vector<Job> active;
    std::map<uint64_t, tl_result> results;
    uint64_t next_ticket = 1;
    size_t in_use = 0, peak = 0;
    uint64_t completed = 0;
    // written by the scheduler thread only, read by tl_server_stats
    std::atomic<uint64_t> admitted{0};
    std::atomic<uint32_t> n_active{0}, peak_active{0};
    bool stop = false;
    std::thread worker;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

void finish(tl_server *sv, Job &j, int32_t status)
{
    tl_result r{};
    r.ticket = j.ticket;
    r.status = status;
    r.sweeps = j.done;
    r.t_submit = j.t_submit;
    r.t_start = j.t_start;
    r.t_done = sv->now();
    if (status == TL_OK && j.s) {
        if (tl_sampler_hash(j.s, r.hash) != TL_OK) r.status = TL_EDEVICE;
        tl_observables o{};
        if (r.status == TL_OK && tl_sampler_observables(j.s, &o) == TL_OK) r.scalar_now = o.scalar_now;
    }
    if (j.ev) (void)hipEventDestroy(j.ev);
    if (j.s) tl_sampler_destroy(j.s);
    j.s = nullptr;
    j.ev = nullptr;
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->in_use -= j.bytes;
    sv->results[j.ticket] = r;
    sv->completed += 1;
    sv->done_cv.notify_all();
}

void scheduler(tl_server *sv)
{
    (void)hipSetDevice(sv->device);
    for (;;) {
        std::vector<Job> admit;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            if (sv->active.empty() && sv->queue.empty())
                sv->cv.wait_for(lk, std::chrono::milliseconds(2), [&] { return sv->stop || !sv->queue.empty(); });
            if (sv->stop) break;
            // admission in arrival order, bounded by slots and the memory budget
            while (!sv->queue.empty() && (int32_t)(sv->active.size() + admit.size()) < sv->max_slots &&
                   sv->in_use + sv->queue.front().bytes <= sv->budget) {
                Job j = sv->queue.front();
                sv->queue.pop_front();
                sv->in_use += j.bytes;
                if (sv->in_use > sv->peak) sv->peak = sv->in_use;
                admit.push_back(j);
            }
        }
        for (Job &j : admit) {
            tl_options o{};
            o.obs_bin = sv->obs_bin;
            j.t_start = sv->now();
            tl_status st = tl_sampler_create(&j.dom, &j.w, j.seed, &o, &j.s);
            if (st == TL_OK && hipEventCreateWithFlags(&j.ev, hipEventDisableTiming) != hipSuccess) st = TL_EDEVICE;
            if (st != TL_OK) {
                finish(sv, j, st);
                continue;
            }
            sv->admitted += 1;
            sv->active.push_back(j);
        }
        sv->n_active = (uint32_t)sv->active.size();
        if (sv->n_active > sv->peak_active) sv->peak_active = sv->n_active.load();
        // advance every chain whose previous quantum has completed
        bool progressed = false;
        for (size_t i = 0; i < sv->active.size();) {
            Job &j = sv->active[i];
            if (j.in_flight) {
                const hipError_t q = hipEventQuery(j.ev);
                if (q == hipErrorNotReady) {
                    ++i;
                    continue;
                }
                j.in_flight = false;
                if (q != hipSuccess) {
                    Job dead = j;
                    sv->active.erase(sv->active.begin() + i);
                    finish(sv, dead, TL_EDEVICE);
                    continue;
                }
            }
            if (j.done >= j.sweeps) {
                Job fin = j;
                sv->active.erase(sv->active.begin() + i);
                finish(sv, fin, TL_OK);
                progressed = true;
                continue;
            }
            uint64_t q = j.sweeps - j.done;
            if (q > sv->quantum) q = sv->quantum;
            tl_status st = tl_sampler_sweep(j.s, q);
            hipStream_t stream = nullptr;
            if (st == TL_OK) stream = tl::sampler_stream(j.s);
            if (st != TL_OK || hipEventRecord(j.ev, stream) != hipSuccess) {
                Job dead = j;
                sv->active.erase(sv->active.begin() + i);
                finish(sv, dead, st != TL_OK ? st : TL_EDEVICE);
                continue;
            }
            j.done += q;
            j.in_flight = true;
            progressed = true;
            ++i;
        }
        if (!progressed && !sv->active.empty()) std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    // shutdown: drain the device work of the remaining chains and release them
    for (Job &j : sv->active) {
        if (j.s) (void)tl_sampler_sync(j.s);
        finish(sv, j, TL_EBUSY);
    }
    sv->active.clear();
}

}  // namespace

extern "C" {

tl_status tl_server_create(size_t hbm_budget_bytes, int32_t max_slots, const tl_options *opt, tl_server **out)
{
    if (!out || hbm_budget_bytes == 0 || max_slots <= 0) return tl::fail(TL_EINVAL, "invalid server arguments");
    *out = nullptr;
    tl_server *sv = new (std::nothrow) tl_server();
    if (!sv) return tl::fail(TL_ENOMEM, "host allocation failed");
    sv->budget = hbm_budget_bytes;
    sv->max_slots = max_slots;
    if (opt && opt->sweeps_per_launch) sv->quantum = opt->sweeps_per_launch;
    if (opt && opt->obs_bin) sv->obs_bin = opt->obs_bin;
    sv->t0 = std::chrono::steady_clock::now();
    if (hipGetDevice(&sv->device) != hipSuccess) {
        delete sv;
        return tl::fail(TL_EDEVICE, "no current device");
    }
    sv->worker = std::thread(scheduler, sv);
    *out = sv;
    return TL_OK;
}

tl_status tl_server_submit(tl_server *sv, const tl_domain *dom, const tl_weights *w, uint64_t seed,
                           uint64_t n_sweeps, uint64_t *ticket)
{
    if (!sv || !dom || !w || !ticket) return tl::fail(TL_EINVAL, "null argument");
    std::vector<uint32_t> thr;
    tl_status st = tl::make_table(*dom, *w, thr);
    if (st != TL_OK) return st;
    const size_t bytes = tl::sampler_device_bytes(*dom, sv->obs_bin);
    if (bytes == 0) return tl::fail(TL_EINVAL, "invalid domain");
    if (bytes > sv->budget) return tl::fail(TL_EBUDGET, "job needs %zu bytes, budget is %zu", bytes, sv->budget);
    if (n_sweeps > 0xFFFFFFFFull) return tl::fail(TL_EINVAL, "sweep count exceeds 2^32");
    std::lock_guard<std::mutex> lk(sv->mu);
    Job j;
    j.ticket = sv->next_ticket++;
    j.dom = *dom;
    j.w = *w;
    j.seed = seed;
    j.sweeps = n_sweeps;
    j.bytes = bytes;
    j.t_submit = sv->now();
    sv->queue.push_back(j);
    *ticket = j.ticket;
    sv->cv.notify_one();
    return TL_OK;
}

tl_status tl_server_poll(tl_server *sv, uint64_t ticket, tl_result *out)
{
    if (!sv || !out) return tl::fail(TL_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->results.find(ticket);
    if (it == sv->results.end()) return TL_EBUSY;
    *out = it->second;
    return TL_OK;
}

tl_status tl_server_wait(tl_server *sv, uint64_t ticket, double timeout_s, tl_result *out)
{
    if (!sv || !out) return tl::fail(TL_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(sv->mu);
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
    while (sv->results.find(ticket) == sv->results.end()) {
        if (sv->done_cv.wait_until(lk, deadline) == std::cv_status::timeout &&
            sv->results.find(ticket) == sv->results.end())
            return TL_EBUSY;
    }
    *out = sv->results[ticket];
    return TL_OK;
}

tl_status tl_server_stats(tl_server *sv, tl_server_counters *out)
{
    if (!sv || !out) return tl::fail(TL_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    out->queued = sv->queue.size();
    out->active = sv->n_active.load();
    out->admitted = sv->admitted;
    out->completed = sv->completed;
    out->bytes_in_use = sv->in_use;
    out->peak_bytes = sv->peak;
    out->peak_active = sv->peak_active;
    return TL_OK;
}

tl_status tl_server_destroy(tl_server *sv)
{
    if (!sv) return TL_OK;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->cv.notify_all();
    }
    if (sv->worker.joinable()) sv->worker.join();
    delete sv;
    return TL_OK;
}

}  // extern "C"
