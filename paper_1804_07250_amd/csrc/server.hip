// Served form: continuous batching of sampling jobs on one stream.
//
// Requests queue in arrival order.  A scheduler thread admits them while a
// slot is free and the device arena (one allocation of the memory budget,
// carved first-fit) has room for the job's two state buffers, its export
// buffer and its row digests.  The GPU then runs in ticks: one launch per
// kernel family advances every admitted job by a few sweeps, one work-group
// per (job, tile) item, so many jobs fill the chip together and a new job
// joins at the next tick.  A job that reaches its sweep count is exported,
// hashed and observed right after its last tick on the same stream; the host
// completes the digest, posts the result and returns the memory.  Every draw
// is keyed by the job's own seed, sweep and site, and a tile with its halo
// computes exactly the sweep of the whole state, so a job's result does not
// depend on what else runs beside it.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string.h>
#include <thread>
#include <vector>

#include "errors.hpp"
#include "internal.hpp"
#include "models.hpp"

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over one device allocation; free blocks coalesce.
class Arena {
public:
    hipError_t init(size_t bytes)
    {
        size_ = bytes / kAlign * kAlign;   // never more than the budget
        if (size_ == 0) return hipErrorInvalidValue;
        hipError_t e = hipMalloc((void **)&base_, size_);
        if (e == hipSuccess) free_[0] = size_;
        return e;
    }
    void release()
    {
        if (base_) (void)hipFree(base_);
        base_ = nullptr;
        free_.clear();
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = align_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void free(size_t off, size_t bytes)
    {
        bytes = align_up(bytes);
        auto it = free_.emplace(off, bytes).first;
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
    uint8_t *at(size_t off) const { return base_ + off; }
    size_t size() const { return size_; }

private:
    uint8_t *base_ = nullptr;
    size_t size_ = 0;
    std::map<size_t, size_t> free_;   // offset -> bytes
};

// Page-locked host blocks in power-of-two size classes, reused across jobs and
// returned to the system only when the server ends.
class PinnedPool {
public:
    void *get(size_t bytes, size_t *cls)
    {
        size_t c = 256;
        while (c < bytes) c <<= 1;
        *cls = c;
        auto &fl = free_[c];
        if (!fl.empty()) {
            void *p = fl.back();
            fl.pop_back();
            return p;
        }
        void *p = nullptr;
        if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess) return nullptr;
        all_.push_back(p);
        return p;
    }
    void put(void *p, size_t cls)
    {
        if (p) free_[cls].push_back(p);
    }
    void release()
    {
        for (void *p : all_) (void)hipHostFree(p);
        all_.clear();
        free_.clear();
    }

private:
    std::map<size_t, std::vector<void *>> free_;
    std::vector<void *> all_;
};

struct Job {
    uint64_t ticket = 0;
    tl_domain dom{};
    uint64_t seed = 0;
    uint64_t sweeps = 0;
    uint64_t enq = 0;   // sweeps enqueued so far
    size_t bytes = 0, off = 0;
    double t_submit = 0, t_start = 0;
    std::unique_ptr<tl::Model> model;
    tl::Thr T{};
    bool metro = false;
    bool uniform = false;
    uint32_t rows = 0, row_bytes = 0, obs_B = 1;
    uint8_t *d_export = nullptr, *d_digest = nullptr;
    unsigned long long *d_bin = nullptr;
    uint8_t *h_res = nullptr;   // pinned: row digests, then the observable
    size_t h_cls = 0;
    bool finishing = false;
    int32_t status = TL_OK;
};

// Device bytes of a job: two state buffers, the canonical export, one digest
// per export row, the observable's counter and, for a masked height-model
// domain, its tables.
size_t job_bytes(const tl::Model &m, uint32_t *rows, uint32_t *row_bytes)
{
    m.export_layout(rows, row_bytes);
    return 2 * align_up(m.state_words() * sizeof(uint32_t)) + align_up((size_t)*rows * *row_bytes) +
           align_up(32 * (size_t)*rows) + kAlign + align_up(m.region_bytes());
}

struct Tick {
    hipEvent_t ev = nullptr;
    uint32_t slot = 0;
};

// Jobs whose last tick has been enqueued: their export, digests and
// observable run on the finishing stream; ev marks the end of that work.
struct Finish {
    hipEvent_t ev = nullptr;
    std::vector<Job *> jobs;
};

}  // namespace

struct tl_server {
    size_t budget = 0;
    int32_t max_slots = 0;
    uint32_t quantum = 8;   // sweeps per tick of a weighted job (2x for one-bit jobs)
    uint32_t order = 0;     // colour order of every job: 0 fixed, 1 random per step
    int device = 0;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv;       // wakes the scheduler
    std::condition_variable done_cv;  // wakes waiters
    std::deque<std::unique_ptr<Job>> queue;
    std::map<uint64_t, tl_result> results;
    uint64_t next_ticket = 1;
    size_t in_use = 0, peak = 0;
    uint64_t completed = 0;
    bool stop = false;
    std::atomic<uint64_t> admitted{0};
    std::atomic<uint32_t> n_active{0}, peak_active{0};
    std::thread worker;

    // scheduler-thread state
    hipStream_t stream = nullptr;
    // a tick's launches of different kernel instantiations run side by side:
    // the first on `stream`, the others on `side`, joined through events
    hipStream_t side = nullptr;
    hipEvent_t ev_upload = nullptr, ev_side = nullptr;
    // the results of finished jobs are produced on `fin`, after their last
    // tick, so that they never hold up the ticks of the other jobs
    hipStream_t fin = nullptr;
    std::deque<Finish> finishing;
    Arena arena;
    PinnedPool pinned;
    std::vector<std::unique_ptr<Job>> active;
    std::deque<Tick> inflight;
    std::vector<hipEvent_t> events;
    static constexpr uint32_t kInflight = 2, kSlots = kInflight + 1;
    uint32_t next_slot = 0;
    // a tick's job descriptors and then its items, staged in one pinned
    // buffer per slot and uploaded with one copy into d_buf
    uint32_t cap_jobs = 0, cap_items = 0;
    uint8_t *d_buf = nullptr;
    uint8_t *h_buf[kSlots] = {};

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

void post(tl_server *sv, Job &j, int32_t status)
{
    tl_result r{};
    r.ticket = j.ticket;
    r.status = status;
    r.sweeps = status == TL_OK ? j.sweeps : 0;
    r.t_submit = j.t_submit;
    r.t_start = j.t_start;
    r.t_done = sv->now();
    if (status == TL_OK) {
        tl::sha256_host(j.h_res, 32 * (size_t)j.rows, r.hash);
        uint64_t v = 0;
        memcpy(&v, j.h_res + 32 * (size_t)j.rows, sizeof(v));
        r.scalar_now = v;
    }
    sv->pinned.put(j.h_res, j.h_cls);
    j.h_res = nullptr;
    if (j.model) j.model->release();
    if (j.bytes) sv->arena.free(j.off, j.bytes);
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->in_use -= j.bytes;
    sv->results[j.ticket] = r;
    sv->completed += 1;
    sv->done_cv.notify_all();
}

// Give an admitted job its device memory and initial state.
int32_t start_job(tl_server *sv, Job &j)
{
    uint8_t *base = sv->arena.at(j.off);
    const size_t sb = align_up(j.model->state_words() * sizeof(uint32_t));
    uint32_t *a = (uint32_t *)base, *b = (uint32_t *)(base + sb);
    j.d_export = base + 2 * sb;
    j.d_digest = j.d_export + align_up((size_t)j.rows * j.row_bytes);
    j.d_bin = (unsigned long long *)(j.d_digest + align_up(32 * (size_t)j.rows));
    j.h_res = (uint8_t *)sv->pinned.get(32 * (size_t)j.rows + 8, &j.h_cls);
    if (!j.h_res) return TL_ENOMEM;
    j.model->attach(a, b);
    if (j.model->attach_region((uint8_t *)j.d_bin + kAlign, sv->stream) != hipSuccess) return TL_EDEVICE;
    uint32_t w = 0, h = 0;
    j.model->cell_box(&w, &h);
    j.obs_B = std::max(w, h);
    if (j.model->init(j.dom.init == TL_INIT_MAX, sv->stream) != hipSuccess) return TL_EDEVICE;
    return TL_OK;
}

// Result of a finished job: canonical export -> row digests -> host, and the
// whole-state observable -> host, after its last tick.
hipError_t enqueue_finish(Job &j, hipStream_t st)
{
    hipError_t e = j.model->export_canonical(j.d_export, st);
    if (e == hipSuccess) e = tl::hash_rows(j.d_export, j.rows, j.row_bytes, j.d_digest, st);
    if (e == hipSuccess) e = hipMemcpyAsync(j.h_res, j.d_digest, 32 * (size_t)j.rows, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemsetAsync(j.d_bin, 0, sizeof(unsigned long long), st);
    if (e == hipSuccess) e = j.model->observe(j.obs_B, 1, j.d_bin, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(j.h_res + 32 * (size_t)j.rows, j.d_bin, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           st);
    return e;
}

hipEvent_t take_event(tl_server *sv)
{
    if (sv->events.empty()) {
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return nullptr;
        return ev;
    }
    hipEvent_t ev = sv->events.back();
    sv->events.pop_back();
    return ev;
}

void post_and_drop(tl_server *sv, Job *jp, int32_t st)
{
    auto it = std::find_if(sv->active.begin(), sv->active.end(),
                           [&](const std::unique_ptr<Job> &p) { return p.get() == jp; });
    if (it == sv->active.end()) return;
    post(sv, *jp, jp->status != TL_OK ? jp->status : st);
    sv->active.erase(it);
}

// Bytes of n job descriptors at the start of a staging buffer (the items
// follow, 16-byte aligned).
size_t staged_jobs_bytes(size_t n) { return (n * sizeof(tl::TileJob) + 15) & ~(size_t)15; }

hipError_t grow(tl_server *sv, uint32_t jobs, uint32_t items)
{
    if (jobs <= sv->cap_jobs && items <= sv->cap_items) return hipSuccess;
    // the staging and device arrays are in use by the ticks in flight
    hipError_t e = hipStreamSynchronize(sv->stream);
    if (e != hipSuccess) return e;
    const uint32_t cj = std::max(jobs, std::max(2 * sv->cap_jobs, 64u));
    const uint32_t ci = std::max(items, std::max(2 * sv->cap_items, 4096u));
    if (sv->d_buf) (void)hipFree(sv->d_buf);
    for (uint32_t s = 0; s < tl_server::kSlots; ++s) {
        if (sv->h_buf[s]) (void)hipHostFree(sv->h_buf[s]);
        sv->h_buf[s] = nullptr;
    }
    sv->d_buf = nullptr;
    sv->cap_jobs = sv->cap_items = 0;
    const size_t bytes = staged_jobs_bytes(cj) + ci * sizeof(tl::TileItem);
    e = hipMalloc(&sv->d_buf, bytes);
    for (uint32_t s = 0; s < tl_server::kSlots && e == hipSuccess; ++s)
        e = hipHostMalloc((void **)&sv->h_buf[s], bytes, hipHostMallocDefault);
    if (e == hipSuccess) {
        sv->cap_jobs = cj;
        sv->cap_items = ci;
    }
    return e;
}

// Retire the oldest tick if it has completed; false if it has not.
bool retire(tl_server *sv)
{
    if (sv->inflight.empty()) return false;
    Tick &tk = sv->inflight.front();
    const hipError_t q = hipEventQuery(tk.ev);
    if (q == hipErrorNotReady) return false;
    const int32_t st = q == hipSuccess ? TL_OK : TL_EDEVICE;
    sv->events.push_back(tk.ev);
    sv->inflight.pop_front();
    if (st != TL_OK) {   // the stream is unusable: fail every admitted job
        (void)hipStreamSynchronize(sv->stream);
        (void)hipStreamSynchronize(sv->fin);
        for (Finish &f : sv->finishing) sv->events.push_back(f.ev);
        sv->finishing.clear();
        while (!sv->inflight.empty()) {
            sv->events.push_back(sv->inflight.front().ev);
            sv->inflight.pop_front();
        }
        for (auto &j : sv->active) post(sv, *j, TL_EDEVICE);
        sv->active.clear();
    }
    sv->n_active = (uint32_t)sv->active.size();
    return true;
}

// Enqueue one tick: every active job with sweeps left advances by its share;
// jobs that reach their count are finished after it.  False if there was
// nothing to do.
bool tick(tl_server *sv)
{
    std::vector<Job *> run, fin;
    for (auto &j : sv->active) {
        if (j->finishing) continue;
        if (j->enq < j->sweeps) run.push_back(j.get());
        else fin.push_back(j.get());
    }
    if (run.empty() && fin.empty()) return false;
    std::vector<tl::TileJob> jobs(run.size());
    std::vector<tl::TilePlan> plans(run.size());
    uint32_t n_items = 0;
    for (size_t i = 0; i < run.size(); ++i) {
        Job &j = *run[i];
        const uint64_t left = j.sweeps - j.enq;
        // one-bit jobs take twice the sweeps per tick (their launch then
        // lasts about as long as the weighted one beside it)
        const uint64_t want = (uint64_t)sv->quantum * (j.uniform ? 2u : 1u);
        const uint32_t smax = (uint32_t)std::min<uint64_t>(left, want);
        if (!j.model->tile_job((uint32_t)j.enq, smax, j.T, j.metro, j.seed, true, &jobs[i], &plans[i])) {
            j.status = TL_EINVAL;
            j.enq = j.sweeps;   // finish (as failed) without running
            plans[i] = tl::TilePlan{};
            continue;
        }
        n_items += plans[i].tiles();
    }
    hipError_t e = grow(sv, (uint32_t)run.size(), n_items);
    if (e != hipSuccess) {   // finish these jobs, as failed, at the next tick
        for (Job *j : run) {
            j->status = TL_EDEVICE;
            j->enq = j->sweeps;
        }
        return true;
    }
    const uint32_t slot = sv->next_slot;
    sv->next_slot = (sv->next_slot + 1) % tl_server::kSlots;
    const size_t joff = staged_jobs_bytes(run.size());
    tl::TileJob *hj = reinterpret_cast<tl::TileJob *>(sv->h_buf[slot]);
    tl::TileItem *hi = reinterpret_cast<tl::TileItem *>(sv->h_buf[slot] + joff);
    tl::TileJob *dj = reinterpret_cast<tl::TileJob *>(sv->d_buf);
    tl::TileItem *di = reinterpret_cast<tl::TileItem *>(sv->d_buf + joff);
    // one launch per kernel: the height jobs of every rule and table layout
    // together (the work-groups take their job's kernel body), by whether the
    // domain has site planes, then the domino jobs
    auto key = [&](size_t i) {
        if (!run[i]->model->height_family()) return 100u;
        return run[i]->model->masked() ? 10u : 0u;
    };
    std::vector<size_t> order(run.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return key(a) < key(b); });
    struct Group {
        uint32_t first, count, threads, lds, key;
    };
    std::vector<Group> groups;
    uint32_t ni = 0;
    for (size_t pos = 0; pos < order.size(); ++pos) {
        const size_t i = order[pos];
        hj[pos] = jobs[i];
        const tl::TilePlan &p = plans[i];
        if (p.tiles() == 0) continue;
        if (groups.empty() || groups.back().key != key(i)) groups.push_back(Group{ni, 0u, 0u, 0u, key(i)});
        Group &gr = groups.back();
        for (uint32_t t = 0; t < p.tiles(); ++t) hi[ni++] = tl::TileItem{(uint32_t)pos, t};
        gr.count += p.tiles();
        gr.threads = std::max(gr.threads, p.threads);
        gr.lds = std::max(gr.lds, p.lds);
    }
    if (ni) {
        e = hipMemcpyAsync(sv->d_buf, sv->h_buf[slot], joff + ni * sizeof(tl::TileItem), hipMemcpyHostToDevice,
                           sv->stream);
        // launches after the first wait for the uploads on the side stream, and
        // the main stream waits for them before anything else of this tick
        const bool split = groups.size() > 1;
        if (split && e == hipSuccess) e = hipEventRecord(sv->ev_upload, sv->stream);
        if (split && e == hipSuccess) e = hipStreamWaitEvent(sv->side, sv->ev_upload, 0);
        for (size_t k = 0; k < groups.size(); ++k) {
            const Group &gr = groups[k];
            hipStream_t st = k == 0 ? sv->stream : sv->side;
            if (e != hipSuccess) break;
            if (gr.key == 100u)
                e = tl::domino_items(dj, di + gr.first, gr.count, gr.threads, gr.lds, sv->order, st);
            else
                e = tl::height_items_mixed(dj, di + gr.first, gr.count, gr.threads, gr.lds, sv->order,
                                           gr.key >= 10u ? 1u : 0u, st);
        }
        if (split && e == hipSuccess) e = hipEventRecord(sv->ev_side, sv->side);
        if (split && e == hipSuccess) e = hipStreamWaitEvent(sv->stream, sv->ev_side, 0);
    }
    for (size_t i = 0; i < run.size(); ++i) {
        Job &j = *run[i];
        if (plans[i].tiles() == 0) continue;
        j.model->swap_buffers();
        j.enq += plans[i].S;
        if (e != hipSuccess) j.status = TL_EDEVICE;
    }
    Tick tk;
    tk.slot = slot;
    Finish f;
    for (auto &jp : sv->active) {
        Job &j = *jp;
        if (j.finishing || j.enq < j.sweeps) continue;
        j.finishing = true;
        f.jobs.push_back(&j);
    }
    tk.ev = take_event(sv);
    if (!tk.ev || hipEventRecord(tk.ev, sv->stream) != hipSuccess) {
        // no event: wait for the stream instead, and fail the jobs it ends
        (void)hipStreamSynchronize(sv->stream);
        for (Job *jp : f.jobs) {
            jp->status = TL_EDEVICE;
            post_and_drop(sv, jp, TL_EDEVICE);
        }
        if (tk.ev) sv->events.push_back(tk.ev);
        return true;
    }
    if (!f.jobs.empty()) {
        // results of the jobs this tick ends, on the finishing stream after it
        hipError_t fe = hipStreamWaitEvent(sv->fin, tk.ev, 0);
        for (Job *jp : f.jobs)
            if (jp->status == TL_OK && (fe != hipSuccess || enqueue_finish(*jp, sv->fin) != hipSuccess))
                jp->status = TL_EDEVICE;
        f.ev = take_event(sv);
        if (!f.ev || hipEventRecord(f.ev, sv->fin) != hipSuccess) {
            (void)hipStreamSynchronize(sv->fin);
            for (Job *jp : f.jobs) post_and_drop(sv, jp, TL_EDEVICE);
            if (f.ev) sv->events.push_back(f.ev);
        } else {
            sv->finishing.push_back(std::move(f));
        }
    }
    sv->inflight.push_back(std::move(tk));
    return true;
}

// Post the jobs of the oldest finishing record if its work has completed;
// false if it has not (or there is none).
bool retire_finished(tl_server *sv)
{
    if (sv->finishing.empty()) return false;
    Finish &f = sv->finishing.front();
    const hipError_t q = hipEventQuery(f.ev);
    if (q == hipErrorNotReady) return false;
    const int32_t st = q == hipSuccess ? TL_OK : TL_EDEVICE;
    for (Job *jp : f.jobs) post_and_drop(sv, jp, st);
    sv->events.push_back(f.ev);
    sv->finishing.pop_front();
    return true;
}

void scheduler(tl_server *sv)
{
    (void)hipSetDevice(sv->device);
    for (;;) {
        std::vector<std::unique_ptr<Job>> admit;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            if (sv->active.empty() && sv->queue.empty() && sv->inflight.empty())
                sv->cv.wait_for(lk, std::chrono::milliseconds(2), [&] { return sv->stop || !sv->queue.empty(); });
            if (sv->stop) break;
            // admission in arrival order, bounded by slots and the arena
            while (!sv->queue.empty() && (int32_t)(sv->active.size() + admit.size()) < sv->max_slots) {
                Job &f = *sv->queue.front();
                if (!sv->arena.alloc(f.bytes, &f.off)) break;
                sv->in_use += f.bytes;
                sv->peak = std::max(sv->peak, sv->in_use);
                admit.push_back(std::move(sv->queue.front()));
                sv->queue.pop_front();
            }
        }
        for (auto &j : admit) {
            j->t_start = sv->now();
            const int32_t st = start_job(sv, *j);
            if (st != TL_OK) {
                post(sv, *j, st);
                continue;
            }
            sv->admitted += 1;
            sv->active.push_back(std::move(j));
        }
        sv->n_active = (uint32_t)sv->active.size();
        if (sv->n_active > sv->peak_active) sv->peak_active = sv->n_active.load();
        bool busy = false;
        while (retire(sv)) busy = true;
        while (retire_finished(sv)) busy = true;
        if (sv->inflight.size() < tl_server::kInflight && tick(sv)) busy = true;
        if (!busy && !(sv->inflight.empty() && sv->finishing.empty()))
            std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    // shutdown: drain the streams, fail what has not finished
    (void)hipStreamSynchronize(sv->stream);
    (void)hipStreamSynchronize(sv->fin);
    while (retire(sv)) {
    }
    while (retire_finished(sv)) {
    }
    for (auto &j : sv->active) post(sv, *j, TL_EBUSY);
    sv->active.clear();
    std::lock_guard<std::mutex> lk(sv->mu);
    for (auto &j : sv->queue) {
        tl_result r{};
        r.ticket = j->ticket;
        r.status = TL_EBUSY;
        r.t_submit = j->t_submit;
        r.t_done = sv->now();
        sv->results[j->ticket] = r;
    }
    sv->queue.clear();
    sv->done_cv.notify_all();
}

void destroy_resources(tl_server *sv)
{
    if (sv->stream) (void)hipStreamSynchronize(sv->stream);
    if (sv->side) (void)hipStreamSynchronize(sv->side);
    if (sv->fin) (void)hipStreamSynchronize(sv->fin);
    for (hipEvent_t e : sv->events)
        if (e) (void)hipEventDestroy(e);
    sv->events.clear();
    if (sv->d_buf) (void)hipFree(sv->d_buf);
    for (uint32_t s = 0; s < tl_server::kSlots; ++s)
        if (sv->h_buf[s]) (void)hipHostFree(sv->h_buf[s]);
    sv->pinned.release();
    sv->arena.release();
    if (sv->ev_upload) (void)hipEventDestroy(sv->ev_upload);
    if (sv->ev_side) (void)hipEventDestroy(sv->ev_side);
    sv->ev_upload = sv->ev_side = nullptr;
    if (sv->side) (void)hipStreamDestroy(sv->side);
    sv->side = nullptr;
    if (sv->fin) (void)hipStreamDestroy(sv->fin);
    sv->fin = nullptr;
    if (sv->stream) (void)hipStreamDestroy(sv->stream);
    sv->stream = nullptr;
}

}  // namespace

extern "C" {

tl_status tl_server_create(size_t hbm_budget_bytes, int32_t max_slots, const tl_options *opt, tl_server **out)
{
    if (!out || hbm_budget_bytes == 0 || max_slots <= 0) return tl::fail(TL_EINVAL, "invalid server arguments");
    if (opt && opt->colour_order > 1) return tl::fail(TL_EINVAL, "unknown colour order %u", opt->colour_order);
    if (opt && opt->device_buf) return tl::fail(TL_EINVAL, "servers allocate their own state pool");
    *out = nullptr;
    std::unique_ptr<tl_server> sv(new (std::nothrow) tl_server());
    if (!sv) return tl::fail(TL_ENOMEM, "host allocation failed");
    sv->budget = hbm_budget_bytes;
    sv->max_slots = max_slots;
    if (opt && opt->sweeps_per_launch) sv->quantum = opt->sweeps_per_launch;
    if (opt) sv->order = opt->colour_order;
    sv->t0 = std::chrono::steady_clock::now();
    if (hipGetDevice(&sv->device) != hipSuccess) return tl::fail(TL_EDEVICE, "no current device");
    hipError_t e = hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sv->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sv->fin, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sv->ev_upload, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sv->ev_side, hipEventDisableTiming);
    if (e == hipSuccess) e = sv->arena.init(hbm_budget_bytes);
    if (e == hipSuccess) e = grow(sv.get(), 64, 4096);
    if (e != hipSuccess) {
        destroy_resources(sv.get());
        return tl::fail(e == hipErrorOutOfMemory ? TL_ENOMEM : TL_EDEVICE, "server set-up: %s",
                        hipGetErrorString(e));
    }
    sv->worker = std::thread(scheduler, sv.get());
    *out = sv.release();
    return TL_OK;
}

tl_status tl_server_submit(tl_server *sv, const tl_domain *dom, const tl_weights *w, uint64_t seed,
                           uint64_t n_sweeps, uint64_t *ticket)
{
    if (!sv || !dom || !w || !ticket) return tl::fail(TL_EINVAL, "null argument");
    std::vector<uint32_t> thr;
    tl_status st = tl::make_table(*dom, *w, thr);
    if (st != TL_OK) return st;
    std::vector<uint32_t> thr_free;
    st = tl::make_free_table(*dom, *w, thr_free);
    if (st != TL_OK) return st;
    std::string why;
    tl_status mst = TL_EINVAL;
    std::unique_ptr<tl::Model> m = tl::make_model(*dom, why, &mst);
    if (!m) return tl::fail(mst, "%s", why.c_str());
    m->order = sv->order;
    m->set_boundary_table(thr_free);
    if (n_sweeps > 0xFFFFFFFFull) return tl::fail(TL_EINVAL, "sweep count exceeds 2^32");
    if (sv->order && n_sweeps * (uint64_t)m->colours() > 0x100000000ull)
        return tl::fail(TL_EINVAL, "step counter would exceed 2^32 (random colour order)");
    std::unique_ptr<Job> j(new (std::nothrow) Job());
    if (!j) return tl::fail(TL_ENOMEM, "host allocation failed");
    j->bytes = job_bytes(*m, &j->rows, &j->row_bytes);
    if (align_up(j->bytes) > sv->budget / kAlign * kAlign)
        return tl::fail(TL_EBUDGET, "job needs %zu bytes, budget is %zu", j->bytes, sv->budget);
    j->dom = *dom;
    j->dom.mask = nullptr;   // the model keeps its own copy of a mask
    j->seed = seed;
    j->sweeps = n_sweeps;
    j->metro = w->rule == TL_METROPOLIS;
    std::copy(thr.begin(), thr.end(), j->T.v);
    j->T.count = (uint32_t)thr.size();
    j->uniform = j->T.uniform();
    j->model = std::move(m);
    std::lock_guard<std::mutex> lk(sv->mu);
    j->ticket = sv->next_ticket++;
    j->t_submit = sv->now();
    *ticket = j->ticket;
    sv->queue.push_back(std::move(j));
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
    destroy_resources(sv);
    delete sv;
    return TL_OK;
}

}  // extern "C"
