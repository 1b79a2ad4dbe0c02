// Batched form: thousands of independent domino chains (Aztec diamonds of
// uneven orders, or domains given by masks, each run on the Aztec diamond it
// is embedded in) advanced together by one persistent launch per call, replayed
// from a captured hipGraph.  Chains are packed into bundles (several small
// chains per work-group, first-fit over the chains longest first) and the
// bundles are handed to work-groups costliest first (LPT order) through an
// atomic counter; each chain lives in LDS for the whole call.  Every draw is keyed by (chain seed, sweep, colour, site), so a chain
// gives the same tiling in the batch as alone.
#include <algorithm>
#include <memory>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "errors.hpp"
#include "internal.hpp"
#include "models.hpp"

struct tl_batch {
    int32_t count = 0;
    std::vector<tl_domain> doms;
    std::vector<uint64_t> seeds;
    tl_weights w{};
    tl::Thr T{};
    bool metro = false;
    uint32_t colour_order = 0;   // 0 fixed, 1 random per step (Section 2.2)
    // mask-domain chains: the model that knows the domain's extremal tilings
    // and export box (nullptr for Aztec chains); attached to the chain's
    // stretch of the pool when used
    std::vector<std::unique_ptr<tl::Model>> masks;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint32_t *planes = nullptr;
    std::vector<tl::BatchChain> chains;
    tl::BatchChain *d_chains = nullptr;
    std::vector<uint32_t> order;   // chains, longest first
    // bundles for each work-group size used so far (built before any capture)
    struct BundleSet {
        uint32_t threads = 0, count = 0;
        tl::BatchBundle *d_bundles = nullptr;
        uint32_t *d_members = nullptr;
    };
    std::vector<BundleSet> sets;
    uint32_t *d_counter = nullptr;
    uint32_t lds_max = 0;
    uint32_t threads = 256;
    uint32_t workgroups = 0;
    uint32_t cus = 0;
    uint64_t t = 0;
    uint64_t sites = 0;
    uint64_t owner_bits = 0;
    hipGraphExec_t graph = nullptr;
    hipGraph_t graph_def = nullptr;
    uint32_t graph_q = 0;
    tl::Timing timing;
    std::vector<hipEvent_t> ev;   // start/stop around graph launches when timing
};

namespace {

tl::DominoDev chain_dev(const tl_batch *b, int32_t i)
{
    const tl::BatchChain &c = b->chains[i];
    tl::DominoDev d;
    d.n = (int)c.n;
    d.omega = ((int)c.n + 1) & 1;
    d.ng = c.ng;
    d.RS = c.RS;
    d.PS = c.PS;
    d.planes = b->planes + c.offset;
    d.spare = nullptr;
    return d;
}

tl_status drop_graph(tl_batch *b)
{
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    if (b->graph_def) (void)hipGraphDestroy(b->graph_def);
    b->graph = nullptr;
    b->graph_def = nullptr;
    b->graph_q = 0;
    return TL_OK;
}

// Bundles for work-groups of `threads`: chains in LPT order go first-fit into
// bundles of at most kBundleMax chains, `threads` (row, group) tasks and the
// LDS of the largest chain, all of one diamond parity (n + 1) & 1, so that a
// colour step is the owner step for every chain of a bundle or for none; a
// chain with more tasks than threads is a bundle alone.  Bundles are ordered by passes per colour step, then tasks.
tl_status bundle_set(tl_batch *b, uint32_t threads, const tl_batch::BundleSet **out)
{
    for (const auto &st : b->sets)
        if (st.threads == threads) {
            *out = &st;
            return TL_OK;
        }
    struct Open {
        uint32_t tasks, lds, parity;
        std::vector<uint32_t> m;
    };
    std::vector<Open> open;
    for (uint32_t ci : b->order) {
        const tl::BatchChain &c = b->chains[ci];
        const uint32_t tasks = c.n * c.ng, lds = c.lds_bytes, parity = (c.n + 1) & 1u;
        bool placed = false;
        if (tasks <= threads)
            for (Open &o : open)
                if (o.parity == parity && o.tasks + tasks <= threads && o.lds + lds <= b->lds_max &&
                    o.m.size() < tl::kBundleMax) {
                    o.tasks += tasks;
                    o.lds += lds;
                    o.m.push_back(ci);
                    placed = true;
                    break;
                }
        if (!placed) open.push_back(Open{tasks, lds, parity, {ci}});
    }
    auto passes = [&](const Open &o) { return (o.tasks + threads - 1) / threads; };
    std::stable_sort(open.begin(), open.end(), [&](const Open &x, const Open &y) {
        return passes(x) != passes(y) ? passes(x) > passes(y) : x.tasks > y.tasks;
    });
    std::vector<tl::BatchBundle> bundles;
    std::vector<uint32_t> members;
    for (const Open &o : open) {
        bundles.push_back(tl::BatchBundle{(uint32_t)members.size(), (uint32_t)o.m.size(), o.tasks, 0u});
        members.insert(members.end(), o.m.begin(), o.m.end());
    }
    tl_batch::BundleSet st;
    st.threads = threads;
    st.count = (uint32_t)bundles.size();
    if (hipMalloc(&st.d_bundles, bundles.size() * sizeof(tl::BatchBundle)) != hipSuccess ||
        hipMalloc(&st.d_members, members.size() * sizeof(uint32_t)) != hipSuccess) {
        if (st.d_bundles) (void)hipFree(st.d_bundles);
        return tl::fail(TL_ENOMEM, "batch bundle tables");
    }
    TL_HIP(hipMemcpy(st.d_bundles, bundles.data(), bundles.size() * sizeof(tl::BatchBundle), hipMemcpyHostToDevice));
    TL_HIP(hipMemcpy(st.d_members, members.data(), members.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    b->sets.push_back(st);
    *out = &b->sets.back();
    return TL_OK;
}

uint32_t workgroups_for(const tl_batch *b, uint32_t threads, uint32_t bundles)
{
    // as many resident work-groups per CU as LDS and threads allow
    uint32_t per_cu = (160u * 1024u) / (b->lds_max + 64u);
    const uint32_t by_threads = 2048u / threads;
    if (per_cu > by_threads) per_cu = by_threads;
    if (per_cu < 1u) per_cu = 1u;
    uint32_t wg = b->cus * per_cu;
    if (wg > bundles) wg = bundles;
    return wg;
}

// The mask model of chain i, attached to the chain's state in the pool.
tl::Model *mask_model(tl_batch *b, int32_t i)
{
    tl::Model *m = b->masks[i].get();
    if (m) {
        uint32_t *st = b->planes + b->chains[i].offset;
        m->attach(st, st);
    }
    return m;
}

tl_status init_all(tl_batch *b)
{
    for (int32_t i = 0; i < b->count; ++i) {
        const bool init_max = b->doms[i].init == TL_INIT_MAX;
        if (tl::Model *m = mask_model(b, i)) {
            TL_HIP(m->init(init_max, b->stream));
            continue;
        }
        const tl::DominoDev d = chain_dev(b, i);
        TL_HIP(tl::domino_init(d, init_max ? 1 : 0, b->stream));
    }
    for (auto &c : b->chains) c.t = 0;
    TL_HIP(hipMemcpyAsync(b->d_chains, b->chains.data(), b->chains.size() * sizeof(tl::BatchChain),
                          hipMemcpyHostToDevice, b->stream));
    b->t = 0;
    return TL_OK;
}

// The bundle set for `threads` must exist (bundle_set) before a capture.
tl_status launch_direct(tl_batch *b, uint32_t nsweeps, uint32_t threads, tl::Timing *tm)
{
    const tl_batch::BundleSet *st = nullptr;
    for (const auto &x : b->sets)
        if (x.threads == threads) st = &x;
    if (!st) return tl::fail(TL_EINVAL, "no bundles for %u threads", threads);
    TL_HIP(tl::domino_batch_sweeps(b->d_chains, st->d_bundles, st->d_members, st->count, b->d_counter, b->planes,
                                   nsweeps, b->T, b->metro ? 1 : 0, b->colour_order, threads,
                                   workgroups_for(b, threads, st->count), b->lds_max, b->stream, tm));
    return TL_OK;
}

}  // namespace

extern "C" {

tl_status tl_batch_create(int32_t n, const tl_domain *doms, const tl_weights *w, const uint64_t *seeds,
                          const tl_options *opt, tl_batch **out)
{
    if (!doms || !w || !seeds || !out || n <= 0) return tl::fail(TL_EINVAL, "invalid batch arguments");
    if (opt && opt->colour_order > 1) return tl::fail(TL_EINVAL, "unknown colour order %u", opt->colour_order);
    if (opt && opt->device_buf) return tl::fail(TL_EINVAL, "batches allocate their own chain pool");
    *out = nullptr;
    // every early return below releases what was set up so far
    struct Destroy {
        void operator()(tl_batch *p) const { (void)tl_batch_destroy(p); }
    };
    std::unique_ptr<tl_batch, Destroy> b(new (std::nothrow) tl_batch());
    if (!b) return tl::fail(TL_ENOMEM, "host allocation failed");
    b->count = n;
    b->doms.assign(doms, doms + n);
    b->seeds.assign(seeds, seeds + n);
    b->w = *w;
    b->metro = w->rule == TL_METROPOLIS;
    b->colour_order = opt ? opt->colour_order : 0u;
    b->masks.resize(n);
    std::vector<uint32_t> thr;
    for (int32_t i = 0; i < n; ++i) {
        tl_domain &d = b->doms[i];
        if (d.model != TL_DOMINO || (d.shape != TL_AZTEC && d.shape != TL_MASK))
            return tl::fail(TL_EINVAL, "batches hold domino chains on Aztec diamonds or masks (chain %d)", i);
        if (d.init != TL_INIT_MIN && d.init != TL_INIT_MAX) return tl::fail(TL_EINVAL, "unknown init (chain %d)", i);
        if (d.shape == TL_MASK) {
            // the host pre-pass (domain checks, Thurston's test, extremal
            // tilings); the chain runs on the Aztec diamond of order
            // ceil((w + h) / 2) that holds the box
            if (d.w < 1 || d.h < 1 || d.w + d.h > 1024)
                return tl::fail(TL_EINVAL, "batched mask boxes need w + h <= 1024 (chain %d)", i);
            std::string why;
            tl_status mst = TL_EINVAL;
            b->masks[i] = tl::make_model(d, why, &mst);
            if (!b->masks[i]) return tl::fail(mst, "chain %d: %s", i, why.c_str());
            d.n = (d.w + d.h + 1) / 2;
            d.mask = nullptr;   // the model keeps its own copy
        }
        if (d.n < 1 || d.n > 512) return tl::fail(TL_EINVAL, "batched Aztec orders must be in [1, 512] (chain %d)", i);
    }
    tl_status st = tl::make_table(doms[0], *w, thr);
    if (st != TL_OK) return st;
    for (size_t i = 0; i < thr.size() && i < 32; ++i) b->T.v[i] = thr[i];
    b->T.count = (uint32_t)std::min<size_t>(thr.size(), 32);
    // layout: chains back to back, each in the single-chain layout
    uint64_t words = 0;
    b->chains.resize(n);
    for (int32_t i = 0; i < n; ++i) {
        tl::BatchChain &c = b->chains[i];
        uint32_t ng, RS;
        size_t PS;
        const size_t wds = tl::domino_words(b->doms[i].n, &ng, &RS, &PS);
        if (b->masks[i] && b->masks[i]->state_words() != wds)
            return tl::fail(TL_EINVAL, "chain %d: mask layout does not match its diamond", i);
        c.offset = words;
        c.PS = PS;
        c.n = (uint32_t)b->doms[i].n;
        c.ng = ng;
        c.RS = RS;
        c.key0 = (uint32_t)seeds[i];
        c.key1 = (uint32_t)(seeds[i] >> 32);
        c.t = 0;
        c.lds_bytes = 4u * c.n * 4u * ng * 4u;
        c.pad = 0;
        words += (wds + 63) / 64 * 64;   // 256-byte aligned chains
        b->lds_max = std::max(b->lds_max, c.lds_bytes);
        b->sites += b->masks[i] ? b->masks[i]->sites() : 2ull * c.n * c.n - 2ull * c.n + 1ull;
        b->owner_bits += 4ull * c.n * c.n;
    }
    if (opt && opt->stream) {
        b->stream = (hipStream_t)opt->stream;
    } else {
        TL_HIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
        b->own_stream = true;
    }
    int dev = 0, cus = 0;
    TL_HIP(hipGetDevice(&dev));
    TL_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    b->cus = (uint32_t)cus;
    if (hipMalloc(&b->planes, words * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&b->d_chains, n * sizeof(tl::BatchChain)) != hipSuccess ||
        hipMalloc(&b->d_counter, sizeof(uint32_t)) != hipSuccess)
        return tl::fail(TL_ENOMEM, "batch state allocation (%zu MB)", (size_t)(words * 4 >> 20));
    // longest chains first
    b->order.resize(n);
    std::iota(b->order.begin(), b->order.end(), 0u);
    std::stable_sort(b->order.begin(), b->order.end(),
                     [&](uint32_t x, uint32_t y) { return b->chains[x].n > b->chains[y].n; });
    if (opt && opt->tile_rows) b->threads = opt->tile_rows;   // work-group size override
    const tl_batch::BundleSet *set = nullptr;
    st = bundle_set(b.get(), b->threads, &set);
    if (st != TL_OK) return st;
    st = init_all(b.get());
    if (st != TL_OK) return st;
    TL_HIP(hipStreamSynchronize(b->stream));
    *out = b.release();
    return TL_OK;
}

tl_status tl_batch_autotune(tl_batch *b, uint32_t probe_sweeps, uint32_t *threads_out, float *ms_out)
{
    if (!b) return tl::fail(TL_EINVAL, "null batch");
    if (b->t != 0) return tl::fail(TL_EINVAL, "autotune runs before the first sweep");
    if (probe_sweeps == 0) probe_sweeps = 1;
    const uint32_t cand[3] = {256u, 512u, 1024u};
    float best = 1e30f;
    uint32_t best_th = b->threads;
    hipEvent_t e0, e1;
    TL_HIP(hipEventCreate(&e0));
    TL_HIP(hipEventCreate(&e1));
    for (uint32_t th : cand) {
        const tl_batch::BundleSet *set = nullptr;
        tl_status sb = bundle_set(b, th, &set);
        if (sb != TL_OK) return sb;
        TL_HIP(hipEventRecord(e0, b->stream));
        tl_status st = launch_direct(b, probe_sweeps, th, nullptr);
        if (st != TL_OK) return st;
        TL_HIP(hipEventRecord(e1, b->stream));
        TL_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        TL_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
            best = ms;
            best_th = th;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->threads = best_th;
    drop_graph(b);
    tl_status st = init_all(b);   // the probes advanced the chains: start again
    if (st != TL_OK) return st;
    TL_HIP(hipStreamSynchronize(b->stream));
    if (threads_out) *threads_out = best_th;
    if (ms_out) *ms_out = best;
    return TL_OK;
}

tl_status tl_batch_sweep(tl_batch *b, uint64_t n)
{
    if (!b) return tl::fail(TL_EINVAL, "null batch");
    if (n == 0) return TL_OK;
    if (b->t + n > 0xFFFFFFFFull) return tl::fail(TL_EINVAL, "sweep counter would exceed 2^32");
    if (b->colour_order && 2 * (b->t + n) > 0x100000000ull)
        return tl::fail(TL_EINVAL, "step counter would exceed 2^32 (random colour order)");
    if (b->graph_q != (uint32_t)n) {
        drop_graph(b);
        const tl_batch::BundleSet *set = nullptr;
        tl_status sb = bundle_set(b, b->threads, &set);   // no allocation inside the capture
        if (sb != TL_OK) return sb;
        TL_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        tl_status st = launch_direct(b, (uint32_t)n, b->threads, nullptr);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(b->stream, &g);
        if (st != TL_OK) return st;
        if (e != hipSuccess) return tl::fail(TL_EDEVICE, "graph capture: %s", hipGetErrorString(e));
        b->graph_def = g;
        TL_HIP(hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0));
        b->graph_q = (uint32_t)n;
    }
    if (b->timing.on) {
        hipEvent_t a, c;
        TL_HIP(b->timing.events(&a, &c));
        TL_HIP(hipEventRecord(a, b->stream));
        TL_HIP(hipGraphLaunch(b->graph, b->stream));
        TL_HIP(hipEventRecord(c, b->stream));
        b->timing.pending.push_back(a);
        b->timing.pending.push_back(c);
        b->timing.pending_steps.push_back(2u * (uint32_t)n);
    } else {
        TL_HIP(hipGraphLaunch(b->graph, b->stream));
    }
    b->t += n;
    return TL_OK;
}

tl_status tl_batch_sync(tl_batch *b)
{
    if (!b) return tl::fail(TL_EINVAL, "null batch");
    TL_HIP(hipStreamSynchronize(b->stream));
    return TL_OK;
}

tl_status tl_batch_reset(tl_batch *b)
{
    if (!b) return tl::fail(TL_EINVAL, "null batch");
    return init_all(b);
}

tl_status tl_batch_info(const tl_batch *b, uint64_t *sites, uint64_t *state_bytes, uint32_t *threads,
                        uint32_t *workgroups)
{
    if (!b) return tl::fail(TL_EINVAL, "null batch");
    if (sites) *sites = b->sites;
    if (state_bytes) *state_bytes = b->owner_bits / 8;
    if (threads) *threads = b->threads;
    if (workgroups) {
        uint32_t nb = (uint32_t)b->count;
        for (const auto &x : b->sets)
            if (x.threads == b->threads) nb = x.count;
        *workgroups = workgroups_for(b, b->threads, nb);
    }
    return TL_OK;
}

tl_status tl_batch_set_timing(tl_batch *b, int enable)
{
    if (!b) return tl::fail(TL_EINVAL, "null batch");
    b->timing.on = enable != 0;
    return TL_OK;
}

tl_status tl_batch_kernel_time(tl_batch *b, double *ms, uint64_t *launches, uint64_t *colour_steps)
{
    if (!b) return tl::fail(TL_EINVAL, "null batch");
    TL_HIP(hipStreamSynchronize(b->stream));
    TL_HIP(b->timing.collect());
    if (ms) *ms = b->timing.ms;
    if (launches) *launches = b->timing.launches;
    if (colour_steps) *colour_steps = b->timing.steps;
    b->timing.ms = 0.0;
    b->timing.launches = b->timing.steps = 0;
    return TL_OK;
}

tl_status tl_batch_export_size(tl_batch *b, int32_t chain, size_t *bytes, uint32_t *rows, uint32_t *row_bytes)
{
    if (!b) return tl::fail(TL_EINVAL, "null batch");
    if (chain < 0 || chain >= b->count) return tl::fail(TL_EINVAL, "chain %d out of range", chain);
    uint32_t r = 2u * b->chains[chain].n, rb = r;
    if (const tl::Model *m = b->masks[chain].get()) m->export_layout(&r, &rb);
    if (bytes) *bytes = (size_t)r * rb;
    if (rows) *rows = r;
    if (row_bytes) *row_bytes = rb;
    return TL_OK;
}

}  // extern "C"

namespace {

// Canonical export of one chain into device memory (the diamond's box, or the
// mask's box).
hipError_t export_chain(tl_batch *b, int32_t chain, uint8_t *dev)
{
    if (tl::Model *m = mask_model(b, chain)) return m->export_canonical(dev, b->stream);
    return tl::domino_export(chain_dev(b, chain), dev, b->stream);
}

}  // namespace

extern "C" {

tl_status tl_batch_export(tl_batch *b, int32_t chain, void *host, size_t bytes)
{
    if (!b || !host) return tl::fail(TL_EINVAL, "null argument");
    size_t need = 0;
    tl_status st = tl_batch_export_size(b, chain, &need, nullptr, nullptr);
    if (st != TL_OK) return st;
    if (bytes < need) return tl::fail(TL_EINVAL, "export buffer has %zu bytes, %zu needed", bytes, need);
    uint8_t *dev = nullptr;
    TL_HIP(hipMalloc(&dev, need));
    hipError_t e = export_chain(b, chain, dev);
    if (e == hipSuccess) e = hipMemcpyAsync(host, dev, need, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    (void)hipFree(dev);
    if (e != hipSuccess) return tl::fail(TL_EDEVICE, "batch export: %s", hipGetErrorString(e));
    return TL_OK;
}

tl_status tl_batch_hash(tl_batch *b, int32_t chain, uint8_t digest[32])
{
    if (!b || !digest) return tl::fail(TL_EINVAL, "null argument");
    size_t need = 0;
    uint32_t rows = 0, rb = 0;
    tl_status st = tl_batch_export_size(b, chain, &need, &rows, &rb);
    if (st != TL_OK) return st;
    uint8_t *dev = nullptr;
    TL_HIP(hipMalloc(&dev, need + 32 * (size_t)rows));
    std::vector<uint8_t> rowd(32 * (size_t)rows);
    hipError_t e = export_chain(b, chain, dev);
    if (e == hipSuccess) e = tl::hash_rows(dev, rows, rb, dev + need, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(rowd.data(), dev + need, rowd.size(), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    (void)hipFree(dev);
    if (e != hipSuccess) return tl::fail(TL_EDEVICE, "batch hash: %s", hipGetErrorString(e));
    tl::sha256_host(rowd.data(), rowd.size(), digest);
    return TL_OK;
}

tl_status tl_batch_destroy(tl_batch *b)
{
    if (!b) return TL_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    b->timing.release();
    if (b->planes) (void)hipFree(b->planes);
    if (b->d_chains) (void)hipFree(b->d_chains);
    for (auto &x : b->sets) {
        if (x.d_bundles) (void)hipFree(x.d_bundles);
        if (x.d_members) (void)hipFree(x.d_members);
    }
    if (b->d_counter) (void)hipFree(b->d_counter);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return TL_OK;
}

}  // extern "C"
