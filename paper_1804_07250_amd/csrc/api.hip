// C-ABI of the Glauber-sweep library (include/tilings.h): sampler objects,
// threshold tables, sweep scheduling, observables, export, import and hashing.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <cstdio>
#include <deque>
#include <thread>

#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tilings.h"
#include "errors.hpp"
#include "exact_ratio.hpp"
#include "internal.hpp"
#include "models.hpp"
#include "region.hpp"

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace tl {
tl_status fail(tl_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}
}  // namespace tl

using tl::fail;

namespace {

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

}  // namespace

struct tl_sampler {
    tl_domain dom{};
    tl_weights w{};
    uint64_t seed = 0;
    tl_options opt{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;                    // device current at creation: the state lives there
    uint64_t t = 0;
    uint64_t samples = 0;
    std::vector<uint32_t> thr;
    std::vector<uint32_t> thr_free;    // six-vertex free north edges
    std::unique_ptr<tl::Model> model;
    unsigned long long *bin_sum = nullptr;  // device accumulators
    unsigned long long *bin_tmp = nullptr;
    uint32_t bins_x = 0, bins_y = 0, B = 1;
    std::vector<uint32_t> cells_per_bin;    // lazily computed on the host

    // Releases whatever was set up (also after a failed create).
    ~tl_sampler()
    {
        if (stream) (void)hipStreamSynchronize(stream);
        if (model) model->release();
        if (bin_sum) (void)hipFree(bin_sum);
        if (bin_tmp) (void)hipFree(bin_tmp);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

namespace {

tl_status make_thresholds(const tl_domain &d, const tl_weights &w, std::vector<uint32_t> &thr)
{
    if (d.flags && (d.model != TL_SIXVERTEX || d.shape != TL_MASK || tl::free_side_of(d.flags) < 0))
        return fail(TL_EINVAL, "free sides are a six-vertex mask option, one side per domain");
    using tl::Ratio;
    const bool metro = w.rule == TL_METROPOLIS;
    if (w.rule != TL_HEATBATH && w.rule != TL_METROPOLIS) return fail(TL_EINVAL, "unknown rule %d", w.rule);
    std::vector<Ratio> R;
    const Ratio one;
    switch (d.model) {
    case TL_DOMINO:
        if (w.kind == TL_W_UNIFORM) {
            R.assign(4, one);
        } else if (w.kind == TL_W_TWO_PERIODIC) {
            if (!finite_pos(w.w[0]) || !finite_pos(w.w[1])) return fail(TL_EINVAL, "two-periodic weights must be > 0");
            const Ratio b2a2 = (Ratio::of(w.w[1]) / Ratio::of(w.w[0])).pow(2);
            R = {one, one, b2a2, b2a2.inv()};
        } else if (w.kind == TL_W_VOLUME_BW) {
            Ratio q[2];
            for (int i = 0; i < 2; ++i) {
                const double num = w.w[2 * i], den = w.w[2 * i + 1];
                if (!finite_pos(num) || (den != 0.0 && !finite_pos(den)))
                    return fail(TL_EINVAL, "volume weights must be > 0");
                q[i] = den > 0.0 ? Ratio::of(num) / Ratio::of(den) : Ratio::of(num);
            }
            // vertical raises the height by 4 at black (x+y even) vertices, lowers it at white ones
            R = {q[0].pow(4), q[0].pow(4), q[1].pow(-4), q[1].pow(-4)};
        } else {
            return fail(TL_EINVAL, "weight kind %d does not apply to dominoes", w.kind);
        }
        break;
    case TL_LOZENGE:
        if (w.kind == TL_W_UNIFORM) {
            R = {one};
        } else if (w.kind == TL_W_VOLUME) {
            if (!finite_pos(w.w[0])) return fail(TL_EINVAL, "volume weight q must be > 0");
            if (w.w[1] != 0.0 && !finite_pos(w.w[1])) return fail(TL_EINVAL, "volume weight denominator must be > 0");
            R = {w.w[1] > 0.0 ? Ratio::of(w.w[0]) / Ratio::of(w.w[1]) : Ratio::of(w.w[0])};
        } else {
            return fail(TL_EINVAL, "weight kind %d does not apply to lozenges", w.kind);
        }
        break;
    case TL_SIXVERTEX: {
        Ratio a2, b2, c2;
        if (w.kind == TL_W_SIXVERTEX6) {
            // With the boundary fixed, each corner of a flipped face moves
            // between two types whose weights multiply to a1 a2, b1 b2 or
            // c1 c2, so the chain sees the six weights only through those
            // products: a^2 = a1 a2, b^2 = b1 b2, c^2 = c1 c2.
            for (int i = 0; i < 6; ++i)
                if (!finite_pos(w.w[i])) return fail(TL_EINVAL, "six-vertex weights must be > 0");
            a2 = Ratio::of(w.w[0]) * Ratio::of(w.w[1]);
            b2 = Ratio::of(w.w[2]) * Ratio::of(w.w[3]);
            c2 = Ratio::of(w.w[4]) * Ratio::of(w.w[5]);
        } else if (w.kind == TL_W_SIXVERTEX) {
            if (!finite_pos(w.w[0]) || !finite_pos(w.w[1]) || !finite_pos(w.w[2]))
                return fail(TL_EINVAL, "six-vertex weights must be > 0");
            a2 = Ratio::of(w.w[0]);
            b2 = Ratio::of(w.w[1]);
            c2 = Ratio::of(w.w[2]);
        } else if (w.kind != TL_W_UNIFORM) {
            return fail(TL_EINVAL, "weight kind %d does not apply to the six-vertex model", w.kind);
        }
        // W_up / W_down = prod over the corners (c/w)^(+1 if the corner's diagonal
        // face is high, -1 otherwise), w = a at NE and SW, b at NW and SE; the
        // exponents of a, b and c are even, so squares suffice.
        for (int mask = 0; mask < 16; ++mask) {
            const int hNE = mask & 1, hNW = (mask >> 1) & 1, hSW = (mask >> 2) & 1, hSE = (mask >> 3) & 1;
            const int ea = 1 - hNE - hSW;   // exponent of a^2
            const int eb = 1 - hNW - hSE;   // exponent of b^2
            const int ec = hNE + hNW + hSW + hSE - 2;   // exponent of c^2
            R.push_back(a2.pow(ea) * b2.pow(eb) * c2.pow(ec));
        }
        break;
    }
    default:
        return fail(TL_EINVAL, "unknown model %d", d.model);
    }
    if (!tl::exact_thresholds(R, metro, thr))
        return fail(TL_EINVAL, "weights too uneven for 32-bit Metropolis thresholds (a ratio above 2^31)");
    return TL_OK;
}

// Table of the free points of a six-vertex domain (empty for any other
// domain).  Such a flip changes only the two cells beside the point's three
// neighbours; reading each cell's type off its corners (a1 none of its four
// edges carries a path, a2 all four, b1 left and right, b2 bottom and top, c1
// bottom and left, c2 right and top) with the neighbours at m, W_up / W_down
// over the context (first diagonal high) + 2 (second diagonal high) is
//   north (cells SW, SE of the point):  (SW ? c2/a1 : a2/c1) (SE ? c1/b2 : b1/c2)
//   south (cells NW, NE):               (NW ? c1/b1 : b2/c2) (NE ? c2/a2 : a1/c1)
//   east  (cells SW, NW; diagonals SW, NW): (SW ? c2/a1 : a2/c1) (NW ? c1/b1 : b2/c2)
//   west  (cells SE, NE; diagonals SE, NE): (SE ? c1/b2 : b1/c2) (NE ? c2/a2 : a1/c1)
tl_status make_free_thresholds(const tl_domain &d, const tl_weights &w, std::vector<uint32_t> &out)
{
    using tl::Ratio;
    out.clear();
    const int side = tl::free_side_of(d.flags);
    if (d.model != TL_SIXVERTEX || d.shape != TL_MASK || side <= 0) return TL_OK;
    Ratio a1, a2, b1, b2, c1, c2;
    if (w.kind == TL_W_SIXVERTEX6) {
        for (int i = 0; i < 6; ++i)
            if (!finite_pos(w.w[i])) return fail(TL_EINVAL, "six-vertex weights must be > 0");
        a1 = Ratio::of(w.w[0]);
        a2 = Ratio::of(w.w[1]);
        b1 = Ratio::of(w.w[2]);
        b2 = Ratio::of(w.w[3]);
        c1 = Ratio::of(w.w[4]);
        c2 = Ratio::of(w.w[5]);
    } else if (w.kind != TL_W_UNIFORM) {
        return fail(TL_EINVAL, "free sides need uniform weights or the six vertex weights");
    }
    std::vector<Ratio> R;
    for (int ctx = 0; ctx < 4; ++ctx) {
        const bool d0 = ctx & 1, d1 = ctx & 2;
        switch (side) {
        case 1: R.push_back((d0 ? c2 / a1 : a2 / c1) * (d1 ? c1 / b2 : b1 / c2)); break;
        case 2: R.push_back((d0 ? c1 / b1 : b2 / c2) * (d1 ? c2 / a2 : a1 / c1)); break;
        case 3: R.push_back((d0 ? c2 / a1 : a2 / c1) * (d1 ? c1 / b1 : b2 / c2)); break;
        default: R.push_back((d0 ? c1 / b2 : b1 / c2) * (d1 ? c2 / a2 : a1 / c1)); break;
        }
    }
    if (!tl::exact_thresholds(R, w.rule == TL_METROPOLIS, out))
        return fail(TL_EINVAL, "weights too uneven for 32-bit Metropolis thresholds (a ratio above 2^31)");
    return TL_OK;
}

tl::Thr table_of(const tl_sampler *s)
{
    tl::Thr T{};
    for (size_t i = 0; i < s->thr.size() && i < 32; ++i) T.v[i] = s->thr[i];
    T.count = (uint32_t)(s->thr.size() < 32 ? s->thr.size() : 32);
    return T;
}

// Sets *flag when the word arrays a and b differ anywhere.
__global__ void __launch_bounds__(256) words_differ_kernel(const uint32_t *a, const uint32_t *b, size_t n,
                                                           uint32_t *flag)
{
    uint32_t acc = 0u;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) acc |= a[i] ^ b[i];
    if (acc) atomicOr(flag, 1u);
}

// Coupling from the past with rounds side by side (one-tile states).  Round R
// is the same computation as in the sequential doubling (both chains over the
// counters [2^(R-1), 2^R), ..., [1, 2), [0, 1)); up to kRounds rounds run at
// once, each on its own stream (the sampler's and two more, so that every
// round has a hardware queue of its own under the default four) with its own
// two chains, issued in pieces of at most kPiece sweeps with at most kRing
// pieces in flight, so that a round made unnecessary by a smaller round that
// met stops after its current pieces.  Rounds are checked in order of R: the
// answer is the smallest R whose chains meet, exactly as when the rounds run
// one after the other.
struct CftpRound {
    static constexpr uint32_t kRing = 2;
    uint32_t R = 0;
    std::unique_ptr<tl::Model> bot, top;
    hipStream_t st = nullptr;
    bool own_stream = false;
    uint32_t *d_flag = nullptr, *h_flag = nullptr;
    tl::TileJob *h_jobs = nullptr, *d_jobs = nullptr;   // kRing x 2 descriptors
    hipEvent_t ring[kRing] = {};
    bool ring_used[kRing] = {};   // a piece has been recorded on ring[i]
    hipEvent_t done = nullptr;
    uint32_t slot = 0;
    std::vector<std::pair<uint32_t, uint32_t>> pieces;   // (first sweep counter, sweeps)
    size_t next = 0;
    bool checked = false;

    hipError_t setup(const tl::Model &m, hipStream_t shared)
    {
        bot = m.twin();
        top = m.twin();
        hipError_t e = bot->allocate();
        if (e == hipSuccess) e = top->allocate();
        if (shared) {
            st = shared;
        } else if (e == hipSuccess) {
            e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
            own_stream = e == hipSuccess;
        }
        if (e == hipSuccess) e = hipMalloc(&d_flag, sizeof(uint32_t));
        if (e == hipSuccess) e = hipHostMalloc((void **)&h_flag, sizeof(uint32_t), hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void **)&h_jobs, 2 * kRing * sizeof(tl::TileJob), hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc(&d_jobs, 2 * kRing * sizeof(tl::TileJob));
        for (uint32_t i = 0; i < kRing && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&ring[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
        return e;
    }
    void teardown()
    {
        if (st) (void)hipStreamSynchronize(st);
        if (bot) bot->release();
        if (top) top->release();
        for (hipEvent_t &ev : ring)
            if (ev) (void)hipEventDestroy(ev);
        if (done) (void)hipEventDestroy(done);
        if (d_jobs) (void)hipFree(d_jobs);
        if (h_jobs) (void)hipHostFree(h_jobs);
        if (h_flag) (void)hipHostFree(h_flag);
        if (d_flag) (void)hipFree(d_flag);
        if (own_stream) (void)hipStreamDestroy(st);
    }
    hipError_t start(uint32_t r_log2, uint32_t piece)
    {
        R = r_log2;
        next = 0;
        checked = false;
        pieces.clear();
        for (int r = (int)R; r >= 0; --r) {
            const uint32_t t0 = r ? 1u << (r - 1) : 0u, count = r ? 1u << (r - 1) : 1u;
            for (uint32_t k = 0; k < count; k += piece) pieces.emplace_back(t0 + k, std::min(piece, count - k));
        }
        hipError_t e = bot->init(false, st);
        if (e == hipSuccess) e = top->init(true, st);
        return e;
    }
};

hipError_t cftp_issue_piece(CftpRound &rd, const tl::Thr &T, uint64_t seed, const tl::TileItem *d_items)
{
    const uint32_t sl = rd.slot % CftpRound::kRing;
    const auto pc = rd.pieces[rd.next];
    tl::TilePlan pb, pt;
    tl::TileJob *hj = rd.h_jobs + 2 * sl;
    if (!rd.bot->tile_job(pc.first, pc.second, T, false, seed, false, &hj[0], &pb) ||
        !rd.top->tile_job(pc.first, pc.second, T, false, seed, false, &hj[1], &pt) || pb.S != pc.second ||
        pb.tiles() != 1 || pt.tiles() != 1)
        return hipErrorInvalidConfiguration;
    hipError_t e = hipMemcpyAsync(rd.d_jobs + 2 * sl, hj, 2 * sizeof(tl::TileJob), hipMemcpyHostToDevice, rd.st);
    if (e == hipSuccess)
        e = rd.bot->height_family()
                ? tl::height_items(rd.d_jobs + 2 * sl, d_items, 2, std::max(pb.threads, pt.threads),
                                   std::max(pb.lds, pt.lds), hj[0].mode, hj[0].kind, pb.order, hj[0].site != nullptr,
                                   rd.st)
                : tl::domino_items(rd.d_jobs + 2 * sl, d_items, 2, std::max(pb.threads, pt.threads),
                                   std::max(pb.lds, pt.lds), pb.order, rd.st);
    if (e == hipSuccess) e = hipEventRecord(rd.ring[sl], rd.st);
    if (e == hipSuccess) {
        rd.ring_used[sl] = true;
        rd.bot->swap_buffers();
        rd.top->swap_buffers();
        ++rd.slot;
        ++rd.next;
    }
    return e;
}

hipError_t cftp_queue_check(CftpRound &rd)
{
    const size_t words = rd.bot->state_words();
    hipError_t e = hipMemsetAsync(rd.d_flag, 0, sizeof(uint32_t), rd.st);
    if (e == hipSuccess) {
        size_t blocks = (words + 255) / 256;
        if (blocks > 2048) blocks = 2048;
        hipLaunchKernelGGL(words_differ_kernel, dim3((uint32_t)blocks), dim3(256), 0, rd.st, rd.bot->state(),
                           rd.top->state(), words, rd.d_flag);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(rd.h_flag, rd.d_flag, sizeof(uint32_t), hipMemcpyDeviceToHost, rd.st);
    if (e == hipSuccess) e = hipEventRecord(rd.done, rd.st);
    if (e == hipSuccess) rd.checked = true;
    return e;
}

// Runs the rounds; on return *R_out is the round whose chains met (*met) or
// the last round, and the sampler's state holds that round's minimal chain.
hipError_t cftp_side_by_side(tl_sampler *s, uint32_t max_log2, const tl::Thr &T, uint32_t *R_out, bool *met)
{
    constexpr uint32_t kRounds = 3, kPiece = 512;
    std::vector<std::unique_ptr<CftpRound>> all;
    std::deque<CftpRound *> active, idle;
    tl::TileItem *d_items = nullptr;
    const tl::TileItem items[2] = {{0u, 0u}, {1u, 0u}};
    hipError_t e = hipMalloc(&d_items, sizeof(items));
    if (e == hipSuccess) e = hipMemcpy(d_items, items, sizeof(items), hipMemcpyHostToDevice);
    for (uint32_t i = 0; i < std::min(kRounds, max_log2) && e == hipSuccess; ++i) {
        all.emplace_back(new CftpRound());
        e = all.back()->setup(*s->model, i == 0 ? s->stream : nullptr);
        idle.push_back(all.back().get());
    }
    uint32_t next_R = 1;
    CftpRound *answer = nullptr;
    *met = false;
    while (e == hipSuccess && !answer) {
        while (!idle.empty() && next_R <= max_log2 && e == hipSuccess) {
            CftpRound *rd = idle.front();
            idle.pop_front();
            e = rd->start(next_R++, kPiece);
            active.push_back(rd);
        }
        bool progress = false;
        for (CftpRound *rd : active) {
            while (e == hipSuccess && rd->next < rd->pieces.size()) {
                // the ring slot is free once the piece that last used it has run
                const uint32_t sl = rd->slot % CftpRound::kRing;
                if (rd->ring_used[sl]) {
                    const hipError_t q = hipEventQuery(rd->ring[sl]);
                    if (q == hipErrorNotReady) break;
                    if (q != hipSuccess) {
                        e = q;
                        break;
                    }
                }
                e = cftp_issue_piece(*rd, T, s->seed, d_items);
                progress = true;
            }
            if (e == hipSuccess && rd->next == rd->pieces.size() && !rd->checked) {
                e = cftp_queue_check(*rd);
                progress = true;
            }
        }
        if (e != hipSuccess) break;
        if (active.empty()) {
            e = hipErrorUnknown;
            break;
        }
        CftpRound *front = active.front();
        if (front->checked) {
            const hipError_t q = hipEventQuery(front->done);
            if (q == hipSuccess) {
                if (*front->h_flag == 0u || front->R == max_log2) {
                    *met = *front->h_flag == 0u;
                    answer = front;
                } else {
                    active.pop_front();
                    idle.push_back(front);
                }
                progress = true;
            } else if (q != hipErrorNotReady) {
                e = q;
            }
        }
        if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    if (e == hipSuccess && answer) {
        *R_out = answer->R;
        e = hipStreamSynchronize(answer->st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(const_cast<uint32_t *>(s->model->state()), answer->bot->state(),
                               s->model->state_words() * sizeof(uint32_t), hipMemcpyDeviceToDevice, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    }
    for (auto &rd : all) rd->teardown();   // waits for the rounds still running
    if (d_items) (void)hipFree(d_items);
    return e;
}

tl_status enqueue_sample(tl_sampler *s)
{
    TL_HIP(s->model->observe(s->B, s->bins_x, s->bin_sum, s->stream));
    s->samples += 1;
    return TL_OK;
}

}  // namespace

namespace tl {
hipStream_t sampler_stream(const tl_sampler *s) { return s->stream; }
tl_status make_table(const tl_domain &d, const tl_weights &w, std::vector<uint32_t> &thr)
{
    return make_thresholds(d, w, thr);
}
tl_status make_free_table(const tl_domain &d, const tl_weights &w, std::vector<uint32_t> &thr)
{
    return make_free_thresholds(d, w, thr);
}
}  // namespace tl

namespace {

// Cache key of a tile shape: model, shape and sizes, table kind, colour
// order and device (architecture and CU count).
std::string tune_key(const tl_sampler *s, bool uniform)
{
    int dev = 0;
    hipDeviceProp_t prop{};
    std::string arch = "?";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount);
    for (char &ch : arch)
        if (ch == ' ') ch = '_';
    const tl_domain &d = s->dom;
    std::string k = "m" + std::to_string(d.model) + ":s" + std::to_string(d.shape) + ":" + std::to_string(d.n) + "," +
                    std::to_string(d.a) + "," + std::to_string(d.b) + "," + std::to_string(d.c) + "," +
                    std::to_string(d.w) + "x" + std::to_string(d.h) + "," + std::to_string(s->model->sites()) +
                    ":f" + std::to_string(d.flags) + ":" + (uniform ? "one-bit" : "weighted") + ":o" +
                    std::to_string(s->opt.colour_order) + ":" + arch;
    return k;
}

// Last entry of `key` in the cache file: rows, groups, sweeps and the tiled
// kernel (2 when the line has no fourth number); false if none.
bool tune_lookup(const char *path, const std::string &key, uint32_t v[4])
{
    FILE *f = path ? std::fopen(path, "r") : nullptr;
    if (!f) return false;
    char line[1024];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char k[768];
        unsigned a, b, c, kk = 2;
        const int got = std::sscanf(line, "%767s %u %u %u %u", k, &a, &b, &c, &kk);
        if (got >= 4 && key == k) {
            v[0] = a;
            v[1] = b;
            v[2] = c;
            v[3] = got == 5 ? kk : 2u;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

}  // namespace

extern "C" {

const char *tl_status_str(tl_status st)
{
    switch (st) {
    case TL_OK: return "ok";
    case TL_EINVAL: return "invalid argument";
    case TL_EUNTILEABLE: return "domain not tileable";
    case TL_ENOMEM: return "out of memory";
    case TL_EBUDGET: return "over memory budget";
    case TL_EDEVICE: return "device error";
    case TL_EBUSY: return "busy";
    }
    return "unknown status";
}

const char *tl_last_error(void) { return g_last_error.c_str(); }

tl_status tl_domain_extremes(const tl_domain *dom, void *tmax, void *tmin, size_t bytes)
{
    if (!dom) return fail(TL_EINVAL, "null argument");
    if (dom->shape != TL_MASK)
        return fail(TL_EINVAL, "extremal states are computed for mask domains");
    if (dom->flags && (dom->model != TL_SIXVERTEX || tl::free_side_of(dom->flags) < 0))
        return fail(TL_EINVAL, "free sides are a six-vertex option, one side per domain");
    if (dom->model == TL_SIXVERTEX || dom->model == TL_LOZENGE) {
        tl::HeightRegion r;
        std::string why;
        const tl::RegionStatus st = dom->model == TL_SIXVERTEX
                                        ? tl::build_sixv_region(dom->mask, dom->w, dom->h,
                                                                tl::free_side_of(dom->flags), r, why)
                                        : tl::build_loz_region(dom->mask, dom->w, dom->h, r, why);
        if (st != tl::kRegionOk)
            return fail(st == tl::kRegionUntileable ? TL_EUNTILEABLE : TL_EINVAL, "%s", why.c_str());
        const size_t need = r.hmax.size() * sizeof(int32_t);
        if ((tmax || tmin) && bytes < need) return fail(TL_EINVAL, "buffers hold %zu bytes, %zu needed", bytes, need);
        if (tmax) memcpy(tmax, r.hmax.data(), need);
        if (tmin) memcpy(tmin, r.hmin.data(), need);
        return TL_OK;
    }
    if (dom->model != TL_DOMINO) return fail(TL_EINVAL, "unknown model %d", dom->model);
    tl::Region r;
    std::string why;
    const tl::RegionStatus st = tl::build_region(dom->mask, dom->w, dom->h, r, why);
    if (st != tl::kRegionOk) return fail(st == tl::kRegionUntileable ? TL_EUNTILEABLE : TL_EINVAL, "%s", why.c_str());
    const size_t need = (size_t)r.w * r.h;
    if ((tmax || tmin) && bytes < need) return fail(TL_EINVAL, "buffers hold %zu bytes, %zu needed", bytes, need);
    if (tmax) memcpy(tmax, r.tmax.data(), need);
    if (tmin) memcpy(tmin, r.tmin.data(), need);
    return TL_OK;
}

tl_status tl_thresholds(const tl_domain *dom, const tl_weights *w, uint32_t *out, uint32_t cap, uint32_t *count)
{
    if (!dom || !w) return fail(TL_EINVAL, "null argument");
    std::vector<uint32_t> thr, thr_free;
    tl_status st = make_thresholds(*dom, *w, thr);
    if (st == TL_OK) st = make_free_thresholds(*dom, *w, thr_free);
    if (st != TL_OK) return st;
    thr.insert(thr.end(), thr_free.begin(), thr_free.end());
    if (count) *count = (uint32_t)thr.size();
    if (out)
        for (uint32_t i = 0; i < cap && i < thr.size(); ++i) out[i] = thr[i];
    return TL_OK;
}

// Bytes of one state buffer inside caller-owned memory, rounded up so that the
// second buffer starts 256-byte aligned like a hipMalloc allocation.
static size_t state_half_bytes(const tl::Model &m)
{
    return (m.state_words() * sizeof(uint32_t) + 255u) & ~(size_t)255u;
}

tl_status tl_sampler_create(const tl_domain *dom, const tl_weights *w, uint64_t seed, const tl_options *opt,
                            tl_sampler **out)
{
    if (!dom || !w || !out) return fail(TL_EINVAL, "null argument");
    *out = nullptr;
    std::unique_ptr<tl_sampler> s(new (std::nothrow) tl_sampler());
    if (!s) return fail(TL_ENOMEM, "host allocation failed");
    s->dom = *dom;
    s->w = *w;
    s->seed = seed;
    if (opt) s->opt = *opt;
    if (dom->init != TL_INIT_MIN && dom->init != TL_INIT_MAX) return fail(TL_EINVAL, "unknown init %d", dom->init);
    if (s->opt.colour_order > 1) return fail(TL_EINVAL, "unknown colour order %u", s->opt.colour_order);
    tl_status st = make_thresholds(*dom, *w, s->thr);
    if (st == TL_OK) st = make_free_thresholds(*dom, *w, s->thr_free);
    if (st != TL_OK) return st;
    std::string why;
    tl_status mst = TL_EINVAL;
    s->model = tl::make_model(*dom, why, &mst);
    if (!s->model) return fail(mst, "%s", why.c_str());
    s->dom.mask = nullptr;   // the model keeps its own copy of a mask
    s->model->order = s->opt.colour_order;
    s->model->set_boundary_table(s->thr_free);
    TL_HIP(hipGetDevice(&s->device));
    if (s->opt.stream) {
        s->stream = (hipStream_t)s->opt.stream;
    } else {
        TL_HIP(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
        s->own_stream = true;
    }
    hipError_t e;
    if (s->opt.device_buf) {
        // the state in caller-owned memory: two buffers, each 256-byte aligned
        const size_t half = state_half_bytes(*s->model), need = 2 * half;
        if (s->opt.device_buf_bytes < need || ((uintptr_t)s->opt.device_buf & 255u))
            return fail(TL_EINVAL, "device_buf must hold %zu bytes, 256-byte aligned", need);
        char *buf = (char *)s->opt.device_buf;
        e = s->model->allocate_into((uint32_t *)buf, (uint32_t *)(buf + half));
    } else {
        e = s->model->allocate();
    }
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? TL_ENOMEM : TL_EDEVICE, "state allocation: %s", hipGetErrorString(e));
    s->B = s->opt.obs_bin ? s->opt.obs_bin : 1u;
    uint32_t cw, ch;
    s->model->cell_box(&cw, &ch);
    s->bins_x = (cw + s->B - 1) / s->B;
    s->bins_y = (ch + s->B - 1) / s->B;
    const size_t nb = (size_t)s->bins_x * s->bins_y;
    if (hipMalloc(&s->bin_sum, nb * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&s->bin_tmp, nb * sizeof(unsigned long long)) != hipSuccess)
        return fail(TL_ENOMEM, "observable buffers");
    TL_HIP(hipMemsetAsync(s->bin_sum, 0, nb * sizeof(unsigned long long), s->stream));
    TL_HIP(s->model->init(dom->init == TL_INIT_MAX, s->stream));
    *out = s.release();
    return TL_OK;
}


tl_status tl_sampler_autotune(tl_sampler *s, uint32_t probe_sweeps, tl_tune_info *out)
{
    if (!s) return fail(TL_EINVAL, "null sampler");
    if (s->opt.kernel == 1) return fail(TL_EINVAL, "the streaming kernel has no tile shape");
    if (probe_sweeps == 0) probe_sweeps = 50;
    const tl::Thr T = table_of(s);
    const bool metro = s->w.rule == TL_METROPOLIS;
    const std::string key = tune_key(s, T.uniform());
    tl_tune_info info{};
    uint32_t cached[4];
    if (tune_lookup(s->opt.tune_cache, key, cached)) {
        s->model->tuned_rows = cached[0];
        s->model->tuned_groups = cached[1];
        s->model->tuned_sweeps = cached[2];
        s->model->tuned_kernel = cached[3];
        info.tile_rows = cached[0];
        info.tile_groups = cached[1];
        info.sweeps_per_launch = cached[2];
        info.kernel = cached[3];
        info.from_cache = 1;
        if (out) *out = info;
        return TL_OK;
    }
    // candidates: the automatic shape first, then heights x widths x sweeps
    struct Cand {
        uint32_t rows, groups, sweeps, kernel;
    };
    std::vector<Cand> cands{{0u, 0u, 0u, 2u}};
    const uint32_t ng = s->model->row_groups();
    std::vector<uint32_t> widths{ng <= 8u ? ng : 8u};
    if (ng > 4u) widths.push_back(4u);
    if (ng > 2u) widths.push_back(2u);
    const bool domino = !s->model->height_family();
    const std::vector<uint32_t> rows = domino ? std::vector<uint32_t>{16u, 24u, 32u, 48u}
                                              : std::vector<uint32_t>{4u, 8u, 16u, 32u};
    const std::vector<uint32_t> sweeps = domino ? std::vector<uint32_t>{12u, 25u} : std::vector<uint32_t>{4u, 6u, 8u, 16u};
    for (uint32_t r : rows)
        for (uint32_t g : widths)
            for (uint32_t sw : sweeps) cands.push_back(Cand{r, g, sw, 2u});
    if (domino) {
        // register tiles: 64 lanes of rows, halo included (the plan trims the
        // sweeps per launch to what the halo covers)
        for (uint32_t r : {24u, 32u, 40u, 48u})
            for (uint32_t g : {2u, 4u})
                if (g <= ng) cands.push_back(Cand{r, g, (64u - r) / 2u, 3u});
    }
    // probe on a copy of the state, from the sampler's sweep counter
    std::unique_ptr<tl::Model> probe = s->model->twin();
    hipError_t e = probe->allocate();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess)
        e = hipMemcpyAsync(const_cast<uint32_t *>(probe->state()), s->model->state(),
                           s->model->state_words() * sizeof(uint32_t), hipMemcpyDeviceToDevice, s->stream);
    tl_options popt = s->opt;
    popt.tile_rows = popt.tile_groups = popt.sweeps_per_launch = 0;
    popt.kernel = 0;
    const uint32_t t0 = (uint32_t)s->t;
    float best = -1.0f;
    Cand pick{0u, 0u, 0u, 2u};
    for (const Cand &c : cands) {
        if (e != hipSuccess) break;
        probe->tuned_rows = c.rows;
        probe->tuned_groups = c.groups;
        probe->tuned_sweeps = c.sweeps;
        probe->tuned_kernel = c.kernel;
        hipError_t pe = probe->sweeps(t0, probe_sweeps, T, metro, s->seed, popt, s->stream);   // warm-up
        if (pe == hipErrorInvalidConfiguration) {   // no launch plan for this shape
            (void)hipGetLastError();
            continue;
        }
        if (pe == hipSuccess) pe = hipEventRecord(e0, s->stream);
        if (pe == hipSuccess) pe = probe->sweeps(t0, probe_sweeps, T, metro, s->seed, popt, s->stream);
        if (pe == hipSuccess) pe = hipEventRecord(e1, s->stream);
        if (pe == hipSuccess) pe = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (pe == hipSuccess) pe = hipEventElapsedTime(&ms, e0, e1);
        if (pe != hipSuccess) {
            e = pe;
            break;
        }
        ++info.candidates;
        if (best < 0.0f || ms < best) {
            best = ms;
            pick = c;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    probe->release();
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? TL_ENOMEM : TL_EDEVICE, "autotune: %s", hipGetErrorString(e));
    if (info.candidates == 0) return fail(TL_EINVAL, "no tile shape has a launch plan for this domain");
    s->model->tuned_rows = pick.rows;
    s->model->tuned_groups = pick.groups;
    s->model->tuned_sweeps = pick.sweeps;
    s->model->tuned_kernel = pick.kernel;
    info.tile_rows = pick.rows;
    info.tile_groups = pick.groups;
    info.sweeps_per_launch = pick.sweeps;
    info.kernel = pick.kernel;
    info.ms_per_sweep = best / (float)probe_sweeps;
    if (s->opt.tune_cache) {
        FILE *f = std::fopen(s->opt.tune_cache, "a");
        if (!f) return fail(TL_EINVAL, "cannot append to the tune cache %s", s->opt.tune_cache);
        std::fprintf(f, "%s %u %u %u %u\n", key.c_str(), pick.rows, pick.groups, pick.sweeps, pick.kernel);
        std::fclose(f);
    }
    if (out) *out = info;
    return TL_OK;
}

tl_status tl_sampler_state_bytes(const tl_domain *dom, size_t *bytes)
{
    if (!dom || !bytes) return fail(TL_EINVAL, "null argument");
    std::string why;
    tl_status mst = TL_EINVAL;
    std::unique_ptr<tl::Model> m = tl::make_model(*dom, why, &mst);
    if (!m) return fail(mst, "%s", why.c_str());
    *bytes = 2 * state_half_bytes(*m);
    return TL_OK;
}

tl_status tl_sampler_sweep(tl_sampler *s, uint64_t n)
{
    if (!s) return fail(TL_EINVAL, "null sampler");
    if (s->t + n > 0xFFFFFFFFull) return fail(TL_EINVAL, "sweep counter would exceed 2^32");
    if (s->model->order && (s->t + n) * (uint64_t)s->model->colours() > 0x100000000ull)
        return fail(TL_EINVAL, "step counter would exceed 2^32 (random colour order)");
    const tl::Thr T = table_of(s);
    const bool metro = s->w.rule == TL_METROPOLIS;
    const uint32_t every = s->opt.obs_every;
    uint64_t done = 0;
    while (done < n) {
        const uint32_t t = (uint32_t)(s->t + done);
        // sweeps until the next sample point (or the end)
        uint64_t chunk = n - done;
        if (every) {
            const uint64_t to_sample = every - (t % every);
            if (to_sample < chunk) chunk = to_sample;
        }
        TL_HIP(s->model->sweeps(t, (uint32_t)chunk, T, metro, s->seed, s->opt, s->stream));
        done += chunk;
        if (every && ((uint64_t)t + chunk) % every == 0) {
            tl_status st = enqueue_sample(s);
            if (st != TL_OK) return st;
        }
    }
    s->t += n;
    return TL_OK;
}

tl_status tl_sampler_sync(tl_sampler *s)
{
    if (!s) return fail(TL_EINVAL, "null sampler");
    TL_HIP(hipStreamSynchronize(s->stream));
    return TL_OK;
}

tl_status tl_sampler_observables(tl_sampler *s, tl_observables *o)
{
    if (!s || !o) return fail(TL_EINVAL, "null argument");
    const size_t nb = (size_t)s->bins_x * s->bins_y;
    if ((o->bin_sum || o->bin_now || o->bin_density) && o->bin_capacity < nb)
        return fail(TL_EINVAL, "bin buffers hold %zu entries, %zu needed", o->bin_capacity, nb);
    TL_HIP(hipMemsetAsync(s->bin_tmp, 0, nb * sizeof(unsigned long long), s->stream));
    TL_HIP(s->model->observe(s->B, s->bins_x, s->bin_tmp, s->stream));
    std::vector<unsigned long long> sum(nb), now(nb);
    TL_HIP(hipMemcpyAsync(sum.data(), s->bin_sum, nb * sizeof(unsigned long long), hipMemcpyDeviceToHost, s->stream));
    TL_HIP(hipMemcpyAsync(now.data(), s->bin_tmp, nb * sizeof(unsigned long long), hipMemcpyDeviceToHost, s->stream));
    TL_HIP(hipStreamSynchronize(s->stream));
    o->sweeps = s->t;
    o->samples = s->samples;
    o->bins_x = s->bins_x;
    o->bins_y = s->bins_y;
    int64_t a = 0, b = 0;
    for (size_t i = 0; i < nb; ++i) {
        a += (int64_t)sum[i];
        b += (int64_t)now[i];
    }
    o->scalar_sum = a;
    o->scalar_now = b;
    if (o->bin_sum) memcpy(o->bin_sum, sum.data(), nb * sizeof(uint64_t));
    if (o->bin_now) memcpy(o->bin_now, now.data(), nb * sizeof(uint64_t));
    if (o->bin_density) {
        if (s->cells_per_bin.empty()) s->cells_per_bin = s->model->cells_per_bin(s->B, s->bins_x, s->bins_y);
        for (size_t i = 0; i < nb; ++i) {
            const uint32_t c = s->cells_per_bin[i];
            o->bin_density[i] = (c && s->samples) ? (double)sum[i] / ((double)s->samples * (double)c) : 0.0;
        }
    }
    return TL_OK;
}

tl_status tl_sampler_export_size(const tl_sampler *s, size_t *bytes, uint32_t *rows, uint32_t *row_bytes)
{
    if (!s) return fail(TL_EINVAL, "null sampler");
    uint32_t r, rb;
    s->model->export_layout(&r, &rb);
    if (bytes) *bytes = (size_t)r * rb;
    if (rows) *rows = r;
    if (row_bytes) *row_bytes = rb;
    return TL_OK;
}

tl_status tl_sampler_export(tl_sampler *s, void *host, size_t bytes, uint64_t *sweep_out)
{
    if (!s || !host) return fail(TL_EINVAL, "null argument");
    uint32_t r, rb;
    s->model->export_layout(&r, &rb);
    const size_t need = (size_t)r * rb;
    if (bytes < need) return fail(TL_EINVAL, "export buffer has %zu bytes, %zu needed", bytes, need);
    uint8_t *dev = nullptr;
    TL_HIP(hipMallocAsync((void **)&dev, need, s->stream));
    hipError_t e = s->model->export_canonical(dev, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(host, dev, need, hipMemcpyDeviceToHost, s->stream);
    (void)hipFreeAsync(dev, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return fail(TL_EDEVICE, "export: %s", hipGetErrorString(e));
    if (sweep_out) *sweep_out = s->t;
    return TL_OK;
}

tl_status tl_sampler_hash(tl_sampler *s, uint8_t digest[32])
{
    if (!s || !digest) return fail(TL_EINVAL, "null argument");
    uint32_t r, rb;
    s->model->export_layout(&r, &rb);
    const size_t need = (size_t)r * rb;
    uint8_t *dev = nullptr;
    TL_HIP(hipMallocAsync((void **)&dev, need + 32 * (size_t)r, s->stream));
    std::vector<uint8_t> rowd(32 * (size_t)r);
    hipError_t e = s->model->export_canonical(dev, s->stream);
    if (e == hipSuccess) e = tl::hash_rows(dev, r, rb, dev + need, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(rowd.data(), dev + need, rowd.size(), hipMemcpyDeviceToHost, s->stream);
    (void)hipFreeAsync(dev, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return fail(TL_EDEVICE, "hash: %s", hipGetErrorString(e));
    tl::sha256_host(rowd.data(), rowd.size(), digest);
    return TL_OK;
}

// ------------------------------------------------ hash without allocation
namespace {
// Staging of tl_sampler_hash_noalloc: the canonical export, then the 32-byte
// digest of every row.  Each GPU holds its own copy at its own address; host
// code uses that address (looked up once per device), never the array's name.
__device__ __align__(256) uint8_t scratch[TL_HASH_NOALLOC_SCRATCH_BYTES];
constexpr int kScratchDevices = 64;
constexpr uint32_t kScratchMaxRows = 32768u;   // every domain's export has at most this many rows
std::mutex g_scratch_mu;                       // guards the table and the host digests, and orders the calls
uint8_t *g_scratch_dev[kScratchDevices];       // address of `scratch` on each device, nullptr until looked up
uint8_t g_rows_host[32u * kScratchMaxRows];    // row digests copied back for the final hash
}  // namespace

tl_status tl_sampler_hash_noalloc(tl_sampler *s, uint8_t digest[32])
{
    if (!s || !digest) return fail(TL_EINVAL, "null argument");
    uint32_t r, rb;
    s->model->export_layout(&r, &rb);
    const size_t need = (size_t)r * rb + 32u * (size_t)r;
    if (r > kScratchMaxRows || need > (size_t)TL_HASH_NOALLOC_SCRATCH_BYTES)
        return fail(TL_EINVAL, "hash_noalloc: the export needs %zu bytes of staging (%u rows), the static buffer "
                               "holds %zu bytes (%u rows); use tl_sampler_hash",
                    need, r, (size_t)TL_HASH_NOALLOC_SCRATCH_BYTES, kScratchMaxRows);
    if (s->device < 0 || s->device >= kScratchDevices) return fail(TL_EINVAL, "device %d out of range", s->device);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    int cur = 0;
    TL_HIP(hipGetDevice(&cur));
    if (cur != s->device) TL_HIP(hipSetDevice(s->device));
    hipError_t e = hipSuccess;
    if (!g_scratch_dev[s->device]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e == hipSuccess && !p) e = hipErrorInvalidSymbol;
        if (e == hipSuccess) g_scratch_dev[s->device] = (uint8_t *)p;
    }
    if (e == hipSuccess) {
        // every byte read below is written first by the same call: nothing to clear
        uint8_t *dev = g_scratch_dev[s->device];
        const size_t rows_at = (size_t)r * rb;
        e = s->model->export_canonical(dev, s->stream);
        if (e == hipSuccess) e = tl::hash_rows(dev, r, rb, dev + rows_at, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(g_rows_host, dev + rows_at, 32u * (size_t)r, hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    }
    if (cur != s->device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return fail(TL_EDEVICE, "hash_noalloc: %s", hipGetErrorString(e));
    tl::sha256_host(g_rows_host, 32u * (size_t)r, digest);
    return TL_OK;
}

tl_status tl_sampler_import(tl_sampler *s, const void *host, size_t bytes, uint64_t sweep)
{
    if (!s || !host) return fail(TL_EINVAL, "null argument");
    uint32_t r, rb;
    s->model->export_layout(&r, &rb);
    if (bytes != (size_t)r * rb) return fail(TL_EINVAL, "import needs exactly %zu bytes", (size_t)r * rb);
    if (sweep > 0xFFFFFFFFull) return fail(TL_EINVAL, "sweep counter exceeds 2^32");
    std::string why;
    hipError_t e = hipSuccess;
    if (!s->model->import_canonical((const uint8_t *)host, s->stream, why, &e)) {
        if (e != hipSuccess) return fail(TL_EDEVICE, "import: %s", hipGetErrorString(e));
        return fail(TL_EINVAL, "import: %s", why.c_str());
    }
    TL_HIP(hipStreamSynchronize(s->stream));
    s->t = sweep;
    return TL_OK;
}

tl_status tl_sampler_destroy(tl_sampler *s)
{
    delete s;   // the destructor synchronises and releases
    return TL_OK;
}

tl_status tl_sampler_reset(tl_sampler *s, uint64_t seed)
{
    if (!s) return fail(TL_EINVAL, "null sampler");
    s->seed = seed;
    s->t = 0;
    s->samples = 0;
    const size_t nb = (size_t)s->bins_x * s->bins_y;
    TL_HIP(hipMemsetAsync(s->bin_sum, 0, nb * sizeof(unsigned long long), s->stream));
    TL_HIP(s->model->init(s->dom.init == TL_INIT_MAX, s->stream));
    return TL_OK;
}

tl_status tl_sampler_cftp(tl_sampler *s, uint32_t max_log2, tl_cftp_info *out)
{
    if (!s) return fail(TL_EINVAL, "null sampler");
    if (max_log2 < 1 || max_log2 > 31) return fail(TL_EINVAL, "max_log2 must be in 1..31");
    if (s->w.rule != TL_HEATBATH) return fail(TL_EINVAL, "coupling from the past needs the heat-bath rule");
    if (s->model->order && max_log2 > 30)
        return fail(TL_EINVAL, "max_log2 must be <= 30 under the random colour order");
    if (s->dom.model == TL_SIXVERTEX) {
        // the moves keep the height order iff raising a diagonal face never
        // lowers the up threshold (for weights a, b, c: a <= c and b <= c)
        for (uint32_t m = 0; m < 16; ++m)
            for (uint32_t k = 0; k < 4; ++k)
                if (!(m >> k & 1u) && s->thr[m] > s->thr[m | (1u << k)])
                    return fail(TL_EINVAL, "coupling from the past needs weights that keep the height order "
                                           "(a <= c and b <= c)");
        // free points: raising a context diagonal must not lower the up threshold
        for (uint32_t m = 0; m < 4 && !s->thr_free.empty(); ++m)
            for (uint32_t k = 0; k < 2; ++k)
                if (!(m >> k & 1u) && s->thr_free[m] > s->thr_free[m | (1u << k)])
                    return fail(TL_EINVAL, "coupling from the past needs free-edge weights that keep the "
                                           "height order");
    }
    {
        // a state that is one tile: the rounds run side by side
        const tl::Thr T1 = table_of(s);
        tl::TileJob j1;
        tl::TilePlan p1;
        if (s->opt.kernel == 0 && s->opt.tile_rows == 0 && s->opt.tile_groups == 0 &&
            s->opt.sweeps_per_launch == 0 && s->model->tile_job(0, 1, T1, false, s->seed, false, &j1, &p1) &&
            p1.tiles() == 1) {
            uint32_t Rm = 0;
            bool met = false;
            TL_HIP(hipStreamSynchronize(s->stream));
            const hipError_t ce = cftp_side_by_side(s, max_log2, T1, &Rm, &met);
            if (ce != hipSuccess)
                return fail(ce == hipErrorOutOfMemory ? TL_ENOMEM : TL_EDEVICE, "coupling from the past: %s",
                            hipGetErrorString(ce));
            uint64_t total = 0;
            for (uint32_t r = 1; r <= Rm; ++r) total += 2ull << r;
            s->t = 1ull << Rm;
            s->samples = 0;
            const size_t nb = (size_t)s->bins_x * s->bins_y;
            TL_HIP(hipMemsetAsync(s->bin_sum, 0, nb * sizeof(unsigned long long), s->stream));
            if (out) {
                out->log2_sweeps = Rm;
                out->sweeps = 1ull << Rm;
                out->total_sweeps = total;
            }
            if (!met) return fail(TL_EBUSY, "the chains have not met within 2^%u sweeps", max_log2);
            return TL_OK;
        }
    }
    std::unique_ptr<tl::Model> top = s->model->twin();
    hipError_t e = top->allocate();
    uint32_t *flag = nullptr;
    if (e == hipSuccess) e = hipMalloc(&flag, sizeof(uint32_t));
    const tl::Thr T = table_of(s);
    const size_t words = s->model->state_words();
    // A state that is one tile runs both chains of a segment in one two-job
    // launch (one work-group each); descriptors are staged per segment.
    const uint32_t kSeg = 32;
    tl::TileJob *h_jobs = nullptr, *d_jobs = nullptr;
    tl::TileItem *d_items = nullptr;
    bool fused = s->opt.kernel == 0 && s->opt.tile_rows == 0 && s->opt.tile_groups == 0 &&
                 s->opt.sweeps_per_launch == 0;
    if (fused && e == hipSuccess) {
        tl::TileJob j;
        tl::TilePlan p;
        fused = s->model->tile_job(0, 1, T, false, s->seed, false, &j, &p) && p.tiles() == 1;
    }
    if (fused && e == hipSuccess) {
        const tl::TileItem items[2] = {{0u, 0u}, {1u, 0u}};
        e = hipHostMalloc((void **)&h_jobs, 2 * kSeg * sizeof(tl::TileJob), hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc(&d_jobs, 2 * kSeg * sizeof(tl::TileJob));
        if (e == hipSuccess) e = hipMalloc(&d_items, sizeof(items));
        if (e == hipSuccess) e = hipMemcpy(d_items, items, sizeof(items), hipMemcpyHostToDevice);
    }
    auto segment = [&](uint32_t slot, uint32_t t0, uint32_t count) -> hipError_t {
        if (!fused) {
            hipError_t err = s->model->sweeps(t0, count, T, false, s->seed, s->opt, s->stream);
            if (err == hipSuccess) err = top->sweeps(t0, count, T, false, s->seed, s->opt, s->stream);
            return err;
        }
        tl::TilePlan pb, pt;
        if (!s->model->tile_job(t0, count, T, false, s->seed, false, &h_jobs[2 * slot], &pb) ||
            !top->tile_job(t0, count, T, false, s->seed, false, &h_jobs[2 * slot + 1], &pt) || pb.S != count ||
            pb.tiles() != 1 || pt.tiles() != 1)
            return hipErrorInvalidConfiguration;
        hipError_t err = hipMemcpyAsync(d_jobs + 2 * slot, h_jobs + 2 * slot, 2 * sizeof(tl::TileJob),
                                        hipMemcpyHostToDevice, s->stream);
        if (err == hipSuccess)
            err = s->model->height_family()
                      ? tl::height_items(d_jobs + 2 * slot, d_items, 2, pb.threads, pb.lds, h_jobs[2 * slot].mode,
                                         h_jobs[2 * slot].kind, pb.order, h_jobs[2 * slot].site != nullptr,
                                         s->stream)
                      : tl::domino_items(d_jobs + 2 * slot, d_items, 2, pb.threads, pb.lds, pb.order, s->stream);
        if (err == hipSuccess) {
            s->model->swap_buffers();
            top->swap_buffers();
        }
        return err;
    };
    uint64_t total = 0;
    uint32_t R = 1, differ = 1;
    for (; e == hipSuccess && R <= max_log2; ++R) {
        e = s->model->init(false, s->stream);
        if (e == hipSuccess) e = top->init(true, s->stream);
        for (int r = (int)R; r >= 0 && e == hipSuccess; --r) {
            const uint32_t t0 = r ? 1u << (r - 1) : 0u, count = r ? 1u << (r - 1) : 1u;
            e = segment((uint32_t)r, t0, count);
        }
        total += 2ull << R;
        if (e == hipSuccess) e = hipMemsetAsync(flag, 0, sizeof(uint32_t), s->stream);
        if (e == hipSuccess) {
            size_t blocks = (words + 255) / 256;
            if (blocks > 2048) blocks = 2048;
            hipLaunchKernelGGL(words_differ_kernel, dim3((uint32_t)blocks), dim3(256), 0, s->stream,
                               s->model->state(), top->state(), words, flag);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(&differ, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e == hipSuccess && !differ) break;
    }
    if (h_jobs) (void)hipHostFree(h_jobs);
    if (d_jobs) (void)hipFree(d_jobs);
    if (d_items) (void)hipFree(d_items);
    top->release();
    if (flag) (void)hipFree(flag);
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? TL_ENOMEM : TL_EDEVICE, "coupling from the past: %s",
                    hipGetErrorString(e));
    const uint32_t Rend = differ ? max_log2 : R;
    s->t = 1ull << Rend;
    s->samples = 0;
    const size_t nb = (size_t)s->bins_x * s->bins_y;
    TL_HIP(hipMemsetAsync(s->bin_sum, 0, nb * sizeof(unsigned long long), s->stream));
    if (out) {
        out->log2_sweeps = Rend;
        out->sweeps = 1ull << Rend;
        out->total_sweeps = total;
    }
    if (differ) return fail(TL_EBUSY, "the chains have not met within 2^%u sweeps", max_log2);
    return TL_OK;
}

tl_status tl_sampler_set_timing(tl_sampler *s, int enable)
{
    if (!s) return fail(TL_EINVAL, "null sampler");
    if (enable < 0) return fail(TL_EINVAL, "timing period must be >= 0");
    s->model->timing.on = enable != 0;
    s->model->timing.every = enable > 0 ? (uint32_t)enable : 1u;
    s->model->timing.counter = 0;
    return TL_OK;
}

tl_status tl_sampler_kernel_time(tl_sampler *s, double *ms, uint64_t *launches, uint64_t *colour_steps,
                                 double *bytes_per_colour_step)
{
    if (!s) return fail(TL_EINVAL, "null sampler");
    TL_HIP(hipStreamSynchronize(s->stream));
    TL_HIP(s->model->timing.collect());
    if (ms) *ms = s->model->timing.ms;
    if (launches) *launches = s->model->timing.launches;
    if (colour_steps) *colour_steps = s->model->timing.steps;
    if (bytes_per_colour_step) *bytes_per_colour_step = s->model->bytes_per_colour_step();
    s->model->timing.ms = 0.0;
    s->model->timing.launches = 0;
    s->model->timing.steps = 0;
    return TL_OK;
}

tl_status tl_sampler_info(const tl_sampler *s, uint64_t *sites, uint32_t *colours)
{
    if (!s) return fail(TL_EINVAL, "null sampler");
    if (sites) *sites = s->model->sites();
    if (colours) *colours = (uint32_t)s->model->colours();
    return TL_OK;
}

tl_status tl_sampler_thresholds(const tl_sampler *s, uint32_t *out, uint32_t cap, uint32_t *count)
{
    if (!s) return fail(TL_EINVAL, "null sampler");
    std::vector<uint32_t> all = s->thr;
    all.insert(all.end(), s->thr_free.begin(), s->thr_free.end());
    if (count) *count = (uint32_t)all.size();
    if (out)
        for (uint32_t i = 0; i < cap && i < all.size(); ++i) out[i] = all[i];
    return TL_OK;
}

}  // extern "C"
