// Host-side model objects: device allocation, sweep scheduling per model and
// the host conversion of canonical exports for import.
#include <limits.h>
#include <stdlib.h>

#include <algorithm>
#include <utility>
#include <string.h>

#include "models.hpp"
#include "host_philox.hpp"
#include "region.hpp"

namespace tl {

namespace {

// Copy a packed extremal state (host) into both state buffers.  With cache, a
// model that owns its device memory keeps a device copy of it (made on the
// first start from it), so that later starts (resets, the rounds of coupling
// from the past) copy on the device.
hipError_t load_state(uint32_t *planes, uint32_t *spare, const std::vector<uint32_t> &host, uint32_t **cache,
                      hipStream_t s)
{
    const size_t bytes = host.size() * sizeof(uint32_t);
    const void *src = host.data();
    hipMemcpyKind kind = hipMemcpyHostToDevice;
    if (cache) {
        if (!*cache) {
            uint32_t *d = nullptr;
            hipError_t e = hipMalloc(&d, bytes);
            if (e == hipSuccess) e = hipMemcpyAsync(d, src, bytes, hipMemcpyHostToDevice, s);
            if (e != hipSuccess) {
                if (d) (void)hipFree(d);
                return e;
            }
            *cache = d;
        }
        src = *cache;
        kind = hipMemcpyDeviceToDevice;
    }
    hipError_t e = hipMemcpyAsync(planes, src, bytes, kind, s);
    if (e == hipSuccess) e = hipMemcpyAsync(spare, src, bytes, kind, s);
    return e;
}

// ------------------------------------------------------------------ domino
// The Aztec diamond of order n, or a domain given by a mask, embedded in the
// Aztec diamond of its region (faces outside the domain stay uncovered, so no
// rotation reaches them and the kernels run unchanged).
class DominoModel : public Model {
public:
    explicit DominoModel(int n) { setup(n); }
    explicit DominoModel(std::shared_ptr<const Region> r) : region_(std::move(r)) { setup(region_->n); }

    std::unique_ptr<Model> twin() const override
    {
        std::unique_ptr<Model> m(region_ ? new DominoModel(region_) : new DominoModel(d_.n));
        m->order = order;
        m->tuned_rows = tuned_rows;
        m->tuned_groups = tuned_groups;
        m->tuned_sweeps = tuned_sweeps;
        m->tuned_kernel = tuned_kernel;
        return m;
    }
    hipError_t allocate() override
    {
        hipError_t e = hipMalloc(&d_.planes, words_ * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMalloc(&d_.spare, words_ * sizeof(uint32_t));
        owned_ = true;
        keep_ext_ = true;
        return e;
    }
    hipError_t allocate_into(uint32_t *state, uint32_t *spare) override
    {
        attach(state, spare);
        keep_ext_ = true;   // a sampler's state: other tables stay library-allocated
        return hipSuccess;
    }
    void release() override
    {
        if (owned_ && d_.planes) (void)hipFree(d_.planes);
        if (owned_ && d_.spare) (void)hipFree(d_.spare);
        d_.planes = d_.spare = nullptr;
        for (uint32_t *&p : ext_)
            if (p) {
                (void)hipFree(p);
                p = nullptr;
            }
        keep_ext_ = false;
        timing.release();
    }
    size_t state_words() const override { return words_; }
    uint32_t row_groups() const override { return d_.ng; }
    void attach(uint32_t *state, uint32_t *spare) override
    {
        d_.planes = state;
        d_.spare = spare;
        owned_ = false;
        keep_ext_ = false;
    }
    bool tile_job(uint32_t t0, uint32_t S_max, const Thr &T, bool metro, uint64_t seed, bool, TileJob *j,
                  TilePlan *p) const override
    {
        DominoTile tile = domino_auto_tile(d_.n, order != 0, !T.uniform());
        tile.reg = 0;   // multi-job launches run LDS tiles
        tile.S = S_max;
        tile.order = order;
        if (!domino_plan(d_, tile, S_max, p)) return false;
        *j = domino_tile_job(d_, *p, t0, T, metro ? 1 : 0, seed);
        return true;
    }
    void swap_buffers() override { std::swap(d_.planes, d_.spare); }
    bool height_family() const override { return false; }
    const uint32_t *state() const override { return d_.planes; }
    hipError_t init(bool init_max, hipStream_t s) override
    {
        if (!region_) return domino_init(d_, init_max ? 1 : 0, s);
        // the extremal tilings of the domain, packed once on the host, go to
        // both buffers (the zero padding included)
        std::vector<uint32_t> &host = init_max ? packed_max_ : packed_min_;
        if (host.empty()) {
            std::string why;
            if (!pack(init_max ? region_->tmax.data() : region_->tmin.data(), host, why))
                return hipErrorInvalidValue;
        }
        return load_state(d_.planes, d_.spare, host, keep_ext_ ? &ext_[init_max ? 1 : 0] : nullptr, s);
    }

    hipError_t sweeps(uint32_t t0, uint32_t n, const Thr &T, bool metro, uint64_t seed, const tl_options &opt,
                      hipStream_t s) override
    {
        if (opt.kernel == 1) {   // one launch per colour step
            for (uint32_t i = 0; i < n; ++i)
                for (uint32_t j = 0; j < 2; ++j) {
                    const uint32_t step = 2u * (t0 + i) + j;
                    const int c = order ? (int)host_step_colour(seed, step, 2u) : (int)j;
                    hipError_t e = domino_colour_step(d_, c, order ? step : t0 + i, T, metro ? 1 : 0, seed, s,
                                                      &timing);
                    if (e != hipSuccess) return e;
                }
            return hipSuccess;
        }
        DominoTile tile = domino_auto_tile(d_.n, order != 0, !T.uniform());
        if (tuned_rows) {
            tile.TR = tuned_rows;
            tile.TG = tuned_groups;
            tile.S = tuned_sweeps;
            tile.reg = tuned_kernel == 3 ? 1u : 0u;
        }
        // tile fields given with the automatic kernel keep their meaning for
        // the LDS tiles
        if (opt.kernel == 0 && (opt.tile_rows || opt.tile_groups || opt.sweeps_per_launch)) tile.reg = 0;
        if (opt.tile_rows) tile.TR = opt.tile_rows;
        if (opt.tile_groups) tile.TG = opt.tile_groups;
        if (opt.sweeps_per_launch) tile.S = opt.sweeps_per_launch;
        tile.order = order;
        if (opt.kernel == 2) tile.reg = 0;
        if (opt.kernel == 3) tile.reg = 1;
        return domino_tiled_sweeps(d_, tile, t0, n, T, metro ? 1 : 0, seed, s, &timing);
    }
    hipError_t observe(uint32_t B, uint32_t bins_x, unsigned long long *bins, hipStream_t s) override
    {
        if (!region_) return domino_observe(d_, B, bins_x, bins, s);
        return domino_observe_box(d_, region_->ox, region_->oy, region_->h, B, bins_x, bins, s);
    }
    void cell_box(uint32_t *w, uint32_t *h) const override
    {
        *w = region_ ? (uint32_t)region_->w : 2u * (uint32_t)d_.n;
        *h = region_ ? (uint32_t)region_->h : 2u * (uint32_t)d_.n;
    }
    static bool face_in(int n, int X, int Y) { return abs(2 * X - 2 * n + 1) + abs(2 * Y - 2 * n + 1) <= 2 * n; }
    // Is face (x, y) of the export box part of the domain?
    bool in_domain(int x, int y) const
    {
        if (region_) return region_->mask[(size_t)y * region_->w + x] != 0;
        return face_in(d_.n, x, y);
    }
    std::vector<uint32_t> cells_per_bin(uint32_t B, uint32_t bx, uint32_t by) const override
    {
        std::vector<uint32_t> c((size_t)bx * by, 0u);
        uint32_t W, H;
        cell_box(&W, &H);
        for (uint32_t y = 0; y < H; ++y)
            for (uint32_t x = 0; x < W; ++x)
                if (in_domain((int)x, (int)y)) c[(size_t)(y / B) * bx + x / B] += 1;
        return c;
    }
    void export_layout(uint32_t *rows, uint32_t *row_bytes) const override { cell_box(row_bytes, rows); }
    hipError_t export_canonical(uint8_t *dev, hipStream_t s) override
    {
        if (!region_) return domino_export(d_, dev, s);
        return domino_export_box(d_, region_->ox, region_->oy, region_->w, region_->h, dev, s);
    }

    bool import_canonical(const uint8_t *f, hipStream_t s, std::string &why, hipError_t *err) override
    {
        std::vector<uint32_t> host;
        if (!pack(f, host, why)) return false;
        hipError_t e = hipMemcpyAsync(d_.planes, host.data(), host.size() * sizeof(uint32_t),
                                      hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { *err = e; return false; }
        return true;
    }
    uint64_t sites() const override
    {
        return region_ ? region_->sites : 2ull * d_.n * d_.n - 2ull * d_.n + 1ull;
    }
    int colours() const override { return 2; }
    // 4 bits per owner site (n^2 owners), read and written: n^2 bytes
    double bytes_per_colour_step() const override { return 2.0 * 4.0 * (double)d_.n * d_.n / 8.0; }

private:
    void setup(int n)
    {
        d_.n = n;
        d_.omega = (n + 1) & 1;
        words_ = domino_words(n, &d_.ng, &d_.RS, &d_.PS);
    }
    // Validate a canonical export (the export box: the diamond's 2n x 2n box, or
    // the domain's w x h box) and pack its crossed edges into owner planes.
    bool pack(const uint8_t *f, std::vector<uint32_t> &host, std::string &why) const
    {
        const int n = d_.n;
        uint32_t W, H;
        cell_box(&W, &H);
        const int ox = region_ ? region_->ox : 0, oy = region_ ? region_->oy : 0;
        host.assign(4 * d_.PS, 0u);
        auto set_owner = [&](int p, int P, int Q) -> bool {
            const int r2 = P + Q - n - 1, k2 = Q - P + n - 1;
            if (r2 < 0 || k2 < 0 || (r2 & 1) || (k2 & 1)) return false;
            const int r = r2 / 2, k = k2 / 2;
            if (r >= n || k >= n) return false;
            host[(size_t)p * d_.PS + (size_t)r * d_.RS + (k >> 5)] |= 1u << (k & 31);
            return true;
        };
        for (int y = 0; y < (int)H; ++y)
            for (int x = 0; x < (int)W; ++x) {
                const uint8_t dir = f[(size_t)y * W + x];
                if (!in_domain(x, y)) {
                    if (dir != 0xFF) { why = "face outside the domain is not 0xFF"; return false; }
                    continue;
                }
                if (dir > 3) { why = "invalid partner code"; return false; }
                const int px = x + (dir == 2) - (dir == 3), py = y + (dir == 0) - (dir == 1);
                if (px < 0 || py < 0 || px >= (int)W || py >= (int)H || !in_domain(px, py) ||
                    f[(size_t)py * W + px] != (uint8_t)(dir ^ 1u)) {
                    why = "faces do not form a domino tiling";
                    return false;
                }
                const int X = x + ox, Y = y + oy;   // face in the diamond's box
                bool ok = true;
                if (dir == 2) {   // vertical segment (X+1,Y)-(X+1,Y+1)
                    ok = (((X + 1 + Y) & 1) == d_.omega) ? set_owner(0, X + 1, Y) : set_owner(1, X + 1, Y + 1);
                } else if (dir == 0) {  // horizontal segment (X,Y+1)-(X+1,Y+1)
                    ok = (((X + Y + 1) & 1) == d_.omega) ? set_owner(2, X, Y + 1) : set_owner(3, X + 1, Y + 1);
                }
                if (!ok) { why = "crossed edge without an interior owner"; return false; }
            }
        return true;
    }

    DominoDev d_;
    size_t words_ = 0;
    bool owned_ = false;
    std::shared_ptr<const Region> region_;
    std::vector<uint32_t> packed_max_, packed_min_;
    bool keep_ext_ = false;                  // keep device copies of the extremal states
    uint32_t *ext_[2] = {nullptr, nullptr};  // T_min, T_max on the device
};

// ------------------------------------------------------- lozenge / six-vertex
class HeightModel : public Model {
public:
    explicit HeightModel(const tl_domain &dom) : dom_(dom)
    {
        d_.model = dom.model;
        d_.a = dom.a;
        d_.b = dom.b;
        d_.c = dom.c;
        d_.N = dom.n;
        height_words(d_);
    }
    // Domain given by a mask: the state box holds the domain's box at its
    // south-west corner (six-vertex: the square of N = max(w, h) cells;
    // lozenge: the w x h x 0 box, i.e. the (w+1) x (h+1) vertices); points that
    // are not sites never flip (site planes); exports and observables use the
    // domain's own box.
    explicit HeightModel(std::shared_ptr<const HeightRegion> r) : region_(std::move(r))
    {
        dom_ = tl_domain{};
        dom_.model = region_->model;
        d_.model = region_->model;
        if (region_->model == TL_LOZENGE) {
            d_.a = region_->w;
            d_.b = region_->h;
            d_.c = 0;
        } else {
            // free points sit on a side of the domain's box: keep them inner
            // points of the state, with a row (column) beyond a free north
            // (east) side and the box two rows (columns) up (right) for a free
            // south (west) one
            const int side = region_->free_sites ? region_->free_side : 0;
            d_.free_side = side;
            d_.ox = side == 4 ? 2 : 0;
            d_.oy = side == 2 ? 2 : 0;
            d_.N = std::max(region_->w + d_.ox + (side == 3 ? 1 : 0), region_->h + d_.oy + (side == 1 ? 1 : 0));
        }
        height_words(d_);
    }
    std::unique_ptr<Model> twin() const override
    {
        std::unique_ptr<Model> m(region_ ? new HeightModel(region_) : new HeightModel(dom_));
        m->order = order;
        m->tuned_rows = tuned_rows;
        m->tuned_groups = tuned_groups;
        m->tuned_sweeps = tuned_sweeps;
        m->tuned_kernel = tuned_kernel;
        m->set_boundary_table(free_thr_);
        return m;
    }
    bool loz() const { return d_.model == TL_LOZENGE; }
    int width() const { return loz() ? d_.a + d_.c + 1 : d_.N + 1; }   // export row length

    hipError_t allocate() override
    {
        const size_t words = height_words(d_);
        hipError_t e = hipMalloc(&d_.planes, words * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMalloc(&d_.spare, words * sizeof(uint32_t));
        owned_ = true;
        keep_ext_ = true;
        if (e != hipSuccess) return e;
        return allocate_region();
    }
    hipError_t allocate_into(uint32_t *state, uint32_t *spare) override
    {
        attach(state, spare);
        keep_ext_ = true;   // a sampler's state: other tables stay library-allocated
        return allocate_region();
    }
    // Bytes of a masked domain's device tables, each 256-byte aligned: site
    // planes, anchors, heights, minimal heights, cells, free-edge planes.
    static size_t al(size_t v) { return (v + 255) / 256 * 256; }
    size_t region_bytes() const override
    {
        if (!region_) return 0;
        HeightDev d = d_;
        const size_t words = height_words(d), V = region_->anchor.size(), C = region_->cells.size();
        return al(words * 4) + 3 * al(V * 4) + al(C) + (region_->free_sites ? al(words * 4) : 0);
    }
    bool masked() const override { return region_ != nullptr; }
    hipError_t attach_region(uint8_t *dev, hipStream_t s) override
    {
        if (!region_) return hipSuccess;
        HeightDev d = d_;
        const size_t words = height_words(d), V = region_->anchor.size(), C = region_->cells.size();
        uint8_t *p = dev;
        site_ = (uint32_t *)p;
        p += al(words * 4);
        anchor_ = (int32_t *)p;
        p += al(V * 4);
        heights_ = (int32_t *)p;
        p += al(V * 4);
        hmin_ = (int32_t *)p;
        p += al(V * 4);
        cells_ = p;
        p += al(C);
        freep_ = region_->free_sites ? (uint32_t *)p : nullptr;
        region_owned_ = false;
        if (site_host_.empty()) pack_points(region_->site, site_host_, [](int32_t v) { return v != 0; });
        if (freep_ && freep_host_.empty()) pack_points(region_->site, freep_host_, [](int32_t v) { return v == 2; });
        hipError_t e = hipMemcpyAsync(site_, site_host_.data(), words * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && freep_)
            e = hipMemcpyAsync(freep_, freep_host_.data(), words * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(anchor_, region_->anchor.data(), V * sizeof(int32_t), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hmin_, region_->hmin.data(), V * sizeof(int32_t), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(cells_, region_->cells.data(), C, hipMemcpyHostToDevice, s);
        d_.site = site_;
        d_.freep = freep_;
        return e;
    }
    // Device copies of a masked domain's site planes, anchors and cells.
    hipError_t allocate_region()
    {
        if (!region_) return hipSuccess;
        const size_t words = height_words(d_);
        hipError_t e = hipSuccess;
        const size_t V = region_->anchor.size(), C = region_->cells.size();
        e = hipMalloc(&site_, words * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMalloc(&anchor_, V * sizeof(int32_t));
        if (e == hipSuccess) e = hipMalloc(&heights_, V * sizeof(int32_t));
        if (e == hipSuccess) e = hipMalloc(&hmin_, V * sizeof(int32_t));
        if (e == hipSuccess) e = hipMalloc(&cells_, C);
        if (e == hipSuccess && region_->free_sites) e = hipMalloc(&freep_, words * sizeof(uint32_t));
        if (e != hipSuccess) return e;
        std::vector<uint32_t> planes;
        pack_points(region_->site, planes, [](int32_t v) { return v != 0; });
        e = hipMemcpy(site_, planes.data(), planes.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess && freep_) {
            pack_points(region_->site, planes, [](int32_t v) { return v == 2; });
            e = hipMemcpy(freep_, planes.data(), planes.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
            d_.freep = freep_;
        }
        if (e == hipSuccess) e = hipMemcpy(anchor_, region_->anchor.data(), V * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(hmin_, region_->hmin.data(), V * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(cells_, region_->cells.data(), C, hipMemcpyHostToDevice);
        d_.site = site_;
        return e;
    }
    void release() override
    {
        if (owned_ && d_.planes) (void)hipFree(d_.planes);
        if (owned_ && d_.spare) (void)hipFree(d_.spare);
        d_.planes = d_.spare = nullptr;
        for (uint32_t *&p : ext_)
            if (p) {
                (void)hipFree(p);
                p = nullptr;
            }
        keep_ext_ = false;
        if (region_owned_)
            for (void *p : {(void *)site_, (void *)anchor_, (void *)heights_, (void *)hmin_, (void *)cells_,
                            (void *)freep_})
                if (p) (void)hipFree(p);
        region_owned_ = true;
        site_ = freep_ = nullptr;
        d_.freep = nullptr;
        anchor_ = heights_ = hmin_ = nullptr;
        cells_ = nullptr;
        d_.site = nullptr;
        timing.release();
    }
    // Bit planes (state layout) of a per-point property of a masked domain:
    // bit of point (I, J) set iff pred(value at J*(w+1) + I).  Six-vertex
    // plane I mod 2, site I / 2; lozenge plane I mod 3, site I / 3.
    template <typename V, typename F>
    void pack_points(const std::vector<V> &vals, std::vector<uint32_t> &host, F pred) const
    {
        host.assign(d_.P * d_.PS, 0u);
        const int w = region_->w, h = region_->h, P = loz() ? 3 : 2;
        for (int J = 0; J <= h; ++J)
            for (int I = 0; I <= w; ++I)
                if (pred((int32_t)vals[(size_t)J * (w + 1) + I])) {
                    const int X = I + d_.ox, Y = J + d_.oy, p = X % P, k = X / P;
                    host[(size_t)p * d_.PS + (size_t)Y * d_.RS + 4 + (k >> 5)] |= 1u << (k & 31);
                }
    }
    // The residual bit of a height: six-vertex floor(h/2) mod 2, lozenge H mod 2.
    bool residual(int32_t v) const { return loz() ? (v & 1) != 0 : ((v >> 1) & 1) != 0; }
    size_t state_words() const override
    {
        HeightDev d = d_;
        return height_words(d);
    }
    uint32_t row_groups() const override { return d_.ng; }
    void attach(uint32_t *state, uint32_t *spare) override
    {
        d_.planes = state;
        d_.spare = spare;
        owned_ = false;
        keep_ext_ = false;
    }
    // Multi-job tiles: a state whose (row, group) tasks fit one work-group (512)
    // and whose planes fit 64 KB of LDS is one tile (no halo, any sweep
    // count), unless spread asks for tiles whose tasks, a quad of lanes each
    // for bit-serial decisions, all run at once (a work-group with fewer lanes
    // than that takes its tasks in turns).  Larger states are cut into tiles
    // spanning up to 8 groups, 32, 16 or 8 rows high: the tallest whose tasks
    // fit 512 lanes, else the one that needs the fewest turns.
    bool tile_job(uint32_t t0, uint32_t S_max, const Thr &T, bool metro, uint64_t seed, bool spread, TileJob *j,
                  TilePlan *p) const override
    {
        const Thr K = kernel_table(T, metro);
        HeightTile tile;
        tile.S = S_max;
        tile.order = order;
        tile.lanes = K.uniform() ? 1u : 4u;
        tile.items = 1;
        const uint32_t whole = height_task_rows(d_.model, d_.rows) * d_.ng;
        if (whole <= 512u && (!spread || whole * tile.lanes <= 512u) &&
            (size_t)d_.P * d_.rows * 4u * (d_.ng + 2u) * 4u <= 64u * 1024u) {
            tile.TR = d_.rows;
            tile.TG = d_.ng;
            if (!height_plan(d_, tile, S_max, p)) return false;
        } else {
            tile.TG = d_.ng <= 8u ? d_.ng : 4u;
            uint32_t best_turns = 0;
            for (uint32_t TR : {32u, 16u, 8u}) {
                tile.TR = TR;
                TilePlan q;
                if (!height_plan(d_, tile, S_max, &q)) continue;
                const uint32_t lanes = height_task_rows(d_.model, q.TR + 2u * q.HR) * (q.TG + 2u * q.HG) * tile.lanes;
                const uint32_t turns = (lanes + 511u) / 512u;
                if (best_turns == 0 || turns < best_turns) {
                    *p = q;
                    best_turns = turns;
                }
                if (turns == 1u) break;
            }
            if (best_turns == 0) return false;
        }
        *j = height_tile_job(d_, *p, t0, K, metro ? 1 : 0, seed);
        return true;
    }
    void swap_buffers() override { std::swap(d_.planes, d_.spare); }
    bool height_family() const override { return true; }
    const uint32_t *state() const override { return d_.planes; }
    hipError_t init(bool init_max, hipStream_t s) override
    {
        if (!region_) return height_init(d_, init_max ? 1 : 0, s);
        // residual bits floor(h/2) mod 2 of the extremal configuration, packed
        // once, into both buffers
        std::vector<uint32_t> &host = init_max ? packed_max_ : packed_min_;
        if (host.empty())
            pack_points(init_max ? region_->hmax : region_->hmin, host,
                        [this](int32_t v) { return v != INT32_MIN && residual(v); });
        return load_state(d_.planes, d_.spare, host, keep_ext_ ? &ext_[init_max ? 1 : 0] : nullptr, s);
    }

    // Six-vertex kernels take one threshold per weight class (sA, sB) (and
    // current state for Metropolis): class 3*sA + sB <-> mask with NE = sA>=1,
    // SW = sA>=2, NW = sB>=1, SE = sB>=2.  When the thresholds depend on
    // sA + sB only (a = b), the table has one entry per sum s = 0..4 (two for
    // Metropolis: current state down, up) instead, and the kernels use those
    // 5 classes.
    // Kernel table: the interior classes (below), and for a domain with free
    // north edges their table at v[kFreeBase ..].
    Thr kernel_table(const Thr &T, bool metro) const
    {
        Thr K = interior_table(T, metro);
        K.nfree = (uint32_t)free_thr_.size();
        for (uint32_t i = 0; i < K.nfree; ++i) K.v[Thr::kFreeBase + i] = free_thr_[i];
        return K;
    }
    void set_boundary_table(const std::vector<uint32_t> &t) override { free_thr_ = t; }
    Thr interior_table(const Thr &T, bool metro) const
    {
        if (loz()) return T;
        auto mask_of = [](int i, int j) {
            return (i >= 1 ? 1u : 0u) | (j >= 1 ? 2u : 0u) | (i >= 2 ? 4u : 0u) | (j >= 2 ? 8u : 0u);
        };
        const uint32_t per = metro ? 2u : 1u;
        bool by_sum = true;
        for (int i = 0; i < 3 && by_sum; ++i)
            for (int j = 0; j < 3; ++j) {
                const int s = i + j, i0 = s < 2 ? s : 2;   // reference class of the sum
                for (uint32_t q = 0; q < per; ++q)
                    if (T.v[per * mask_of(i, j) + q] != T.v[per * mask_of(i0, s - i0) + q]) by_sum = false;
            }
        Thr K{};
        uint32_t n = 0;
        if (by_sum) {
            for (int s = 0; s <= 4; ++s) {
                const int i0 = s < 2 ? s : 2;
                for (uint32_t q = 0; q < per; ++q) K.v[n++] = T.v[per * mask_of(i0, s - i0) + q];
            }
            K.count = n;
            return K;
        }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                const uint32_t mask = (i >= 1 ? 1u : 0u) | (j >= 1 ? 2u : 0u) | (i >= 2 ? 4u : 0u) | (j >= 2 ? 8u : 0u);
                if (metro) {
                    K.v[n++] = T.v[2 * mask];
                    K.v[n++] = T.v[2 * mask + 1];
                } else {
                    K.v[n++] = T.v[mask];
                }
            }
        K.count = n;
        return K;
    }
    hipError_t sweeps(uint32_t t0, uint32_t n, const Thr &T, bool metro, uint64_t seed, const tl_options &opt,
                      hipStream_t s) override
    {
        const Thr K = kernel_table(T, metro);
        if (opt.kernel == 1) {
            const uint32_t colours = loz() ? 3u : 4u;
            for (uint32_t i = 0; i < n; ++i)
                for (uint32_t j = 0; j < colours; ++j) {
                    const uint32_t step = colours * (t0 + i) + j;
                    const int c = order ? (int)host_step_colour(seed, step, colours) : (int)j;
                    hipError_t e = height_colour_step(d_, c, order ? step : t0 + i, K, metro ? 1 : 0, seed, s,
                                                      &timing);
                    if (e != hipSuccess) return e;
                }
            return hipSuccess;
        }
        HeightTile tile = height_auto_tile(d_, K.uniform(), metro);
        if (tuned_rows) {
            tile.TR = tuned_rows;
            tile.TG = tuned_groups;
            tile.S = tuned_sweeps;
        }
        if (opt.tile_rows) tile.TR = opt.tile_rows;
        if (opt.tile_groups) tile.TG = opt.tile_groups;
        if (opt.sweeps_per_launch) tile.S = opt.sweeps_per_launch;
        tile.order = order;
        tile.lanes = K.uniform() ? 1u : 4u;
        return height_tiled_sweeps(d_, tile, t0, n, K, metro ? 1 : 0, seed, s, &timing);
    }
    hipError_t observe(uint32_t B, uint32_t bins_x, unsigned long long *bins, hipStream_t s) override
    {
        if (region_ && loz())
            return loz_region_observe(d_, anchor_, hmin_, region_->w, region_->h, heights_, B, bins_x, bins, s);
        if (region_)
            return sixv_region_observe(d_, anchor_, cells_, region_->w, region_->h, heights_, B, bins_x, bins, s);
        return height_observe(d_, B, bins_x, bins, s);
    }
    void cell_box(uint32_t *w, uint32_t *h) const override
    {
        if (region_) {
            *w = (uint32_t)region_->cw;
            *h = (uint32_t)region_->ch;
        } else if (loz()) {
            *w = (uint32_t)(d_.a + d_.c + 1);
            *h = (uint32_t)(d_.b + d_.c + 1);
        } else {
            *w = *h = (uint32_t)d_.N;
        }
    }
    bool in_hex(int X, int Y) const
    {
        const int x = X - d_.c, y = Y - d_.c;
        return x >= -d_.c && x <= d_.a && y >= -d_.c && y <= d_.b && x - y >= -d_.b && x - y <= d_.a;
    }
    int hmin(int X, int Y) const { return std::max(0, std::max(d_.c - X, d_.c - Y)); }
    int hmax(int X, int Y) const { return std::min(d_.c, std::min(d_.a + d_.c - X, d_.b + d_.c - Y)); }
    std::vector<uint32_t> cells_per_bin(uint32_t B, uint32_t bx, uint32_t by) const override
    {
        std::vector<uint32_t> cnt((size_t)bx * by, 0u);
        uint32_t w, h;
        cell_box(&w, &h);
        for (uint32_t Y = 0; Y < h; ++Y)
            for (uint32_t X = 0; X < w; ++X) {
                const bool in = region_ ? region_->cells[(size_t)Y * w + X] != 0 : (!loz() || in_hex((int)X, (int)Y));
                if (in) cnt[(size_t)(Y / B) * bx + X / B] += 1;
            }
        return cnt;
    }
    void export_layout(uint32_t *rows, uint32_t *row_bytes) const override
    {
        *rows = region_ ? (uint32_t)region_->h + 1u : d_.rows;
        *row_bytes = 4u * (uint32_t)(region_ ? region_->w + 1 : width());
    }
    hipError_t export_canonical(uint8_t *dev, hipStream_t s) override
    {
        if (region_ && loz())
            return loz_region_export(d_, anchor_, region_->w, region_->h, reinterpret_cast<int32_t *>(dev), s);
        if (region_)
            return sixv_region_export(d_, anchor_, region_->w, region_->h, reinterpret_cast<int32_t *>(dev), s);
        return height_export(d_, reinterpret_cast<int32_t *>(dev), s);
    }
    // Masked domain: off the domain INT32_MIN, boundary points their fixed
    // heights; six-vertex sites one away from their four neighbours with the
    // parity of I + J; lozenge sites with steps 0 or -1 to their six
    // neighbours along (1,0), (0,1), (1,1).
    bool import_region(const int32_t *H, std::vector<uint32_t> &host, std::string &why) const
    {
        const int w = region_->w, h = region_->h, PW = w + 1;
        std::vector<int32_t> vals((size_t)PW * (h + 1), INT32_MIN);
        for (int J = 0; J <= h; ++J)
            for (int I = 0; I <= w; ++I) {
                const size_t v = (size_t)J * PW + I;
                const int32_t a = region_->anchor[v], x = H[v];
                if (a != INT32_MAX) {
                    if (x != a) {
                        why = a == INT32_MIN ? "point off the domain is not INT32_MIN" : "boundary height violated";
                        return false;
                    }
                    if (a != INT32_MIN) vals[v] = x;
                    continue;
                }
                if (loz()) {
                    // forward neighbours: x minus 0 or 1; backward ones: x plus 0 or 1
                    const int32_t fw[3] = {H[v + 1], H[v + PW], H[v + PW + 1]};
                    const int32_t bw[3] = {H[v - 1], H[v - PW], H[v - PW - 1]};
                    for (int q = 0; q < 3; ++q)
                        if (fw[q] == INT32_MIN || bw[q] == INT32_MIN || (x - fw[q] != 0 && x - fw[q] != 1) ||
                            (bw[q] - x != 0 && bw[q] - x != 1)) {
                            why = "height step not in {0, -1}";
                            return false;
                        }
                    vals[v] = x;
                    continue;
                }
                // a point of the free side has no neighbour across it
                const int fs = region_->site[v] == 2 ? region_->free_side : 0;
                int32_t nb[4];
                int cnt = 0;
                if (fs != 4) nb[cnt++] = H[v - 1];    // west
                if (fs != 3) nb[cnt++] = H[v + 1];    // east
                if (fs != 2) nb[cnt++] = H[v - PW];   // south
                if (fs != 1) nb[cnt++] = H[v + PW];   // north
                for (int q = 0; q < cnt; ++q)
                    if (const int32_t y = nb[q]; y == INT32_MIN || (x > y ? x - y : y - x) != 1) {
                        why = "ice rule violated";
                        return false;
                    }
                if (((int64_t)x - I - J) & 1) {
                    why = "height parity differs from I + J";
                    return false;
                }
                vals[v] = x;
            }
        pack_points(vals, host, [this](int32_t x) { return x != INT32_MIN && residual(x); });
        return true;
    }
    bool import_canonical(const uint8_t *raw, hipStream_t s, std::string &why, hipError_t *err) override
    {
        if (region_) {
            std::vector<int32_t> H((size_t)(region_->w + 1) * (region_->h + 1));
            memcpy(H.data(), raw, H.size() * sizeof(int32_t));
            std::vector<uint32_t> host;
            if (!import_region(H.data(), host, why)) return false;
            hipError_t e = hipMemcpyAsync(d_.planes, host.data(), host.size() * sizeof(uint32_t),
                                          hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) { *err = e; return false; }
            return true;
        }
        const int W = width(), R = (int)d_.rows;
        std::vector<int32_t> h((size_t)W * R);
        memcpy(h.data(), raw, h.size() * sizeof(int32_t));
        auto at = [&](int X, int Y) { return h[(size_t)Y * W + X]; };
        std::vector<uint32_t> host(d_.P * d_.PS, 0u);
        auto setbit = [&](uint32_t p, uint32_t y, uint32_t k) {
            host[p * d_.PS + (size_t)y * d_.RS + 4 + (k >> 5)] |= 1u << (k & 31u);
        };
        if (loz()) {
            for (int Y = 0; Y < R; ++Y)
                for (int X = 0; X < W; ++X) {
                    const int32_t v = at(X, Y);
                    if (!in_hex(X, Y)) {
                        if (v != INT32_MIN) { why = "vertex outside the hexagon is not INT32_MIN"; return false; }
                        continue;
                    }
                    if (v < hmin(X, Y) || v > hmax(X, Y)) { why = "height outside [H_min, H_max]"; return false; }
                    const int dx[3] = {1, 0, 1}, dy[3] = {0, 1, 1};
                    for (int q = 0; q < 3; ++q) {
                        const int X2 = X + dx[q], Y2 = Y + dy[q];
                        if (X2 < W && Y2 < R && in_hex(X2, Y2)) {
                            const int dlt = at(X2, Y2) - v;
                            if (dlt != 0 && dlt != -1) { why = "height step not in {0, -1}"; return false; }
                        }
                    }
                    if (v & 1) setbit((uint32_t)(X % 3), (uint32_t)Y, (uint32_t)(X / 3));
                }
        } else {
            const int N = d_.N;
            for (int J = 0; J <= N; ++J)
                for (int I = 0; I <= N; ++I) {
                    const int32_t v = at(I, J);
                    const bool edge = I == 0 || J == 0 || I == N || J == N;
                    if (edge) {
                        const int want = J == 0 ? I : (I == 0 ? J : (J == N ? N - I : N - J));
                        if (v != want) { why = "domain-wall boundary heights violated"; return false; }
                    }
                    if (I < N && std::abs(at(I + 1, J) - v) != 1) { why = "ice rule violated"; return false; }
                    if (J < N && std::abs(at(I, J + 1) - v) != 1) { why = "ice rule violated"; return false; }
                    if (v < 0) { why = "negative height"; return false; }
                    if ((v >> 1) & 1) setbit((uint32_t)(I & 1), (uint32_t)J, (uint32_t)(I >> 1));
                }
        }
        hipError_t e = hipMemcpyAsync(d_.planes, host.data(), host.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { *err = e; return false; }
        return true;
    }
    uint64_t sites() const override
    {
        if (region_) return region_->sites;
        if (loz()) {
            uint64_t n = 0;
            for (int Y = 1; Y < (int)d_.rows - 1; ++Y) {
                const int lo = std::max(0, Y - d_.b), hi = std::min(d_.a + d_.c, Y + d_.a);
                if (hi - lo - 1 > 0) n += (uint64_t)(hi - lo - 1);
            }
            return n;
        }
        return (uint64_t)(d_.N - 1) * (uint64_t)(d_.N - 1);
    }
    int colours() const override { return loz() ? 3 : 4; }
    // one bit per site read and written once per colour step (the streaming
    // formulation), counted over the sites, not the padded box of the planes
    double bytes_per_colour_step() const override { return 2.0 * (double)sites() / 8.0; }

private:
    tl_domain dom_;
    HeightDev d_;
    bool owned_ = false;
    bool keep_ext_ = false;                  // keep device copies of the extremal states
    uint32_t *ext_[2] = {nullptr, nullptr};  // minimal, maximal state on the device
    std::shared_ptr<const HeightRegion> region_;
    uint32_t *site_ = nullptr, *freep_ = nullptr;
    bool region_owned_ = true;   // false: the tables live in caller-owned memory (attach_region)
    std::vector<uint32_t> site_host_, freep_host_;   // packed planes the asynchronous uploads read
    int32_t *anchor_ = nullptr, *heights_ = nullptr, *hmin_ = nullptr;
    std::vector<uint32_t> free_thr_;
    uint8_t *cells_ = nullptr;
    std::vector<uint32_t> packed_max_, packed_min_;
};

}  // namespace

std::unique_ptr<Model> make_model(const tl_domain &d, std::string &why, tl_status *status)
{
    if (status) *status = TL_EINVAL;
    if (d.shape == TL_MASK && d.flags && (d.model != TL_SIXVERTEX || free_side_of(d.flags) < 0)) {
        why = "free sides are a six-vertex option, one side per domain";
        return nullptr;
    }
    if (d.model == TL_SIXVERTEX && d.shape == TL_MASK) {
        auto r = std::make_shared<HeightRegion>();
        const RegionStatus st = build_sixv_region(d.mask, d.w, d.h, free_side_of(d.flags), *r, why);
        if (st != kRegionOk) {
            if (status && st == kRegionUntileable) *status = TL_EUNTILEABLE;
            return nullptr;
        }
        return std::unique_ptr<Model>(new HeightModel(std::shared_ptr<const HeightRegion>(std::move(r))));
    }
    if (d.model == TL_LOZENGE && d.shape == TL_MASK) {
        auto r = std::make_shared<HeightRegion>();
        const RegionStatus st = build_loz_region(d.mask, d.w, d.h, *r, why);
        if (st != kRegionOk) {
            if (status && st == kRegionUntileable) *status = TL_EUNTILEABLE;
            return nullptr;
        }
        return std::unique_ptr<Model>(new HeightModel(std::shared_ptr<const HeightRegion>(std::move(r))));
    }
    if (d.model == TL_DOMINO && d.shape == TL_MASK) {
        auto r = std::make_shared<Region>();
        const RegionStatus st = build_region(d.mask, d.w, d.h, *r, why);
        if (st != kRegionOk) {
            if (status && st == kRegionUntileable) *status = TL_EUNTILEABLE;
            return nullptr;
        }
        return std::unique_ptr<Model>(new DominoModel(std::shared_ptr<const Region>(std::move(r))));
    }
    if (d.model == TL_DOMINO) {
        if (d.shape != TL_AZTEC) { why = "dominoes support the Aztec diamond and mask shapes"; return nullptr; }
        if (d.n < 1 || d.n > 16384) { why = "Aztec order must be in [1, 16384]"; return nullptr; }
        return std::unique_ptr<Model>(new DominoModel(d.n));
    }
    if (d.model == TL_LOZENGE) {
        if (d.shape != TL_HEXAGON) { why = "lozenges support the hexagon shape"; return nullptr; }
        if (d.a < 1 || d.b < 1 || d.c < 1 || d.a + d.c > 32767 || d.b + d.c > 32767) {
            why = "hexagon sides must be >= 1 with a+c, b+c <= 32767";
            return nullptr;
        }
        return std::unique_ptr<Model>(new HeightModel(d));
    }
    if (d.model == TL_SIXVERTEX) {
        if (d.shape != TL_DWBC_SQUARE) { why = "the six-vertex model supports the domain-wall square"; return nullptr; }
        if (d.n < 1 || d.n > 32767) { why = "six-vertex N must be in [1, 32767]"; return nullptr; }
        return std::unique_ptr<Model>(new HeightModel(d));
    }
    why = "unknown model";
    return nullptr;
}

}  // namespace tl

namespace tl {

size_t sampler_device_bytes(const tl_domain &d, uint32_t obs_bin)
{
    std::string why;
    if (d.shape == TL_MASK || !make_model(d, why)) return 0;
    const uint32_t B = obs_bin ? obs_bin : 1u;
    size_t words = 0, cells_w = 0, cells_h = 0;
    if (d.model == TL_DOMINO) {
        uint32_t ng, RS;
        size_t PS;
        words = domino_words(d.n, &ng, &RS, &PS);
        cells_w = cells_h = 2u * (uint32_t)d.n;
    } else {
        HeightDev h;
        h.model = d.model;
        h.a = d.a;
        h.b = d.b;
        h.c = d.c;
        h.N = d.n;
        words = height_words(h);
        cells_w = d.model == TL_LOZENGE ? (size_t)(d.a + d.c + 1) : (size_t)d.n;
        cells_h = d.model == TL_LOZENGE ? (size_t)(d.b + d.c + 1) : (size_t)d.n;
    }
    const size_t bins = ((cells_w + B - 1) / B) * ((cells_h + B - 1) / B);
    return 2 * words * sizeof(uint32_t) + 2 * bins * sizeof(unsigned long long);
}

}  // namespace tl
