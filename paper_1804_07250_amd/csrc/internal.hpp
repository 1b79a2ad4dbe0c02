// Host-side interfaces between the C-ABI layer (api.hip) and the per-model
// kernel launchers.  Every launcher enqueues on the given stream and returns the
// HIP status of the launch.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>
#include "../../include/tilings.h"

#include <vector>

namespace tl {

// Threshold values handed to a colour-step kernel by value.
struct Thr {
    uint32_t v[32];
    uint32_t count;
    // six-vertex free north edges: nfree entries at v[kFreeBase ..]
    uint32_t nfree;
    static constexpr uint32_t kFreeBase = 24;
    // every threshold is 2^31: one random bit per site decides
    bool uniform() const
    {
        for (uint32_t i = 0; i < count; ++i)
            if (v[i] != 0x80000000u) return false;
        for (uint32_t i = 0; i < nfree; ++i)
            if (v[kFreeBase + i] != 0x80000000u) return false;
        return count > 0;
    }
};

// Optional per-launch kernel timing: when enabled, sweep kernels are launched
// with hipExtLaunchKernelGGL and a start/stop event pair recorded by the
// dispatch itself; collect() (after the stream has been synchronised) adds the
// elapsed times.  `steps` counts the colour steps each launch performed.
struct Timing {
    bool on = false;
    uint32_t every = 1;       // time one launch in `every`
    uint64_t counter = 0;
    std::vector<hipEvent_t> pool;
    std::vector<hipEvent_t> pending;      // start, stop, start, stop, ...
    std::vector<uint32_t> pending_steps;
    double ms = 0.0;
    uint64_t launches = 0, steps = 0;

    hipError_t events(hipEvent_t *a, hipEvent_t *b)
    {
        for (hipEvent_t *e : {a, b}) {
            if (!pool.empty()) {
                *e = pool.back();
                pool.pop_back();
            } else {
                hipError_t err = hipEventCreate(e);
                if (err != hipSuccess) return err;
            }
        }
        return hipSuccess;
    }
    hipError_t collect()
    {
        for (size_t i = 0; i + 1 < pending.size(); i += 2) {
            float t = 0.f;
            hipError_t e = hipEventElapsedTime(&t, pending[i], pending[i + 1]);
            if (e != hipSuccess) return e;
            ms += t;
            launches += 1;
            steps += pending_steps[i / 2];
            pool.push_back(pending[i]);
            pool.push_back(pending[i + 1]);
        }
        pending.clear();
        pending_steps.clear();
        return hipSuccess;
    }
    void release()
    {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        for (hipEvent_t e : pending) (void)hipEventDestroy(e);
        pool.clear();
        pending.clear();
    }
};

template <typename F, typename... Args>
hipError_t launch(Timing *tm, uint32_t steps, F kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t s,
                  Args... args)
{
    if (tm && tm->on && (tm->counter++ % tm->every) == 0) {
        hipEvent_t a, b;
        hipError_t e = tm->events(&a, &b);
        if (e != hipSuccess) return e;
        hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, a, b, 0, args...);
        tm->pending.push_back(a);
        tm->pending.push_back(b);
        tm->pending_steps.push_back(steps);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- domino
// Aztec diamond of order n in the owner frame: the owner colour
// omega = (n+1) mod 2 has its n^2 sites on the grid (r, k) in [0, n)^2; each
// owner site keeps the four crossing bits of its edges N, S, E, W (so every edge
// of the lattice is stored once, 4 bits per owner vertex = 2 bits per face).
// Plane p (N=0, S=1, E=2, W=3) row r word w lives at planes[p*PS + r*RS + w].
// RS = 4*(ng+1) words (ng groups of 4 words cover the row, 4 zero pad words),
// n+1 rows (row n is zero padding).
struct DominoDev {
    int n = 0;
    int omega = 0;
    uint32_t ng = 0;   // groups of 128 sites per row
    uint32_t RS = 0;   // row stride in words
    size_t PS = 0;     // plane stride in words
    uint32_t *planes = nullptr;   // current state
    uint32_t *spare = nullptr;    // second buffer of the tiled kernel (same layout)
};
// Tile of the multi-sweep kernel: TR owner rows x TG groups of 4 words, run for
// up to S sweeps per launch with an S-row halo above and below and a one-group
// halo left and right (a dimension covered by one tile needs no halo).
// Words per LDS row of a domino tile of LG groups: the groups, one more group
// (the neighbour the shifted planes read), rounded to an odd number of 4-word
// slots so that 16 consecutive rows of one group fall in distinct banks.
inline __host__ __device__ uint32_t domino_lds_row_words(uint32_t LG)
{
    const uint32_t slots = LG + 1u;
    return 4u * (slots | 1u);
}
struct DominoTile {
    uint32_t TR = 32, TG = 4, S = 8;
    uint32_t order = 0;   // colour order: 0 fixed, 1 random per step
    uint32_t reg = 0;     // 1: register-resident tiles (a lane per row, a wavefront per group column)
};
size_t domino_words(int n, uint32_t *ng, uint32_t *RS, size_t *PS);
hipError_t domino_init(const DominoDev &d, int init_max, hipStream_t s);
// One colour step; t is the sweep counter of the draws (the step index under
// the random colour order).
hipError_t domino_colour_step(const DominoDev &d, int colour, uint32_t t, const Thr &T, int metropolis,
                              uint64_t seed, hipStream_t s, Timing *tm = nullptr);
// Sweeps t0 .. t0+n-1 with the tiled kernel; swaps d.planes / d.spare.
hipError_t domino_tiled_sweeps(DominoDev &d, const DominoTile &tile, uint32_t t0, uint32_t n, const Thr &T,
                               int metropolis, uint64_t seed, hipStream_t s, Timing *tm = nullptr);
DominoTile domino_auto_tile(int n, bool random_order, bool weighted = false);
hipError_t domino_export(const DominoDev &d, uint8_t *faces, hipStream_t s);
hipError_t domino_observe(const DominoDev &d, uint32_t B, uint32_t bins_x, unsigned long long *bins,
                          hipStream_t s);
// The same over a w x h box of faces at face offset (ox, oy) in the diamond's
// box (a domain embedded in the diamond); bins are counted in box coordinates.
hipError_t domino_export_box(const DominoDev &d, int ox, int oy, int w, int h, uint8_t *faces, hipStream_t s);
hipError_t domino_observe_box(const DominoDev &d, int ox, int oy, int h, uint32_t B, uint32_t bins_x,
                              unsigned long long *bins, hipStream_t s);

// ------------------------------------------------------------ batched chains
// One entry per domino chain of a batch; planes of chain i start at word
// `offset` of the batch buffer and use the DominoDev layout of its order n.
struct BatchChain {
    uint64_t offset;
    uint64_t PS;
    uint32_t n, ng, RS;
    uint32_t key0, key1;
    uint32_t t;        // sweeps done, advanced by the kernel
    uint32_t lds_bytes;
    uint32_t pad;
};
// A bundle: chains members[first .. first+count) that one work-group advances
// together.  A bundle of several chains has at most as many (row, group)
// tasks as the work-group has threads; a single chain may have more.
constexpr uint32_t kBundleMax = 16;
struct BatchBundle {
    uint32_t first, count, tasks, pad;
};
// Advance every chain of bundles[0..nbundles) by nsweeps sweeps: one
// persistent launch; work-groups take bundles from an atomic counter (reset by
// a small kernel first, so the pair can be captured in a graph).
// colour_order: 0 fixed, 1 random per step (chain by chain, from its key).
hipError_t domino_batch_sweeps(BatchChain *chains, const BatchBundle *bundles, const uint32_t *members,
                               uint32_t nbundles, uint32_t *counter, uint32_t *planes, uint32_t nsweeps, const Thr &T,
                               int metropolis, uint32_t colour_order, uint32_t threads, uint32_t workgroups,
                               uint32_t lds_bytes, hipStream_t s, Timing *tm = nullptr);

// ------------------------------------------------------ height-function models
// Bit-planes of a 1-bit height residual: plane p, row y, word w at
// planes[p*PS + y*RS + 4 + w] (a zero pad group before and after each row).
struct HeightDev {
    int model = 0;          // TL_LOZENGE or TL_SIXVERTEX
    int a = 0, b = 0, c = 0;  // hexagon sides (lozenge)
    int N = 0;              // grid size (six-vertex)
    uint32_t P = 0;         // planes: 3 (lozenge, X mod 3) or 2 (six-vertex, I mod 2)
    uint32_t rows = 0;      // b+c+1 or N+1
    uint32_t K = 0;         // sites per plane row
    uint32_t ng = 0, RS = 0;
    size_t PS = 0;
    uint32_t *planes = nullptr, *spare = nullptr;
    // six-vertex domain given by a mask: bit planes (same layout as the state)
    // of the points that may flip, and of those on its free side (or
    // nullptr); nullptr for the domain-wall square
    const uint32_t *site = nullptr;
    const uint32_t *freep = nullptr;
    int free_side = 0;      // side of the free points: 1 north, 2 south, 3 east, 4 west
    int ox = 0, oy = 0;     // six-vertex mask: state point of the mask box's point (0, 0)
};
struct HeightTile {
    uint32_t TR = 32, TG = 4, S = 8;
    uint32_t order = 0;   // colour order: 0 fixed, 1 random per step
    uint32_t lanes = 1;   // lanes per task: 1 (one-bit decisions) or 4 (bit-serial, a quad per task)
    uint32_t items = 0;   // 1: a share of a multi-job launch (work-groups of at most 512 lanes)
};
size_t height_words(HeightDev &d);
hipError_t height_init(const HeightDev &d, int init_max, hipStream_t s);
hipError_t height_colour_step(const HeightDev &d, int colour, uint32_t t, const Thr &T, int metropolis,
                              uint64_t seed, hipStream_t s, Timing *tm = nullptr);
hipError_t height_tiled_sweeps(HeightDev &d, const HeightTile &tile, uint32_t t0, uint32_t n, const Thr &T,
                               int metropolis, uint64_t seed, hipStream_t s, Timing *tm = nullptr);
HeightTile height_auto_tile(const HeightDev &d, bool uniform, bool metropolis = false);
// int32 canonical export into dev (rows x (row length) values)
hipError_t height_export(const HeightDev &d, int32_t *dev, hipStream_t s);
hipError_t height_observe(const HeightDev &d, uint32_t B, uint32_t bins_x, unsigned long long *bins, hipStream_t s);
// Six-vertex domain given by a mask (w x h cells in the state's box): the
// (h+1) x (w+1) heights, anchored at the boundary points (anchor: boundary
// height, INT32_MIN off the domain, INT32_MAX at sites); type-c cells of the
// domain (cells: w*h bytes, 1 = in the domain) into bins, through `heights`,
// a (w+1)*(h+1) int32 scratch buffer.
hipError_t sixv_region_export(const HeightDev &d, const int32_t *anchor, int w, int h, int32_t *out, hipStream_t s);
hipError_t sixv_region_observe(const HeightDev &d, const int32_t *anchor, const uint8_t *cells, int w, int h,
                               int32_t *heights, uint32_t B, uint32_t bins_x, unsigned long long *bins,
                               hipStream_t s);
// Lozenge domain given by a mask (w x h squares, c = 0 box): the (h+1) x (w+1)
// heights anchored as above; the volume H - H_min of its vertices into bins
// of B x B vertices (hmin: INT32_MIN off the domain).
hipError_t loz_region_export(const HeightDev &d, const int32_t *anchor, int w, int h, int32_t *out, hipStream_t s);
hipError_t loz_region_observe(const HeightDev &d, const int32_t *anchor, const int32_t *hmin, int w, int h,
                              int32_t *heights, uint32_t B, uint32_t bins_x, unsigned long long *bins,
                              hipStream_t s);

// ------------------------------------------------------ planned tile launches
// One launch of a tiled multi-sweep kernel, planned on the host: S sweeps,
// tiles_x * tiles_y tiles of TR rows x TG groups with HR halo rows and HG halo
// groups on each side, `threads` per work-group (one (row, group) task per
// thread and row pass), `lds` bytes of LDS per work-group.
struct TilePlan {
    uint32_t S = 0, TR = 0, TG = 0, HR = 0, HG = 0, tiles_x = 0, tiles_y = 0, threads = 0, lds = 0;
    uint32_t order = 0;   // colour order of the launch (the halo covers it)
    uint32_t reg = 0;     // domino: register-resident tiles
    uint32_t tiles() const { return tiles_x * tiles_y; }
};
// Largest launch of at most S_max sweeps the tile shape allows (tile sizes
// clamped as the single-state launches clamp them); false if none fits.
bool domino_plan(const DominoDev &d, const DominoTile &tile, uint32_t S_max, TilePlan *p);
// Thread rows of a height tile of LR rows: lozenge one per row, six-vertex
// one per row pair (each colour step updates rows of one parity only).
inline uint32_t height_task_rows(int model, uint32_t LR) { return model == TL_LOZENGE ? LR : (LR + 1u) / 2u; }
bool height_plan(const HeightDev &d, const HeightTile &tile, uint32_t S_max, TilePlan *p);

// One state's share of a multi-job launch (served form): the state it reads
// and the buffer it writes, its geometry, launch plan, thresholds and key.
// A work-group handles one item (job, tile).
enum { kModeHeatBath = 0, kModeMetropolis = 1, kModeUniform = 2 };
// Layout of a height-model kernel table: classes (lozenge; six-vertex 9 classes
// (sA, sB) [x2 Metropolis]) or six-vertex 5 classes by sA + sB (heat-bath).
enum { kTableClass = 0, kTableSum = 1 };
// Six-vertex tables by sA + sB: 5 entries (heat-bath) or 5 x 2 (Metropolis).
inline uint32_t table_kind(const Thr &K)
{
    return K.count == 5u || K.count == 10u ? (uint32_t)kTableSum : (uint32_t)kTableClass;
}
struct TileJob {
    const uint32_t *in;
    uint32_t *out;
    uint64_t PS;
    uint32_t RS, ng, rows, P, K;      // domino: rows = n, P = 4, K = 0
    int32_t model, a, b, c, N, omega;   // heights: model and sides; domino: omega
    uint32_t t0, S, TR, TG, HR, HG, tiles_x;
    uint32_t mode;                      // kMode*
    uint32_t kind;                      // kTable* (height models)
    uint32_t order;                     // colour order: 0 fixed, 1 random per step
    uint32_t key0, key1;
    const uint32_t *site;               // six-vertex site planes of a masked domain, or nullptr
    const uint32_t *freep;              // planes of its free points, or nullptr
    int32_t free_side;                  // their side: 1 north, 2 south, 3 east, 4 west
    Thr T;                              // kernel table (heights: weight classes)
};
struct TileItem {
    uint32_t job, tile;
};
TileJob domino_tile_job(const DominoDev &d, const TilePlan &p, uint32_t t0, const Thr &T, int metropolis,
                        uint64_t seed);
TileJob height_tile_job(const HeightDev &d, const TilePlan &p, uint32_t t0, const Thr &T, int metropolis,
                        uint64_t seed);
// One launch over items[0..n_items) (device arrays): threads and LDS bytes per
// work-group at least the largest any item's plan asks for.
// Every job of a launch has colour order `order`.
hipError_t domino_items(const TileJob *jobs, const TileItem *items, uint32_t n_items, uint32_t threads,
                        uint32_t lds, uint32_t order, hipStream_t s);
// Height items of one launch share one rule and one table kind (one kernel
// instantiation each); a heat-bath launch also runs one-bit jobs.
// Every job has colour order `order`, and site planes iff `masked`.
hipError_t height_items(const TileJob *jobs, const TileItem *items, uint32_t n_items, uint32_t threads,
                        uint32_t lds, uint32_t mode, uint32_t kind, uint32_t order, uint32_t masked, hipStream_t s);
// Height items of any rules and table kinds in one launch.
hipError_t height_items_mixed(const TileJob *jobs, const TileItem *items, uint32_t n_items, uint32_t threads,
                              uint32_t lds, uint32_t order, uint32_t masked, hipStream_t s);

// ----------------------------------------------------------------- hashing
// SHA-256 of each of `rows` rows of `row_bytes` bytes at `data` (device), into
// 32-byte digests at `digests` (device).
hipError_t hash_rows(const uint8_t *data, uint32_t rows, uint32_t row_bytes, uint8_t *digests,
                     hipStream_t s);
void sha256_host(const uint8_t *data, size_t len, uint8_t out[32]);

}  // namespace tl
