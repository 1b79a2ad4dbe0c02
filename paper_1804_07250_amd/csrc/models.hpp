// Per-model state objects behind the C-ABI: each owns its device bit-planes and
// knows how to initialise, sweep, observe, export and import its state.
#pragma once
#include <memory>
#include <string>
#include <vector>

#include "../../include/tilings.h"
#include "internal.hpp"

namespace tl {

class Model {
public:
    virtual ~Model() {}
    // A fresh model of the same domain (nothing allocated).
    virtual std::unique_ptr<Model> twin() const = 0;
    // Threshold table of the free north-edge points of a six-vertex domain.
    virtual void set_boundary_table(const std::vector<uint32_t> &) {}
    virtual hipError_t allocate() = 0;
    // The same with the state in caller-owned buffers of state_words() words
    // each (freed by the caller); other buffers are allocated as usual.
    virtual hipError_t allocate_into(uint32_t *state, uint32_t *spare) = 0;
    virtual void release() = 0;
    virtual hipError_t init(bool init_max, hipStream_t s) = 0;
    // Sweeps t0 .. t0+n-1, every colour in order 0..K-1 within a sweep.
    virtual hipError_t sweeps(uint32_t t0, uint32_t n, const Thr &T, bool metropolis, uint64_t seed,
                              const tl_options &opt, hipStream_t s) = 0;
    // Add the per-cell observable of the current state to bins of B x B cells.
    virtual hipError_t observe(uint32_t B, uint32_t bins_x, unsigned long long *bins, hipStream_t s) = 0;
    virtual void cell_box(uint32_t *w, uint32_t *h) const = 0;
    virtual std::vector<uint32_t> cells_per_bin(uint32_t B, uint32_t bins_x, uint32_t bins_y) const = 0;
    virtual void export_layout(uint32_t *rows, uint32_t *row_bytes) const = 0;
    virtual hipError_t export_canonical(uint8_t *dev, hipStream_t s) = 0;
    // Validate a canonical export on the host and upload it; false on error
    // (why set for invalid input, *err set for HIP failures).
    virtual bool import_canonical(const uint8_t *host, hipStream_t s, std::string &why, hipError_t *err) = 0;
    virtual uint64_t sites() const = 0;
    virtual int colours() const = 0;
    // Algorithmic bytes of one colour step: the packed state read and written once.
    virtual double bytes_per_colour_step() const = 0;

    // Multi-job launches (served form).  The state lives in two caller-owned
    // buffers of state_words() words each (attach; release() leaves them);
    // tile_job plans the next launch of at most S_max sweeps from sweep t0 and
    // describes it (tile shape: small states in one tile, larger ones in row
    // tiles; with spread, a height-model state whose tasks would take turns in
    // one work-group goes to row tiles too, for launches that last as long as
    // their slowest work-group), and swap_buffers() follows that launch.
    virtual size_t state_words() const = 0;
    virtual void attach(uint32_t *state, uint32_t *spare) = 0;
    virtual bool tile_job(uint32_t t0, uint32_t S_max, const Thr &T, bool metro, uint64_t seed, bool spread,
                          TileJob *j, TilePlan *p) const = 0;
    virtual void swap_buffers() = 0;
    virtual bool height_family() const = 0;
    // Device tables of a masked height-model domain placed in caller-owned
    // memory (served jobs): region_bytes() bytes at dev, filled with
    // asynchronous copies on stream s from host copies the model keeps; the
    // caller keeps the memory until the model is released.
    virtual size_t region_bytes() const { return 0; }
    virtual hipError_t attach_region(uint8_t *, hipStream_t) { return hipSuccess; }
    // Masked domain (the kernels read site planes).
    virtual bool masked() const { return false; }
    // Current state buffer (state_words() words; equal buffers <=> equal states).
    virtual const uint32_t *state() const = 0;
    Timing timing;
    // Colour order of sweeps and tile jobs: 0 = colours 0..K-1 in every sweep,
    // 1 = a random colour per step (step s = K t + i draws its colour and uses
    // sweep counter s for its site draws).
    uint32_t order = 0;
    // Tile shape for sweeps whose options leave it automatic (0 = the
    // automatic shape), as picked by the autotuner.
    uint32_t tuned_rows = 0, tuned_groups = 0, tuned_sweeps = 0;
    uint32_t tuned_kernel = 2;   // dominoes: 2 LDS tiles, 3 register tiles
    // Groups of 128 sites per state row (the tile-width unit).
    virtual uint32_t row_groups() const = 0;
};

// nullptr on error, with why set and *status (nullable) the error code:
// TL_EINVAL, or TL_EUNTILEABLE for a mask domain without tilings.
std::unique_ptr<Model> make_model(const tl_domain &d, std::string &why, tl_status *status = nullptr);
// Device bytes a sampler of this domain allocates (state, spare buffer, bins
// of edge obs_bin), or 0 if the domain is invalid.
size_t sampler_device_bytes(const tl_domain &d, uint32_t obs_bin);


}  // namespace tl
