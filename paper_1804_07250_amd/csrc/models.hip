// Host-side model objects: device allocation, sweep scheduling per model and
// the host conversion of canonical exports for import.
#include <stdlib.h>
#include <string.h>

#include "models.hpp"

namespace tl {

namespace {

// ------------------------------------------------------------------ domino
class DominoModel : public Model {
public:
    explicit DominoModel(int n) { d_.n = n; d_.omega = (n + 1) & 1; }

    hipError_t allocate() override
    {
        const size_t words = domino_words(d_.n, &d_.ng, &d_.RS, &d_.PS);
        hipError_t e = hipMalloc(&d_.planes, words * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMalloc(&d_.spare, words * sizeof(uint32_t));
        return e;
    }
    void release() override
    {
        if (d_.planes) (void)hipFree(d_.planes);
        if (d_.spare) (void)hipFree(d_.spare);
        d_.planes = d_.spare = nullptr;
        timing.release();
    }
    hipError_t init(bool init_max, hipStream_t s) override { return domino_init(d_, init_max ? 1 : 0, s); }

    hipError_t sweeps(uint32_t t0, uint32_t n, const Thr &T, bool metro, uint64_t seed, const tl_options &opt,
                      hipStream_t s) override
    {
        if (opt.kernel == 1) {   // one launch per colour step
            for (uint32_t i = 0; i < n; ++i)
                for (int c = 0; c < 2; ++c) {
                    hipError_t e = domino_colour_step(d_, c, t0 + i, T, metro ? 1 : 0, seed, s, &timing);
                    if (e != hipSuccess) return e;
                }
            return hipSuccess;
        }
        DominoTile tile = domino_auto_tile(d_.n);
        if (opt.tile_rows) tile.TR = opt.tile_rows;
        if (opt.tile_groups) tile.TG = opt.tile_groups;
        if (opt.sweeps_per_launch) tile.S = opt.sweeps_per_launch;
        return domino_tiled_sweeps(d_, tile, t0, n, T, metro ? 1 : 0, seed, s, &timing);
    }
    hipError_t observe(uint32_t B, uint32_t bins_x, unsigned long long *bins, hipStream_t s) override
    {
        return domino_observe(d_, B, bins_x, bins, s);
    }
    void cell_box(uint32_t *w, uint32_t *h) const override { *w = *h = 2u * (uint32_t)d_.n; }
    static bool face_in(int n, int X, int Y) { return abs(2 * X - 2 * n + 1) + abs(2 * Y - 2 * n + 1) <= 2 * n; }
    std::vector<uint32_t> cells_per_bin(uint32_t B, uint32_t bx, uint32_t by) const override
    {
        std::vector<uint32_t> c((size_t)bx * by, 0u);
        const int W = 2 * d_.n;
        for (int Y = 0; Y < W; ++Y)
            for (int X = 0; X < W; ++X)
                if (face_in(d_.n, X, Y)) c[(size_t)(Y / B) * bx + X / B] += 1;
        return c;
    }
    void export_layout(uint32_t *rows, uint32_t *row_bytes) const override
    {
        *rows = 2u * (uint32_t)d_.n;
        *row_bytes = 2u * (uint32_t)d_.n;
    }
    hipError_t export_canonical(uint8_t *dev, hipStream_t s) override { return domino_export(d_, dev, s); }

    bool import_canonical(const uint8_t *f, hipStream_t s, std::string &why, hipError_t *err) override
    {
        const int n = d_.n, W = 2 * n;
        std::vector<uint32_t> host(4 * d_.PS, 0u);
        auto set_owner = [&](int p, int P, int Q) -> bool {
            const int r2 = P + Q - n - 1, k2 = Q - P + n - 1;
            if (r2 < 0 || k2 < 0 || (r2 & 1) || (k2 & 1)) return false;
            const int r = r2 / 2, k = k2 / 2;
            if (r >= n || k >= n) return false;
            host[(size_t)p * d_.PS + (size_t)r * d_.RS + (k >> 5)] |= 1u << (k & 31);
            return true;
        };
        for (int Y = 0; Y < W; ++Y)
            for (int X = 0; X < W; ++X) {
                const uint8_t dir = f[(size_t)Y * W + X];
                if (!face_in(n, X, Y)) {
                    if (dir != 0xFF) { why = "face outside the diamond is not 0xFF"; return false; }
                    continue;
                }
                if (dir > 3) { why = "invalid partner code"; return false; }
                const int PX = X + (dir == 2) - (dir == 3), PY = Y + (dir == 0) - (dir == 1);
                if (PX < 0 || PY < 0 || PX >= W || PY >= W || !face_in(n, PX, PY) ||
                    f[(size_t)PY * W + PX] != (uint8_t)(dir ^ 1u)) {
                    why = "faces do not form a domino tiling";
                    return false;
                }
                bool ok = true;
                if (dir == 2) {   // vertical segment (X+1,Y)-(X+1,Y+1)
                    ok = (((X + 1 + Y) & 1) == d_.omega) ? set_owner(0, X + 1, Y) : set_owner(1, X + 1, Y + 1);
                } else if (dir == 0) {  // horizontal segment (X,Y+1)-(X+1,Y+1)
                    ok = (((X + Y + 1) & 1) == d_.omega) ? set_owner(2, X, Y + 1) : set_owner(3, X + 1, Y + 1);
                }
                if (!ok) { why = "crossed edge without an interior owner"; return false; }
            }
        hipError_t e = hipMemcpyAsync(d_.planes, host.data(), host.size() * sizeof(uint32_t),
                                      hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { *err = e; return false; }
        return true;
    }
    uint64_t sites() const override { return 2ull * d_.n * d_.n - 2ull * d_.n + 1ull; }
    int colours() const override { return 2; }
    // 4 bits per owner site (n^2 owners), read and written: n^2 bytes
    double bytes_per_colour_step() const override { return 2.0 * 4.0 * (double)d_.n * d_.n / 8.0; }

private:
    DominoDev d_;
};

}  // namespace

std::unique_ptr<Model> make_model(const tl_domain &d, std::string &why)
{
    if (d.model == TL_DOMINO) {
        if (d.shape != TL_AZTEC) { why = "dominoes support the Aztec diamond shape"; return nullptr; }
        if (d.n < 1 || d.n > 16384) { why = "Aztec order must be in [1, 16384]"; return nullptr; }
        return std::unique_ptr<Model>(new DominoModel(d.n));
    }
    why = "model not supported";
    return nullptr;
}

}  // namespace tl
