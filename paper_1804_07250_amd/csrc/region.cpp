// Host pre-pass for general domino domains (Section 1.1; Thurston's
// tileability test with the extremal tilings, linear in the domain's size).
//
// Boundary edges always bound a domino, so walking the boundary fixes the
// heights there.  Any height function obeys h(v) <= h(u) + 1 across an edge
// u -> v with a black face on its left and h(v) <= h(u) + 3 with a white one,
// so h <= U(v) = min over boundary vertices b of h(b) + dist(b, v) (edge
// lengths 1 and 3); symmetrically h >= L(v) with lengths 3 and 1 walked
// backwards.  The domain is tileable iff U and L equal the boundary heights
// on the boundary; then U is the height function of T_max and L that of
// T_min.  Distances take small integer lengths, so a bucket queue (Dial's
// method) keeps the work linear.
#include "region.hpp"
#include "../../include/tilings.h"

#include <limits.h>
#include <stdint.h>

#include <algorithm>

namespace tl {

namespace {

constexpr int32_t kUnset = INT32_MIN;

struct Grid {
    int w, h, parity;
    const std::vector<uint8_t> &m;
    int vw() const { return w + 1; }
    bool in(int x, int y) const { return x >= 0 && y >= 0 && x < w && y < h && m[(size_t)y * w + x]; }
    bool black(int x, int y) const { return ((x + y + parity) & 1) == 0; }
};

// The four edges out of vertex (i, j): neighbour and the faces on the left
// and the right of the walk.
struct Step {
    int di, dj, lx, ly, rx, ry;
};
constexpr Step kSteps[4] = {
    {1, 0, 0, 0, 0, -1},     // east:  left (i, j),       right (i, j-1)
    {-1, 0, -1, -1, -1, 0},  // west:  left (i-1, j-1),   right (i-1, j)
    {0, 1, -1, 0, 0, 0},     // north: left (i-1, j),     right (i, j)
    {0, -1, 0, -1, -1, -1},  // south: left (i, j-1),     right (i-1, j-1)
};

int floor_div2(int v) { return v >= 0 ? v / 2 : -((-v + 1) / 2); }

bool connected(const std::vector<uint8_t> &sel, int W, int H, size_t expected)
{
    if (expected == 0) return true;
    size_t start = 0;
    while (!sel[start]) ++start;
    std::vector<uint8_t> seen(sel.size(), 0);
    std::vector<size_t> stack{start};
    seen[start] = 1;
    size_t count = 1;
    while (!stack.empty()) {
        const size_t c = stack.back();
        stack.pop_back();
        const int x = (int)(c % W), y = (int)(c / W);
        const int nx[4] = {x + 1, x - 1, x, x}, ny[4] = {y, y, y + 1, y - 1};
        for (int k = 0; k < 4; ++k) {
            if (nx[k] < 0 || ny[k] < 0 || nx[k] >= W || ny[k] >= H) continue;
            const size_t d = (size_t)ny[k] * W + nx[k];
            if (sel[d] && !seen[d]) {
                seen[d] = 1;
                ++count;
                stack.push_back(d);
            }
        }
    }
    return count == expected;
}

// Multi-source shortest paths with edge lengths len_black / len_white, the
// sources being the boundary vertices at key sign * hb.
std::vector<int32_t> bound(const Grid &g, const std::vector<int32_t> &hb, int sign, int len_black, int len_white)
{
    const int VW = g.vw();
    const size_t V = hb.size();
    std::vector<int32_t> dist(V, kUnset);
    int32_t kmin = INT32_MAX;
    for (size_t v = 0; v < V; ++v)
        if (hb[v] != kUnset) kmin = std::min(kmin, sign * hb[v]);
    std::vector<std::vector<uint32_t>> buckets;
    auto push = [&](uint32_t v, int32_t key) {
        dist[v] = key;
        const size_t b = (size_t)(key - kmin);
        if (b >= buckets.size()) buckets.resize(b + 1);
        buckets[b].push_back(v);
    };
    for (size_t v = 0; v < V; ++v)
        if (hb[v] != kUnset) push((uint32_t)v, sign * hb[v]);
    for (size_t b = 0; b < buckets.size(); ++b) {
        for (size_t q = 0; q < buckets[b].size(); ++q) {
            const uint32_t v = buckets[b][q];
            const int32_t d = (int32_t)b + kmin;
            if (dist[v] != d) continue;   // a shorter path reached v first
            const int i = (int)(v % VW), j = (int)(v / VW);
            for (const Step &s : kSteps) {
                const bool l = g.in(i + s.lx, j + s.ly), r = g.in(i + s.rx, j + s.ry);
                if (!l && !r) continue;
                const uint32_t u = (uint32_t)((j + s.dj) * VW + i + s.di);
                const int32_t nd = d + (g.black(i + s.lx, j + s.ly) ? len_black : len_white);
                if (dist[u] == kUnset || nd < dist[u]) push(u, nd);
            }
        }
        std::vector<uint32_t>().swap(buckets[b]);
    }
    return dist;
}

// Canonical export of the tiling with height function hv (sign * dist).
bool tiling_of(const Grid &g, const std::vector<int32_t> &dist, int sign, std::vector<uint8_t> &out)
{
    const int VW = g.vw();
    out.assign((size_t)g.w * g.h, 0xFF);
    auto H = [&](int i, int j) { return (int64_t)sign * dist[(size_t)j * VW + i]; };
    for (int y = 0; y < g.h; ++y)
        for (int x = 0; x < g.w; ++x) {
            if (!g.in(x, y)) continue;
            // edge (two corners), partner code, partner face
            const int e[4][4] = {{x, y + 1, x + 1, y + 1}, {x, y, x + 1, y}, {x + 1, y, x + 1, y + 1}, {x, y, x, y + 1}};
            const int px[4] = {x, x, x + 1, x - 1}, py[4] = {y + 1, y - 1, y, y};
            int code = -1;
            for (int k = 0; k < 4; ++k) {
                const int64_t dh = H(e[k][0], e[k][1]) - H(e[k][2], e[k][3]);
                if (dh != 3 && dh != -3) continue;
                if (code >= 0 || !g.in(px[k], py[k])) return false;
                code = k;
            }
            if (code < 0) return false;
            out[(size_t)y * g.w + x] = (uint8_t)code;
        }
    return true;
}

}  // namespace

void region_embedding(int w, int h, int *n, int *ox, int *oy)
{
    const int N = (w + h + 1) / 2;
    const int m = floor_div2(h - w);
    const int D = ((m - N) & 1) == 0 ? m : m - 1;
    *n = N;
    *ox = (N + D) / 2;
    *oy = (N - D) / 2;
}

namespace {

// Copy the mask (0/1) and check it describes an accepted domain: non-empty,
// edge-connected, no pinch vertex, no hole.
RegionStatus validate_mask(const uint8_t *mask, int w, int h, std::vector<uint8_t> &m, uint64_t &count,
                           std::string &why)
{
    if (!mask || w < 1 || h < 1 || (int64_t)w + h > 32768) {
        why = "mask domain needs a mask and 1 <= w, h with w + h <= 32768";
        return kRegionInvalid;
    }
    m.assign((size_t)w * h, 0);
    count = 0;
    for (size_t i = 0; i < m.size(); ++i) {
        m[i] = mask[i] ? 1 : 0;
        count += m[i];
    }
    if (count == 0) {
        why = "empty domain";
        return kRegionInvalid;
    }
    auto in = [&](int x, int y) { return x >= 0 && y >= 0 && x < w && y < h && m[(size_t)y * w + x]; };
    // pinch vertices: exactly two diagonally opposite cells inside
    for (int j = 0; j <= h; ++j)
        for (int i = 0; i <= w; ++i) {
            const bool sw = in(i - 1, j - 1), se = in(i, j - 1), nw = in(i - 1, j), ne = in(i, j);
            if ((sw && ne && !se && !nw) || (se && nw && !sw && !ne)) {
                why = "domain pinched at vertex (" + std::to_string(i) + ", " + std::to_string(j) + ")";
                return kRegionInvalid;
            }
        }
    if (!connected(m, w, h, count)) {
        why = "domain is not connected";
        return kRegionInvalid;
    }
    // holes: the complement in the box grown by one cell must be connected
    const int W2 = w + 2, H2 = h + 2;
    std::vector<uint8_t> out((size_t)W2 * H2, 1);
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) out[(size_t)(y + 1) * W2 + x + 1] = m[(size_t)y * w + x] ? 0 : 1;
    if (!connected(out, W2, H2, (size_t)W2 * H2 - count)) {
        why = "domain has a hole";
        return kRegionInvalid;
    }
    return kRegionOk;
}

}  // namespace

RegionStatus build_region(const uint8_t *mask, int w, int h, Region &r, std::string &why)
{
    const RegionStatus vs = validate_mask(mask, w, h, r.mask, r.faces, why);
    if (vs != kRegionOk) return vs;
    r.w = w;
    r.h = h;
    region_embedding(w, h, &r.n, &r.ox, &r.oy);
    const Grid g{w, h, r.n & 1, r.mask};
    r.sites = 0;
    for (int j = 1; j < h; ++j)
        for (int i = 1; i < w; ++i)
            r.sites += g.in(i - 1, j - 1) && g.in(i, j - 1) && g.in(i - 1, j) && g.in(i, j);

    // boundary heights, walking the boundary edges from the lowest, then
    // leftmost, vertex of the domain
    const int VW = w + 1;
    const size_t V = (size_t)VW * (h + 1);
    std::vector<int32_t> hb(V, kUnset);
    size_t start = 0;
    for (int j = 0, found = 0; j <= h && !found; ++j)
        for (int i = 0; i <= w && !found; ++i)
            if (g.in(i - 1, j - 1) || g.in(i, j - 1) || g.in(i - 1, j) || g.in(i, j)) {
                start = (size_t)j * VW + i;
                found = 1;
            }
    hb[start] = 0;
    std::vector<size_t> stack{start};
    while (!stack.empty()) {
        const size_t v = stack.back();
        stack.pop_back();
        const int i = (int)(v % VW), j = (int)(v / VW);
        for (const Step &s : kSteps) {
            const bool l = g.in(i + s.lx, j + s.ly), rr = g.in(i + s.rx, j + s.ry);
            if (l == rr) continue;   // interior edge, or no edge of the domain
            const size_t u = (size_t)(j + s.dj) * VW + i + s.di;
            const int32_t hu = hb[v] + (g.black(i + s.lx, j + s.ly) ? 1 : -1);
            if (hb[u] == kUnset) {
                hb[u] = hu;
                stack.push_back(u);
            } else if (hb[u] != hu) {
                why = "no tiling: the boundary heights do not close up";
                return kRegionUntileable;
            }
        }
    }
    const std::vector<int32_t> up = bound(g, hb, 1, 1, 3);
    const std::vector<int32_t> down = bound(g, hb, -1, 3, 1);
    for (size_t v = 0; v < V; ++v)
        if (hb[v] != kUnset && (up[v] != hb[v] || down[v] != -hb[v])) {
            why = "no tiling: no height function meets the boundary heights";
            return kRegionUntileable;
        }
    if (!tiling_of(g, up, 1, r.tmax) || !tiling_of(g, down, -1, r.tmin)) {
        why = "no tiling: extremal heights do not describe a tiling";
        return kRegionUntileable;
    }
    return kRegionOk;
}

// Six-vertex domains.  Neighbouring heights differ by exactly 1, so the
// configurations are the functions that are 1-Lipschitz along the cell sides
// of the domain, agree with the boundary and have the parity of I + J: the
// largest is min_b h(b) + dist(b, v), the smallest max_b h(b) - dist(b, v)
// (unit lengths, a bucket queue from all boundary points at once), and one
// exists iff both meet the boundary heights.
int free_side_of(uint32_t flags)
{
    switch (flags) {
    case 0: return 0;
    case TL_FREE_NORTH: return 1;
    case TL_FREE_SOUTH: return 2;
    case TL_FREE_EAST: return 3;
    case TL_FREE_WEST: return 4;
    default: return -1;
    }
}

RegionStatus build_sixv_region(const uint8_t *mask, int w, int h, int free_side, HeightRegion &r,
                               std::string &why)
{
    uint64_t ncells = 0;
    const RegionStatus vs = validate_mask(mask, w, h, r.cells, ncells, why);
    if (vs != kRegionOk) return vs;
    r.model = 2;   // TL_SIXVERTEX
    r.w = w;
    r.h = h;
    r.cw = w;
    r.ch = h;
    r.free_sites = 0;
    r.free_side = free_side;
    const int PW = w + 1;
    const size_t V = (size_t)PW * (h + 1);
    auto in = [&](int x, int y) { return x >= 0 && y >= 0 && x < w && y < h && r.cells[(size_t)y * w + x] != 0; };
    std::vector<uint8_t> pt(V, 0);
    r.site.assign(V, 0);
    r.sites = 0;
    size_t start = V;
    for (int J = 0; J <= h; ++J)
        for (int I = 0; I <= w; ++I) {
            const bool a = in(I - 1, J - 1), b = in(I, J - 1), c = in(I - 1, J), d = in(I, J);
            const size_t v = (size_t)J * PW + I;
            pt[v] = a || b || c || d;
            r.site[v] = a && b && c && d;
            r.sites += r.site[v];
            if (pt[v] && start == V) start = v;
        }
    // Steps out of point (I, J): neighbour offset, the two cells beside the
    // edge (above / below for horizontal steps, right / left for vertical
    // ones) and the direction sign of the boundary increment.
    struct Edge {
        int dI, dJ, ax, ay, bx, by, sign;
    };
    static constexpr Edge kE[4] = {{1, 0, 0, 0, 0, -1, 1},
                                   {-1, 0, -1, 0, -1, -1, -1},
                                   {0, 1, 0, 0, -1, 0, 1},
                                   {0, -1, 0, -1, -1, -1, -1}};
    // Is a boundary edge (cells a, b beside it, a != b) a side of the free
    // kind: horizontal steps have a above and b below, vertical ones a to the
    // right and b to the left; the domain's cell is the one inside.
    auto free_edge = [&](const Edge &e, bool a, bool b) {
        switch (free_side) {
        case 1: return e.dJ == 0 && b;   // north side of the cell below
        case 2: return e.dJ == 0 && a;   // south side of the cell above
        case 3: return e.dI == 0 && b;   // east side of the cell to the left
        case 4: return e.dI == 0 && a;   // west side of the cell to the right
        default: return false;
        }
    };
    std::vector<int32_t> hb(V, kUnset);
    {
        const int I0 = (int)(start % PW), J0 = (int)(start / PW);
        hb[start] = (I0 + J0) & 1;
        std::vector<size_t> stack{start};
        while (!stack.empty()) {
            const size_t v = stack.back();
            stack.pop_back();
            const int I = (int)(v % PW), J = (int)(v / PW);
            for (const Edge &e : kE) {
                const bool a = in(I + e.ax, J + e.ay), b = in(I + e.bx, J + e.by);
                if (a == b) continue;   // interior side, or no side of the domain
                if (free_edge(e, a, b)) continue;   // a free leg
                const size_t u = (size_t)(J + e.dJ) * PW + I + e.dI;
                const int32_t hu = hb[v] + e.sign * (a ? 1 : -1);
                if (hb[u] == kUnset) {
                    hb[u] = hu;
                    stack.push_back(u);
                } else if (hb[u] != hu) {
                    why = "no configuration: the boundary heights do not close up";
                    return kRegionUntileable;
                }
            }
        }
    }
    // boundary points the walk did not reach: free (code 2) when every boundary
    // edge at them is a free side, otherwise the fixed boundary is in pieces
    for (size_t v = 0; v < V; ++v) {
        if (!pt[v] || r.site[v] || hb[v] != kUnset) continue;
        const int I = (int)(v % PW), J = (int)(v / PW);
        bool all_free = free_side != 0;
        for (const Edge &e : kE) {
            const bool a = in(I + e.ax, J + e.ay), b = in(I + e.bx, J + e.by);
            if (a != b && !free_edge(e, a, b)) all_free = false;
        }
        if (!all_free) {
            why = free_side ? "free edges split the fixed boundary" : "boundary not connected";
            return kRegionInvalid;
        }
        r.site[v] = 2;
        r.sites += 1;
        r.free_sites += 1;
    }
    auto bound = [&](int sign) {
        std::vector<int32_t> dist(V, kUnset);
        int32_t kmin = INT32_MAX;
        for (size_t v = 0; v < V; ++v)
            if (hb[v] != kUnset) kmin = std::min(kmin, sign * hb[v]);
        std::vector<std::vector<uint32_t>> buckets;
        auto push = [&](size_t v, int32_t key) {
            dist[v] = key;
            const size_t b = (size_t)(key - kmin);
            if (b >= buckets.size()) buckets.resize(b + 1);
            buckets[b].push_back((uint32_t)v);
        };
        for (size_t v = 0; v < V; ++v)
            if (hb[v] != kUnset) push(v, sign * hb[v]);
        for (size_t b = 0; b < buckets.size(); ++b) {
            for (size_t q = 0; q < buckets[b].size(); ++q) {
                const uint32_t v = buckets[b][q];
                const int32_t d = (int32_t)b + kmin;
                if (dist[v] != d) continue;
                const int I = (int)(v % PW), J = (int)(v / PW);
                for (const Edge &e : kE) {
                    if (!in(I + e.ax, J + e.ay) && !in(I + e.bx, J + e.by)) continue;
                    const size_t u = (size_t)(J + e.dJ) * PW + I + e.dI;
                    if (dist[u] == kUnset || d + 1 < dist[u]) push(u, d + 1);
                }
            }
            std::vector<uint32_t>().swap(buckets[b]);
        }
        return dist;
    };
    const std::vector<int32_t> up = bound(1), down = bound(-1);
    r.hmax.assign(V, INT32_MIN);
    r.hmin.assign(V, INT32_MIN);
    r.anchor.assign(V, INT32_MIN);
    for (size_t v = 0; v < V; ++v) {
        if (!pt[v]) continue;
        if (hb[v] != kUnset && (up[v] != hb[v] || down[v] != -hb[v])) {
            why = "no configuration meets the boundary heights";
            return kRegionUntileable;
        }
        r.hmax[v] = up[v];
        r.hmin[v] = -down[v];
        r.anchor[v] = r.site[v] ? INT32_MAX : hb[v];
    }
    return kRegionOk;
}

// Lozenge domains.  Triangle (x, y, t) has edge-neighbours: t = 0 -> (x, y, 1),
// (x, y-1, 1), (x+1, y, 1); t = 1 -> (x, y, 0), (x, y+1, 0), (x-1, y, 0).
RegionStatus build_loz_region(const uint8_t *mask, int w, int h, HeightRegion &r, std::string &why)
{
    if (!mask || w < 1 || h < 1 || (int64_t)w + h > 32766) {
        why = "lozenge mask domain needs a mask and 1 <= w, h with w + h <= 32766";
        return kRegionInvalid;
    }
    const size_t T = (size_t)w * h * 2;
    std::vector<uint8_t> m(T);
    uint64_t count = 0;
    for (size_t i = 0; i < T; ++i) {
        m[i] = mask[i] ? 1 : 0;
        count += m[i];
    }
    if (!count) {
        why = "empty domain";
        return kRegionInvalid;
    }
    auto in = [&](int x, int y, int t) {
        return x >= 0 && y >= 0 && x < w && y < h && m[((size_t)y * w + x) * 2 + t] != 0;
    };
    // the six triangles at point (X, Y), counter-clockwise from the edge (1,0)
    auto ring = [&](int X, int Y, bool out[6]) {
        out[0] = in(X, Y, 0);
        out[1] = in(X, Y, 1);
        out[2] = in(X - 1, Y, 0);
        out[3] = in(X - 1, Y - 1, 1);
        out[4] = in(X - 1, Y - 1, 0);
        out[5] = in(X, Y - 1, 1);
    };
    const int PW = w + 1;
    const size_t V = (size_t)PW * (h + 1);
    std::vector<uint8_t> pt(V, 0);
    r.site.assign(V, 0);
    r.sites = 0;
    size_t start = V;
    for (int Y = 0; Y <= h; ++Y)
        for (int X = 0; X <= w; ++X) {
            bool rg[6];
            ring(X, Y, rg);
            int n = 0, runs = 0;
            for (int i = 0; i < 6; ++i) {
                n += rg[i];
                runs += rg[i] && !rg[(i + 5) % 6];
            }
            if (n > 0 && n < 6 && runs > 1) {
                why = "domain pinched at vertex (" + std::to_string(X) + ", " + std::to_string(Y) + ")";
                return kRegionInvalid;
            }
            const size_t v = (size_t)Y * PW + X;
            pt[v] = n > 0;
            r.site[v] = n == 6;
            r.sites += r.site[v];
            if (pt[v] && start == V) start = v;
        }
    // connectivity of the triangles, and of the complement in the box grown by
    // one square (no holes)
    auto components_ok = [&](int W, int H, auto sel, uint64_t expected) {
        std::vector<uint8_t> seen((size_t)W * H * 2, 0);
        size_t first = seen.size();
        for (size_t i = 0; i < seen.size() && first == seen.size(); ++i)
            if (sel((int)((i / 2) % W), (int)((i / 2) / W), (int)(i & 1))) first = i;
        if (first == seen.size()) return expected == 0;
        std::vector<size_t> stack{first};
        seen[first] = 1;
        uint64_t got = 1;
        while (!stack.empty()) {
            const size_t c = stack.back();
            stack.pop_back();
            const int x = (int)((c / 2) % W), y = (int)((c / 2) / W), t = (int)(c & 1);
            const int nb[3][3] = {{x, y, 1 - t}, {x, t ? y + 1 : y - 1, 1 - t}, {t ? x - 1 : x + 1, y, 1 - t}};
            for (const auto &q : nb) {
                if (q[0] < 0 || q[1] < 0 || q[0] >= W || q[1] >= H || !sel(q[0], q[1], q[2])) continue;
                const size_t d = ((size_t)q[1] * W + q[0]) * 2 + q[2];
                if (!seen[d]) {
                    seen[d] = 1;
                    ++got;
                    stack.push_back(d);
                }
            }
        }
        return got == expected;
    };
    if (!components_ok(w, h, in, count)) {
        why = "domain is not connected";
        return kRegionInvalid;
    }
    if (!components_ok(w + 2, h + 2, [&](int x, int y, int t) { return !in(x - 1, y - 1, t); },
                       (uint64_t)(w + 2) * (h + 2) * 2 - count)) {
        why = "domain has a hole";
        return kRegionInvalid;
    }
    // Steps out of a point: offset, the triangle on the left and on the right.
    struct Step {
        int dX, dY, lx, ly, lt, rx, ry, rt;
    };
    static constexpr Step kS[6] = {{1, 0, 0, 0, 0, 0, -1, 1},     {0, 1, -1, 0, 0, 0, 0, 1},
                                   {1, 1, 0, 0, 1, 0, 0, 0},      {-1, 0, -1, -1, 1, -1, 0, 0},
                                   {0, -1, 0, -1, 1, -1, -1, 0},  {-1, -1, -1, -1, 0, -1, -1, 1}};
    std::vector<int32_t> hb(V, kUnset);
    {
        const int X0 = (int)(start % PW), Y0 = (int)(start / PW);
        hb[start] = X0 + Y0;
        std::vector<size_t> stack{start};
        while (!stack.empty()) {
            const size_t v = stack.back();
            stack.pop_back();
            const int X = (int)(v % PW), Y = (int)(v / PW);
            for (const Step &s : kS) {
                const bool li = in(X + s.lx, Y + s.ly, s.lt), ri = in(X + s.rx, Y + s.ry, s.rt);
                if (li == ri) continue;
                // bounding edge: +1 along a lower-right triangle's counter-clockwise
                // walk, -1 along an upper-left one's
                const int inc = li ? (s.lt == 0 ? 1 : -1) : (s.rt == 0 ? -1 : 1);
                const size_t u = (size_t)(Y + s.dY) * PW + X + s.dX;
                const int32_t hu = hb[v] + inc;
                if (hb[u] == kUnset) {
                    hb[u] = hu;
                    stack.push_back(u);
                } else if (hb[u] != hu) {
                    why = "no tiling: the boundary heights do not close up";
                    return kRegionUntileable;
                }
            }
        }
    }
    auto bound = [&](int sign, int len_lr, int len_ul) {
        std::vector<int32_t> dist(V, kUnset);
        int32_t kmin = INT32_MAX;
        for (size_t v = 0; v < V; ++v)
            if (hb[v] != kUnset) kmin = std::min(kmin, sign * hb[v]);
        std::vector<std::vector<uint32_t>> buckets;
        auto push = [&](size_t v, int32_t key) {
            dist[v] = key;
            const size_t b = (size_t)(key - kmin);
            if (b >= buckets.size()) buckets.resize(b + 1);
            buckets[b].push_back((uint32_t)v);
        };
        for (size_t v = 0; v < V; ++v)
            if (hb[v] != kUnset) push(v, sign * hb[v]);
        for (size_t b = 0; b < buckets.size(); ++b) {
            for (size_t q = 0; q < buckets[b].size(); ++q) {
                const uint32_t v = buckets[b][q];
                const int32_t d = (int32_t)b + kmin;
                if (dist[v] != d) continue;
                const int X = (int)(v % PW), Y = (int)(v / PW);
                for (const Step &s : kS) {
                    if (!in(X + s.lx, Y + s.ly, s.lt) && !in(X + s.rx, Y + s.ry, s.rt)) continue;
                    const size_t u = (size_t)(Y + s.dY) * PW + X + s.dX;
                    const int32_t nd = d + (s.lt == 0 ? len_lr : len_ul);
                    if (dist[u] == kUnset || nd < dist[u]) push(u, nd);
                }
            }
            std::vector<uint32_t>().swap(buckets[b]);
        }
        return dist;
    };
    const std::vector<int32_t> up = bound(1, 1, 2), down = bound(-1, 2, 1);
    r.model = 1;   // TL_LOZENGE
    r.w = w;
    r.h = h;
    r.cw = w + 1;
    r.ch = h + 1;
    r.cells.assign(V, 0);
    r.hmax.assign(V, INT32_MIN);
    r.hmin.assign(V, INT32_MIN);
    r.anchor.assign(V, INT32_MIN);
    int32_t lowest = INT32_MAX;
    for (size_t v = 0; v < V; ++v) {
        if (!pt[v]) continue;
        if (hb[v] != kUnset && (up[v] != hb[v] || down[v] != -hb[v])) {
            why = "no tiling: no height function meets the boundary heights";
            return kRegionUntileable;
        }
        const int XY = (int)(v % PW) + (int)(v / PW);
        r.hmax[v] = (up[v] - XY) / 3;    // exact: h' - X - Y is a multiple of 3
        r.hmin[v] = (-down[v] - XY) / 3;
        lowest = std::min(lowest, r.hmin[v]);
    }
    for (size_t v = 0; v < V; ++v) {
        if (!pt[v]) continue;
        r.cells[v] = 1;
        r.hmax[v] -= lowest;
        r.hmin[v] -= lowest;
        r.anchor[v] = r.site[v] ? INT32_MAX : r.hmin[v];
    }
    return kRegionOk;
}

}  // namespace tl
