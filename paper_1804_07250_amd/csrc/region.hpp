// General domino domains (Section 1.1): a simply-connected union of faces
// given by a mask, its embedding in an Aztec diamond, and the host pre-pass
// that decides tileability and builds the extremal tilings (Thurston).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace tl {

// Mask of h rows by w faces (row 0 southmost) and what the samplers derive
// from it.  The diamond of order n holds the box at face offset (ox, oy);
// tmax / tmin are canonical exports (h x w, partner 0:N 1:S 2:E 3:W, 0xFF
// outside the domain) of T_max and T_min.
struct Region {
    int w = 0, h = 0;
    int n = 0, ox = 0, oy = 0;
    std::vector<uint8_t> mask;          // 1 = face in the domain
    std::vector<uint8_t> tmax, tmin;
    uint64_t faces = 0;                 // faces of the domain
    uint64_t sites = 0;                 // vertices with all four faces in the domain
};

enum RegionStatus { kRegionOk = 0, kRegionInvalid = 1, kRegionUntileable = 2 };

// Aztec order n = ceil((w+h)/2) and offset: ox + oy = n, ox - oy = D with
// m = floor((h-w)/2), D = m if m - n is even, else m - 1.
void region_embedding(int w, int h, int *n, int *ox, int *oy);

// Validate the mask (non-empty, edge-connected, no pinch vertex, no hole),
// embed it and compute T_max / T_min.  Heights: a face of the diamond's box
// is black when its coordinates sum to an even number; walking an edge with a
// black face on its left the height changes by +1 (the edge bounds a domino)
// or -3 (a domino covers it), with a white face on its left by -1 or +3.
RegionStatus build_region(const uint8_t *mask, int w, int h, Region &r, std::string &why);

// The six-vertex model on a domain (Section 1.2 with the domains of Section
// 1.1): the model's vertices are the cells of a w x h mask, heights live on the
// (w+1) x (h+1) cell corners (point (I, J) at index J*(w+1) + I), sites are the
// corners whose four cells all lie in the domain.  Domain-wall type boundary:
// legs through the south and west sides of cells carry paths, legs through the
// north and east sides are empty; walking a boundary edge in +x the height
// rises by 1 if the domain is above it and falls by 1 if below, in +y it rises
// if the domain is to its right and falls if to its left; the lowest, then
// leftmost, point gets height (I + J) mod 2.
struct SixvRegion {
    int w = 0, h = 0;
    std::vector<uint8_t> mask;           // w*h cells, 1 = in the domain
    std::vector<uint8_t> site;           // (w+1)*(h+1) points, 1 = site
    std::vector<int32_t> anchor;         // boundary height; INT32_MIN off the domain; INT32_MAX at sites
    std::vector<int32_t> hmax, hmin;     // extremal configurations (INT32_MIN off the domain)
    uint64_t sites = 0, cells = 0;
};
RegionStatus build_sixv_region(const uint8_t *mask, int w, int h, SixvRegion &r, std::string &why);

}  // namespace tl
