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

// A height-function model on a domain given by a mask over a box of w x h
// unit squares: heights on the (w+1) x (h+1) points (point (I, J) at index
// J*(w+1) + I), the sites those whose surrounding cells all lie in the domain,
// the other points of the domain fixed by its boundary.  Observable cells:
// six-vertex, the cw x ch = w x h cells (the model's vertices); lozenge, the
// (w+1) x (h+1) points of the domain.
struct HeightRegion {
    int model = 0;                       // TL_SIXVERTEX or TL_LOZENGE
    int w = 0, h = 0;
    int cw = 0, ch = 0;                  // box of the observable cells
    std::vector<uint8_t> cells;          // cw*ch, 1 = cell of the domain
    std::vector<uint8_t> site;           // (w+1)*(h+1) points, 1 = site, 2 = point of the free side
    std::vector<int32_t> anchor;         // boundary height; INT32_MIN off the domain; INT32_MAX at sites
    std::vector<int32_t> hmax, hmin;     // extremal states (INT32_MIN off the domain)
    uint64_t sites = 0;                  // points that may move (free ones included)
    uint64_t free_sites = 0;
    int free_side = 0;                   // six-vertex: 0 none, 1 north, 2 south, 3 east, 4 west
};

// Six-vertex (Section 1.2 with the domains of Section 1.1): the model's
// vertices are the cells of a w x h mask, sites are the corners whose four
// cells lie in the domain.  Domain-wall type boundary: legs through the south
// and west sides of cells carry paths, legs through the north and east sides
// are empty; walking a boundary edge in +x the height rises by 1 if the domain
// is above it and falls by 1 if below, in +y it rises if the domain is to its
// right and falls if to its left; the lowest, then leftmost, point gets height
// (I + J) mod 2.  With a free side (free_side 1 north, 2 south, 3 east,
// 4 west) the legs through that side of cells are free: boundary points all
// of whose boundary edges are such sides move (code 2: the three neighbours
// off that side only); the remaining fixed boundary must be one piece.
RegionStatus build_sixv_region(const uint8_t *mask, int w, int h, int free_side, HeightRegion &r,
                               std::string &why);
// Free side of a domain's flags (0 none, 1..4), or -1 for an invalid set.
int free_side_of(uint32_t flags);

// Lozenges (Section 1.2's triangular lattice: Z^2 with the diagonals (1,1);
// the domains of Section 1.1): mask[(y*w + x)*2 + t] selects triangle t of unit
// square (x, y), t = 0 the lower-right {(x,y), (x+1,y), (x+1,y+1)}, t = 1 the
// upper-left {(x,y), (x,y+1), (x+1,y+1)}.  Sites are the points whose six
// triangles lie in the domain.  Thurston's heights h' = 3H + X + Y rise by 1
// along the bounding edges of a lower-right triangle walked counter-clockwise
// and fall by 2 across the edge its lozenge covers (signs flipped for
// upper-left triangles); H_max / H_min are the shortest-path bounds from the
// boundary (lengths 1 and 2), normalised so that the smallest H_min is 0.
RegionStatus build_loz_region(const uint8_t *mask, int w, int h, HeightRegion &r, std::string &why);

}  // namespace tl
