"""The six-vertex model on general domains (Section 1.2 with the domains of
Section 1.1; the paper's L-shaped example has "domain-wall type" boundary
conditions).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

Conventions.  A domain is a mask of h rows by w cells (row 0 southmost);
cell (x, y) is a vertex of the six-vertex model when mask[y, x] is true.
Heights live on the corner points (I, J), 0 <= I <= w, 0 <= J <= h, of the
cells; the points of the domain are the corners of its cells, its sites the
points whose four cells all belong to it.  The canonical export is the
(h+1) x (w+1) array of heights, INT32_MIN off the domain.

Domain-wall type boundary: every leg (an edge of the model leaving the
domain) through the south or west side of a cell carries a path, every leg
through the north or east side is empty.  With the height rule of Figure
"sixvertexh" (crossing an occupied edge in +x or +y adds 1, an empty one
subtracts 1) the heights along the boundary follow: walking a boundary edge
in +x adds 1 if the domain lies above it (the south side of a cell) and
subtracts 1 if below; walking one in +y adds 1 if the domain lies to its
right (a west side) and subtracts 1 if to its left.  They are fixed up to one
constant, chosen so that the lowest, then leftmost, point has height
(I + J) mod 2 (the domain-wall square gets h(0, 0) = 0).  Heights of
neighbouring points differ by exactly 1, so the configurations are the
integer functions that are 1-Lipschitz along the edges of the domain, agree
with the boundary, and have the parity of I + J; the largest is
min over boundary points b of h(b) + dist(b, v), the smallest
max_b h(b) - dist(b, v), and a configuration exists iff both agree with the
boundary heights on the boundary.  On the N x N square these are the
domain-wall boundary, N - |I + J - N| and |I - J|.
"""
from __future__ import annotations

import ctypes
import heapq

import numpy as np

from .region import Untileable, check_region

I32MIN = np.iinfo(np.int32).min


def _cells(mask):
    m = np.asarray(mask, dtype=bool)
    h, w = m.shape
    return m, w, h, (lambda x, y: 0 <= x < w and 0 <= y < h and bool(m[y, x]))


def sixv_points(mask):
    """(points, sites): the corner points of the domain's cells and the
    points with all four cells in the domain, as boolean (h+1) x (w+1) arrays."""
    m = np.asarray(mask, dtype=bool)
    h, w = m.shape
    P = np.zeros((h + 2, w + 2), dtype=bool)
    P[1:-1, 1:-1] = m
    sw, se, nw, ne = P[:-1, :-1], P[:-1, 1:], P[1:, :-1], P[1:, 1:]
    return sw | se | nw | ne, sw & se & nw & ne


def _edges(inside, I, J):
    """Edges out of point (I, J) along cell sides of the domain: (neighbour,
    number of domain cells beside the edge, boundary increment of the walk)."""
    # +x: cells above (I, J) and below (I, J-1)
    for (I2, J2), a, b, sign in (((I + 1, J), (I, J), (I, J - 1), 1), ((I - 1, J), (I - 1, J), (I - 1, J - 1), -1)):
        ia, ib = inside(*a), inside(*b)
        if ia or ib:
            yield (I2, J2), ia + ib, sign * (1 if ia else -1)
    # +y: cells right (I, J) and left (I-1, J)
    for (I2, J2), r, l, sign in (((I, J + 1), (I, J), (I - 1, J), 1), ((I, J - 1), (I, J - 1), (I - 1, J - 1), -1)):
        ir, il = inside(*r), inside(*l)
        if ir or il:
            yield (I2, J2), ir + il, sign * (1 if ir else -1)


def _free_edge(inside, u, v, side="north"):
    """Is the boundary edge u-v the `side` side (north, south, east or west)
    of a domain cell?"""
    (I, J), (I2, J2) = u, v
    if side in ("north", "south"):
        if J != J2:
            return False
        below, above = inside(min(I, I2), J - 1), inside(min(I, I2), J)
        return (below and not above) if side == "north" else (above and not below)
    if I != I2:
        return False
    left, right = inside(I - 1, min(J, J2)), inside(I, min(J, J2))
    return (left and not right) if side == "east" else (right and not left)


def _side(free_north, free_side):
    if free_side is not None and free_side not in ("north", "south", "east", "west"):
        raise ValueError("unknown free side %r" % (free_side,))
    return free_side or ("north" if free_north else None)


def sixv_boundary_heights(mask, free_north=False, free_side=None):
    """Heights of the fixed boundary points under the domain-wall type
    boundary; raises Untileable if the walk around the boundary does not close
    up.  With a free side (free_side one of north, south, east, west;
    free_north for north) the legs through those sides of cells are free:
    those boundary edges are not walked, and the points whose boundary edges
    are all such edges are free (absent from the result)."""
    side = _side(free_north, free_side)
    m, w, h, inside = _cells(mask)
    pts, sites = sixv_points(m)
    order = [(I, J) for J in range(h + 1) for I in range(w + 1) if pts[J, I]]
    I0, J0 = order[0]
    hb = {(I0, J0): (I0 + J0) % 2}
    stack = [(I0, J0)]
    while stack:
        u = stack.pop()
        for v, ncells, dh in _edges(inside, *u):
            if ncells != 1 or (side and _free_edge(inside, u, v, side)):
                continue
            hv = hb[u] + dh
            if v in hb:
                if hb[v] != hv:
                    raise Untileable("boundary heights do not close up")
            else:
                hb[v] = hv
                stack.append(v)
    return hb


def sixv_free_points(mask, side="north"):
    """Points whose boundary edges are all `side` sides of domain cells."""
    m, w, h, inside = _cells(mask)
    pts, sites = sixv_points(m)
    free = np.zeros_like(pts)
    for J in range(h + 1):
        for I in range(w + 1):
            if not pts[J, I] or sites[J, I]:
                continue
            bnd = [(v, ncells) for v, ncells, _ in _edges(inside, I, J) if ncells == 1]
            free[J, I] = all(_free_edge(inside, (I, J), v, side) for v, _ in bnd)
    return free


def sixv_extremal_heights(mask, free_north=False, free_side=None):
    """(h_max, h_min) as (h+1) x (w+1) int64 arrays (I32MIN off the domain);
    raises Untileable when no configuration meets the boundary, ValueError
    when free edges split the fixed boundary into several pieces."""
    side = _side(free_north, free_side)
    m, w, h, inside = _cells(mask)
    check_region(m)
    pts, sites = sixv_points(m)
    hb = sixv_boundary_heights(m, free_side=side)
    free = sixv_free_points(m, side) if side else np.zeros_like(pts)
    if any(not sites[J, I] and not free[J, I] for J in range(h + 1) for I in range(w + 1)
           if pts[J, I] and (I, J) not in hb):
        raise ValueError("the fixed boundary is not one piece")

    def bound(sign):
        dist = {v: sign * x for v, x in hb.items()}
        heap = [(d, v) for v, d in dist.items()]
        heapq.heapify(heap)
        while heap:
            d, u = heapq.heappop(heap)
            if d > dist[u]:
                continue
            for v, _, _ in _edges(inside, *u):
                if v not in dist or d + 1 < dist[v]:
                    dist[v] = d + 1
                    heapq.heappush(heap, (d + 1, v))
        return dist

    up, down = bound(1), bound(-1)
    for b, x in hb.items():
        if up[b] != x or down[b] != -x:
            raise Untileable("no configuration meets the boundary heights")
    hmax = np.full((h + 1, w + 1), I32MIN, dtype=np.int64)
    hmin = np.full((h + 1, w + 1), I32MIN, dtype=np.int64)
    for (I, J), d in up.items():
        hmax[J, I] = d
    for (I, J), d in down.items():
        hmin[J, I] = -d
    return hmax, hmin


def sixv_c_vertices(mask, heights):
    """Cells of type c (both diagonal pairs of corner heights equal)."""
    m = np.asarray(mask, dtype=bool)
    H = np.asarray(heights)
    isc = (H[:-1, :-1] == H[1:, 1:]) & (H[:-1, 1:] == H[1:, :-1])
    return isc & m


class SixVertexRegionOracle:
    """The serial six-vertex chain (same moves, draws and contexts as the
    domain-wall square) on a general domain with domain-wall type boundary."""

    def __init__(self, mask, thr, metropolis=False, seed=0, obs_every=0, bin_=1, init="min",
                 random_colours=False, free_north=False, thr_free=None, free_side=None):
        from . import _p, lib
        self._lib, self._pp = lib, _p
        m = np.asarray(mask, dtype=bool)
        self.mask = m
        self.h_, self.w = m.shape
        pts, sites = sixv_points(m)
        self.points = pts
        side = _side(free_north, free_side)
        self.free = sixv_free_points(m, side) if side else np.zeros_like(pts)
        # site codes: 1 interior, 2 on the free side; the side's code for the
        # C step, and the offsets of the draws (two rows / columns for a free
        # south / west side, whose points then sit inside the model's box)
        self.site = np.ascontiguousarray(sites.astype(np.uint8) + 2 * self.free.astype(np.uint8))
        self.side_code = {None: 0, "north": 1, "south": 2, "east": 3, "west": 4}[side]
        self.ox = 2 if side == "west" else 0
        self.oy = 2 if side == "south" else 0
        self.thr_free = np.asarray(thr_free if thr_free is not None else [0] * 8, dtype=np.uint32)
        self.hmax, self.hmin = sixv_extremal_heights(m, free_side=side)
        self.H = np.ascontiguousarray((self.hmax if init == "max" else self.hmin).astype(np.int32))
        self.thr = np.asarray(thr, dtype=np.uint32)
        self.metropolis = metropolis
        self.random_colours = random_colours
        self.seed = seed
        self.t = 0
        self.cells = (self.h_, self.w)
        self.obs_every = obs_every
        self.bin = bin_
        nbx, nby = -(-self.w // bin_), -(-self.h_ // bin_)
        self.bin_sum = np.zeros(nbx * nby, dtype=np.uint64)
        self.scalar_sum = np.zeros(1, dtype=np.int64)
        self.samples = np.zeros(1, dtype=np.uint64)

    def _sweep(self, n):
        p = self._pp
        self._lib().or_sixvr_sweeps(self.w, self.h_, p(self.H, ctypes.c_int32), p(self.site, ctypes.c_uint8),
                                    p(self.thr, ctypes.c_uint32), p(self.thr_free, ctypes.c_uint32),
                                    int(self.metropolis), self.seed, self.t, n, int(self.random_colours),
                                    self.side_code, self.ox, self.oy)
        self.t += n

    def sweep(self, nsweeps):
        if not self.obs_every:
            self._sweep(nsweeps)
            return
        for _ in range(nsweeps):
            t = self.t
            self._sweep(1)
            if (t + 1) % self.obs_every == 0:
                v, bs = self.observe()
                self.bin_sum += bs
                self.scalar_sum += v
                self.samples += 1

    def export(self):
        out = self.H.copy()
        out[~self.points] = I32MIN
        return out

    def load(self, H):
        H = np.asarray(H, dtype=np.int64)
        if H.shape != self.H.shape:
            raise ValueError("wrong shape")
        fixed = self.points & (self.site == 0)
        if not (H[fixed] == self.hmin[fixed]).all() or not (H[~self.points] == I32MIN).all():
            raise ValueError("boundary heights differ")
        self.H[:] = np.where(self.points, H, 0).astype(np.int32)

    def flip(self, I, J, up):
        p = self._pp
        return self._lib().or_sixvr_flip(self.w, self.h_, p(self.H, ctypes.c_int32), p(self.site, ctypes.c_uint8),
                                         self.side_code, I, J, int(up))

    def observe(self, bin_=None):
        """Type-c cells, in total and per bin of bin_ x bin_ cells."""
        b = bin_ or self.bin
        c = sixv_c_vertices(self.mask, self.H)
        nbx, nby = -(-self.w // b), -(-self.h_ // b)
        bs = np.zeros(nbx * nby, dtype=np.uint64)
        ys, xs = np.nonzero(c)
        np.add.at(bs, (ys // b) * nbx + xs // b, 1)
        return int(c.sum()), bs

    def in_domain_cells(self):
        return self.mask.copy()

    def sites(self):
        """Points that may flip (interior sites and free-edge points)."""
        return [(I, J) for J in range(self.h_ + 1) for I in range(self.w + 1) if self.site[J, I]]
