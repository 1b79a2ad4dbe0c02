"""Lozenge tilings of general domains (the simply-connected domains of Section
1.1 on the triangular lattice of Section 1.2: partial hexagons, the paper's
"weird region").

TEST INFRASTRUCTURE ONLY, like the rest of this package.

Conventions.  The triangular lattice is Z^2 with the diagonals (1,1).  Unit
square (x, y) of a w x h box holds two triangles: t = 0, the lower-right one
{(x,y), (x+1,y), (x+1,y+1)}, and t = 1, the upper-left one {(x,y), (x,y+1),
(x+1,y+1)}.  A domain is a boolean mask[y, x, t] (row 0 southmost).  Heights
H live on the (w+1) x (h+1) vertices; along (1,0), (0,1) and (1,1) they change
by 0 or -1 (the plane-partition height of the hexagon).  Canonical export:
int32 (h+1) x (w+1), INT32_MIN off the domain.

Thurston's heights: h' = 3 H + X + Y.  Walking an edge of a lower-right
triangle counter-clockwise, h' rises by 1 if the edge bounds its lozenge and
falls by 2 if the lozenge covers it; for an upper-left triangle the signs
flip.  Boundary edges always bound a lozenge, so the domain fixes h' on its
boundary (up to a constant).  Every height function obeys
h'(v) <= h'(u) + 1 across an edge u -> v with a lower-right triangle on its
left and h'(v) <= h'(u) + 2 with an upper-left one, so the largest one is the
least upper bound from the boundary, the smallest the greatest lower bound
(lengths 2 and 1 for -h'), and the domain is tileable iff both meet the
boundary heights.  Heights are normalised so that the smallest value of
H_min over the domain is 0 (the hexagon's empty box).
"""
from __future__ import annotations

import ctypes
import heapq
from collections import deque

import numpy as np

from .region import Untileable

I32MIN = np.iinfo(np.int32).min


def _tri(mask):
    m = np.asarray(mask, dtype=bool)
    if m.ndim != 3 or m.shape[2] != 2:
        raise ValueError("a lozenge domain is a (h, w, 2) mask")
    h, w = m.shape[:2]
    return m, w, h, (lambda x, y, t: 0 <= x < w and 0 <= y < h and bool(m[y, x, t]))


def _neighbours(x, y, t):
    """Triangles sharing an edge with triangle (x, y, t)."""
    if t == 0:
        return ((x, y, 1), (x, y - 1, 1), (x + 1, y, 1))
    return ((x, y, 0), (x, y + 1, 0), (x - 1, y, 0))


def _around(X, Y):
    """The six triangles at vertex (X, Y), counter-clockwise from the edge (1,0)."""
    return ((X, Y, 0), (X, Y, 1), (X - 1, Y, 0), (X - 1, Y - 1, 1), (X - 1, Y - 1, 0), (X, Y - 1, 1))


def _steps(X, Y):
    """Edges out of vertex (X, Y): (neighbour, triangle on the left, on the right)."""
    return (((X + 1, Y), (X, Y, 0), (X, Y - 1, 1)), ((X, Y + 1), (X - 1, Y, 0), (X, Y, 1)),
            ((X + 1, Y + 1), (X, Y, 1), (X, Y, 0)), ((X - 1, Y), (X - 1, Y - 1, 1), (X - 1, Y, 0)),
            ((X, Y - 1), (X, Y - 1, 1), (X - 1, Y - 1, 0)), ((X - 1, Y - 1), (X - 1, Y - 1, 0), (X - 1, Y - 1, 1)))


def check_loz_region(mask):
    """Raise ValueError unless the triangles form an accepted domain:
    non-empty, connected through edges, no vertex where the domain's
    triangles form two or more separate fans, no hole."""
    m, w, h, inside = _tri(mask)
    if not m.any():
        raise ValueError("empty domain")
    for Y in range(h + 1):
        for X in range(w + 1):
            ring = [inside(*t) for t in _around(X, Y)]
            if 0 < sum(ring) < 6 and sum(1 for i in range(6) if ring[i] and not ring[i - 1]) > 1:
                raise ValueError("domain pinched at vertex (%d, %d)" % (X, Y))

    def components(sel, W, H):
        seen = set()
        count = 0
        for y0 in range(H):
            for x0 in range(W):
                for t0 in (0, 1):
                    if not sel(x0, y0, t0) or (x0, y0, t0) in seen:
                        continue
                    count += 1
                    seen.add((x0, y0, t0))
                    q = deque([(x0, y0, t0)])
                    while q:
                        for n in _neighbours(*q.popleft()):
                            if 0 <= n[0] < W and 0 <= n[1] < H and sel(*n) and n not in seen:
                                seen.add(n)
                                q.append(n)
        return count

    if components(inside, w, h) != 1:
        raise ValueError("domain is not connected")
    outside = lambda x, y, t: not inside(x - 1, y - 1, t)   # the box grown by one square
    if components(outside, w + 2, h + 2) != 1:
        raise ValueError("domain has a hole")


def loz_points(mask):
    """(points, sites) as boolean (h+1) x (w+1) arrays: vertices of the
    domain's triangles, and vertices with all six triangles inside."""
    m, w, h, inside = _tri(mask)
    pts = np.zeros((h + 1, w + 1), dtype=bool)
    sites = np.zeros((h + 1, w + 1), dtype=bool)
    for Y in range(h + 1):
        for X in range(w + 1):
            ring = [inside(*t) for t in _around(X, Y)]
            pts[Y, X] = any(ring)
            sites[Y, X] = all(ring)
    return pts, sites


def loz_extremal_heights(mask):
    """(H_max, H_min) as int64 (h+1) x (w+1) arrays (I32MIN off the domain);
    raises Untileable."""
    m, w, h, inside = _tri(mask)
    check_loz_region(m)
    pts, sites = loz_points(m)
    order = [(X, Y) for Y in range(h + 1) for X in range(w + 1) if pts[Y, X]]
    X0, Y0 = order[0]
    hb = {(X0, Y0): X0 + Y0}
    stack = [(X0, Y0)]
    while stack:
        u = stack.pop()
        for v, left, right in _steps(*u):
            li, ri = inside(*left), inside(*right)
            if li == ri:
                continue
            # bounding edge: +1 along a lower-right triangle's counter-clockwise
            # walk, -1 along an upper-left one's
            inc = (1 if left[2] == 0 else -1) if li else (-1 if right[2] == 0 else 1)
            hv = hb[u] + inc
            if v in hb:
                if hb[v] != hv:
                    raise Untileable("boundary heights do not close up")
            else:
                hb[v] = hv
                stack.append(v)

    def bound(sign, len_lr, len_ul):
        dist = {v: sign * x for v, x in hb.items()}
        heap = [(d, v) for v, d in dist.items()]
        heapq.heapify(heap)
        while heap:
            d, u = heapq.heappop(heap)
            if d > dist[u]:
                continue
            for v, left, right in _steps(*u):
                if not (inside(*left) or inside(*right)):
                    continue
                nd = d + (len_lr if left[2] == 0 else len_ul)
                if v not in dist or nd < dist[v]:
                    dist[v] = nd
                    heapq.heappush(heap, (nd, v))
        return dist

    up, down = bound(1, 1, 2), bound(-1, 2, 1)
    for b, x in hb.items():
        if up[b] != x or down[b] != -x:
            raise Untileable("no height function meets the boundary heights")
    Hmax = np.full((h + 1, w + 1), I32MIN, dtype=np.int64)
    Hmin = np.full((h + 1, w + 1), I32MIN, dtype=np.int64)
    for (X, Y), d in up.items():
        Hmax[Y, X] = (d - X - Y) // 3
    for (X, Y), d in down.items():
        Hmin[Y, X] = (-d - X - Y) // 3
    shift = Hmin[pts].min()
    Hmax[pts] -= shift
    Hmin[pts] -= shift
    return Hmax, Hmin


def hexagon_mask(a, b, c):
    """The a x b x c hexagon as a triangle mask in its (a+c) x (b+c) box
    (X = x + c, Y = y + c): the triangles with all three vertices in it."""
    def vin(X, Y):
        x, y = X - c, Y - c
        return -c <= x <= a and -c <= y <= b and -b <= x - y <= a
    w, h = a + c, b + c
    m = np.zeros((h, w, 2), dtype=bool)
    for y in range(h):
        for x in range(w):
            m[y, x, 0] = vin(x, y) and vin(x + 1, y) and vin(x + 1, y + 1)
            m[y, x, 1] = vin(x, y) and vin(x, y + 1) and vin(x + 1, y + 1)
    return m


class LozengeRegionOracle:
    """The serial lozenge chain (same moves, draws and contexts as the
    hexagon) on a general domain."""

    def __init__(self, mask, thr, metropolis=False, seed=0, obs_every=0, bin_=1, init="min",
                 random_colours=False):
        from . import _p, lib
        self._lib, self._pp = lib, _p
        m = np.asarray(mask, dtype=bool)
        self.mask = m
        self.h_, self.w = m.shape[:2]
        self.points, sites = loz_points(m)
        self.site = np.ascontiguousarray(sites, dtype=np.uint8)
        self.Hmax, self.Hmin = loz_extremal_heights(m)
        self.H = np.ascontiguousarray(np.where(self.points, self.Hmax if init == "max" else self.Hmin, 0)
                                      .astype(np.int32))
        self.thr = np.asarray(thr, dtype=np.uint32)
        self.metropolis = metropolis
        self.random_colours = random_colours
        self.seed = seed
        self.t = 0
        self.cells = (self.h_ + 1, self.w + 1)
        self.obs_every = obs_every
        self.bin = bin_
        nbx, nby = -(-(self.w + 1) // bin_), -(-(self.h_ + 1) // bin_)
        self.bin_sum = np.zeros(nbx * nby, dtype=np.uint64)
        self.scalar_sum = np.zeros(1, dtype=np.int64)
        self.samples = np.zeros(1, dtype=np.uint64)

    def _sweep(self, n):
        p = self._pp
        self._lib().or_lozr_sweeps(self.w, self.h_, p(self.H, ctypes.c_int32), p(self.site, ctypes.c_uint8),
                                   p(self.thr, ctypes.c_uint32), int(self.metropolis), self.seed, self.t, n,
                                   int(self.random_colours))
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
        fixed = self.points & ~self.site.astype(bool)
        if H.shape != self.H.shape or not (H[fixed] == self.Hmin[fixed]).all() or \
                not (H[~self.points] == I32MIN).all():
            raise ValueError("not a height function of the domain")
        self.H[:] = np.where(self.points, H, 0).astype(np.int32)

    def flip(self, X, Y, up):
        p = self._pp
        return self._lib().or_lozr_flip(self.w, self.h_, p(self.H, ctypes.c_int32), p(self.site, ctypes.c_uint8),
                                        X, Y, int(up))

    def observe(self, bin_=None):
        """Volume H - H_min, in total and per bin of bin_ x bin_ vertices."""
        b = bin_ or self.bin
        q = np.where(self.points, self.H.astype(np.int64) - self.Hmin, 0)
        nbx, nby = -(-(self.w + 1) // b), -(-(self.h_ + 1) // b)
        bs = np.zeros(nbx * nby, dtype=np.uint64)
        ys, xs = np.nonzero(q)
        np.add.at(bs, (ys // b) * nbx + xs // b, q[ys, xs].astype(np.uint64))
        return int(q.sum()), bs

    def in_domain_cells(self):
        return self.points.copy()

    def sites(self):
        return [(X, Y) for Y in range(self.h_ + 1) for X in range(self.w + 1) if self.site[Y, X]]
