"""Domino tilings of general domains (Section 1.1): a finite, simply-connected
union of square-lattice faces, its embedding in an Aztec diamond, Thurston's
tileability test with the extremal tilings T_max and T_min, and the serial
chain on the embedded domain.

TEST INFRASTRUCTURE ONLY, like the rest of this package: the product package
never imports it, and it shares no code with the HIP path.

Conventions.  A domain is a mask of h rows by w columns (row 0 southmost);
face (x, y) belongs to it when mask[y, x] is true.  Its canonical export has
the same shape: the partner direction of each face (0 = north, 1 = south,
2 = east, 3 = west) and 0xFF outside the domain.

Embedding.  The chain runs on the Aztec diamond of order
n = ceil((w + h) / 2); the box of the domain sits at face offset (ox, oy)
with ox + oy = n and ox - oy = D, where m = floor((h - w) / 2) and D = m if
m - n is even, else m - 1.  Faces of the diamond outside the domain stay
uncovered; a 2 x 2 block of two parallel dominoes lies inside the domain, so
the rotations of Section 2.2 never reach those faces.  The draws are the
diamond's (site (r, k) of the owner grid), so the embedding fixes them.

Height function (Section 1.1, Figure "hf"): a face (X, Y) of the diamond's
box is black when X + Y is even.  Along an edge walked with a black face on
its left the height rises by 1 where the edge bounds a domino and falls by 3
where a domino covers it; with a white face on its left the signs flip.
Boundary edges always bound a domino, so the domain fixes the heights on its
boundary (up to one constant).  Every height function therefore satisfies
h(v) <= h(u) + len(u -> v) with len 1 (black on the left) or 3 (white on the
left), hence h(v) <= min over boundary vertices b of h(b) + dist(b, v).
Thurston's characterisation: the domain is tileable iff this bound agrees
with the boundary heights on the boundary, and then the bound is the height
function of T_max.  T_min is the mirror statement (lengths 3 and 1, bound
from below).  The dominoes of a height function sit on the edges where it
changes by 3.  The chain's up move (the vertical pair) raises the height at
black vertices (X + Y even) and lowers it at white ones.  The two brick
tilings of an Aztec diamond are its extremes: the vertical one is T_max for
odd orders and T_min for even orders.
"""
from __future__ import annotations

import heapq

import numpy as np
from scipy import ndimage

NORTH, SOUTH, EAST, WEST = 0, 1, 2, 3


class Untileable(ValueError):
    """The domain has no domino tiling."""


def region_embedding(w, h):
    """(n, ox, oy): order of the Aztec diamond that holds a w x h box of faces
    and the box's face offset in it (the embedding stated in the module
    docstring)."""
    n = (w + h + 1) // 2
    m = (h - w) // 2
    D = m if (m - n) % 2 == 0 else m - 1
    return n, (n + D) // 2, (n - D) // 2


def check_region(mask):
    """Raise ValueError unless the mask describes a domain the samplers
    accept: non-empty, its faces connected through edges, no vertex where
    exactly two diagonally opposite faces belong to it (a pinch), and no hole
    (the faces outside it, in the box grown by one face, connected)."""
    m = np.asarray(mask, dtype=bool)
    if m.ndim != 2 or not m.any():
        raise ValueError("empty domain")
    P = np.zeros((m.shape[0] + 2, m.shape[1] + 2), dtype=bool)
    P[1:-1, 1:-1] = m
    # the four faces around every vertex (i, j) of the grown box
    sw, se, nw, ne = P[:-1, :-1], P[:-1, 1:], P[1:, :-1], P[1:, 1:]
    pinch = (sw & ne & ~se & ~nw) | (se & nw & ~sw & ~ne)
    if pinch.any():
        j, i = np.argwhere(pinch)[0]
        raise ValueError("domain pinched at vertex (%d, %d)" % (i, j))

    def components(sel):
        # connected components through shared edges
        return ndimage.label(sel, structure=[[0, 1, 0], [1, 1, 1], [0, 1, 0]])[1]

    if components(P) != 1:
        raise ValueError("domain is not connected")
    if components(~P) != 1:
        raise ValueError("domain has a hole")


def _edge_faces(u, v):
    """(left face, right face) of the unit edge walked from vertex u to v."""
    (i, j), (i2, j2) = u, v
    if i2 == i + 1:
        return (i, j), (i, j - 1)
    if i2 == i - 1:
        return (i - 1, j - 1), (i - 1, j)
    if j2 == j + 1:
        return (i - 1, j), (i, j)
    return (i, j - 1), (i - 1, j - 1)


def extremal_heights(mask, parity=0):
    """Heights of T_max and T_min on the vertices of the domain (Thurston's
    algorithm as characterised in the module docstring).  Face (x, y) of the
    mask is black when x + y + parity is even.  Returns (hmax, hmin), dicts
    vertex -> height, both 0 at the lowest, then leftmost, vertex; raises
    Untileable."""
    m = np.asarray(mask, dtype=bool)
    h, w = m.shape
    inside = lambda f: 0 <= f[0] < w and 0 <= f[1] < h and m[f[1], f[0]]
    black = lambda f: (f[0] + f[1] + parity) % 2 == 0

    def edges(u):
        i, j = u
        for v in ((i + 1, j), (i - 1, j), (i, j + 1), (i, j - 1)):
            left, right = _edge_faces(u, v)
            a, b = inside(left), inside(right)
            if a or b:
                yield v, left, a and b

    verts = sorted({(i, j) for j in range(h + 1) for i in range(w + 1)
                    if any(True for _ in edges((i, j)))}, key=lambda p: (p[1], p[0]))
    # boundary heights: along boundary edges the height moves by +-1
    start = verts[0]
    hb = {start: 0}
    stack = [start]
    while stack:
        u = stack.pop()
        for v, left, interior in edges(u):
            if interior:
                continue
            hv = hb[u] + (1 if black(left) else -1)
            if v in hb:
                if hb[v] != hv:
                    raise Untileable("boundary heights do not close up")
            else:
                hb[v] = hv
                stack.append(v)

    def bound(len_black, len_white, sign):
        dist = {v: sign * d for v, d in hb.items()}
        heap = [(d, v) for v, d in dist.items()]
        heapq.heapify(heap)
        while heap:
            d, u = heapq.heappop(heap)
            if d > dist[u]:
                continue
            for v, left, _ in edges(u):
                nd = d + (len_black if black(left) else len_white)
                if v not in dist or nd < dist[v]:
                    dist[v] = nd
                    heapq.heappush(heap, (nd, v))
        return dist

    up = bound(1, 3, 1)         # h(v) <= h(u) + len(u -> v)
    down = bound(3, 1, -1)      # -h(v) <= -h(u) + len'(u -> v)
    for b, hv in hb.items():
        if up[b] != hv or down[b] != -hv:
            raise Untileable("no height function meets the boundary heights")
    hmax = up
    hmin = {v: -d for v, d in down.items()}
    return hmax, hmin


def tiling_from_heights(mask, heights):
    """Canonical export of the tiling whose height function is `heights`:
    the dominoes cover the interior edges where the height changes by 3."""
    m = np.asarray(mask, dtype=bool)
    h, w = m.shape
    f = np.full((h, w), 255, dtype=np.uint8)
    for y in range(h):
        for x in range(w):
            if not m[y, x]:
                continue
            # edges of the face and the neighbour across each
            sides = (((x, y + 1), (x + 1, y + 1), NORTH, (x, y + 1)),
                     ((x, y), (x + 1, y), SOUTH, (x, y - 1)),
                     ((x + 1, y), (x + 1, y + 1), EAST, (x + 1, y)),
                     ((x, y), (x, y + 1), WEST, (x - 1, y)))
            for a, b, code, (px, py) in sides:
                if abs(heights[a] - heights[b]) == 3:
                    if not (0 <= px < w and 0 <= py < h and m[py, px]) or f[y, x] != 255:
                        raise AssertionError("not the height function of a tiling")
                    f[y, x] = code
            if f[y, x] == 255:
                raise AssertionError("face (%d, %d) left uncovered" % (x, y))
    return f


def extremal_tilings(mask, parity=0):
    """(T_max, T_min) as canonical exports; raises Untileable."""
    hmax, hmin = extremal_heights(mask, parity)
    return tiling_from_heights(mask, hmax), tiling_from_heights(mask, hmin)


def square_tmin(side):
    """T_min of the side x side square (side even) in closed form, for squares
    too large for extremal_tilings.  Counting rows y from the south and
    mirroring the northern half (yy = min(y, side - 1 - y)), row y holds
    horizontal dominoes on columns yy .. side - 1 - yy and vertical dominoes
    on either side; a vertical domino at distance xx = min(x, side - 1 - x)
    from the nearer side pairs with the row towards the middle when yy - xx
    is odd and with the row away from it otherwise.  extremal_tilings is the
    definition; the tests check this form against it for every even side up
    to 16."""
    if side < 2 or side % 2:
        raise ValueError("square_tmin takes an even side")
    y, x = np.mgrid[0:side, 0:side]
    yy = np.minimum(y, side - 1 - y)
    xx = np.minimum(x, side - 1 - x)
    horiz = (x >= yy) & (x < side - yy)
    towards_middle = (yy - xx) % 2 == 1
    south = y < side // 2
    vert = np.where(towards_middle == south, NORTH, SOUTH)
    f = np.where(horiz, np.where((x - yy) % 2 == 0, EAST, WEST), vert)
    return f.astype(np.uint8)


def region_heights(faces, parity=0):
    """Height function of a tiling (canonical export of a domain), 0 at the
    lowest, then leftmost, vertex of the domain (same rule as above)."""
    f = np.asarray(faces)
    h, w = f.shape
    inside = lambda c: 0 <= c[0] < w and 0 <= c[1] < h and f[c[1], c[0]] != 255
    black = lambda c: (c[0] + c[1] + parity) % 2 == 0
    verts = sorted({(i, j) for j in range(h + 1) for i in range(w + 1)
                    if any(inside(c) for c in ((i - 1, j - 1), (i, j - 1), (i - 1, j), (i, j)))},
                   key=lambda p: (p[1], p[0]))
    out = {verts[0]: 0}
    stack = [verts[0]]
    while stack:
        u = stack.pop()
        i, j = u
        for v in ((i + 1, j), (i - 1, j), (i, j + 1), (i, j - 1)):
            left, right = _edge_faces(u, v)
            if not (inside(left) or inside(right)):
                continue
            covered = inside(left) and inside(right) and (
                (f[left[1], left[0]], (right[0] - left[0], right[1] - left[1])) in
                ((EAST, (1, 0)), (WEST, (-1, 0)), (NORTH, (0, 1)), (SOUTH, (0, -1))))
            d = 1 if black(left) else -1
            hv = out[u] + (-3 * d if covered else d)
            if v in out:
                if out[v] != hv:
                    raise AssertionError("inconsistent heights")
            else:
                out[v] = hv
                stack.append(v)
    return out


class DominoRegionOracle:
    """The serial domino chain (Section 2.2) on a general domain, run on the
    Aztec diamond the domain is embedded in (module docstring).  Same
    interface as DominoOracle, in the domain's own coordinates."""

    def __init__(self, mask, thr, metropolis=False, seed=0, obs_every=0, bin_=1, init="min",
                 random_colours=False):
        from . import DominoOracle
        m = np.asarray(mask, dtype=bool)
        check_region(m)
        self.mask = m
        self.h, self.w = m.shape
        self.n, self.ox, self.oy = region_embedding(self.w, self.h)
        self.parity = (self.ox + self.oy) % 2
        self.chain = DominoOracle(self.n, thr, metropolis=metropolis, seed=seed, random_colours=random_colours)
        # init None: no start state yet (load one); skips the extremal tilings
        if init is not None:
            self.tmax, self.tmin = extremal_tilings(m, self.parity)
            self.load(self.tmax if init == "max" else self.tmin)
        self.metropolis = metropolis
        self.seed = seed
        self.cells = (self.h, self.w)
        self.obs_every = obs_every
        self.bin = bin_
        nbx, nby = -(-self.w // bin_), -(-self.h // bin_)
        self.bin_sum = np.zeros(nbx * nby, dtype=np.uint64)
        self.scalar_sum = np.zeros(1, dtype=np.int64)
        self.samples = np.zeros(1, dtype=np.uint64)

    @property
    def t(self):
        return self.chain.t

    @t.setter
    def t(self, v):
        self.chain.t = v

    @property
    def thr(self):
        return self.chain.thr

    def sweep(self, nsweeps):
        if not self.obs_every:
            self.chain.sweep(nsweeps)
            return
        for _ in range(nsweeps):
            t = self.chain.t
            self.chain.sweep(1)
            if (t + 1) % self.obs_every == 0:
                v, bs = self.observe()
                self.bin_sum += bs
                self.scalar_sum += v
                self.samples += 1

    def export(self):
        return self.chain.export()[self.oy:self.oy + self.h, self.ox:self.ox + self.w].copy()

    def load(self, faces):
        f = np.ascontiguousarray(faces, dtype=np.uint8)
        if f.shape != self.mask.shape or not np.array_equal(f != 255, self.mask):
            raise ValueError("not a domino tiling of the domain")
        n = self.n
        full = np.full((2 * n, 2 * n), 255, dtype=np.uint8)
        full[self.oy:self.oy + self.h, self.ox:self.ox + self.w] = f
        self.chain.load(full, allow_uncovered=True)

    def observe(self, bin_=None):
        """Faces covered by horizontal dominoes, in total and per bin of
        bin_ x bin_ faces of the domain's box."""
        b = bin_ or self.bin
        f = self.export()
        horiz = (f == EAST) | (f == WEST)
        nbx, nby = -(-self.w // b), -(-self.h // b)
        bs = np.zeros(nbx * nby, dtype=np.uint64)
        ys, xs = np.nonzero(horiz)
        np.add.at(bs, (ys // b) * nbx + xs // b, 1)
        return int(horiz.sum()), bs

    def in_domain_cells(self):
        return self.mask.copy()

    def flip(self, x, y, up):
        return self.chain.flip(x + self.ox, y + self.oy, up)

    def sites(self):
        """Vertices of the domain with all four faces in it (the rotation
        sites), in the domain's coordinates."""
        m = self.mask
        return [(i, j) for j in range(1, self.h) for i in range(1, self.w)
                if m[j - 1, i - 1] and m[j - 1, i] and m[j, i - 1] and m[j, i]]
