"""Serial CPU oracle for the parallel Glauber sweep (arXiv:1804.07250).

TEST INFRASTRUCTURE ONLY: the product package never imports this module.  Only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code with the HIP path.

Parts:
  * ``liboracle.so`` (plain C, built with gcc from the ``*.c`` files here): the
    Philox4x32-10 generator, the per-site uniform and one serial chain per model
    (domino: the paper's T_b / T_w tilestate arrays with Rotate + Update of
    Section 2.2; lozenge and six-vertex: full int32 heights, Section 1.2);
  * exact threshold tables (``fractions.Fraction``): T = floor(2^32 p) with
    p = W_up / (W_up + W_down) (heat-bath) or the lazy Metropolis pair, from the
    weights of Section 1.1.1 (edge and volume weights) and Section 1.2 (vertex
    weights a, b, c);
  * the canonical hash (row digests, then one digest over them).
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = ["philox.c", "domino.c", "lozenge.c", "sixvertex.c", "sixvertex_region.c", "lozenge_region.c"]
TWO32 = 1 << 32


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, serial, no OpenMP)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-o", tmp] + srcs)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i32p = ctypes.POINTER(ctypes.c_int32)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.or_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.or_site_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_uint32, ctypes.c_uint32]
        L.or_site_uniform.restype = ctypes.c_uint32
        L.or_set_reverse_order.argtypes = [ctypes.c_int]
        L.or_domino_array_len.argtypes = [ctypes.c_int]
        L.or_domino_vertex_state.argtypes = [ctypes.c_int, u8p, u8p, ctypes.c_int, ctypes.c_int]
        L.or_domino_brick.argtypes = [ctypes.c_int, u8p, u8p]
        L.or_domino_from_faces.argtypes = [ctypes.c_int, u8p, u8p, u8p, ctypes.c_int]
        L.or_domino_to_faces.argtypes = [ctypes.c_int, u8p, u8p, u8p]
        L.or_domino_flip.argtypes = [ctypes.c_int, u8p, u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.or_domino_sweeps.argtypes = [ctypes.c_int, u8p, u8p, u32p, ctypes.c_int, ctypes.c_uint64,
                                       ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p]
        L.or_domino_observe.argtypes = [ctypes.c_int, u8p, u8p, ctypes.c_uint32, ctypes.c_void_p]
        L.or_domino_observe.restype = ctypes.c_int64
        L.or_lozenge_min.argtypes = [ctypes.c_int] * 3 + [i32p]
        L.or_lozenge_max.argtypes = [ctypes.c_int] * 3 + [i32p]
        L.or_lozenge_flip.argtypes = [ctypes.c_int] * 3 + [i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.or_lozenge_sweeps.argtypes = [ctypes.c_int] * 3 + [i32p, u32p, ctypes.c_int, ctypes.c_uint64,
                                                             ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                                             ctypes.c_void_p]
        L.or_lozenge_observe.argtypes = [ctypes.c_int] * 3 + [i32p, ctypes.c_uint32, ctypes.c_void_p]
        L.or_lozenge_observe.restype = ctypes.c_int64
        L.or_sixv_min.argtypes = [ctypes.c_int, i32p]
        L.or_sixv_max.argtypes = [ctypes.c_int, i32p]
        L.or_sixv_flip.argtypes = [ctypes.c_int, i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.or_sixv_sweeps.argtypes = [ctypes.c_int, i32p, u32p, ctypes.c_int, ctypes.c_uint64,
                                     ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p]
        L.or_sixvr_flip.argtypes = [ctypes.c_int, ctypes.c_int, i32p, u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int]
        L.or_sixvr_sweeps.argtypes = [ctypes.c_int, ctypes.c_int, i32p, u8p, u32p, u32p, ctypes.c_int,
                                      ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int]
        L.or_lozr_flip.argtypes = [ctypes.c_int, ctypes.c_int, i32p, u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.or_lozr_sweeps.argtypes = [ctypes.c_int, ctypes.c_int, i32p, u8p, u32p, ctypes.c_int, ctypes.c_uint64,
                                     ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int]
        L.or_step_colour.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
        L.or_step_colour.restype = ctypes.c_uint32
        L.or_sixv_observe.argtypes = [ctypes.c_int, i32p, ctypes.c_uint32, ctypes.c_void_p]
        L.or_sixv_observe.restype = ctypes.c_int64
        _lib = L
    return _lib


def _p(arr, ctype):
    return arr.ctypes.data_as(ctypes.POINTER(ctype))


class _Obs(ctypes.Structure):
    _fields_ = [("obs_every", ctypes.c_uint32), ("bin", ctypes.c_uint32),
                ("bin_sum", ctypes.POINTER(ctypes.c_uint64)),
                ("scalar_sum", ctypes.POINTER(ctypes.c_int64)),
                ("samples", ctypes.POINTER(ctypes.c_uint64))]


# --------------------------------------------------------------------------- RNG

def philox4x32_10(ctr, key):
    """Philox4x32-10 (Salmon et al., SC'11) of a 4-word counter and 2-word key."""
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32), _p(out, ctypes.c_uint32))
    return [int(v) for v in out]


def set_reverse_order(rev: bool):
    lib().or_set_reverse_order(int(rev))


def site_uniform(seed, r, k, t, c):
    return int(lib().or_site_uniform(seed, r, k, t, c))


def step_colour(seed, step, K):
    """Colour of colour step `step` under the random colour order."""
    return int(lib().or_step_colour(seed, step, K))


# --------------------------------------------------------------------- thresholds

def _floor32(p: Fraction) -> int:
    v = (p.numerator * TWO32) // p.denominator
    if not 0 <= v < TWO32:
        raise ValueError("threshold out of range")
    return v


def table_from_ratios(ratios, metropolis: bool):
    """Thresholds from exact up/down weight ratios R per context.

    heat-bath:        T = floor(2^32 R / (1 + R))            (new state up iff u < T)
    lazy Metropolis:  current down: T = floor(2^32 min(1, R) / 2)
                      current up:   T = 2^32 - floor(2^32 min(1, 1/R) / 2)
                      laid out as [ctx*2 + current_is_up].
    """
    out = []
    for R in ratios:
        R = Fraction(R)
        if R <= 0:
            raise ValueError("weights must be positive")
        if not metropolis:
            out.append(_floor32(R / (1 + R)))
        else:
            out.append(_floor32(min(Fraction(1), R) / 2))
            f = _floor32(min(Fraction(1), 1 / R) / 2)
            if f == 0:   # 2^32 does not fit a 32-bit table
                raise ValueError("threshold out of range")
            out.append(TWO32 - f)
    return out


def domino_ratios(kind="uniform", a=1, b=1):
    """Up (vertical pair) / down (horizontal pair) weight ratio per context
    2c + (x mod 2).  Two-periodic edge weights: a crossed edge weighs a when its
    even (x+y even) endpoint has x even, b otherwise.  At an even vertex all four
    of its edges share one weight (ratio 1); at an odd vertex with x even the
    vertical pair crosses its E/W edges (even endpoints at odd x: weight b) and
    the horizontal pair its N/S edges (weight a), so R = b^2/a^2; x odd: a^2/b^2."""
    if kind == "uniform":
        return [Fraction(1)] * 4
    a, b = Fraction(a), Fraction(b)
    if kind == "volume":
        # Volume weights prod_v q_v^h(v) (Section 1.1.1), q = a at black (x+y
        # even) vertices and b at white ones.  A rotation moves the height of
        # its vertex by 4; the vertical pair is the higher state at black
        # vertices and the lower one at white vertices, so R = a^4 at black
        # sites and b^-4 at white sites.
        return [a ** 4, a ** 4, b ** -4, b ** -4]
    return [Fraction(1), Fraction(1), (b * b) / (a * a), (a * a) / (b * b)]


def lozenge_ratios(q):
    """Volume weight q^volume: adding one cube multiplies the weight by q."""
    return [Fraction(q)]


def sixv_ratios(a, b, c_squared):
    """W_up / W_down for each mask of diagonal faces at height m+1 (NE=1, NW=2,
    SW=4, SE=8).  Corners NE and SW carry a, NW and SE carry b when not of type
    c; a corner whose diagonal face is high is of type c in the up state only.
    Only c^2 enters because exactly four corners change."""
    a, b, c2 = Fraction(a), Fraction(b), Fraction(c_squared)
    wts = [a, b, a, b]  # NE, NW, SW, SE
    out = []
    for mask in range(16):
        R = Fraction(1)
        nhigh = 0
        for bit, w in enumerate(wts):
            if mask >> bit & 1:
                R /= w
                nhigh += 1
            else:
                R *= w
        # c^(nhigh - (4 - nhigh)) = (c^2)^(nhigh - 2)
        e = nhigh - 2
        R *= c2 ** e
        out.append(R)
    return out


def sixv_vertex_type(hSW, hSE, hNW, hNE):
    """Type of the vertex surrounded by four faces of these heights (Section
    1.2, Figure "sixvertexh": a path crosses an edge where the height rises by
    1 towards +x or +y).  a1: no path edge, a2: all four, b1: left and right,
    b2: bottom and top, c1: bottom and left, c2: right and top."""
    bottom, top = hSE - hSW == 1, hNE - hNW == 1
    left, right = hNW - hSW == 1, hNE - hSE == 1
    return {(False, False, False, False): "a1", (True, True, True, True): "a2",
            (True, True, False, False): "b1", (False, False, True, True): "b2",
            (True, False, True, False): "c1", (False, True, False, True): "c2"}[(left, right, bottom, top)]


def sixv_ratios6(a1, a2, b1, b2, c1, c2):
    """W_up / W_down for each mask of diagonal faces at height m+1 (NE=1, NW=2,
    SW=4, SE=8) with the six vertex weights of Section 1.2: the flipped face at
    m-1 or m+1, its four edge neighbours at m, the diagonal faces at m+1 or
    m-1 by the mask; the weight of each state is the product over the four
    corners of the flipped face of the weight of the corner's type."""
    w = {"a1": Fraction(a1), "a2": Fraction(a2), "b1": Fraction(b1), "b2": Fraction(b2),
         "c1": Fraction(c1), "c2": Fraction(c2)}
    out = []
    for mask in range(16):
        m = 10

        def weight(f):
            diag = {(1, 1): 0, (-1, 1): 1, (-1, -1): 2, (1, -1): 3}
            h = {(0, 0): f, (1, 0): m, (-1, 0): m, (0, 1): m, (0, -1): m}
            for pos, bit in diag.items():
                h[pos] = m + 1 if mask >> bit & 1 else m - 1
            W = Fraction(1)
            for cx, cy in ((0, 0), (-1, 0), (-1, -1), (0, -1)):   # corners NE, NW, SW, SE
                W *= w[sixv_vertex_type(h[(cx, cy)], h[(cx + 1, cy)], h[(cx, cy + 1)], h[(cx + 1, cy + 1)])]
            return W

        out.append(weight(m + 1) / weight(m - 1))
    return out


# Free sides of a six-vertex domain: the point's missing neighbour, its three
# neighbours and the two diagonal points of its context (first, second), as
# offsets (dI, dJ) from the point.
FREE_SIDES = {
    "north": {"missing": (0, 1), "diag": ((-1, -1), (1, -1))},
    "south": {"missing": (0, -1), "diag": ((-1, 1), (1, 1))},
    "east": {"missing": (1, 0), "diag": ((-1, -1), (-1, 1))},
    "west": {"missing": (-1, 0), "diag": ((1, -1), (1, 1))},
}


def sixv_free_ratios6(a1, a2, b1, b2, c1, c2, side="north"):
    """W_up / W_down of a flip at a point of a free side (the boundary
    variation of the c-flip, Section 1.2), for each context (first diagonal
    at m+1) + 2 (second diagonal at m+1): the point at m-1 or m+1, its three
    neighbours at m, its two diagonal points on the domain's side at m+1 or
    m-1; the weight of a state is the product over the two cells the point
    touches (the cells beside its three neighbours' edges) of the weight of
    the cell's type."""
    w = {"a1": Fraction(a1), "a2": Fraction(a2), "b1": Fraction(b1), "b2": Fraction(b2),
         "c1": Fraction(c1), "c2": Fraction(c2)}
    miss = FREE_SIDES[side]["missing"]
    d0, d1 = FREE_SIDES[side]["diag"]
    out = []
    for ctx in range(4):
        m = 10
        h = {(1, 0): m, (-1, 0): m, (0, 1): m, (0, -1): m}
        del h[miss]
        h[d0] = m + 1 if ctx & 1 else m - 1
        h[d1] = m + 1 if ctx & 2 else m - 1

        def weight(f):
            hh = dict(h)
            hh[(0, 0)] = f
            W = Fraction(1)
            # the cells with the point as a corner whose four corners are all known
            for cx, cy in ((0, 0), (-1, 0), (-1, -1), (0, -1)):
                corners = [(cx, cy), (cx + 1, cy), (cx, cy + 1), (cx + 1, cy + 1)]
                if all(c in hh for c in corners):
                    W *= w[sixv_vertex_type(*[hh[c] for c in corners])]
            return W

        out.append(weight(m + 1) / weight(m - 1))
    return out


# --------------------------------------------------------------------- hashing

def canonical_hash(arr2d: np.ndarray) -> str:
    """SHA-256 over the concatenated SHA-256 digests of the rows of the
    canonical export (little-endian bytes)."""
    a = np.ascontiguousarray(arr2d)
    h = hashlib.sha256()
    for row in a:
        h.update(hashlib.sha256(row.tobytes()).digest())
    return h.hexdigest()


# ----------------------------------------------------------------------- models

class _Chain:
    """random_colours: the paper's random colour choice per step (or_step_colour)
    instead of the fixed order 0 .. K-1 within a sweep."""
    metropolis = False
    random_colours = False

    def _obs(self, obs_every, bin_, nbins):
        self.bin_sum = np.zeros(nbins, dtype=np.uint64)
        self.scalar_sum = np.zeros(1, dtype=np.int64)
        self.samples = np.zeros(1, dtype=np.uint64)
        self.obs_every = obs_every
        self.bin = bin_
        self._o = _Obs(obs_every, bin_, _p(self.bin_sum, ctypes.c_uint64),
                       _p(self.scalar_sum, ctypes.c_int64), _p(self.samples, ctypes.c_uint64))


class DominoOracle(_Chain):
    """Aztec diamond of order n; state = the paper's split tilestate arrays."""

    def __init__(self, n, thr, metropolis=False, seed=0, obs_every=0, bin_=1, init="min", random_colours=False):
        self.n = n
        self.random_colours = random_colours
        L = lib()
        m = L.or_domino_array_len(n)
        self.Tb = np.zeros(m, dtype=np.uint8)
        self.Tw = np.zeros(m, dtype=np.uint8)
        L.or_domino_brick(n, _p(self.Tb, ctypes.c_uint8), _p(self.Tw, ctypes.c_uint8))
        if init == "max":
            self.load(domino_vertical_brick(self.export()))
        self.thr = np.asarray(thr, dtype=np.uint32)
        self.metropolis = metropolis
        self.seed = seed
        self.t = 0
        self.cells = (2 * n, 2 * n)
        nb = -(-2 * n // bin_)
        self._obs(obs_every, bin_, nb * nb)

    def sweep(self, nsweeps):
        lib().or_domino_sweeps(self.n, _p(self.Tb, ctypes.c_uint8), _p(self.Tw, ctypes.c_uint8),
                               _p(self.thr, ctypes.c_uint32), int(self.metropolis), self.seed,
                               self.t, nsweeps, int(self.random_colours), ctypes.byref(self._o))
        self.t += nsweeps

    def export(self):
        f = np.zeros((2 * self.n, 2 * self.n), dtype=np.uint8)
        lib().or_domino_to_faces(self.n, _p(self.Tb, ctypes.c_uint8), _p(self.Tw, ctypes.c_uint8),
                                 _p(f, ctypes.c_uint8))
        return f

    def load(self, faces, allow_uncovered=False):
        """Load a canonical export; with allow_uncovered, faces of the diamond
        marked 0xFF stay uncovered (a tiling of a region inside the diamond)."""
        f = np.ascontiguousarray(faces, dtype=np.uint8)
        rc = lib().or_domino_from_faces(self.n, _p(f, ctypes.c_uint8), _p(self.Tb, ctypes.c_uint8),
                                        _p(self.Tw, ctypes.c_uint8), int(allow_uncovered))
        if rc != 0:
            raise ValueError("not a domino tiling of the Aztec diamond")

    def vertex_state(self, X, Y):
        return int(lib().or_domino_vertex_state(self.n, _p(self.Tb, ctypes.c_uint8),
                                                _p(self.Tw, ctypes.c_uint8), X, Y))

    def flip(self, X, Y, up):
        return lib().or_domino_flip(self.n, _p(self.Tb, ctypes.c_uint8), _p(self.Tw, ctypes.c_uint8),
                                    X, Y, int(up))

    def observe(self, bin_=None):
        b = bin_ or self.bin
        nb = -(-2 * self.n // b)
        bs = np.zeros(nb * nb, dtype=np.uint64)
        v = lib().or_domino_observe(self.n, _p(self.Tb, ctypes.c_uint8), _p(self.Tw, ctypes.c_uint8),
                                    b, bs.ctypes.data)
        return int(v), bs

    def in_domain_cells(self):
        n = self.n
        Y, X = np.mgrid[0:2 * n, 0:2 * n]
        return (np.abs(2 * X - 2 * n + 1) + np.abs(2 * Y - 2 * n + 1) <= 2 * n)

    def sites(self):
        """Box vertices (X, Y) that are interior (the rotation sites)."""
        n = self.n
        return [(X, Y) for Y in range(2 * n + 1) for X in range(2 * n + 1)
                if abs(X - n) + abs(Y - n) <= n - 1]


class LozengeOracle(_Chain):
    def __init__(self, a, b, c, thr, metropolis=False, seed=0, obs_every=0, bin_=1, init="min",
                 random_colours=False):
        self.a, self.b, self.c = a, b, c
        self.random_colours = random_colours
        self.W, self.H = a + c + 1, b + c + 1
        self.Hs = np.zeros(self.W * self.H, dtype=np.int32)
        f = lib().or_lozenge_min if init == "min" else lib().or_lozenge_max
        f(a, b, c, _p(self.Hs, ctypes.c_int32))
        self.thr = np.asarray(thr, dtype=np.uint32)
        self.metropolis = metropolis
        self.seed = seed
        self.t = 0
        self.cells = (self.H, self.W)
        self._obs(obs_every, bin_, (-(-self.W // bin_)) * (-(-self.H // bin_)))

    def sweep(self, nsweeps):
        lib().or_lozenge_sweeps(self.a, self.b, self.c, _p(self.Hs, ctypes.c_int32),
                                _p(self.thr, ctypes.c_uint32), int(self.metropolis), self.seed,
                                self.t, nsweeps, int(self.random_colours), ctypes.byref(self._o))
        self.t += nsweeps

    def export(self):
        return self.Hs.reshape(self.H, self.W).copy()

    def load(self, Hs):
        self.Hs[:] = np.asarray(Hs, dtype=np.int32).reshape(-1)

    def flip(self, X, Y, up):
        return lib().or_lozenge_flip(self.a, self.b, self.c, _p(self.Hs, ctypes.c_int32), X, Y, int(up))

    def observe(self, bin_=None):
        b = bin_ or self.bin
        bs = np.zeros((-(-self.W // b)) * (-(-self.H // b)), dtype=np.uint64)
        v = lib().or_lozenge_observe(self.a, self.b, self.c, _p(self.Hs, ctypes.c_int32), b,
                                     bs.ctypes.data)
        return int(v), bs

    def in_domain_cells(self):
        return self.export() != np.iinfo(np.int32).min

    def sites(self):
        a, b, c = self.a, self.b, self.c
        out = []
        for Y in range(self.H):
            for X in range(self.W):
                x, y = X - c, Y - c
                if -c < x < a and -c < y < b and -b < x - y < a:
                    out.append((X, Y))
        return out


class SixVertexOracle(_Chain):
    def __init__(self, N, thr, metropolis=False, seed=0, obs_every=0, bin_=1, init="min", random_colours=False):
        self.N = N
        self.random_colours = random_colours
        self.h = np.zeros((N + 1) * (N + 1), dtype=np.int32)
        f = lib().or_sixv_min if init == "min" else lib().or_sixv_max
        f(N, _p(self.h, ctypes.c_int32))
        self.thr = np.asarray(thr, dtype=np.uint32)
        self.metropolis = metropolis
        self.seed = seed
        self.t = 0
        self.cells = (N, N)
        self._obs(obs_every, bin_, (-(-N // bin_)) ** 2)

    def sweep(self, nsweeps):
        lib().or_sixv_sweeps(self.N, _p(self.h, ctypes.c_int32), _p(self.thr, ctypes.c_uint32),
                             int(self.metropolis), self.seed, self.t, nsweeps, int(self.random_colours),
                             ctypes.byref(self._o))
        self.t += nsweeps

    def export(self):
        return self.h.reshape(self.N + 1, self.N + 1).copy()

    def load(self, h):
        self.h[:] = np.asarray(h, dtype=np.int32).reshape(-1)

    def flip(self, I, J, up):
        return lib().or_sixv_flip(self.N, _p(self.h, ctypes.c_int32), I, J, int(up))

    def observe(self, bin_=None):
        b = bin_ or self.bin
        bs = np.zeros((-(-self.N // b)) ** 2, dtype=np.uint64)
        v = lib().or_sixv_observe(self.N, _p(self.h, ctypes.c_int32), b, bs.ctypes.data)
        return int(v), bs

    def in_domain_cells(self):
        return np.ones((self.N, self.N), dtype=bool)

    def sites(self):
        return [(I, J) for J in range(1, self.N) for I in range(1, self.N)]


def domino_vertical_brick(horizontal):
    """The all-vertical tiling of an Aztec diamond from the all-horizontal one
    (canonical export, row 0 southmost): the mirror image in the diagonal X = Y,
    under which a partner to the east (+X) becomes one to the north (+Y),
    west -> south, north -> east and south -> west.  The two brick tilings are
    the extremal tilings of Section 1.1.4: every rotation available from either
    one moves the height function the same way."""
    remap = np.array([2, 3, 0, 1] + [255] * 252, dtype=np.uint8)
    return remap[np.ascontiguousarray(horizontal.T)]


def cftp_segments(R):
    """Sweeps from time -2^R to time 0 as (first sweep counter, count), in
    time order.  The draws of each time step are fixed once for all rounds
    (the reading of the seed list of the CFTP host function in Section 2.2):
    time tau in [-2^r, -2^(r-1)), r >= 1, uses sweep counter tau + 3 * 2^(r-1),
    so that segment r is the counters [2^(r-1), 2^r) in order, and time -1
    uses counter 0."""
    segs = [(1 << (r - 1), 1 << (r - 1)) for r in range(R, 0, -1)]
    segs.append((0, 1))
    return segs


def cftp(make, max_log2=30, first_log2=1):
    """Coupling from the past (Section 1.1.4; the CFTP host function of
    Section 2.2).  make(init) returns a fresh chain started from the maximal
    ("max") or minimal ("min") state.  For R = first_log2, first_log2 + 1, ...
    both chains run the same sweeps from time -2^R to 0; the first R at which
    they end equal gives the exact sample.  Returns (R, final export)."""
    for R in range(first_log2, max_log2 + 1):
        top, bottom = make("max"), make("min")
        for t0, count in cftp_segments(R):
            for ch in (top, bottom):
                ch.t = t0
                ch.sweep(count)
        a, b = top.export(), bottom.export()
        if np.array_equal(a, b):
            return R, b
    raise RuntimeError("no coalescence within 2^%d sweeps" % max_log2)


def bin_density(bin_sum, samples, in_domain, bin_):
    """density[bin] = bin_sum / (samples * in-domain cells of the bin); 0 for
    bins without in-domain cells or before any sample (fp64, one division)."""
    Hc, Wc = in_domain.shape
    by, bx = -(-Hc // bin_), -(-Wc // bin_)
    cnt = np.zeros((by, bx), dtype=np.float64)
    for y in range(by):
        for x in range(bx):
            cnt[y, x] = in_domain[y * bin_:(y + 1) * bin_, x * bin_:(x + 1) * bin_].sum()
    out = np.zeros((by, bx), dtype=np.float64)
    s = np.asarray(bin_sum, dtype=np.float64).reshape(by, bx)
    m = (cnt > 0) & (samples > 0)
    out[m] = s[m] / (float(samples) * cnt[m])
    return out


from .region import (DominoRegionOracle, Untileable, check_region, extremal_heights,  # noqa: E402
                     extremal_tilings, region_embedding, region_heights, tiling_from_heights, square_tmin)
from .sixv_region import (SixVertexRegionOracle, sixv_boundary_heights, sixv_c_vertices,  # noqa: E402
                          sixv_extremal_heights, sixv_free_points, sixv_points)
from .loz_region import (LozengeRegionOracle, check_loz_region, hexagon_mask, loz_extremal_heights,  # noqa: E402
                         loz_points)
