"""Pins for the oracle's general domains (Section 1.1: simply-connected
domains, height functions, T_max / T_min and Thurston's tileability test).

* the brute-force tiling enumerator used below reproduces Kasteleyn's closed
  form for rectangles (and the Fibonacci numbers for 2 x n strips);
* tileability by Thurston's test agrees with brute force on every accepted
  domain of a 3 x 4 box and on random domains up to 5 x 6;
* T_max / T_min are tilings of the domain whose heights are the pointwise
  maximum / minimum over all tilings (the definition of Section 1.1);
* the brick tilings are the extremes of Aztec diamonds;
* rotations through the embedded chain reach exactly the enumerated tilings
  (connectivity, Section 1.1.2), and the chain's visits follow the uniform
  law; coupling from the past on a domain coalesces for every start state.
"""
import math
from collections import Counter

import numpy as np
import pytest

import oracle
from oracle_helpers import bfs, chi_square_pvalue
from test_oracle_cftp import chi_square_of_samples, run_from

N, S, E, W = 0, 1, 2, 3


def brute_tilings(mask):
    """Every tiling of the domain by exhaustive search: the first uncovered
    face in row-major order (rows from the south) pairs with its east or its
    north neighbour, since its west and south neighbours are covered."""
    m = np.asarray(mask, dtype=bool)
    h, w = m.shape
    f = np.full((h, w), 255, dtype=np.uint8)
    order = [(x, y) for y in range(h) for x in range(w) if m[y, x]]
    out = []

    def rec(i):
        while i < len(order) and f[order[i][1], order[i][0]] != 255:
            i += 1
        if i == len(order):
            out.append(f.copy())
            return
        x, y = order[i]
        if x + 1 < w and m[y, x + 1] and f[y, x + 1] == 255:
            f[y, x], f[y, x + 1] = E, W
            rec(i + 1)
            f[y, x], f[y, x + 1] = 255, 255
        if y + 1 < h and m[y + 1, x] and f[y + 1, x] == 255:
            f[y, x], f[y + 1, x] = N, S
            rec(i + 1)
            f[y, x], f[y + 1, x] = 255, 255

    rec(0)
    return out


def kasteleyn(m, n):
    """Number of domino tilings of an m x n rectangle (Kasteleyn's product)."""
    p = 1.0
    for j in range(1, (m + 1) // 2 + 1):
        for k in range(1, (n + 1) // 2 + 1):
            p *= 4 * math.cos(math.pi * j / (m + 1)) ** 2 + 4 * math.cos(math.pi * k / (n + 1)) ** 2
    return round(p) if (m * n) % 2 == 0 else 0


def accepted(mask):
    try:
        oracle.check_region(mask)
        return True
    except ValueError:
        return False


def random_domain(rng, w, h, fill):
    """A random simply-connected domain grown face by face in a w x h box."""
    while True:
        m = np.zeros((h, w), dtype=bool)
        m[rng.integers(h), rng.integers(w)] = True
        target = max(2, int(fill * w * h))
        tries = 0
        while m.sum() < target and tries < 50 * w * h:
            tries += 1
            ys, xs = np.nonzero(m)
            k = rng.integers(len(xs))
            dx, dy = [(1, 0), (-1, 0), (0, 1), (0, -1)][rng.integers(4)]
            x, y = xs[k] + dx, ys[k] + dy
            if 0 <= x < w and 0 <= y < h and not m[y, x]:
                m[y, x] = True
                if not accepted(m):
                    m[y, x] = False
        if accepted(m):
            return m


def ones(h, w):
    return np.ones((h, w), dtype=bool)


def l_shape(a, b, c):
    """An a x a square with a b x c rectangle cut out of its north-east corner."""
    m = ones(a, a)
    m[a - b:, a - c:] = False
    return m


# ------------------------------------------------------------------- pins

@pytest.mark.parametrize("h,w", [(2, 1), (2, 5), (2, 9), (3, 4), (4, 4), (4, 5), (3, 6), (5, 6), (6, 6), (3, 3)])
def test_brute_force_matches_kasteleyn(h, w):
    assert len(brute_tilings(ones(h, w))) == kasteleyn(h, w)


def test_strips_are_fibonacci():
    fib = [1, 1]
    while len(fib) < 13:
        fib.append(fib[-1] + fib[-2])
    for n in range(1, 12):
        assert len(brute_tilings(ones(2, n))) == fib[n]


def test_embedding_holds_the_box():
    for w in range(1, 41):
        for h in range(1, 41):
            n, ox, oy = oracle.region_embedding(w, h)
            assert n == (w + h + 1) // 2 and ox + oy == n and ox >= 0 and oy >= 0
            for y in (0, h - 1):
                for x in (0, w - 1):
                    X, Y = x + ox, y + oy
                    assert abs(2 * X - 2 * n + 1) + abs(2 * Y - 2 * n + 1) <= 2 * n, (w, h)


def test_region_checks():
    assert accepted(ones(3, 3))
    assert accepted(l_shape(4, 2, 2))
    ring = ones(3, 3)
    ring[1, 1] = False
    with pytest.raises(ValueError, match="hole"):
        oracle.check_region(ring)
    diag = np.array([[1, 0], [0, 1]], dtype=bool)
    with pytest.raises(ValueError, match="pinch"):
        oracle.check_region(diag)
    pinch = ones(3, 3)
    pinch[0, 1] = pinch[1, 0] = False     # faces (0,0) and (1,1) meet at a corner only
    with pytest.raises(ValueError):
        oracle.check_region(pinch)
    two = np.array([[1, 0, 1]], dtype=bool)
    with pytest.raises(ValueError, match="connected"):
        oracle.check_region(two)
    with pytest.raises(ValueError):
        oracle.check_region(np.zeros((2, 2), dtype=bool))


def check_extremes(mask, parity=0):
    """Thurston's answer against brute force: tileability, and T_max / T_min
    as the pointwise extremes of the heights of every tiling."""
    tilings = brute_tilings(mask)
    if not tilings:
        with pytest.raises(oracle.Untileable):
            oracle.extremal_heights(mask, parity)
        return 0
    hmax, hmin = oracle.extremal_heights(mask, parity)
    hs = [oracle.region_heights(t, parity) for t in tilings]
    for v in hmax:
        assert hmax[v] == max(h[v] for h in hs) and hmin[v] == min(h[v] for h in hs)
    tmax, tmin = oracle.extremal_tilings(mask, parity)
    keys = {t.tobytes() for t in tilings}
    assert tmax.tobytes() in keys and tmin.tobytes() in keys
    assert oracle.region_heights(tmax, parity) == hmax and oracle.region_heights(tmin, parity) == hmin
    return len(tilings)


def test_every_domain_of_a_3x4_box():
    tileable = untileable = 0
    for bits in range(1, 1 << 12):
        m = np.array([(bits >> i) & 1 for i in range(12)], dtype=bool).reshape(3, 4)
        if not accepted(m):
            continue
        for parity in (0, 1):
            c = check_extremes(m, parity)
        tileable += c > 0
        untileable += c == 0
    # both outcomes occur, including balanced domains without tilings
    assert tileable > 100 and untileable > 100


def test_balanced_untileable_domain():
    # equal black and white faces, yet no tiling: Thurston's bound fails
    m = np.array([[1, 0, 0, 1],
                  [1, 1, 1, 1],
                  [1, 0, 0, 1]], dtype=bool)[::-1]
    colours = [(x + y) % 2 for y in range(3) for x in range(4) if m[y, x]]
    assert colours.count(0) == colours.count(1)
    assert brute_tilings(m) == []
    for parity in (0, 1):
        with pytest.raises(oracle.Untileable):
            oracle.extremal_heights(m, parity)


def test_mutilated_chessboard_and_odd_area():
    board = ones(8, 8)
    board[0, 0] = board[7, 7] = False
    with pytest.raises(oracle.Untileable):
        oracle.extremal_heights(board)
    with pytest.raises(oracle.Untileable):
        oracle.extremal_heights(ones(3, 3))


@pytest.mark.parametrize("seed", range(12))
def test_random_domains_against_brute_force(seed):
    rng = np.random.default_rng(seed)
    w, h = [(4, 4), (5, 5), (5, 6), (6, 5)][seed % 4]
    m = random_domain(rng, w, h, 0.75)
    check_extremes(m, seed % 2)


def test_rectangles_and_l_shapes_extremes():
    for m in (ones(4, 4), ones(3, 6), ones(5, 4), l_shape(4, 2, 2), l_shape(6, 2, 4), l_shape(5, 3, 1)):
        assert check_extremes(m, 0) == len(brute_tilings(m))


def test_closed_form_tmin_of_squares():
    # the closed form used for squares too large for the general algorithm
    # equals its T_min on every even side up to 16; odd sides are refused
    for side in range(2, 18, 2):
        m = np.ones((side, side), dtype=bool)
        n, ox, oy = oracle.region_embedding(side, side)
        _, tmin = oracle.extremal_tilings(m, (ox + oy) % 2)
        assert np.array_equal(oracle.square_tmin(side), tmin), side
    with pytest.raises(ValueError):
        oracle.square_tmin(7)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 9])
def test_aztec_extremes_are_the_bricks(n):
    d = oracle.DominoOracle(n, [0] * 4)
    mask = d.in_domain_cells()
    horizontal = d.export()
    vertical = oracle.domino_vertical_brick(horizontal)
    tmax, tmin = oracle.extremal_tilings(mask, 0)
    if n % 2:
        assert (tmax == vertical).all() and (tmin == horizontal).all()
    else:
        assert (tmax == horizontal).all() and (tmin == vertical).all()


def region_chain(mask, seed=1, init="min", thr=None, **kw):
    thr = thr if thr is not None else oracle.table_from_ratios(oracle.domino_ratios(), False)
    return oracle.DominoRegionOracle(mask, thr, seed=seed, init=init, **kw)


def reachable(ch):
    d = ch.chain
    get = lambda: (d.Tb.copy(), d.Tw.copy())

    def put(s):
        d.Tb[:] = s[0]
        d.Tw[:] = s[1]

    return bfs(ch, get, put, lambda: ch.export().tobytes())


@pytest.mark.parametrize("name", ["square4", "rect3x6", "l6", "l5", "random0", "random1"])
def test_rotations_connect_every_tiling(name):
    m = {"square4": ones(4, 4), "rect3x6": ones(3, 6), "l6": l_shape(6, 2, 4), "l5": l_shape(5, 3, 1),
         "random0": random_domain(np.random.default_rng(100), 5, 5, 0.8),
         "random1": random_domain(np.random.default_rng(101), 6, 5, 0.8)}[name]
    tilings = {t.tobytes() for t in brute_tilings(m)}
    if not tilings:
        pytest.skip("untileable draw")
    for init in ("min", "max"):
        ch = region_chain(m, init=init)
        assert set(reachable(ch)) == tilings


def test_chain_keeps_the_domain_and_stays_a_tiling():
    m = l_shape(8, 4, 2)
    ch = region_chain(m, seed=5)
    ch.sweep(40)
    f = ch.export()
    assert np.array_equal(f != 255, m)
    ch.load(f)              # load validates the tiling of the domain
    # the faces of the diamond outside the domain stay uncovered
    full = ch.chain.export()
    assert int((full != 255).sum()) == int(m.sum())
    with pytest.raises(ValueError):
        bad = f.copy()
        bad[0, 0] = 255
        ch.load(bad)


def test_uniform_law_on_a_square():
    m = ones(4, 4)
    tilings = brute_tilings(m)
    assert len(tilings) == 36
    probs = {t.tobytes(): 1.0 / 36 for t in tilings}
    assert chi_square_pvalue(region_chain(m, seed=7), probs, 8000, 6) > 1e-3


def test_observables_on_a_domain():
    m = l_shape(8, 3, 4)
    ch = region_chain(m, seed=3, obs_every=2, bin_=3)
    ch.sweep(9)
    f = ch.export()
    v, bs = ch.observe()
    assert v == int(((f == E) | (f == W)).sum())
    assert int(ch.samples[0]) == 4 and bs.sum() == v


def test_cftp_on_domains_coalesces_from_every_state():
    for m in (l_shape(4, 2, 2), ones(3, 4)):
        states = [np.frombuffer(k, dtype=np.uint8).reshape(m.shape) for k in
                  {t.tobytes() for t in brute_tilings(m)}]
        for seed in range(4):
            make = lambda init, s=seed: region_chain(m, seed=s, init=init)
            R, sample = oracle.cftp(make)
            for st in states:
                assert np.array_equal(run_from(make, st, R), sample)


def test_cftp_law_on_an_l_shape():
    m = l_shape(4, 2, 2)
    tilings = brute_tilings(m)
    probs = {t.tobytes(): 1.0 / len(tilings) for t in tilings}
    samples = [oracle.cftp(lambda init, s=s: region_chain(m, seed=s, init=init))[1] for s in range(3000)]
    assert chi_square_of_samples(samples, probs) > 1e-3
    assert len(Counter(x.tobytes() for x in samples)) == len(tilings)
