"""Helpers for the oracle pin tests: breadth-first enumeration through the
oracle's own flip primitive, and a chi-square comparison of visit counts with
an exact stationary law."""
from collections import Counter

import numpy as np
from scipy import stats


def bfs(chain, get, put, key):
    """All states reachable from the chain's current state by single flips."""
    start = get()
    seen = {key(): start}
    frontier = [start]
    sites = chain.sites()
    while frontier:
        nxt = []
        for st in frontier:
            for (X, Y) in sites:
                for up in (0, 1):
                    put(st)
                    if chain.flip(X, Y, up):
                        k = key()
                        if k not in seen:
                            snap = get()
                            seen[k] = snap
                            nxt.append(snap)
        frontier = nxt
    put(start)
    return seen


def chi_square_pvalue(chain, probs, n_samples, thin, burn=20):
    """Visit frequencies of the chain (sampled every `thin` sweeps) against the
    exact probabilities `probs` (dict state-key -> p)."""
    chain.sweep(burn)
    counts = Counter()
    for _ in range(n_samples):
        chain.sweep(thin)
        counts[chain.export().tobytes()] += 1
    assert set(counts) <= set(probs), "chain visited a state outside the enumeration"
    keys = list(probs)
    obs = np.array([counts.get(k, 0) for k in keys], dtype=np.float64)
    exp = np.array([probs[k] for k in keys], dtype=np.float64) * n_samples
    stat = float(((obs - exp) ** 2 / exp).sum())
    return float(stats.chi2.sf(stat, len(keys) - 1))
