"""Seeded synthetic workload generators (inputs only: domain sizes, seeds,
arrival times).  They hold none of the sampler's arithmetic and serve the
GPU path, the tests and the oracle alike.

* batched Aztec chains: orders drawn uniformly from [16, 512] by numpy's PCG64
  seeded with 0x5EED; chain i has seed i;
* served six-vertex requests: N uniform over {64, 128, 256, 512, 1024},
  exponential inter-arrival times at a given rate (PCG64 seeded with the
  request-stream seed), weights alternating between (a, b, c) = (1, 1, sqrt 2)
  and (1, 1, 1) by request index, request seed = request index.
"""
import numpy as np

BATCH_SEED = 0x5EED
SERVE_SIZES = (64, 128, 256, 512, 1024)


def batch_orders(count=4096, lo=16, hi=512, seed=BATCH_SEED):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [int(v) for v in rng.integers(lo, hi + 1, size=count)]


def serve_requests(count, rate_per_s=200.0, seed=0x5E4E, sizes=SERVE_SIZES):
    """List of dicts: arrival time (s), N, weights (a^2, b^2, c^2), rule
    (lazy Metropolis thresholds), seed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    ns = rng.integers(0, len(sizes), size=count)
    t = np.cumsum(gaps)
    out = []
    for i in range(count):
        w2 = (1.0, 1.0, 2.0) if i % 2 == 0 else (1.0, 1.0, 1.0)
        out.append({"arrival": float(t[i]), "N": int(sizes[ns[i]]), "w2": w2, "metropolis": True, "seed": i})
    return out
