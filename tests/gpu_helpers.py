"""Shared pieces of the GPU parity tests: library loading (skips the module when
there is no GPU) and builders for matching oracle chains."""
import os
import sys

import numpy as np
import pytest


def need_gpu():
    try:
        import torch
        ok = torch.cuda.is_available()
    except Exception:
        ok = False
    if not ok:
        pytest.skip("no GPU")
    import paper_1804_07250_amd as tl
    tl.lib()
    return tl


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def vertical_brick_faces(n):
    """Canonical export of the all-vertical brick tiling of the Aztec diamond
    (every face column covered from its south end)."""
    W = 2 * n
    f = np.full((W, W), 255, dtype=np.uint8)
    for X in range(W):
        start = None
        for Y in range(W):
            if abs(2 * X - 2 * n + 1) + abs(2 * Y - 2 * n + 1) <= 2 * n:
                if start is None:
                    start = Y
                f[Y, X] = 0 if (Y - start) % 2 == 0 else 1
    return f
