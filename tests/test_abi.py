"""The C-ABI library loads without a GPU, exports every function that
include/tilings.h declares, and computes its threshold tables on the host equal
to the oracle's exact-rational tables for the workload weights."""
import ctypes
import math
import os
import re
from fractions import Fraction

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"\b(tl_[a-z_0-9]+)\s*\(", txt)
    return sorted(set(names))


def test_library_exports_declared_symbols():
    import paper_1804_07250_amd as tl
    L = tl.lib()
    names = declared_functions()
    assert "tl_sampler_create" in names and "tl_sampler_sweep" in names and "tl_sampler_observables" in names
    for name in names:
        assert hasattr(L, name), name


def test_status_strings_and_errors_without_gpu():
    import paper_1804_07250_amd as tl
    assert tl.lib().tl_status_str(tl.TL_EINVAL) == b"invalid argument"
    with pytest.raises(tl.TlError) as e:
        tl.thresholds(tl.domain(tl.TL_DOMINO, n=4), tl.weights(tl.TL_W_TWO_PERIODIC, 1.0, -1.0))
    assert e.value.status == tl.TL_EINVAL
    with pytest.raises(tl.TlError):
        tl.thresholds(tl.domain(tl.TL_DOMINO, n=4), tl.weights(tl.TL_W_VOLUME, 0.5))
    with pytest.raises(tl.TlError):
        tl.thresholds(tl.domain(tl.TL_SIXVERTEX, n=4), tl.weights(tl.TL_W_SIXVERTEX, 1.0, float("nan"), 1.0))


@pytest.mark.parametrize("metro", [False, True])
def test_thresholds_equal_exact_tables(metro):
    import paper_1804_07250_amd as tl
    rule = tl.TL_METROPOLIS if metro else tl.TL_HEATBATH
    cases = [
        (tl.domain(tl.TL_DOMINO, n=8), tl.weights(tl.TL_W_UNIFORM, rule=rule), oracle.domino_ratios()),
        (tl.domain(tl.TL_DOMINO, n=8), tl.weights(tl.TL_W_TWO_PERIODIC, 1.0, 0.5, rule=rule),
         oracle.domino_ratios("two", 1, Fraction(1, 2))),
        (tl.domain(tl.TL_LOZENGE, a=3, b=3, c=3), tl.weights(tl.TL_W_VOLUME, 1999.0, 2000.0, rule=rule),
         oracle.lozenge_ratios(Fraction(1999, 2000))),
        (tl.domain(tl.TL_SIXVERTEX, n=8), tl.weights(tl.TL_W_SIXVERTEX, 1.0, 1.0, 2.0, rule=rule),
         oracle.sixv_ratios(1, 1, 2)),
        (tl.domain(tl.TL_SIXVERTEX, n=8), tl.weights(tl.TL_W_SIXVERTEX, 1.0, 1.0, 1.0, rule=rule),
         oracle.sixv_ratios(1, 1, 1)),
        (tl.domain(tl.TL_SIXVERTEX, n=8), tl.weights(tl.TL_W_SIXVERTEX, 4.0, 1.0, 4.0, rule=rule),
         oracle.sixv_ratios(2, 1, 4)),
        (tl.domain(tl.TL_SIXVERTEX, n=8), tl.weights(tl.TL_W_SIXVERTEX6, 1.0, 2.0, 1.5, 0.5, 1.0, 3.0, rule=rule),
         oracle.sixv_ratios6(1, 2, Fraction(3, 2), Fraction(1, 2), 1, 3)),
        (tl.domain(tl.TL_DOMINO, n=8), tl.weights(tl.TL_W_VOLUME_BW, 20.0, 1.0, 1.0, 20.0, rule=rule),
         oracle.domino_ratios("volume", 20, Fraction(1, 20))),
        (tl.domain(tl.TL_DOMINO, n=8), tl.weights(tl.TL_W_VOLUME_BW, 5.0, 4.0, 2.0, 3.0, rule=rule),
         oracle.domino_ratios("volume", Fraction(5, 4), Fraction(2, 3))),
    ]
    for dom, w, ratios in cases:
        assert tl.thresholds(dom, w) == oracle.table_from_ratios(ratios, metro)


def test_state_bytes_on_the_host():
    """tl_sampler_state_bytes needs no device: two bit-plane buffers, each a
    multiple of 256 bytes and at least one bit per site of the domain."""
    import numpy as np
    import paper_1804_07250_amd as tl
    cases = [(tl.domain(tl.TL_DOMINO, n=64), 2 * 64 * 64 * 2 * 2),
             (tl.domain(tl.TL_LOZENGE, a=50, b=40, c=30), 51 * 41),
             (tl.domain(tl.TL_SIXVERTEX, n=128), 127 * 127),
             (tl.domain(tl.TL_DOMINO, mask=np.ones((30, 50), dtype=bool)), 30 * 50 * 2),
             (tl.domain(tl.TL_SIXVERTEX, mask=np.ones((20, 32), dtype=bool), free_north=True), 20 * 31)]
    sizes = []
    for dom, bits in cases:
        n = tl.state_bytes(dom)
        assert n % 512 == 0 and n // 2 >= bits // 8
        sizes.append(n)
    assert tl.state_bytes(tl.domain(tl.TL_DOMINO, n=128)) > sizes[0]
    one = np.zeros((3, 3), dtype=bool)
    one[1, 1] = True
    with pytest.raises(tl.TlError) as e:
        tl.state_bytes(tl.domain(tl.TL_DOMINO, mask=one))
    assert e.value.status == tl.TL_EUNTILEABLE
    with pytest.raises(tl.TlError) as e:
        tl.state_bytes(tl.domain(tl.TL_DOMINO, n=0))
    assert e.value.status == tl.TL_EINVAL
    assert tl.lib().tl_sampler_state_bytes(None, None) == tl.TL_EINVAL


def test_batches_and_servers_refuse_caller_state():
    import ctypes
    import paper_1804_07250_amd as tl
    L = tl.lib()
    dom = tl.domain(tl.TL_DOMINO, n=8)
    w = tl.weights(tl.TL_W_UNIFORM)
    seeds = (ctypes.c_uint64 * 1)(1)
    opt = tl.options(device_buf=256, device_buf_bytes=1 << 20)
    h = ctypes.c_void_p()
    assert L.tl_batch_create(1, ctypes.byref(dom), ctypes.byref(w), seeds, ctypes.byref(opt),
                             ctypes.byref(h)) == tl.TL_EINVAL
    assert L.tl_server_create(1 << 20, 4, ctypes.byref(opt), ctypes.byref(h)) == tl.TL_EINVAL
