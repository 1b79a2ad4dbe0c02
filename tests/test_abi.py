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
