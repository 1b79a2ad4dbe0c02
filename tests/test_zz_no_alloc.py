"""tl_sampler_hash_noalloc (the hash for callers that cannot allocate) against
tl_sampler_hash on the same states: two calls in a row, the second on a
smaller state, then the largest benchmark state, an oversized export (refused)
and a small state checked against the oracle's digest as well."""
import pytest

import oracle
from gpu_helpers import need_gpu, say

pytestmark = pytest.mark.gpu


def test_noalloc_hash_equals_hash_on_shrinking_states():
    tl = need_gpu()
    cases = [
        ("domino n=300", tl.domain(tl.TL_DOMINO, n=300), tl.weights(tl.TL_W_UNIFORM), 40),
        ("lozenge 20^3", tl.domain(tl.TL_LOZENGE, a=20, b=20, c=20), tl.weights(tl.TL_W_VOLUME, 0.9), 30),
        ("six-vertex N=17", tl.domain(tl.TL_SIXVERTEX, n=17), tl.weights(tl.TL_W_SIXVERTEX, 1.0, 1.0, 2.0), 25),
    ]
    for name, dom, w, sweeps in cases:
        say("hash_noalloc: %s" % name)
        s = tl.Sampler(dom, w, 3)
        s.sweep(sweeps)
        a = s.hash_noalloc()
        assert a == s.hash(), name
        # a second call on the same state gives the same digest
        assert s.hash_noalloc() == a, name
        s.destroy()


def test_noalloc_hash_benchmark_state_and_oracle():
    tl = need_gpu()
    say("hash_noalloc: order-2048 Aztec diamond")
    s = tl.Sampler(tl.domain(tl.TL_DOMINO, n=2048), tl.weights(tl.TL_W_UNIFORM), 7)
    s.sweep(10)
    assert s.hash_noalloc() == s.hash()
    s.destroy()
    say("hash_noalloc: order-24 Aztec diamond against the oracle")
    n, seed, sweeps = 24, 5, 20
    s = tl.Sampler(tl.domain(tl.TL_DOMINO, n=n), tl.weights(tl.TL_W_UNIFORM), seed)
    s.sweep(sweeps)
    o = oracle.DominoOracle(n, oracle.table_from_ratios(oracle.domino_ratios(), False), seed=seed)
    o.sweep(sweeps)
    assert s.hash_noalloc() == oracle.canonical_hash(o.export())
    s.destroy()


def test_noalloc_hash_refuses_oversized_export():
    tl = need_gpu()
    say("hash_noalloc: oversized export")
    s = tl.Sampler(tl.domain(tl.TL_DOMINO, n=3300), tl.weights(tl.TL_W_UNIFORM), 1)
    with pytest.raises(tl.TlError) as e:
        s.hash_noalloc()
    assert e.value.status == tl.TL_EINVAL and "static buffer" in str(e.value)
    # the sampler is untouched and the allocating hash still works
    assert len(s.hash()) == 64
    s.destroy()
