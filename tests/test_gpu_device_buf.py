"""Samplers whose state lives in caller-owned device memory (tl_options
device_buf, the ownership rule of the C-ABI): the chain equals the oracle's and
a library-allocated sampler's bit for bit, the caller's memory really holds the
state, and too-small or misaligned buffers are refused."""
import numpy as np
import pytest

import oracle
from gpu_helpers import need_gpu, say

pytestmark = pytest.mark.gpu


def buffer_for(tl, dom, extra=0):
    import torch
    n = tl.state_bytes(dom)
    buf = torch.zeros(n + extra, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    return buf, n


def l_shape(n, cut_w, cut_h):
    m = np.ones((n, n), dtype=bool)
    m[n - cut_h:, n - cut_w:] = False
    return m


def domains(tl):
    stoch = tl.weights(tl.TL_W_SIXVERTEX6, 1.0, 1.0, 0.25, 0.75, 0.25, 0.75)
    return {
        "aztec300": (tl.domain(tl.TL_DOMINO, n=300), tl.weights(tl.TL_W_TWO_PERIODIC, 1.0, 0.5)),
        "hexagon90": (tl.domain(tl.TL_LOZENGE, a=90, b=80, c=70), tl.weights(tl.TL_W_VOLUME, 2.0, 3.0)),
        "sixv200": (tl.domain(tl.TL_SIXVERTEX, n=200), tl.weights(tl.TL_W_SIXVERTEX, 1.0, 1.0, 2.0)),
        "domino_l": (tl.domain(tl.TL_DOMINO, mask=l_shape(70, 20, 30)), tl.weights(tl.TL_W_UNIFORM)),
        "sixv_free": (tl.domain(tl.TL_SIXVERTEX, mask=np.ones((40, 64), dtype=bool), free_north=True), stoch),
        "loz_mask": (tl.domain(tl.TL_LOZENGE, mask=oracle.hexagon_mask(20, 24, 18)),
                     tl.weights(tl.TL_W_VOLUME, 1.0, 2.0)),
    }


KERNELS = {"auto": {}, "step": {"kernel": 1}, "tiled": {"kernel": 2, "tile_rows": 8, "sweeps_per_launch": 3}}
CASES = [("aztec300", "auto", 0), ("aztec300", "step", 1), ("hexagon90", "auto", 0), ("hexagon90", "tiled", 0),
         ("sixv200", "auto", 1), ("domino_l", "tiled", 0), ("sixv_free", "auto", 0), ("loz_mask", "step", 0)]


@pytest.mark.parametrize("name,kernel,order", CASES, ids=["%s-%s-%d" % c for c in CASES])
def test_equals_library_allocated_sampler(name, kernel, order):
    tl = need_gpu()
    say("device_buf %s %s order=%d" % (name, kernel, order))
    dom, w = domains(tl)[name]
    buf, n = buffer_for(tl, dom)
    a = tl.Sampler(dom, w, 31, tl.options(colour_order=order, obs_every=2, obs_bin=5, **KERNELS[kernel]))
    b = tl.Sampler(dom, w, 31, tl.options(colour_order=order, obs_every=2, obs_bin=5, device_buf=buf.data_ptr(),
                                          device_buf_bytes=n, **KERNELS[kernel]))
    b.sync()
    assert int(buf.count_nonzero()) > 0          # the initial state was written there
    for k in (1, 4, 9):
        a.sweep(k)
        b.sweep(k)
        assert (a.export() == b.export()).all(), "after %d sweeps" % k
    assert a.hash() == b.hash()
    oa, ob = a.observables(), b.observables()
    assert (oa["bin_sum"] == ob["bin_sum"]).all() and oa["scalar_now"] == ob["scalar_now"]
    before = buf.clone()
    b.destroy()
    import torch
    torch.cuda.synchronize()
    assert torch.equal(buf, before)              # not freed or cleared by the library


def test_equals_oracle_and_holds_the_state():
    tl = need_gpu()
    import torch
    n_az = 40
    dom = tl.domain(tl.TL_DOMINO, n=n_az)
    w = tl.weights(tl.TL_W_UNIFORM)
    buf, n = buffer_for(tl, dom)
    # one launch per colour step updates the state in place (buffer 0)
    s = tl.Sampler(dom, w, 12, tl.options(kernel=1, device_buf=buf.data_ptr(), device_buf_bytes=n))
    o = oracle.DominoOracle(n_az, oracle.table_from_ratios(oracle.domino_ratios(), False), seed=12)
    for k in (1, 7, 30):
        s.sweep(k)
        o.sweep(k)
        assert (s.export() == o.export()).all()
    # a fresh sampler given a copy of that memory exports the same tiling
    s.sync()
    buf2, _ = buffer_for(tl, dom)
    c = tl.Sampler(dom, w, 99, tl.options(kernel=1, device_buf=buf2.data_ptr(), device_buf_bytes=n))
    c.sync()
    assert not (c.export() == o.export()).all()
    buf2[: n // 2].copy_(buf[: n // 2])
    torch.cuda.synchronize()
    assert (c.export() == o.export()).all()


def test_cftp_with_caller_state():
    tl = need_gpu()
    say("device_buf cftp")
    m = l_shape(24, 8, 10)
    w = tl.weights(tl.TL_W_SIXVERTEX, 1.0, 1.0, 2.0)
    dom = tl.domain(tl.TL_SIXVERTEX, mask=m)
    buf, n = buffer_for(tl, dom)
    a = tl.Sampler(dom, w, 5)
    b = tl.Sampler(dom, w, 5, tl.options(device_buf=buf.data_ptr(), device_buf_bytes=n))
    ia, ib = a.cftp(20), b.cftp(20)
    assert ia == ib
    assert (a.export() == b.export()).all()


def test_second_sampler_reuses_the_buffer():
    tl = need_gpu()
    dom = tl.domain(tl.TL_LOZENGE, a=30, b=30, c=30)
    w = tl.weights(tl.TL_W_VOLUME, 1.0, 2.0)
    buf, n = buffer_for(tl, dom)
    ref = tl.Sampler(dom, w, 3)
    ref.sweep(12)
    for _ in range(2):
        s = tl.Sampler(dom, w, 3, tl.options(device_buf=buf.data_ptr(), device_buf_bytes=n))
        s.sweep(12)
        assert (s.export() == ref.export()).all()
        s.destroy()


def test_rejects_small_or_misaligned_buffers():
    tl = need_gpu()
    dom = tl.domain(tl.TL_SIXVERTEX, n=64)
    w = tl.weights(tl.TL_W_SIXVERTEX, 1.0, 1.0, 1.0)
    buf, n = buffer_for(tl, dom, extra=512)
    assert n % 512 == 0
    for ptr, size in ((buf.data_ptr(), n - 1), (buf.data_ptr() + 4, n), (buf.data_ptr() + 128, n)):
        with pytest.raises(tl.TlError) as e:
            tl.Sampler(dom, w, 1, tl.options(device_buf=ptr, device_buf_bytes=size))
        assert e.value.status == tl.TL_EINVAL
    s = tl.Sampler(dom, w, 1, tl.options(device_buf=buf.data_ptr() + 256, device_buf_bytes=n))
    s.sweep(2)
