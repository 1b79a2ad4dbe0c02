"""Python binding of the MI355X Glauber-sweep library ``libtilings.so``.

Argument marshalling only: every step of the sweep, the observables, the export
and the row hashing run in the library's HIP kernels.  The names follow the
C-ABI of ``include/tilings.h``.  Importing this module loads the library and
raises if it has not been built (``python -m paper_1804_07250_amd.build`` or
``__graft_entry__.build()``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtilings.so")

TL_OK, TL_EINVAL, TL_EUNTILEABLE, TL_ENOMEM, TL_EBUDGET, TL_EDEVICE, TL_EBUSY = 0, -1, -2, -3, -4, -5, -6
TL_DOMINO, TL_LOZENGE, TL_SIXVERTEX = 0, 1, 2
TL_AZTEC, TL_HEXAGON, TL_DWBC_SQUARE, TL_MASK = 0, 1, 2, 3
TL_INIT_MIN, TL_INIT_MAX = 0, 1
TL_HEATBATH, TL_METROPOLIS = 0, 1
TL_W_UNIFORM, TL_W_TWO_PERIODIC, TL_W_VOLUME, TL_W_SIXVERTEX, TL_W_VOLUME_BW, TL_W_SIXVERTEX6 = 0, 1, 2, 3, 4, 5


class TlError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s (status %d): %s" % (_status_name(status), status, message))
        self.status = status


def _status_name(st):
    return {0: "TL_OK", -1: "TL_EINVAL", -2: "TL_EUNTILEABLE", -3: "TL_ENOMEM", -4: "TL_EBUDGET",
            -5: "TL_EDEVICE", -6: "TL_EBUSY"}.get(st, "TL_?")


class tl_domain(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("shape", ctypes.c_int32), ("n", ctypes.c_int32),
                ("a", ctypes.c_int32), ("b", ctypes.c_int32), ("c", ctypes.c_int32),
                ("init", ctypes.c_int32), ("w", ctypes.c_int32), ("h", ctypes.c_int32),
                ("mask", ctypes.POINTER(ctypes.c_uint8)), ("flags", ctypes.c_uint32)]


class tl_weights(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("rule", ctypes.c_int32), ("w", ctypes.c_double * 6)]


class tl_options(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_void_p), ("obs_every", ctypes.c_uint32), ("obs_bin", ctypes.c_uint32),
                ("sweeps_per_launch", ctypes.c_uint32), ("tile_rows", ctypes.c_uint32),
                ("kernel", ctypes.c_uint32), ("tile_groups", ctypes.c_uint32), ("colour_order", ctypes.c_uint32),
                ("device_buf", ctypes.c_void_p), ("device_buf_bytes", ctypes.c_size_t),
                ("tune_cache", ctypes.c_char_p)]


class tl_observables(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_uint64), ("samples", ctypes.c_uint64), ("scalar_now", ctypes.c_int64),
                ("scalar_sum", ctypes.c_int64), ("bins_x", ctypes.c_uint32), ("bins_y", ctypes.c_uint32),
                ("bin_sum", ctypes.POINTER(ctypes.c_uint64)), ("bin_now", ctypes.POINTER(ctypes.c_uint64)),
                ("bin_density", ctypes.POINTER(ctypes.c_double)), ("bin_capacity", ctypes.c_size_t)]


class tl_tune_info(ctypes.Structure):
    _fields_ = [("tile_rows", ctypes.c_uint32), ("tile_groups", ctypes.c_uint32),
                ("sweeps_per_launch", ctypes.c_uint32), ("candidates", ctypes.c_uint32),
                ("from_cache", ctypes.c_uint32), ("ms_per_sweep", ctypes.c_float), ("kernel", ctypes.c_uint32)]


class tl_cftp_info(ctypes.Structure):
    _fields_ = [("log2_sweeps", ctypes.c_uint32), ("sweeps", ctypes.c_uint64), ("total_sweeps", ctypes.c_uint64)]


_lib = None


def lib():
    """Load libtilings.so (raises if it is missing: no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libtilings.so is not built: run __graft_entry__.build() or "
                              "python -m paper_1804_07250_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32
        L.tl_sampler_create.argtypes = [ctypes.POINTER(tl_domain), ctypes.POINTER(tl_weights), u64,
                                        ctypes.POINTER(tl_options), ctypes.POINTER(vp)]
        L.tl_sampler_sweep.argtypes = [vp, u64]
        L.tl_sampler_sync.argtypes = [vp]
        L.tl_sampler_observables.argtypes = [vp, ctypes.POINTER(tl_observables)]
        L.tl_sampler_export_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(u32),
                                             ctypes.POINTER(u32)]
        L.tl_sampler_export.argtypes = [vp, vp, ctypes.c_size_t, ctypes.POINTER(u64)]
        L.tl_sampler_hash.argtypes = [vp, ctypes.POINTER(ctypes.c_uint8)]
        L.tl_sampler_hash_noalloc.argtypes = [vp, ctypes.POINTER(ctypes.c_uint8)]
        L.tl_sampler_import.argtypes = [vp, vp, ctypes.c_size_t, u64]
        L.tl_sampler_destroy.argtypes = [vp]
        L.tl_sampler_info.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u32)]
        L.tl_sampler_reset.argtypes = [vp, u64]
        L.tl_sampler_cftp.argtypes = [vp, u32, ctypes.POINTER(tl_cftp_info)]
        L.tl_sampler_set_timing.argtypes = [vp, i32]
        L.tl_sampler_kernel_time.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(u64),
                                             ctypes.POINTER(u64), ctypes.POINTER(ctypes.c_double)]
        L.tl_sampler_thresholds.argtypes = [vp, ctypes.POINTER(u32), u32, ctypes.POINTER(u32)]
        L.tl_sampler_autotune.argtypes = [vp, u32, ctypes.POINTER(tl_tune_info)]
        L.tl_thresholds.argtypes = [ctypes.POINTER(tl_domain), ctypes.POINTER(tl_weights),
                                    ctypes.POINTER(u32), u32, ctypes.POINTER(u32)]
        L.tl_thresholds.restype = i32
        L.tl_status_str.argtypes = [i32]
        L.tl_status_str.restype = ctypes.c_char_p
        L.tl_last_error.restype = ctypes.c_char_p
        for name in ("tl_sampler_create", "tl_sampler_sweep", "tl_sampler_sync", "tl_sampler_observables",
                     "tl_sampler_export_size", "tl_sampler_export", "tl_sampler_hash", "tl_sampler_hash_noalloc",
                     "tl_sampler_import",
                     "tl_sampler_destroy", "tl_sampler_info", "tl_sampler_thresholds", "tl_sampler_reset",
                     "tl_sampler_set_timing", "tl_sampler_kernel_time", "tl_sampler_cftp",
                     "tl_domain_extremes", "tl_sampler_state_bytes", "tl_sampler_autotune"):
            getattr(L, name).restype = i32
        _lib = L
    return _lib


def _check(st):
    if st != TL_OK:
        raise TlError(st, lib().tl_last_error().decode())


TL_FREE_NORTH, TL_FREE_SOUTH, TL_FREE_EAST, TL_FREE_WEST = 1, 2, 4, 8
FREE_SIDE_FLAGS = {"north": TL_FREE_NORTH, "south": TL_FREE_SOUTH, "east": TL_FREE_EAST, "west": TL_FREE_WEST}


def domain(model, n=0, a=0, b=0, c=0, init=TL_INIT_MIN, mask=None, free_north=False, free_side=None):
    """A domain: the model's fixed shape (Aztec diamond of order n, a x b x c
    hexagon, N x N domain-wall square), or with `mask` the TL_MASK shape:
    (h, w) cells for dominoes and six-vertex domains, (h, w, 2) unit
    triangles for lozenges, row 0 southmost, nonzero = inside.  free_side
    ("north", "south", "east" or "west"; free_north for "north"): six-vertex
    domains with that side free.  The returned struct keeps the mask's bytes
    alive; the library copies them when a sampler is created."""
    if mask is not None:
        m = np.ascontiguousarray(np.asarray(mask) != 0, dtype=np.uint8)
        if m.ndim != (3 if model == TL_LOZENGE else 2) or (model == TL_LOZENGE and m.shape[2] != 2):
            raise ValueError("mask must be (h, w) cells, or (h, w, 2) triangles for lozenges")
        d = tl_domain(model, TL_MASK, 0, 0, 0, 0, init, m.shape[1], m.shape[0],
                      m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                      FREE_SIDE_FLAGS[free_side] if free_side else (TL_FREE_NORTH if free_north else 0))
        d._mask = m
        return d
    shape = {TL_DOMINO: TL_AZTEC, TL_LOZENGE: TL_HEXAGON, TL_SIXVERTEX: TL_DWBC_SQUARE}[model]
    return tl_domain(model, shape, n, a, b, c, init)


def domain_extremes(dom):
    """Extremal states of a mask domain as canonical exports (host only):
    dominoes (T_max, T_min), six-vertex (h_max, h_min); raises TlError
    (TL_EUNTILEABLE when the domain has no tiling / configuration)."""
    if dom.model in (TL_SIXVERTEX, TL_LOZENGE):
        tmax = np.empty((dom.h + 1, dom.w + 1), dtype=np.int32)
    else:
        tmax = np.empty((dom.h, dom.w), dtype=np.uint8)
    tmin = np.empty_like(tmax)
    _check(lib().tl_domain_extremes(ctypes.byref(dom), tmax.ctypes.data_as(ctypes.c_void_p),
                                    tmin.ctypes.data_as(ctypes.c_void_p), tmax.nbytes))
    return tmax, tmin


def weights(kind=TL_W_UNIFORM, *w, rule=TL_HEATBATH):
    arr = (ctypes.c_double * 6)(*([float(v) for v in w] + [0.0] * (6 - len(w))))
    return tl_weights(kind, rule, arr)


def options(stream=None, obs_every=0, obs_bin=1, sweeps_per_launch=0, tile_rows=0, kernel=0, tile_groups=0,
            colour_order=0, device_buf=None, device_buf_bytes=0, tune_cache=None):
    """colour_order: 0 = colours 0..K-1 in every sweep, 1 = a random colour per step.
    device_buf: caller-owned device memory (an address, e.g. a tensor's data_ptr())
    holding the sampler's state, at least state_bytes(domain) bytes.
    tune_cache: path of the tile-shape cache of Sampler.autotune."""
    return tl_options(stream, obs_every, obs_bin, sweeps_per_launch, tile_rows, kernel, tile_groups, colour_order,
                      device_buf, device_buf_bytes,
                      None if tune_cache is None else os.fsencode(tune_cache))


def state_bytes(dom):
    """Device bytes of a sampler's state for this domain (host only)."""
    n = ctypes.c_size_t()
    _check(lib().tl_sampler_state_bytes(ctypes.byref(dom), ctypes.byref(n)))
    return n.value


def thresholds(dom: tl_domain, w: tl_weights):
    """The library's threshold table for (dom, w) (host only)."""
    cnt = ctypes.c_uint32()
    _check(lib().tl_thresholds(ctypes.byref(dom), ctypes.byref(w), None, 0, ctypes.byref(cnt)))
    buf = (ctypes.c_uint32 * max(1, cnt.value))()
    _check(lib().tl_thresholds(ctypes.byref(dom), ctypes.byref(w), buf, cnt.value, ctypes.byref(cnt)))
    return [int(v) for v in buf[:cnt.value]]


class Sampler:
    """One chain: ``tl_sampler_create`` / ``sweep`` / ``observables`` / ``export`` /
    ``hash`` / ``import_`` / ``destroy``."""

    def __init__(self, dom: tl_domain, w: tl_weights, seed: int, opt: tl_options | None = None):
        self._h = ctypes.c_void_p()
        self._opt = opt
        _check(lib().tl_sampler_create(ctypes.byref(dom), ctypes.byref(w), seed,
                                       ctypes.byref(opt) if opt is not None else None, ctypes.byref(self._h)))
        self.dom = dom
        size = ctypes.c_size_t()
        rows, rb = ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().tl_sampler_export_size(self._h, ctypes.byref(size), ctypes.byref(rows), ctypes.byref(rb)))
        self.export_bytes, self.rows, self.row_bytes = size.value, rows.value, rb.value

    @property
    def handle(self):
        return self._h

    def sweep(self, n: int):
        _check(lib().tl_sampler_sweep(self._h, n))

    def sync(self):
        _check(lib().tl_sampler_sync(self._h))

    def reset(self, seed: int):
        _check(lib().tl_sampler_reset(self._h, seed))

    def autotune(self, probe_sweeps: int = 0):
        """Pick the tiled kernel's tile shape by measurement (the chain does not
        change).  Returns {"tile_rows", "tile_groups", "sweeps_per_launch",
        "candidates", "from_cache", "ms_per_sweep", "kernel"}."""
        info = tl_tune_info()
        _check(lib().tl_sampler_autotune(self._h, int(probe_sweeps), ctypes.byref(info)))
        return {k: getattr(info, k) for k, _ in tl_tune_info._fields_}

    def cftp(self, max_log2: int = 24):
        """Exact sample by coupling from the past (raises TlError TL_EBUSY if the
        chains have not met within 2^max_log2 sweeps).  Returns
        {"log2_sweeps", "sweeps", "total_sweeps"}."""
        info = tl_cftp_info()
        _check(lib().tl_sampler_cftp(self._h, int(max_log2), ctypes.byref(info)))
        return {"log2_sweeps": info.log2_sweeps, "sweeps": info.sweeps, "total_sweeps": info.total_sweeps}

    def set_timing(self, period: int):
        """Time every `period`-th sweep launch with dispatch events (0 = off)."""
        _check(lib().tl_sampler_set_timing(self._h, int(period)))

    def kernel_time(self):
        """(total kernel ms, launches, colour steps, algorithmic bytes per colour step)."""
        ms, la, st, bp = ctypes.c_double(), ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_double()
        _check(lib().tl_sampler_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(la), ctypes.byref(st),
                                            ctypes.byref(bp)))
        return ms.value, la.value, st.value, bp.value

    def info(self):
        s, c = ctypes.c_uint64(), ctypes.c_uint32()
        _check(lib().tl_sampler_info(self._h, ctypes.byref(s), ctypes.byref(c)))
        return s.value, c.value

    def thresholds(self):
        cnt = ctypes.c_uint32()
        _check(lib().tl_sampler_thresholds(self._h, None, 0, ctypes.byref(cnt)))
        buf = (ctypes.c_uint32 * max(1, cnt.value))()
        _check(lib().tl_sampler_thresholds(self._h, buf, cnt.value, ctypes.byref(cnt)))
        return [int(v) for v in buf[:cnt.value]]

    def observables(self):
        o = tl_observables()
        _check(lib().tl_sampler_observables(self._h, ctypes.byref(o)))
        nb = o.bins_x * o.bins_y
        bs = np.zeros(nb, dtype=np.uint64)
        bn = np.zeros(nb, dtype=np.uint64)
        bd = np.zeros(nb, dtype=np.float64)
        o.bin_sum = bs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        o.bin_now = bn.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        o.bin_density = bd.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        o.bin_capacity = nb
        _check(lib().tl_sampler_observables(self._h, ctypes.byref(o)))
        shape = (o.bins_y, o.bins_x)
        return {"sweeps": o.sweeps, "samples": o.samples, "scalar_now": o.scalar_now,
                "scalar_sum": o.scalar_sum, "bin_sum": bs.reshape(shape), "bin_now": bn.reshape(shape),
                "bin_density": bd.reshape(shape)}

    def export(self) -> np.ndarray:
        buf = np.empty(self.export_bytes, dtype=np.uint8)
        t = ctypes.c_uint64()
        _check(lib().tl_sampler_export(self._h, buf.ctypes.data, buf.nbytes, ctypes.byref(t)))
        if self.dom.model == TL_DOMINO:
            return buf.reshape(self.rows, self.row_bytes)
        return buf.view(np.int32).reshape(self.rows, self.row_bytes // 4)

    def hash(self) -> str:
        d = (ctypes.c_uint8 * 32)()
        _check(lib().tl_sampler_hash(self._h, d))
        return bytes(d).hex()

    def hash_noalloc(self) -> str:
        """The canonical hash through the entry point that allocates nothing
        (static staging buffer; see tl_sampler_hash_noalloc)."""
        d = (ctypes.c_uint8 * 32)()
        _check(lib().tl_sampler_hash_noalloc(self._h, d))
        return bytes(d).hex()

    def import_(self, arr: np.ndarray, sweep: int):
        a = np.ascontiguousarray(arr)
        _check(lib().tl_sampler_import(self._h, a.ctypes.data, a.nbytes, sweep))

    def destroy(self):
        if self._h:
            lib().tl_sampler_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
