"""Python binding of the batched and served forms (tl_batch_*, tl_server_*).

Argument marshalling only; the batched kernel, the scheduler thread and all
device work live in libtilings.so.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import TL_EBUSY, TL_OK, TlError, _check, lib, tl_domain, tl_options, tl_weights


class tl_result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int32), ("sweeps", ctypes.c_uint64),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_done", ctypes.c_double),
                ("hash", ctypes.c_uint8 * 32), ("scalar_now", ctypes.c_int64)]


class tl_server_counters(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_uint64), ("active", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("bytes_in_use", ctypes.c_uint64), ("peak_bytes", ctypes.c_uint64),
                ("peak_active", ctypes.c_uint32)]


_bound = False


def _bind():
    global _bound
    if _bound:
        return lib()
    L = lib()
    vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32
    sigs = {
        "tl_batch_create": [i32, ctypes.POINTER(tl_domain), ctypes.POINTER(tl_weights), ctypes.POINTER(u64),
                            ctypes.POINTER(tl_options), ctypes.POINTER(vp)],
        "tl_batch_autotune": [vp, u32, ctypes.POINTER(u32), ctypes.POINTER(ctypes.c_float)],
        "tl_batch_sweep": [vp, u64],
        "tl_batch_sync": [vp],
        "tl_batch_reset": [vp],
        "tl_batch_info": [vp, ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(u32), ctypes.POINTER(u32)],
        "tl_batch_set_timing": [vp, i32],
        "tl_batch_kernel_time": [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(u64), ctypes.POINTER(u64)],
        "tl_batch_export_size": [vp, i32, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(u32), ctypes.POINTER(u32)],
        "tl_batch_export": [vp, i32, vp, ctypes.c_size_t],
        "tl_batch_hash": [vp, i32, ctypes.POINTER(ctypes.c_uint8)],
        "tl_batch_destroy": [vp],
        "tl_server_create": [ctypes.c_size_t, i32, ctypes.POINTER(tl_options), ctypes.POINTER(vp)],
        "tl_server_submit": [vp, ctypes.POINTER(tl_domain), ctypes.POINTER(tl_weights), u64, u64,
                             ctypes.POINTER(u64)],
        "tl_server_poll": [vp, u64, ctypes.POINTER(tl_result)],
        "tl_server_wait": [vp, u64, ctypes.c_double, ctypes.POINTER(tl_result)],
        "tl_server_stats": [vp, ctypes.POINTER(tl_server_counters)],
        "tl_server_destroy": [vp],
    }
    for name, args in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = i32
    _bound = True
    return L


class Batch:
    """Independent domino chains advanced together (tl_batch_*)."""

    def __init__(self, doms, w: tl_weights, seeds, opt: tl_options | None = None):
        L = _bind()
        n = len(doms)
        self.n = n
        self._doms = list(doms)   # keeps mask bytes alive until the library has copied them
        arr = (tl_domain * n)(*doms)
        sd = (ctypes.c_uint64 * n)(*[int(s) for s in seeds])
        self._h = ctypes.c_void_p()
        _check(L.tl_batch_create(n, arr, ctypes.byref(w), sd, ctypes.byref(opt) if opt is not None else None,
                                 ctypes.byref(self._h)))

    def autotune(self, probe_sweeps=2):
        th, ms = ctypes.c_uint32(), ctypes.c_float()
        _check(_bind().tl_batch_autotune(self._h, probe_sweeps, ctypes.byref(th), ctypes.byref(ms)))
        return th.value, ms.value

    def sweep(self, n):
        _check(_bind().tl_batch_sweep(self._h, n))

    def sync(self):
        _check(_bind().tl_batch_sync(self._h))

    def reset(self):
        _check(_bind().tl_batch_reset(self._h))

    def info(self):
        s, b, th, wg = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_uint32()
        _check(_bind().tl_batch_info(self._h, ctypes.byref(s), ctypes.byref(b), ctypes.byref(th), ctypes.byref(wg)))
        return {"sites": s.value, "state_bytes": b.value, "threads": th.value, "workgroups": wg.value}

    def set_timing(self, on):
        _check(_bind().tl_batch_set_timing(self._h, int(on)))

    def kernel_time(self):
        ms, la, st = ctypes.c_double(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(_bind().tl_batch_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(la), ctypes.byref(st)))
        return ms.value, la.value, st.value

    def export(self, chain):
        """Canonical export of one chain: the diamond's 2n x 2n box, or the
        mask's h x w box."""
        size, rows, rb = ctypes.c_size_t(), ctypes.c_uint32(), ctypes.c_uint32()
        _check(_bind().tl_batch_export_size(self._h, chain, ctypes.byref(size), ctypes.byref(rows), ctypes.byref(rb)))
        buf = np.empty((rows.value, rb.value), dtype=np.uint8)
        _check(_bind().tl_batch_export(self._h, chain, buf.ctypes.data, buf.nbytes))
        return buf

    def hash(self, chain):
        d = (ctypes.c_uint8 * 32)()
        _check(_bind().tl_batch_hash(self._h, chain, d))
        return bytes(d).hex()

    def destroy(self):
        if self._h:
            _bind().tl_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Server:
    """Continuous-batching request loop (tl_server_*)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int, opt: tl_options | None = None):
        L = _bind()
        self._h = ctypes.c_void_p()
        _check(L.tl_server_create(hbm_budget_bytes, max_slots, ctypes.byref(opt) if opt is not None else None,
                                  ctypes.byref(self._h)))

    def submit(self, dom: tl_domain, w: tl_weights, seed: int, n_sweeps: int) -> int:
        t = ctypes.c_uint64()
        _check(_bind().tl_server_submit(self._h, ctypes.byref(dom), ctypes.byref(w), seed, n_sweeps,
                                        ctypes.byref(t)))
        return t.value

    @staticmethod
    def _res(r):
        return {"ticket": r.ticket, "status": r.status, "sweeps": r.sweeps, "t_submit": r.t_submit,
                "t_start": r.t_start, "t_done": r.t_done, "hash": bytes(r.hash).hex(), "scalar_now": r.scalar_now}

    def poll(self, ticket):
        r = tl_result()
        st = _bind().tl_server_poll(self._h, ticket, ctypes.byref(r))
        if st == TL_EBUSY:
            return None
        _check(st)
        return self._res(r)

    def wait(self, ticket, timeout_s=600.0):
        r = tl_result()
        st = _bind().tl_server_wait(self._h, ticket, timeout_s, ctypes.byref(r))
        if st == TL_EBUSY:
            raise TimeoutError("job %d not done after %.1f s" % (ticket, timeout_s))
        _check(st)
        return self._res(r)

    def stats(self):
        c = tl_server_counters()
        _check(_bind().tl_server_stats(self._h, ctypes.byref(c)))
        return {k: getattr(c, k) for k, _ in tl_server_counters._fields_}

    def destroy(self):
        if self._h:
            _bind().tl_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


__all__ = ["Batch", "Server", "TL_OK", "TlError"]
