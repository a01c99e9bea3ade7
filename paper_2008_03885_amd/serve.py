"""ctypes binding of the solve server in include/mg_serve.h (argument marshalling only).

The server, its worker thread, admission and batching live in libmgmi.so; this module
converts arguments and keeps the caller's device tensors alive until their request
completes.
"""
import ctypes

from . import mg

_LL, _I, _D, _V, _SZ = ctypes.c_longlong, ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t


class mg_server_config(ctypes.Structure):
    _fields_ = [("base", mg.mg_config), ("hbm_budget", _SZ), ("max_slots", _I), ("chunk_steps", _I),
                ("stream_groups", _I)]


class mg_completion(ctypes.Structure):
    _fields_ = [("tag", _LL), ("n", _I), ("status", _I), ("t_submit", _D), ("t_admit", _D),
                ("t_done", _D), ("result", mg.mg_result)]


class mg_server_stats(ctypes.Structure):
    _fields_ = [("submitted", _LL), ("completed", _LL), ("rejected", _LL), ("queued", _I),
                ("active", _I), ("peak_active", _I), ("batches", _I), ("batches_created", _LL),
                ("batches_released", _LL), ("bytes_held", _SZ), ("peak_bytes_held", _SZ),
                ("replays", _LL)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_SIGS = {
    "mg_serve_batch_bytes": (_SZ, [ctypes.POINTER(mg.mg_config), _I, _I]),
    "mg_server_create": (_I, [ctypes.POINTER(mg_server_config), ctypes.POINTER(_V)]),
    "mg_server_submit": (_I, [_V, _LL, _I, _V, _V]),
    "mg_server_poll": (_I, [_V, ctypes.POINTER(mg_completion), _I, _D]),
    "mg_server_stats_get": (_I, [_V, ctypes.POINTER(mg_server_stats)]),
    "mg_server_destroy": (_I, [_V]),
    "mg_server_clock": (_D, []),
}
_bound = False


def lib():
    global _bound
    L = mg.lib()
    if not _bound:
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _bound = True
    return L


def mg_serve_batch_bytes(base, n, slots):
    return lib().mg_serve_batch_bytes(ctypes.byref(base), n, slots)


def mg_server_clock():
    return lib().mg_server_clock()


def make_server_config(hbm_budget, max_slots=16, chunk_steps=2, stream_groups=0, **base_kwargs):
    base_kwargs.setdefault("dim", 2)
    base_kwargs.setdefault("n", 65)
    return mg_server_config(base=mg.make_config(**base_kwargs), hbm_budget=int(hbm_budget),
                            max_slots=max_slots, chunk_steps=chunk_steps, stream_groups=stream_groups)


def mg_server_create(cfg):
    h = _V()
    st = lib().mg_server_create(ctypes.byref(cfg), ctypes.byref(h))
    if st != mg.MG_OK:
        raise mg.MGError(st, mg.last_error() or "mg_server_create failed")
    return h.value


def mg_server_submit(s, tag, n, f_ptr, u_ptr):
    return lib().mg_server_submit(_V(s), tag, n, _V(f_ptr), _V(u_ptr))


def mg_server_poll(s, max_items=64, timeout_s=0.0):
    buf = (mg_completion * max_items)()
    k = lib().mg_server_poll(_V(s), buf, max_items, float(timeout_s))
    if k < 0:
        raise mg.MGError(-k, mg.last_error() or "server failure")
    return [buf[i] for i in range(k)]


def mg_server_stats_get(s):
    st = mg_server_stats()
    mg._check(lib().mg_server_stats_get(_V(s), ctypes.byref(st)))
    return st.as_dict()


def mg_server_destroy(s):
    mg._check(lib().mg_server_destroy(_V(s)))


class Server:
    """A server on the current device.  submit(tag, f, u) takes float64 CUDA tensors of
    shape (n, n) and holds them until the request completes; poll() returns completions."""

    def __init__(self, hbm_budget, max_slots=16, chunk_steps=2, stream_groups=0, **base_kwargs):
        import torch
        torch.cuda.init()  # torch owns the device set-up; the server runs on its current device
        self.cfg = make_server_config(hbm_budget, max_slots, chunk_steps, stream_groups, **base_kwargs)
        self.h = mg_server_create(self.cfg)
        self._live = {}

    def submit(self, tag, f, u):
        import torch
        for t in (f, u):
            assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.dim() == 2
        assert f.shape == u.shape and f.shape[0] == f.shape[1]
        st = mg_server_submit(self.h, tag, f.shape[0], f.data_ptr(), u.data_ptr())
        if st == mg.MG_OK:
            self._live[tag] = (f, u)
        return st

    def poll(self, max_items=64, timeout_s=0.0):
        out = mg_server_poll(self.h, max_items, timeout_s)
        for c in out:
            self._live.pop(c.tag, None)
        return out

    def wait_all(self, count, timeout_s=120.0):
        """Polls until `count` completions arrived (raises on timeout)."""
        import time
        got, t_end = [], time.monotonic() + timeout_s
        while len(got) < count:
            left = t_end - time.monotonic()
            if left <= 0:
                raise TimeoutError("%d of %d requests completed" % (len(got), count))
            got += self.poll(64, min(left, 1.0))
        return got

    def stats(self):
        return mg_server_stats_get(self.h)

    def close(self):
        if self.h:
            mg_server_destroy(self.h)
            self.h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
