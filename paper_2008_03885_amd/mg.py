"""ctypes binding of the C ABI in include/mg.h (argument marshalling only).

Every numerical step runs in the HIP library libmgmi.so; this module only converts
arguments.  Device arrays are passed as raw pointers, e.g. torch tensors on the GPU
through ``tensor.data_ptr()``.  Importing this module does not touch the GPU; the
library is loaded on first use and a missing library raises at once.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmgmi.so")

MG_OK, MG_EINVAL, MG_ENOMEM, MG_EDEVICE, MG_ENOCONV, MG_ENUMERIC, MG_EBUSY = range(7)
MG_COARSE_NG, MG_COARSE_GALERKIN, MG_COARSE_NG2, MG_COARSE_G2 = 0, 1, 2, 3
MG_SMOOTH_JACOBI, MG_SMOOTH_RBJ, MG_SMOOTH_RBGS = 0, 1, 2
MG_PREC_FP64, MG_PREC_MIXED = 0, 1
MG_MAX_HISTORY = 512
STATUS_NAMES = {0: "MG_OK", 1: "MG_EINVAL", 2: "MG_ENOMEM", 3: "MG_EDEVICE", 4: "MG_ENOCONV",
                5: "MG_ENUMERIC", 6: "MG_EBUSY"}


class mg_config(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("n", ctypes.c_int), ("order", ctypes.c_int),
        ("coarse", ctypes.c_int), ("smoother", ctypes.c_int), ("omega", ctypes.c_double),
        ("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("gamma", ctypes.c_int),
        ("prolong", ctypes.c_int), ("restrict_op", ctypes.c_int), ("n_coarsest", ctypes.c_int),
        ("precision", ctypes.c_int), ("rtol", ctypes.c_double), ("max_cycles", ctypes.c_int),
        ("inner_cycles", ctypes.c_int),
    ]


class mg_result(ctypes.Structure):
    _fields_ = [
        ("cycles", ctypes.c_int), ("outer_steps", ctypes.c_int), ("status", ctypes.c_int),
        ("floor_hit", ctypes.c_int), ("rel_residual", ctypes.c_double),
        ("conv_factor", ctypes.c_double), ("history_len", ctypes.c_int),
        ("history", ctypes.c_double * MG_MAX_HISTORY),
    ]

    def hist(self):
        return [self.history[i] for i in range(self.history_len)]


class MGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


_lib = None
_V = ctypes.c_void_p
_I = ctypes.c_int
_SIGS = {
    "mg_setup": (_I, [ctypes.POINTER(mg_config), _V, ctypes.POINTER(_V)]),
    "mg_footprint_bytes": (ctypes.c_size_t, [ctypes.POINTER(mg_config)]),
    "mg_solve": (_I, [_V, _V, _V, ctypes.POINTER(mg_result)]),
    "mg_run_cycles": (_I, [_V, _V, _V, _I, ctypes.POINTER(mg_result)]),
    "mg_solve_async": (_I, [_V, _V, _V]),
    "mg_query": (_I, [_V, ctypes.POINTER(mg_result)]),
    "mg_residual_norm": (_I, [_V, _V, _V, ctypes.POINTER(ctypes.c_double)]),
    "mg_residual_norm_noalloc": (_I, [_I, _I, _I, _V, _V, _V, _V]),
    "mg_destroy": (_I, [_V]),
    "mg_last_error": (ctypes.c_char_p, []),
    "mg_level_size": (_I, [_V, _I]),
    "mg_kernel_smooth": (_I, [_V, _I, _I, _V, _V, _V]),
    "mg_kernel_smooth_colour": (_I, [_V, _I, _I, _I, _V, _V, _V]),
    "mg_kernel_residual": (_I, [_V, _I, _I, _V, _V, _V]),
    "mg_kernel_residual_restrict": (_I, [_V, _I, _I, _V, _V, _V]),
    "mg_kernel_prolong_correct": (_I, [_V, _I, _I, _V, _V, _V]),
    "mg_kernel_presmooth_restrict": (_I, [_V, _I, _I, _V, _V, _V, _V]),
    "mg_kernel_prolong_postsmooth": (_I, [_V, _I, _I, _V, _V, _V, _V]),
    "mg_kernel_coarsest_solve": (_I, [_V, _I, _V, _V]),
    "mg_level_operator": (_I, [_V, _I, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "mg_synchronize": (_I, [_V]),
}


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is missing: build it first "
                               "(python -c 'import __graft_entry__ as g; g.build()')" % LIB_PATH)
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(l, name)
            fn.restype = res
            fn.argtypes = args
        _lib = l
    return _lib


def last_error():
    return lib().mg_last_error().decode()


def _check(status, allow=(MG_OK,)):
    if status not in allow:
        raise MGError(status, last_error())
    return status


def make_config(dim=2, n=129, order=4, coarse=MG_COARSE_NG, omega=0.0, nu1=2, nu2=1, gamma=1,
                prolong=3, restrict_op=1, n_coarsest=9, precision=MG_PREC_FP64, rtol=1e-10,
                max_cycles=100, inner_cycles=4, smoother=MG_SMOOTH_JACOBI):
    return mg_config(dim, n, order, coarse, smoother, omega, nu1, nu2, gamma, prolong, restrict_op,
                     n_coarsest, precision, rtol, max_cycles, inner_cycles)


def mg_footprint_bytes(cfg):
    return lib().mg_footprint_bytes(ctypes.byref(cfg))


def mg_setup(cfg, stream=0):
    h = _V()
    _check(lib().mg_setup(ctypes.byref(cfg), _V(stream), ctypes.byref(h)))
    return h.value


def mg_solve(h, f_ptr, u_ptr, allow=(MG_OK, MG_ENOCONV, MG_ENUMERIC)):
    res = mg_result()
    st = _check(lib().mg_solve(_V(h), _V(f_ptr), _V(u_ptr), ctypes.byref(res)), allow)
    return st, res


def mg_run_cycles(h, f_ptr, u_ptr, ncycles):
    res = mg_result()
    st = _check(lib().mg_run_cycles(_V(h), _V(f_ptr), _V(u_ptr), int(ncycles), ctypes.byref(res)))
    return st, res


def mg_solve_async(h, f_ptr, u_ptr):
    _check(lib().mg_solve_async(_V(h), _V(f_ptr), _V(u_ptr)))


def mg_query(h):
    res = mg_result()
    st = lib().mg_query(_V(h), ctypes.byref(res))
    if st == MG_EBUSY:
        return st, None
    _check(st, (MG_OK, MG_ENOCONV, MG_ENUMERIC))
    return st, res


def mg_residual_norm(h, f_ptr, u_ptr):
    rel = ctypes.c_double()
    _check(lib().mg_residual_norm(_V(h), _V(f_ptr), _V(u_ptr), ctypes.byref(rel)))
    return rel.value


def mg_residual_norm_noalloc(dim, n, order, f_ptr, u_ptr, rel_ptr, stream=0):
    """Enqueues the relative residual norm into the device double at rel_ptr (no handle,
    no allocation); returns the status."""
    return _check(lib().mg_residual_norm_noalloc(int(dim), int(n), int(order), _V(f_ptr), _V(u_ptr),
                                                 _V(rel_ptr), _V(stream)))


def mg_destroy(h):
    _check(lib().mg_destroy(_V(h)))


def mg_level_size(h, level):
    return lib().mg_level_size(_V(h), int(level))


def mg_level_operator(h, level):
    a = (ctypes.c_double * 7)()
    b = (ctypes.c_double * 7)()
    _check(lib().mg_level_operator(_V(h), int(level), a, b))
    return list(a), list(b)


def mg_kernel_smooth(h, level, fp32, f_ptr, uin_ptr, uout_ptr):
    _check(lib().mg_kernel_smooth(_V(h), int(level), int(fp32), _V(f_ptr), _V(uin_ptr), _V(uout_ptr)))


def mg_kernel_smooth_colour(h, level, fp32, colour, f_ptr, uin_ptr, uout_ptr):
    _check(lib().mg_kernel_smooth_colour(_V(h), int(level), int(fp32), int(colour), _V(f_ptr),
                                         _V(uin_ptr), _V(uout_ptr)))


def mg_kernel_residual(h, level, fp32, f_ptr, u_ptr, r_ptr):
    _check(lib().mg_kernel_residual(_V(h), int(level), int(fp32), _V(f_ptr), _V(u_ptr), _V(r_ptr)))


def mg_kernel_residual_restrict(h, level, fp32, f_ptr, u_ptr, fc_ptr):
    _check(lib().mg_kernel_residual_restrict(_V(h), int(level), int(fp32), _V(f_ptr), _V(u_ptr),
                                             _V(fc_ptr)))


def mg_kernel_prolong_correct(h, level, fp32, v_ptr, uin_ptr, uout_ptr):
    _check(lib().mg_kernel_prolong_correct(_V(h), int(level), int(fp32), _V(v_ptr), _V(uin_ptr),
                                           _V(uout_ptr)))


def mg_kernel_presmooth_restrict(h, level, fp32, f_ptr, uin_ptr, uout_ptr, fc_ptr):
    _check(lib().mg_kernel_presmooth_restrict(_V(h), int(level), int(fp32), _V(f_ptr), _V(uin_ptr),
                                              _V(uout_ptr), _V(fc_ptr)))


def mg_kernel_prolong_postsmooth(h, level, fp32, v_ptr, uin_ptr, f_ptr, uout_ptr):
    _check(lib().mg_kernel_prolong_postsmooth(_V(h), int(level), int(fp32), _V(v_ptr), _V(uin_ptr),
                                              _V(f_ptr), _V(uout_ptr)))


def mg_kernel_coarsest_solve(h, fp32, g_ptr, v_ptr):
    _check(lib().mg_kernel_coarsest_solve(_V(h), int(fp32), _V(g_ptr), _V(v_ptr)))


def mg_synchronize(h):
    _check(lib().mg_synchronize(_V(h)))


class Solver:
    """A handle bound to torch's current HIP stream; f and u are torch tensors of shape
    (n,)*dim, float64, on the GPU."""

    def __init__(self, **cfg_kwargs):
        import torch
        self.cfg = make_config(**cfg_kwargs)
        self.stream = torch.cuda.current_stream().cuda_stream
        self.h = mg_setup(self.cfg, self.stream)

    def _ptrs(self, f, u):
        import torch
        for t in (f, u):
            assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
            assert tuple(t.shape) == (self.cfg.n,) * self.cfg.dim
        return f.data_ptr(), u.data_ptr()

    def solve(self, f, u):
        return mg_solve(self.h, *self._ptrs(f, u))

    def run_cycles(self, f, u, k):
        return mg_run_cycles(self.h, *self._ptrs(f, u), k)

    def residual_norm(self, f, u):
        return mg_residual_norm(self.h, *self._ptrs(f, u))

    def close(self):
        if self.h:
            mg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
