"""ctypes binding of the C ABI in include/mg_rbc.h (argument marshalling only).

Red-black coarsening multigrid for the 2D five-point Poisson problem; every numerical step
runs in the HIP library libmgmi.so.  Device arrays are raw pointers (``tensor.data_ptr()``
of FP64 CUDA tensors).  A missing library raises on first use.
"""
import ctypes

from paper_2008_03885_amd import mg

MG_RBC_NG, MG_RBC_G1, MG_RBC_GN = 0, 1, 2
MG_RBC_MAX_COARSEST = 256

_V = ctypes.c_void_p
_I = ctypes.c_int


class mg_rbc_config(ctypes.Structure):
    _fields_ = [("n", _I), ("levels", _I), ("coarse", _I), ("gamma", _I), ("nu1", _I),
                ("nu2", _I), ("omega", ctypes.c_double), ("rtol", ctypes.c_double),
                ("max_cycles", _I)]


_SIGS = {
    "mg_rbc_setup": (_I, [ctypes.POINTER(mg_rbc_config), _V, ctypes.POINTER(_V)]),
    "mg_rbc_destroy": (None, [_V]),
    "mg_rbc_level_size": (_I, [_V, _I]),
    "mg_rbc_level_pitch": (_I, [_V, _I]),
    "mg_rbc_cycles": (_I, [_V, _V, _V, _I]),
    "mg_rbc_solve": (_I, [_V, _V, _V, ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_double)]),
    "mg_rbc_residual_norm": (_I, [_V, _V, _V, ctypes.POINTER(ctypes.c_double)]),
    "mg_rbc_kernel_smooth": (_I, [_V, _I, _I, _V, _V, _V]),
    "mg_rbc_kernel_restrict": (_I, [_V, _I, _V, _V, _V]),
    "mg_rbc_kernel_prolong": (_I, [_V, _I, _V, _V, _V]),
    "mg_rbc_kernel_coarsest": (_I, [_V, _V, _V]),
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        l = mg.lib()
        for name, (res, args) in _SIGS.items():
            fn = getattr(l, name)
            fn.restype = res
            fn.argtypes = args
        _lib = l
    return _lib


def make_config(n=129, levels=2, coarse=MG_RBC_G1, gamma=1, nu1=1, nu2=1, omega=0.0, rtol=1e-10,
                max_cycles=100):
    return mg_rbc_config(n, levels, coarse, gamma, nu1, nu2, omega, rtol, max_cycles)


def _check(status, allow=(mg.MG_OK,)):
    if status not in allow:
        raise mg.MGError(status, mg.last_error())
    return status


def setup(cfg, stream=0):
    h = _V()
    _check(lib().mg_rbc_setup(ctypes.byref(cfg), _V(stream), ctypes.byref(h)))
    return h.value


def destroy(h):
    lib().mg_rbc_destroy(_V(h))


def level_size(h, level):
    return lib().mg_rbc_level_size(_V(h), int(level))


def level_pitch(h, level):
    return lib().mg_rbc_level_pitch(_V(h), int(level))


def cycles(h, f_ptr, u_ptr, count):
    _check(lib().mg_rbc_cycles(_V(h), _V(f_ptr), _V(u_ptr), int(count)))


def solve(h, f_ptr, u_ptr, max_cycles, allow=(mg.MG_OK, mg.MG_ENOCONV, mg.MG_ENUMERIC)):
    """Returns (status, cycles, residual history)."""
    k = _I()
    hist = (ctypes.c_double * (max_cycles + 1))()
    st = _check(lib().mg_rbc_solve(_V(h), _V(f_ptr), _V(u_ptr), ctypes.byref(k), hist), allow)
    return st, k.value, list(hist[:k.value + 1])


def residual_norm(h, f_ptr, u_ptr):
    out = ctypes.c_double()
    _check(lib().mg_rbc_residual_norm(_V(h), _V(f_ptr), _V(u_ptr), ctypes.byref(out)))
    return out.value


def kernel_smooth(h, level, colour, f_ptr, uin_ptr, uout_ptr):
    _check(lib().mg_rbc_kernel_smooth(_V(h), int(level), int(colour), _V(f_ptr), _V(uin_ptr),
                                      _V(uout_ptr)))


def kernel_restrict(h, level, f_ptr, u_ptr, fc_ptr):
    _check(lib().mg_rbc_kernel_restrict(_V(h), int(level), _V(f_ptr), _V(u_ptr), _V(fc_ptr)))


def kernel_prolong(h, level, ec_ptr, uin_ptr, uout_ptr):
    _check(lib().mg_rbc_kernel_prolong(_V(h), int(level), _V(ec_ptr), _V(uin_ptr), _V(uout_ptr)))


def kernel_coarsest(h, f_ptr, u_ptr):
    _check(lib().mg_rbc_kernel_coarsest(_V(h), _V(f_ptr), _V(u_ptr)))
