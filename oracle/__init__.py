"""Plain FP64 CPU oracle for the multigrid hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the GPU library and the GPU library never
imports it.

Contents
  ``mg_oracle.c``  plain C multigrid (operators, transfers, Galerkin stencils, cycles);
                   bound here through ctypes.
  ``lfa.py``       local Fourier analysis from the paper's symbols (section 2.2,
                   appendices A.2 and A.4, section 5.3).
  ``dst.py``       exact discrete solve by sine transforms (eigenvalues from the
                   appendix A.4 symbol) and manufactured-solution helpers.
  ``explicit.py``  explicit sparse matrices of every operator on tiny grids
                   (brute-force R*A*P and cycle iteration matrices).

Arrays are numpy float64, shape (n, n) or (n, n, n), index [z][y][x] (x fastest),
including the boundary points.  Stencils are arrays of shape (2R+1,)*dim indexed
[oz+R][oy+R][ox+R].
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mg_oracle.c")
_LIB = os.path.join(_HERE, "libmgoracle.so")

RESTRICT_FW, RESTRICT_CUBIC = 1, 3
PROLONG_LINEAR, PROLONG_CUBIC = 1, 3
COARSE_NG, COARSE_GALERKIN = 0, 1
# second-order coarse operators for a fourth-order fine operator (section 3.1):
# rediscretized (eq. L_H_2d) and "Galerkin" from the second-order operator (eq. L_H_2G_2d)
COARSE_NG2, COARSE_G2 = 2, 3
# smoothers: omega-Jacobi (section 5.3), omega red-black Jacobi (section 3.1 eq. S_rb with
# the Jacobi partial step; red = odd index sum) and omega red-black Gauss-Seidel (eqs. S_rb,
# S_GS: the partial step sweeps its colour in lexicographic order)
SMOOTH_JACOBI, SMOOTH_RBJ, SMOOTH_RBGS = 0, 1, 2
MAX_RADIUS = 6


def build(force=True):
    """Compile mg_oracle.c with gcc (plain -O3, no FMA contraction, OpenMP loops)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wno-aggressive-loop-optimizations", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd, cwd=_HERE)
    os.replace(tmp, _LIB)
    return _LIB


class _Config(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int), ("order", ctypes.c_int),
                ("coarse", ctypes.c_int), ("restrict_op", ctypes.c_int), ("prolong", ctypes.c_int),
                ("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("gamma", ctypes.c_int),
                ("n_coarsest", ctypes.c_int), ("omega", ctypes.c_double), ("smoother", ctypes.c_int)]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.c_int


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        sig = {
            "or_num_levels": (_I, [_I, _I]),
            "or_fine_stencil": (_I, [_I, _I, ctypes.c_double, _D]),
            "or_galerkin_stencil": (_I, [_I, _I, _D, _I, _I, _D]),
            "or_apply": (None, [_I, _I, _I, _D, _D, _D]),
            "or_residual": (None, [_I, _I, _I, _D, _D, _D, _D]),
            "or_jacobi": (None, [_I, _I, _I, _D, ctypes.c_double, _D, _D, _D]),
            "or_jacobi_colour": (None, [_I, _I, _I, _D, ctypes.c_double, _I, _D, _D, _D]),
            "or_gs_colour": (None, [_I, _I, _I, _D, ctypes.c_double, _I, _D, _D, _D]),
            "or_restrict": (None, [_I, _I, _I, _D, _D]),
            "or_prolong_add": (None, [_I, _I, _I, _D, _D]),
            "or_norm": (ctypes.c_double, [_I, _I, _D]),
            "or_residual_norm_ld": (ctypes.c_double, [_I, _I, _I, _D, _D, _D]),
            "or_mg_create": (ctypes.c_void_p, [ctypes.POINTER(_Config)]),
            "or_mg_destroy": (None, [ctypes.c_void_p]),
            "or_mg_levels": (_I, [ctypes.c_void_p]),
            "or_mg_level_stencil": (_I, [ctypes.c_void_p, _I, ctypes.POINTER(_I), _D]),
            "or_mg_cycle": (None, [ctypes.c_void_p, _D, _D]),
            "or_mg_coarsest_solve": (None, [ctypes.c_void_p, _D, _D]),
            "or_mg_solve": (_I, [ctypes.c_void_p, _D, _D, ctypes.c_double, _I, _D]),
            "or_num_threads": (_I, []),
            "or_set_num_threads": (None, [_I]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _p(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _grid_dim(a):
    n = a.shape[0]
    assert all(s == n for s in a.shape) and a.ndim in (2, 3), a.shape
    return a.ndim, n


def _stencil_radius(s):
    return (s.shape[0] - 1) // 2


def num_threads():
    return _load().or_num_threads()


def set_num_threads(threads):
    """OpenMP threads of the oracle's outer loops (3D grids; 2D loops run on one thread)."""
    _load().or_set_num_threads(int(threads))


def num_levels(n, n_coarsest=9):
    return _load().or_num_levels(n, n_coarsest)


def fine_stencil(dim, order, h):
    R = order // 2
    s = np.zeros((2 * R + 1,) * dim)
    _load().or_fine_stencil(dim, order, h, _p(s))
    return s


def galerkin_stencil(s_fine, restrict_op=RESTRICT_FW, prolong=PROLONG_CUBIC):
    dim = s_fine.ndim
    sf = np.ascontiguousarray(s_fine, dtype=np.float64)
    buf = np.zeros((2 * MAX_RADIUS + 1) ** dim)
    Rc = _load().or_galerkin_stencil(dim, _stencil_radius(sf), _p(sf), restrict_op, prolong, _p(buf))
    return buf[: (2 * Rc + 1) ** dim].reshape((2 * Rc + 1,) * dim).copy()


def apply(s, u):
    dim, n = _grid_dim(u)
    out = np.empty_like(u)
    s = np.ascontiguousarray(s, dtype=np.float64)
    _load().or_apply(dim, n, _stencil_radius(s), _p(s), _p(u), _p(out))
    return out


def residual(s, f, u):
    dim, n = _grid_dim(u)
    out = np.empty_like(u)
    s = np.ascontiguousarray(s, dtype=np.float64)
    _load().or_residual(dim, n, _stencil_radius(s), _p(s), _p(f), _p(u), _p(out))
    return out


def jacobi(s, omega, f, u):
    dim, n = _grid_dim(u)
    out = np.empty_like(u)
    s = np.ascontiguousarray(s, dtype=np.float64)
    _load().or_jacobi(dim, n, _stencil_radius(s), _p(s), float(omega), _p(f), _p(u), _p(out))
    return out


def jacobi_colour(s, omega, colour, f, u):
    """One partial step on colour 1 (odd index sum), 2 (even) or 0 (every point)."""
    dim, n = _grid_dim(u)
    out = np.empty_like(u)
    s = np.ascontiguousarray(s, dtype=np.float64)
    _load().or_jacobi_colour(dim, n, _stencil_radius(s), _p(s), float(omega), int(colour), _p(f),
                             _p(u), _p(out))
    return out


def gs_colour(s, omega, colour, f, u):
    """One Gauss-Seidel partial step (section 3.1 eq. S_GS) on colour 1 (odd index sum),
    2 (even) or 0 (every point): the colour's points in lexicographic order, in place."""
    dim, n = _grid_dim(u)
    out = np.empty_like(u)
    s = np.ascontiguousarray(s, dtype=np.float64)
    _load().or_gs_colour(dim, n, _stencil_radius(s), _p(s), float(omega), int(colour), _p(f),
                         _p(u), _p(out))
    return out


def restrict(d, restrict_op=RESTRICT_FW):
    dim, nf = _grid_dim(d)
    nc = (nf - 1) // 2 + 1
    out = np.zeros((nc,) * dim)
    _load().or_restrict(dim, nf, restrict_op, _p(d), _p(out))
    return out


def prolong_add(v, u, prolong=PROLONG_CUBIC):
    """u += I_H^h v (in place); returns u."""
    dim, nf = _grid_dim(u)
    assert v.shape[0] == (nf - 1) // 2 + 1
    _load().or_prolong_add(dim, nf, prolong, _p(v), _p(u))
    return u


def norm(v):
    dim, n = _grid_dim(v)
    return _load().or_norm(dim, n, _p(v))


def residual_norm_ld(s, f, u):
    dim, n = _grid_dim(u)
    s = np.ascontiguousarray(s, dtype=np.float64)
    return _load().or_residual_norm_ld(dim, n, _stencil_radius(s), _p(s), _p(f), _p(u))


def jacobi_omega_star(dim):
    """Closed-form omega* of omega-Jacobi for the fourth-order operator (derivation in
    lfa.jacobi_optimum): 10/13 in 2D, 9/11 in 3D."""
    return {2: 10.0 / 13.0, 3: 9.0 / 11.0}[dim]


def jacobi_omega(dim, order=4):
    """omega* of omega-Jacobi for every order: second order 4/5, 6/7 (section 5.3);
    fourth order 10/13, 9/11; sixth order 490/653, 147/185 (lfa.jacobi_optimum)."""
    return {2: {2: 4.0 / 5.0, 3: 6.0 / 7.0}, 4: {2: 10.0 / 13.0, 3: 9.0 / 11.0},
            6: {2: 490.0 / 653.0, 3: 147.0 / 185.0}}[order][dim]


def rbgs_omega(dim, order=4, coarse=COARSE_NG):
    """Default omega of red-black Gauss-Seidel (2D): the minimiser of the LFA two-grid factor
    of the V(2,1) cycle with cubic interpolation, to two decimals, per fine order and coarse
    operator (rediscretized, or the second-order rediscretized one)."""
    table = {(4, COARSE_NG): 1.16, (4, COARSE_NG2): 0.98, (6, COARSE_NG): 1.18, (6, COARSE_NG2): 1.0,
             (2, COARSE_NG): 1.0, (2, COARSE_NG2): 1.0}
    assert dim == 2
    return table[(order, coarse)]


def rbj_omega(dim, order=4, coarse=COARSE_NG):
    """Default omega of red-black Jacobi: the minimiser of the LFA two-grid factor of the
    V(2,1) cycle with cubic interpolation, to two decimals, per (dim, fine order, coarse
    operator)."""
    table = {
        (2, 4): (1.13, 1.0, 0.98, 0.97), (2, 6): (1.13, 1.02, 0.99, 0.99), (2, 2): (1.0, 0.98, 1.0, 0.98),
        (3, 4): (1.17, 1.09, 1.09, 1.08), (3, 6): (1.15, 1.1, 1.09, 1.08), (3, 2): (1.13, 1.09, 1.13, 1.09),
    }
    return table[(dim, order)][coarse]


class Multigrid:
    """The (lmax+1)-level gamma-cycle of section 2.2 on the CPU, in FP64."""

    def __init__(self, dim, n, order=4, coarse=COARSE_NG, restrict_op=RESTRICT_FW,
                 prolong=PROLONG_CUBIC, nu1=2, nu2=1, gamma=1, n_coarsest=9, omega=None,
                 smoother=SMOOTH_JACOBI):
        if omega is None:
            omega = (jacobi_omega(dim, order) if smoother == SMOOTH_JACOBI else
                     {SMOOTH_RBJ: rbj_omega, SMOOTH_RBGS: rbgs_omega}[smoother](dim, order, coarse))
        self.cfg = _Config(dim, n, order, coarse, restrict_op, prolong, nu1, nu2, gamma,
                           n_coarsest, float(omega), smoother)
        self.dim, self.n = dim, n
        self._h = _load().or_mg_create(ctypes.byref(self.cfg))
        if not self._h:
            raise ValueError("invalid multigrid configuration")

    def close(self):
        if self._h:
            _load().or_mg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def levels(self):
        return _load().or_mg_levels(self._h)

    def level_stencil(self, l):
        buf = np.zeros((2 * MAX_RADIUS + 1) ** self.dim)
        n = ctypes.c_int()
        R = _load().or_mg_level_stencil(self._h, l, ctypes.byref(n), _p(buf))
        return n.value, buf[: (2 * R + 1) ** self.dim].reshape((2 * R + 1,) * self.dim).copy()

    def cycle(self, u, f):
        _load().or_mg_cycle(self._h, _p(u), _p(f))
        return u

    def coarsest_solve(self, g):
        v = np.zeros_like(g)
        _load().or_mg_coarsest_solve(self._h, _p(g), _p(v))
        return v

    def solve(self, u, f, rtol=1e-10, max_cycles=100):
        """Cycles until the relative residual is <= rtol; returns (cycles, history)."""
        hist = np.zeros(max_cycles + 1)
        c = _load().or_mg_solve(self._h, _p(u), _p(f), float(rtol), int(max_cycles), _p(hist))
        return c, hist[: c + 1].copy()
