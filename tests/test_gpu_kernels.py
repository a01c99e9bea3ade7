"""Each hot-path kernel against the oracle's same step, element by element (GPU).

FP64 tolerances: the kernels evaluate the same sums in another order (difference form,
fused multiply-adds), so results differ by a few units in the last place of the
largest term; the bounds below are 1e-13 of that scale.  FP32 kernels are compared with
the FP64 oracle applied to the same FP32-rounded inputs, to 2e-5 of the scale.
"""
import numpy as np
import pytest

import oracle
import blocks
from gpu_util import Handle, assert_close, dev, host, rand_grid, stream, torch
from paper_2008_03885_amd import inputs, mg

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-13, 2e-5

# (dim, finest n, coarse, prolong, level): level sides cover single-block grids,
# ragged last blocks (257, 1025 vs 252/250-column blocks) and the Galerkin kernels.
CASES_2D = [
    (2, 9, 0, 3, 0), (2, 17, 0, 3, 0), (2, 65, 0, 3, 0), (2, 257, 0, 3, 0), (2, 1025, 0, 3, 0),
    (2, 1025, 0, 3, 2), (2, 257, 1, 3, 1), (2, 257, 1, 3, 2), (2, 1025, 1, 3, 1),
    (2, 513, 1, 1, 1), (2, 513, 1, 1, 2),
    # second-order coarse operators (section 3.1): rediscretized and "Galerkin"
    (2, 257, 2, 3, 1), (2, 257, 3, 3, 1), (2, 257, 3, 3, 2), (2, 513, 3, 1, 1),
]


def _scale_u(u, f, s):
    R = (s.shape[0] - 1) // 2
    return np.abs(u).max() + np.abs(f).max() / s[(R,) * s.ndim]


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("dim,n,coarse,prolong,level", CASES_2D)
def test_smooth(dim, n, coarse, prolong, level, fp32):
    H = Handle(dim, n, coarse=coarse, prolong=prolong)
    try:
        n_l, s = H.level(level)
        u = rand_grid(n_l, dim, 1)
        f = rand_grid(n_l, dim, 2) * s[(s.shape[0] // 2,) * dim]
        if fp32:
            u, f = u.astype(np.float32).astype(np.float64), f.astype(np.float32).astype(np.float64)
        ud, fd = dev(u, fp32), dev(f, fp32)
        out = dev(np.full_like(u, np.nan), fp32)
        mg.mg_kernel_smooth(H.h, level, fp32, fd.data_ptr(), ud.data_ptr(), out.data_ptr())
        ref = oracle.jacobi(s, H.omega, f, u)
        assert_close(host(out), ref, (TOL32 if fp32 else TOL64) * _scale_u(u, f, s), "smooth")
        # zero initial guess (u_in = NULL)
        mg.mg_kernel_smooth(H.h, level, fp32, fd.data_ptr(), None, out.data_ptr())
        ref0 = oracle.jacobi(s, H.omega, f, np.zeros_like(u))
        assert_close(host(out), ref0, (TOL32 if fp32 else TOL64) * _scale_u(u, f, s), "smooth0")
    finally:
        H.close()


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("dim,n,coarse,prolong,level", CASES_2D)
def test_residual(dim, n, coarse, prolong, level, fp32):
    H = Handle(dim, n, coarse=coarse, prolong=prolong)
    try:
        n_l, s = H.level(level)
        d = s[(s.shape[0] // 2,) * dim]
        u = rand_grid(n_l, dim, 3)
        f = rand_grid(n_l, dim, 4) * d
        if fp32:
            u, f = u.astype(np.float32).astype(np.float64), f.astype(np.float32).astype(np.float64)
        out = dev(np.full_like(u, np.nan), fp32)
        fd, ud = dev(f, fp32), dev(u, fp32)  # keep the tensors alive across the launch
        mg.mg_kernel_residual(H.h, level, fp32, fd.data_ptr(), ud.data_ptr(), out.data_ptr())
        ref = oracle.residual(s, f, u)
        scale = np.abs(f).max() + d * np.abs(u).max()
        assert_close(host(out), ref, (TOL32 if fp32 else TOL64) * scale * 4, "residual")
    finally:
        H.close()


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("dim,n,coarse,prolong,level", [c for c in CASES_2D if c[1] > 9])
def test_residual_restrict(dim, n, coarse, prolong, level, fp32):
    H = Handle(dim, n, coarse=coarse, prolong=prolong)
    try:
        n_l, s = H.level(level)
        if level >= H.oracle.levels - 1:
            pytest.skip("coarsest level has no coarser level")
        d = s[(s.shape[0] // 2,) * dim]
        u = rand_grid(n_l, dim, 5)
        f = rand_grid(n_l, dim, 6) * d
        if fp32:
            u, f = u.astype(np.float32).astype(np.float64), f.astype(np.float32).astype(np.float64)
        nc = (n_l - 1) // 2 + 1
        out = dev(np.full((nc,) * dim, np.nan), fp32)
        fd, ud = dev(f, fp32), dev(u, fp32)
        mg.mg_kernel_residual_restrict(H.h, level, fp32, fd.data_ptr(), ud.data_ptr(), out.data_ptr())
        ref = oracle.restrict(oracle.residual(s, f, u))
        scale = np.abs(f).max() + d * np.abs(u).max()
        assert_close(host(out), ref, (TOL32 if fp32 else TOL64) * scale * 4, "resid_restrict")
    finally:
        H.close()


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("dim,n,coarse,prolong,level", [c for c in CASES_2D if c[1] > 9])
def test_prolong_correct(dim, n, coarse, prolong, level, fp32):
    H = Handle(dim, n, coarse=coarse, prolong=prolong)
    try:
        n_l, s = H.level(level)
        if level >= H.oracle.levels - 1:
            pytest.skip("coarsest level has no coarser level")
        nc = (n_l - 1) // 2 + 1
        u = rand_grid(n_l, dim, 7)
        v = rand_grid(nc, dim, 8)
        if fp32:
            u, v = u.astype(np.float32).astype(np.float64), v.astype(np.float32).astype(np.float64)
        ud, vd = dev(u, fp32), dev(v, fp32)
        out = dev(np.full_like(u, np.nan), fp32)
        mg.mg_kernel_prolong_correct(H.h, level, fp32, vd.data_ptr(), ud.data_ptr(), out.data_ptr())
        ref = oracle.prolong_add(v, u.copy(), prolong)
        scale = np.abs(u).max() + 2 * np.abs(v).max()
        assert_close(host(out), ref, (TOL32 if fp32 else TOL64) * scale, "prolong")
        # in place
        mg.mg_kernel_prolong_correct(H.h, level, fp32, vd.data_ptr(), ud.data_ptr(), ud.data_ptr())
        assert_close(host(ud), ref, (TOL32 if fp32 else TOL64) * scale, "prolong in place")
    finally:
        H.close()


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("dim,coarse,prolong", [(2, 0, 3), (2, 1, 3), (2, 1, 1)])
def test_coarsest_solve(dim, coarse, prolong, fp32):
    H = Handle(dim, 65 if dim == 2 else 33, coarse=coarse, prolong=prolong)
    try:
        L = H.oracle.levels
        n_c, s = H.level(L - 1)
        g = rand_grid(n_c, dim, 9)
        if fp32:
            g = g.astype(np.float32).astype(np.float64)
        out = dev(np.full_like(g, np.nan), fp32)
        gd = dev(g, fp32)
        mg.mg_kernel_coarsest_solve(H.h, fp32, gd.data_ptr(), out.data_ptr())
        ref = H.oracle.coarsest_solve(g)
        tol = (1e-6 if fp32 else 1e-12) * np.abs(ref).max()
        assert_close(host(out), ref, tol, "coarsest")
    finally:
        H.close()


def test_level_operators_match_oracle_stencils():
    """The library's 1D-factor Galerkin recursion reproduces the oracle's coarse stencils
    (built by the definition R*L*P on the infinite grid)."""
    for coarse, prolong in ((0, 3), (1, 3), (1, 1), (2, 3), (3, 3), (3, 1)):
        H = Handle(2, 257, coarse=coarse, prolong=prolong)
        try:
            for l in range(H.oracle.levels):
                _, s = H.level(l)
                a, b = mg.mg_level_operator(H.h, l)
                a, b = np.array(a), np.array(b)
                dense = np.outer(b, a) + np.outer(a, b)  # [y][x]
                R = (s.shape[0] - 1) // 2
                full = np.zeros((7, 7))
                full[3 - R:4 + R, 3 - R:4 + R] = s
                assert np.abs(dense - full).max() <= 1e-12 * np.abs(full).max()
        finally:
            H.close()


def test_full_size_sweep_4097():
    """Level-0 sweep and residual at the benchmark size, every element."""
    n = 4097
    H = Handle(2, n)
    try:
        _, s = H.level(0)
        u = rand_grid(n, 2, 11)
        f = rand_grid(n, 2, 12) * s[2, 2]
        out = dev(np.full_like(u, np.nan))
        ud, fd = dev(u), dev(f)
        mg.mg_kernel_smooth(H.h, 0, 0, fd.data_ptr(), ud.data_ptr(), out.data_ptr())
        assert_close(host(out), oracle.jacobi(s, H.omega, f, u), TOL64 * _scale_u(u, f, s), "sweep")
        nc = (n - 1) // 2 + 1
        fc = dev(np.full((nc, nc), np.nan))
        mg.mg_kernel_residual_restrict(H.h, 0, 0, fd.data_ptr(), ud.data_ptr(), fc.data_ptr())
        ref = oracle.restrict(oracle.residual(s, f, u))
        assert_close(host(fc), ref, TOL64 * 4 * (np.abs(f).max() + s[2, 2] * np.abs(u).max()), "rr")
        v = rand_grid(nc, 2, 13)
        vd = dev(v)
        mg.mg_kernel_prolong_correct(H.h, 0, 0, vd.data_ptr(), ud.data_ptr(), out.data_ptr())
        ref = oracle.prolong_add(v, u.copy(), 3)
        assert_close(host(out), ref, TOL64 * (np.abs(u).max() + 2 * np.abs(v).max()), "prolong")
    finally:
        H.close()


def test_kernels_are_deterministic():
    n = 1025
    H = Handle(2, n, coarse=1)
    try:
        u, f = dev(rand_grid(n, 2, 14)), dev(rand_grid(n, 2, 15))
        a, b = dev(np.zeros((n, n))), dev(np.zeros((n, n)))
        for out in (a, b):
            mg.mg_kernel_smooth(H.h, 0, 0, f.data_ptr(), u.data_ptr(), out.data_ptr())
        assert np.array_equal(host(a), host(b))
    finally:
        H.close()


FUSED_CASES = [
    # dim, n, coarse, prolong, level, nu1, nu2
    (2, 17, 0, 3, 0, 2, 1), (2, 65, 0, 3, 0, 2, 1), (2, 257, 0, 3, 0, 2, 1), (2, 1025, 0, 3, 0, 2, 1),
    (2, 257, 0, 3, 1, 0, 1), (2, 257, 0, 3, 0, 1, 2), (2, 257, 0, 1, 0, 3, 2), (2, 129, 0, 3, 0, 3, 0),
    (2, 257, 1, 3, 1, 2, 1), (2, 513, 1, 3, 2, 2, 2), (2, 513, 1, 1, 1, 1, 1), (2, 1025, 1, 3, 1, 3, 0),
]


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("dim,n,coarse,prolong,level,nu1,nu2", FUSED_CASES)
def test_presmooth_restrict(dim, n, coarse, prolong, level, nu1, nu2, fp32):
    """nu1 sweeps, defect and full weighting in one kernel = the oracle's steps in turn."""
    H = Handle(dim, n, coarse=coarse, prolong=prolong, nu1=nu1, nu2=nu2)
    try:
        n_l, s = H.level(level)
        d = s[(s.shape[0] // 2,) * dim]
        u = rand_grid(n_l, dim, 21)
        f = rand_grid(n_l, dim, 22) * d
        if fp32:
            u, f = u.astype(np.float32).astype(np.float64), f.astype(np.float32).astype(np.float64)
        nc = (n_l - 1) // 2 + 1
        ud, fd = dev(u, fp32), dev(f, fp32)
        uo = dev(np.full_like(u, np.nan), fp32)
        fc = dev(np.full((nc,) * dim, np.nan), fp32)
        mg.mg_kernel_presmooth_restrict(H.h, level, fp32, fd.data_ptr(), ud.data_ptr(),
                                        uo.data_ptr(), fc.data_ptr())
        ref = u.copy()
        for _ in range(nu1):
            ref = oracle.jacobi(s, H.omega, f, ref)
        ref_fc = oracle.restrict(oracle.residual(s, f, ref))
        tol = TOL32 if fp32 else TOL64
        scale_u = _scale_u(u, f, s) * (1 + nu1)
        assert_close(host(uo), ref, tol * scale_u * 4, "smoothed u")
        assert_close(host(fc), ref_fc, tol * 8 * (np.abs(f).max() + d * scale_u), "coarse rhs")
        # zero initial guess
        mg.mg_kernel_presmooth_restrict(H.h, level, fp32, fd.data_ptr(), None, uo.data_ptr(),
                                        fc.data_ptr())
        ref = np.zeros_like(u)
        for _ in range(nu1):
            ref = oracle.jacobi(s, H.omega, f, ref)
        assert_close(host(uo), ref, tol * scale_u * 4, "smoothed u (zero guess)")
        assert_close(host(fc), oracle.restrict(oracle.residual(s, f, ref)),
                     tol * 8 * (np.abs(f).max() + d * scale_u), "coarse rhs (zero guess)")
    finally:
        H.close()


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("dim,n,coarse,prolong,level,nu1,nu2", FUSED_CASES)
def test_prolong_postsmooth(dim, n, coarse, prolong, level, nu1, nu2, fp32):
    """Interpolation, correction and nu2 sweeps in one kernel = the oracle's steps in turn."""
    H = Handle(dim, n, coarse=coarse, prolong=prolong, nu1=nu1, nu2=nu2)
    try:
        n_l, s = H.level(level)
        d = s[(s.shape[0] // 2,) * dim]
        nc = (n_l - 1) // 2 + 1
        u = rand_grid(n_l, dim, 23)
        v = rand_grid(nc, dim, 24)
        f = rand_grid(n_l, dim, 25) * d
        if fp32:
            u, v, f = (a.astype(np.float32).astype(np.float64) for a in (u, v, f))
        ud, vd, fd = dev(u, fp32), dev(v, fp32), dev(f, fp32)
        uo = dev(np.full_like(u, np.nan), fp32)
        mg.mg_kernel_prolong_postsmooth(H.h, level, fp32, vd.data_ptr(), ud.data_ptr(), fd.data_ptr(),
                                        uo.data_ptr())
        ref = oracle.prolong_add(v, u.copy(), prolong)
        for _ in range(nu2):
            ref = oracle.jacobi(s, H.omega, f, ref)
        tol = TOL32 if fp32 else TOL64
        scale = (np.abs(u).max() + 2 * np.abs(v).max() + np.abs(f).max() / d) * (1 + nu2)
        assert_close(host(uo), ref, tol * scale * 4, "post")
    finally:
        H.close()


# Fused passes with red-black smoothing: min(1, nu) red-black sweeps per pass.  Sides up
# to 513 take the LDS tile kernels, larger ones the row-marching kernels.
RB_FUSED_CASES = [
    # dim, n, coarse, prolong, level, nu1, nu2
    (2, 65, 0, 3, 0, 2, 1), (2, 257, 0, 3, 0, 1, 1), (2, 257, 0, 1, 0, 0, 2), (2, 1025, 0, 3, 0, 2, 1),
    (2, 1025, 0, 1, 0, 1, 0), (2, 1025, 1, 3, 1, 1, 2), (2, 2049, 1, 3, 1, 2, 1), (2, 1025, 3, 3, 0, 2, 2),
]


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("dim,n,coarse,prolong,level,nu1,nu2", RB_FUSED_CASES)
def test_red_black_fused_passes(dim, n, coarse, prolong, level, nu1, nu2, fp32):
    """The fused pre pass (a red-black sweep, the defect, full weighting) and post pass
    (interpolation, correction, a red-black sweep) = the oracle's partial steps in turn."""
    H = Handle(dim, n, coarse=coarse, prolong=prolong, nu1=nu1, nu2=nu2, smoother=1)
    try:
        n_l, s = H.level(level)
        d = s[(s.shape[0] // 2,) * dim]
        nc = (n_l - 1) // 2 + 1
        u = rand_grid(n_l, dim, 51)
        f = rand_grid(n_l, dim, 52) * d
        v = rand_grid(nc, dim, 53)
        if fp32:
            u, f, v = (a.astype(np.float32).astype(np.float64) for a in (u, f, v))
        ud, fd, vd = dev(u, fp32), dev(f, fp32), dev(v, fp32)
        tol = TOL32 if fp32 else TOL64

        def rb_sweeps(x, count):
            for _ in range(count):
                x = oracle.jacobi_colour(s, H.omega, 2, f, oracle.jacobi_colour(s, H.omega, 1, f, x))
            return x

        uo = dev(np.full_like(u, np.nan), fp32)
        fc = dev(np.full((nc,) * dim, np.nan), fp32)
        for start in (u, None):
            u0 = u if start is not None else np.zeros_like(u)
            mg.mg_kernel_presmooth_restrict(H.h, level, fp32, fd.data_ptr(),
                                            ud.data_ptr() if start is not None else None,
                                            uo.data_ptr(), fc.data_ptr())
            ref = rb_sweeps(u0, min(1, nu1))
            scale_u = _scale_u(u, f, s) * 3
            assert_close(host(uo), ref, tol * scale_u * 4, "pre u")
            assert_close(host(fc), oracle.restrict(oracle.residual(s, f, ref)),
                         tol * 8 * (np.abs(f).max() + d * scale_u), "pre coarse rhs")
        mg.mg_kernel_prolong_postsmooth(H.h, level, fp32, vd.data_ptr(), ud.data_ptr(), fd.data_ptr(),
                                        uo.data_ptr())
        ref = rb_sweeps(oracle.prolong_add(v, u.copy(), prolong), min(1, nu2))
        scale = (np.abs(u).max() + 2 * np.abs(v).max() + np.abs(f).max() / d) * 3
        assert_close(host(uo), ref, tol * scale * 4, "post")
    finally:
        H.close()


# Sixth-order fine operator (section 3.3): radius-3 separable kernels on level 0.
SIXTH_CASES = [
    # dim, n, coarse, prolong, level
    (2, 65, 0, 1, 0), (2, 257, 0, 3, 0), (2, 1025, 0, 1, 0), (2, 1025, 3, 3, 1), (2, 257, 1, 1, 1),
    (3, 33, 0, 3, 0), (3, 65, 0, 1, 0), (3, 129, 0, 3, 0), (3, 65, 1, 3, 1), (3, 257, 0, 3, 0),
    (3, 17, 0, 3, 0),
]


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("dim,n,coarse,prolong,level", SIXTH_CASES)
def test_sixth_order_steps(dim, n, coarse, prolong, level, fp32):
    """Sweep, colour step, defect, defect + full weighting and (2D) the fused passes with
    the sixth-order operator, against the oracle's same steps."""
    H = Handle(dim, n, coarse=coarse, prolong=prolong, order=6, nu1=1, nu2=1)
    try:
        n_l, s = H.level(level)
        d = s[(s.shape[0] // 2,) * dim]
        u = rand_grid(n_l, dim, 61)
        f = rand_grid(n_l, dim, 62) * d
        nc = (n_l - 1) // 2 + 1
        v = rand_grid(nc, dim, 63)
        if fp32:
            u, f, v = (a.astype(np.float32).astype(np.float64) for a in (u, f, v))
        ud, fd, vd = dev(u, fp32), dev(f, fp32), dev(v, fp32)
        tol = TOL32 if fp32 else TOL64
        su = _scale_u(u, f, s)
        out = dev(np.full_like(u, np.nan), fp32)
        mg.mg_kernel_smooth(H.h, level, fp32, fd.data_ptr(), ud.data_ptr(), out.data_ptr())
        assert_close(host(out), oracle.jacobi(s, H.omega, f, u), tol * su * 4, "sweep")
        mg.mg_kernel_smooth_colour(H.h, level, fp32, 1, fd.data_ptr(), ud.data_ptr(), out.data_ptr())
        assert_close(host(out), oracle.jacobi_colour(s, H.omega, 1, f, u), tol * su * 4, "red step")
        mg.mg_kernel_residual(H.h, level, fp32, fd.data_ptr(), ud.data_ptr(), out.data_ptr())
        scale = np.abs(f).max() + d * np.abs(u).max()
        assert_close(host(out), oracle.residual(s, f, u), tol * scale * 8, "defect")
        fc = dev(np.full((nc,) * dim, np.nan), fp32)
        mg.mg_kernel_residual_restrict(H.h, level, fp32, fd.data_ptr(), ud.data_ptr(), fc.data_ptr())
        assert_close(host(fc), oracle.restrict(oracle.residual(s, f, u)), tol * scale * 8, "defect+FW")
        if dim == 2:
            mg.mg_kernel_presmooth_restrict(H.h, level, fp32, fd.data_ptr(), ud.data_ptr(),
                                            out.data_ptr(), fc.data_ptr())
            ref = oracle.jacobi(s, H.omega, f, u)
            assert_close(host(out), ref, tol * su * 8, "pre u")
            assert_close(host(fc), oracle.restrict(oracle.residual(s, f, ref)), tol * scale * 16, "pre fc")
            mg.mg_kernel_prolong_postsmooth(H.h, level, fp32, vd.data_ptr(), ud.data_ptr(),
                                            fd.data_ptr(), out.data_ptr())
            ref = oracle.jacobi(s, H.omega, f, oracle.prolong_add(v, u.copy(), prolong))
            sc = (np.abs(u).max() + 2 * np.abs(v).max() + np.abs(f).max() / d) * 2
            assert_close(host(out), ref, tol * sc * 4, "post")
    finally:
        H.close()


CASES_3D = [
    # dim, finest n, coarse, prolong, level
    (3, 9, 0, 3, 0), (3, 17, 0, 3, 0), (3, 33, 0, 3, 0), (3, 65, 0, 3, 0), (3, 65, 0, 3, 1),
    (3, 33, 1, 3, 1), (3, 65, 1, 3, 1), (3, 65, 1, 3, 2), (3, 33, 1, 1, 1),
    (3, 65, 2, 3, 1), (3, 65, 3, 3, 1), (3, 65, 3, 3, 2),
]


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("dim,n,coarse,prolong,level", CASES_3D)
def test_smooth_3d(dim, n, coarse, prolong, level, fp32):
    test_smooth(dim, n, coarse, prolong, level, fp32)


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("dim,n,coarse,prolong,level", CASES_3D)
def test_residual_3d(dim, n, coarse, prolong, level, fp32):
    test_residual(dim, n, coarse, prolong, level, fp32)


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("dim,n,coarse,prolong,level", [c for c in CASES_3D if c[1] > 9])
def test_residual_restrict_3d(dim, n, coarse, prolong, level, fp32):
    test_residual_restrict(dim, n, coarse, prolong, level, fp32)


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("dim,n,coarse,prolong,level", [c for c in CASES_3D if c[1] > 9])
def test_prolong_correct_3d(dim, n, coarse, prolong, level, fp32):
    test_prolong_correct(dim, n, coarse, prolong, level, fp32)


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("wide,ys,w128", [("0", "1", "1"), ("1", "1", "1"), ("1", "2", "1"), ("1", "2", "0")])
@pytest.mark.parametrize("n,prolong", [(33, 3), (65, 3), (65, 1), (129, 3)])
def test_3d_tile_shapes(n, prolong, wide, ys, w128, fp32, monkeypatch):
    """The cross kernels' other tile shapes (wide sweep and interpolation tiles with one or
    two rows per thread: FP32 sweeps with two rows take 128-column tiles unless
    MG_X3_W128=0; 16 x 7 coarse defect tiles), which the large levels take, against the
    oracle on small and ragged grids; and the small-level shapes forced."""
    for var in ("MG_X3_W", "MG_P3_W", "MG_XRR_TALL"):
        monkeypatch.setenv(var, wide)
    monkeypatch.setenv("MG_X3_YS", ys)
    monkeypatch.setenv("MG_X3_W128", w128)
    test_smooth(3, n, 0, prolong, 0, fp32)
    test_residual(3, n, 0, prolong, 0, fp32)
    test_residual_restrict(3, n, 0, prolong, 0, fp32)
    test_prolong_correct(3, n, 0, prolong, 0, fp32)


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("rows", ["1", "2"])
@pytest.mark.parametrize("n,level", [(33, 1), (65, 1), (65, 2), (129, 1), (257, 1)])
def test_3d_galerkin_sweep_kernels(n, level, rows, fp32, monkeypatch):
    """Galerkin levels: the wavefront-pencil sweep (MG_GPEN_ROWS=2: twice the rows per
    wavefront) and the separable defect + full weighting against the oracle's assembled
    Galerkin stencils, on one strip of 58 columns up to ragged multi-strip, multi-band
    levels."""
    monkeypatch.setenv("MG_GPEN_ROWS", rows)
    test_smooth(3, n, 1, 3, level, fp32)
    test_residual(3, n, 1, 3, level, fp32)
    test_residual_restrict(3, n, 1, 3, level, fp32)


# Red-black partial steps (section 3.1 eq. S_rb): (dim, finest n, coarse, level).  Level
# sides cover single blocks, ragged blocks and 3D plane bands.
CASES_RB = [
    (2, 17, 0, 0), (2, 257, 0, 0), (2, 1025, 0, 1), (2, 257, 1, 1),
    (2, 513, 3, 1), (2, 257, 1, 2), (2, 1025, 0, 0), (2, 257, 2, 1),
    (3, 17, 0, 0), (3, 65, 0, 0), (3, 129, 0, 0), (3, 65, 1, 1),
    (3, 129, 1, 1), (3, 65, 3, 2), (3, 33, 2, 1),
    (3, 9, 0, 0), (3, 257, 2, 1),
]


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("n", [9, 17, 65, 129, 257])
def test_red_black_sweep_3d_one_pass(n, fp32):
    """The one-pass 3D red-black sweep (60 x 8 tiles with a two-column frame) on grids
    from one tile to ragged multi-tile, multi-band ones."""
    H = Handle(3, n, smoother=1)
    try:
        _, s = H.level(0)
        u = rand_grid(n, 3, 71)
        f = rand_grid(n, 3, 72) * s[2, 2, 2]
        if fp32:
            u, f = u.astype(np.float32).astype(np.float64), f.astype(np.float32).astype(np.float64)
        ud, fd = dev(u, fp32), dev(f, fp32)
        out = dev(np.full_like(u, np.nan), fp32)
        mg.mg_kernel_smooth_colour(H.h, 0, fp32, 3, fd.data_ptr(), ud.data_ptr(), out.data_ptr())
        ref = oracle.jacobi_colour(s, H.omega, 2, f, oracle.jacobi_colour(s, H.omega, 1, f, u))
        assert_close(host(out), ref, 2 * (TOL32 if fp32 else TOL64) * _scale_u(u, f, s), "red-black sweep")
    finally:
        H.close()


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("dim,n,coarse,level", CASES_RB)
def test_smooth_colour(dim, n, coarse, level, fp32):
    """One partial step per colour against the oracle's; the other colour is copied
    bit for bit."""
    H = Handle(dim, n, coarse=coarse, smoother=1)
    try:
        n_l, s = H.level(level)
        u = rand_grid(n_l, dim, 41)
        f = rand_grid(n_l, dim, 42) * s[(s.shape[0] // 2,) * dim]
        if fp32:
            u, f = u.astype(np.float32).astype(np.float64), f.astype(np.float32).astype(np.float64)
        ud, fd = dev(u, fp32), dev(f, fp32)
        idx = np.indices(u.shape).sum(axis=0)
        tol = (TOL32 if fp32 else TOL64) * _scale_u(u, f, s)
        for colour in (1, 2, 0):
            out = dev(np.full_like(u, np.nan), fp32)
            mg.mg_kernel_smooth_colour(H.h, level, fp32, colour, fd.data_ptr(), ud.data_ptr(),
                                       out.data_ptr())
            got = host(out)
            ref = oracle.jacobi_colour(s, H.omega, colour, f, u)
            assert_close(got, ref, tol, "colour %d" % colour)
            if colour:
                keep = (idx % 2) != (colour % 2)
                assert np.array_equal(got[keep], u[keep])
            out0 = dev(np.full_like(u, np.nan), fp32)
            mg.mg_kernel_smooth_colour(H.h, level, fp32, colour, fd.data_ptr(), None, out0.data_ptr())
            ref0 = oracle.jacobi_colour(s, H.omega, colour, f, np.zeros_like(u))
            assert_close(host(out0), ref0, tol, "colour %d, zero guess" % colour)
        # a whole red-black sweep in one pass (3D: cross levels only)
        ref = oracle.jacobi_colour(s, H.omega, 2, f, oracle.jacobi_colour(s, H.omega, 1, f, u))
        out = dev(np.full_like(u, np.nan), fp32)
        if dim == 3 and coarse in (1, 3) and level > 0:
            with pytest.raises(mg.MGError):
                mg.mg_kernel_smooth_colour(H.h, level, fp32, 3, fd.data_ptr(), ud.data_ptr(),
                                           out.data_ptr())
        else:
            mg.mg_kernel_smooth_colour(H.h, level, fp32, 3, fd.data_ptr(), ud.data_ptr(), out.data_ptr())
            assert_close(host(out), ref, 2 * tol, "red-black sweep")
            mg.mg_kernel_smooth_colour(H.h, level, fp32, 3, fd.data_ptr(), None, out.data_ptr())
            ref0 = oracle.jacobi_colour(s, H.omega, 2, f,
                                        oracle.jacobi_colour(s, H.omega, 1, f, np.zeros_like(u)))
            assert_close(host(out), ref0, 2 * tol, "red-black sweep, zero guess")
        with pytest.raises(mg.MGError):
            mg.mg_kernel_smooth_colour(H.h, level, fp32, 4, fd.data_ptr(), ud.data_ptr(),
                                       out.data_ptr())
    finally:
        H.close()


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("coarse,prolong", [(0, 3), (1, 3)])
def test_coarsest_solve_3d(coarse, prolong, fp32):
    test_coarsest_solve(3, coarse, prolong, fp32)


def test_full_size_sweep_513_3d_fp32():
    """The FP32 level-0 sweep at 513^3 (128 x 16 tiles from point 1, two rows per thread),
    every element, against the FP64 oracle on the same FP32-rounded inputs."""
    n = 513
    H = Handle(3, n, precision=1)
    try:
        _, s = H.level(0)
        u = rand_grid(n, 3, 33).astype(np.float32).astype(np.float64)
        f = (rand_grid(n, 3, 34) * s[2, 2, 2]).astype(np.float32).astype(np.float64)
        ud, fd = dev(u, True), dev(f, True)
        out = dev(np.full_like(u, np.nan), True)
        mg.mg_kernel_smooth(H.h, 0, 1, fd.data_ptr(), ud.data_ptr(), out.data_ptr())
        assert_close(host(out), oracle.jacobi(s, H.omega, f, u), TOL32 * _scale_u(u, f, s), "sweep fp32")
        mg.mg_kernel_residual(H.h, 0, 1, fd.data_ptr(), ud.data_ptr(), out.data_ptr())
        scale = np.abs(f).max() + s[2, 2, 2] * np.abs(u).max()
        assert_close(host(out), oracle.residual(s, f, u), TOL32 * 4 * scale, "residual fp32")
    finally:
        H.close()


def test_full_size_1025_3d_fp32_sampled():
    """The 1025^3 level-0 FP32 kernels in the launch shapes that the 1025^3 benchmark
    times (sweep tiles of 128 x 16 points and 64-plane chunks from point 1, coarse defect
    tiles from column 1, interpolation tiles from point 1 with the last plane band taking
    the boundary plane): every point of blocks placed across tile, chunk and grid edges,
    against the oracle applied to the same blocks of the FP32 inputs (tests/blocks.py)."""
    t = torch()
    n = 1025
    nc = (n - 1) // 2 + 1
    print("1025^3 FP32 level-0 kernels, sampled blocks", flush=True)
    h = mg.mg_setup(mg.make_config(dim=3, n=n, coarse=1, gamma=2, nu1=2, nu2=2, precision=1,
                                   inner_cycles=1), stream())
    try:
        s = oracle.fine_stencil(3, 4, 1.0 / (n - 1))
        om = oracle.jacobi_omega(3)
        gen = t.Generator(device="cuda")
        gen.manual_seed(inputs.SEED_BASE + 1025)

        def field(m, scale):
            a = (t.rand((m, m, m), generator=gen, device="cuda", dtype=t.float32) * 2 - 1) * scale
            for ax in range(3):
                a.narrow(ax, 0, 1).zero_()
                a.narrow(ax, m - 1, 1).zero_()
            return a

        u, f = field(n, 1.0), field(n, float(s[2, 2, 2]))
        out = t.full_like(u, float("nan"))
        # centres on the sweep's tile edges (x 1 + 128k, y 1 + 16k, z 1 + 64k) and the grid's
        per = [blocks.starts(n, blocks.SWEEP_B, c) for c in
               ([0, 64, 65, 512, 961, n - 1], [0, 16, 17, 513, 1009, n - 1], [0, 128, 129, 513, 897, n - 1])]
        sts = [(a, b, c) for a in per[0] for b in per[1] for c in per[2]]
        B = blocks.SWEEP_B
        mg.mg_kernel_smooth(h, 0, 1, f.data_ptr(), u.data_ptr(), out.data_ptr())
        for st in sts:
            c = blocks.core(st, B, n, blocks.SWEEP_M)
            ref = oracle.jacobi(s, om, blocks.cut(f, st, B), blocks.cut(u, st, B))
            assert_close(blocks.cut(out, st, B)[c], ref[c], TOL32 * 2, "sweep %s" % (st,))
        mg.mg_kernel_residual(h, 0, 1, f.data_ptr(), u.data_ptr(), out.data_ptr())
        for st in sts:
            c = blocks.core(st, B, n, blocks.SWEEP_M)
            ref = oracle.residual(s, blocks.cut(f, st, B), blocks.cut(u, st, B))
            assert_close(blocks.cut(out, st, B)[c], ref[c], TOL32 * 8 * s[2, 2, 2], "residual %s" % (st,))
        del out
        # defect + full weighting: coarse tile edges (x 1 + 16k, y 7k, z 31k coarse)
        B, CB = blocks.RR_B, blocks.RR_CB
        fc = t.full((nc,) * 3, float("nan"), device="cuda", dtype=t.float32)
        mg.mg_kernel_residual_restrict(h, 0, 1, f.data_ptr(), u.data_ptr(), fc.data_ptr())
        per = [blocks.starts(n, B, c, even=True) for c in
               ([0, 62, 64, 496, 992, n - 1], [0, 14, 16, 504, 1010, n - 1], [0, 32, 34, 514, 994, n - 1])]
        for st in [(a, b, c) for a in per[0] for b in per[1] for c in per[2]]:
            c = blocks.core(blocks.coarse(st), CB, nc, blocks.RR_M)
            ref = oracle.restrict(oracle.residual(s, blocks.cut(f, st, B), blocks.cut(u, st, B)))
            got = blocks.cut(fc, blocks.coarse(st), CB)
            assert_close(got[c], ref[c], TOL32 * 8 * s[2, 2, 2], "defect + FW %s" % (st,))
        del fc
        # interpolation + correction: tiles x 1 + 64k, y 1 + 8k, bands of 64 planes from 0
        B, CB = blocks.PRO_B, blocks.PRO_CB
        v = field(nc, 1.0)
        out = t.full_like(u, float("nan"))
        mg.mg_kernel_prolong_correct(h, 0, 1, v.data_ptr(), u.data_ptr(), out.data_ptr())
        per = [blocks.starts(n, B, c, even=True) for c in
               ([0, 64, 66, 512, 960, n - 1], [0, 8, 10, 512, 1016, n - 1], [0, 64, 66, 512, 960, n - 1])]
        for st in [(a, b, c) for a in per[0] for b in per[1] for c in per[2]]:
            c = blocks.core(st, B, n, blocks.PRO_M)
            ref = oracle.prolong_add(blocks.cut(v, blocks.coarse(st), CB), blocks.cut(u, st, B))
            assert_close(blocks.cut(out, st, B)[c], ref[c], TOL32 * 3, "interpolation %s" % (st,))
    finally:
        mg.mg_destroy(h)


def test_full_size_sweep_513_3d():
    """Level-0 sweep and defect + full weighting at 513^3, every element."""
    n = 513
    H = Handle(3, n)
    try:
        _, s = H.level(0)
        u = rand_grid(n, 3, 31)
        f = rand_grid(n, 3, 32) * s[2, 2, 2]
        ud, fd = dev(u), dev(f)
        out = dev(np.full_like(u, np.nan))
        mg.mg_kernel_smooth(H.h, 0, 0, fd.data_ptr(), ud.data_ptr(), out.data_ptr())
        assert_close(host(out), oracle.jacobi(s, H.omega, f, u), TOL64 * _scale_u(u, f, s), "sweep")
        del out
        nc = (n - 1) // 2 + 1
        fc = dev(np.full((nc,) * 3, np.nan))
        mg.mg_kernel_residual_restrict(H.h, 0, 0, fd.data_ptr(), ud.data_ptr(), fc.data_ptr())
        ref = oracle.restrict(oracle.residual(s, f, u))
        assert_close(host(fc), ref, TOL64 * 4 * (np.abs(f).max() + s[2, 2, 2] * np.abs(u).max()), "rr")
    finally:
        H.close()


GS_CASES = [
    # finest n, order, coarse, level: fourth- and sixth-order cross levels, one strip, several
    # strips and bands, a ragged last strip, and a five-point level (Jacobi partial step)
    (9, 4, 0, 0), (33, 4, 0, 0), (257, 4, 0, 0), (1025, 4, 0, 0), (1025, 4, 0, 1), (4097, 4, 0, 0),
    (129, 6, 0, 0), (2049, 6, 0, 0), (257, 4, 2, 1),
]


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("n,order,coarse,level", GS_CASES)
def test_gauss_seidel_partial_steps(n, order, coarse, level, fp32):
    """Red-black Gauss-Seidel partial steps (section 3.1 eq. S_GS) against the oracle's
    lexicographic sweep of the colour; the other colour and the boundary are copied bit
    for bit."""
    print("gs partial step n=%d order=%d coarse=%d level=%d fp32=%d" % (n, order, coarse, level, fp32),
          flush=True)
    H = Handle(2, n, coarse=coarse, order=order, smoother=mg.MG_SMOOTH_RBGS)
    try:
        n_l, s = H.level(level)
        u = rand_grid(n_l, 2, 61)
        f = rand_grid(n_l, 2, 62) * s[(s.shape[0] // 2,) * 2]
        if fp32:
            u, f = u.astype(np.float32).astype(np.float64), f.astype(np.float32).astype(np.float64)
        ud, fd = dev(u, fp32), dev(f, fp32)
        idx = np.indices(u.shape).sum(axis=0)
        tol = (TOL32 if fp32 else TOL64) * _scale_u(u, f, s) * 2
        red = None
        for colour in (1, 2):
            src = ud if colour == 1 else dev(red, fp32)
            base = u if colour == 1 else red
            out = dev(np.full_like(u, np.nan), fp32)
            mg.mg_kernel_smooth_colour(H.h, level, fp32, colour, fd.data_ptr(), src.data_ptr(), out.data_ptr())
            got = host(out)
            ref = oracle.gs_colour(s, H.omega, colour, f, base)
            if not np.abs(got - ref).max() <= tol:  # name the omega and colour the result matches
                for w in (H.omega, 0.98, 1.0, 1.16, 10.0 / 13.0):
                    for c in (1, 2):
                        print("diag omega %.4f colour %d: gs %.3e jacobi %.3e" % (
                            w, c, np.abs(got - oracle.gs_colour(s, w, c, f, base)).max(),
                            np.abs(got - oracle.jacobi_colour(s, w, c, f, base)).max()), flush=True)
                bad = np.argwhere(np.abs(got - ref) > tol)
                print("diag first bad points", bad[:8].tolist(), len(bad), flush=True)
            assert_close(got, ref, tol, "colour %d" % colour)
            keep = (idx % 2) != (colour % 2)
            assert np.array_equal(got[keep], base[keep])
            red = got
    finally:
        H.close()


def test_gauss_seidel_entry_rejects_other_colours():
    H = Handle(2, 65, smoother=mg.MG_SMOOTH_RBGS)
    try:
        a = dev(np.zeros((65, 65)))
        b = dev(np.zeros((65, 65)))
        for colour in (0, 3):
            with pytest.raises(mg.MGError):
                mg.mg_kernel_smooth_colour(H.h, 0, 0, colour, a.data_ptr(), a.data_ptr(), b.data_ptr())
        with pytest.raises(mg.MGError):
            mg.mg_kernel_presmooth_restrict(H.h, 0, 0, a.data_ptr(), a.data_ptr(), b.data_ptr(), b.data_ptr())
    finally:
        H.close()


@pytest.mark.parametrize("fp32", [0, 1])
@pytest.mark.parametrize("dim,n,coarse,level", [(2, 17, 0, 0), (2, 65, 0, 0), (2, 1025, 0, 1), (2, 257, 2, 1),
                                                (3, 17, 0, 0), (3, 65, 0, 0), (3, 129, 2, 1)])
def test_cubic_restriction(dim, n, coarse, level, fp32):
    """Defect + cubic-adjoint restriction (appendix A.4, the 1/1024 operator) against the
    oracle's defect and restriction."""
    print("cubic restriction dim=%d n=%d level=%d fp32=%d" % (dim, n, level, fp32), flush=True)
    H = Handle(dim, n, coarse=coarse, restrict_op=3, precision=fp32)
    try:
        n_l, s = H.level(level)
        nc = (n_l - 1) // 2 + 1
        d = s[(s.shape[0] // 2,) * dim]
        u = rand_grid(n_l, dim, 71)
        f = rand_grid(n_l, dim, 72) * d
        if fp32:
            u, f = u.astype(np.float32).astype(np.float64), f.astype(np.float32).astype(np.float64)
        ud, fd = dev(u, fp32), dev(f, fp32)
        fc = dev(np.full((nc,) * dim, np.nan), fp32)
        mg.mg_kernel_residual_restrict(H.h, level, fp32, fd.data_ptr(), ud.data_ptr(), fc.data_ptr())
        ref = oracle.restrict(oracle.residual(s, f, u), oracle.RESTRICT_CUBIC)
        scale = np.abs(f).max() + d * np.abs(u).max()
        assert_close(host(fc), ref, (TOL32 if fp32 else TOL64) * scale * 16, "defect + cubic restriction")
    finally:
        H.close()
