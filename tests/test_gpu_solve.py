"""Whole-cycle and whole-solve parity of the HIP path with the oracle (GPU).

Bar (FP64): after the same fixed number of cycles, ||u_gpu - u_oracle|| <= 1e-12 ||u_oracle||;
the recorded relative residuals agree to 1e-9 relative plus 5e-14 absolute (near the
rounding floor, about 6e-13 at n = 1025, both are dominated by rounding noise that the
two implementations produce in different orders).  Converged solves are checked against the exact discrete solution
(sine transform) within the bound ||L^{-1}|| ||r|| that the final residual implies.
"""
import numpy as np
import pytest

import oracle
from gpu_util import Handle, dev, host, rand_grid, stream, torch
from oracle import dst
from paper_2008_03885_amd import inputs, mg

pytestmark = pytest.mark.gpu


def _fixed_cycles(H, f, cycles):
    fd = dev(f)
    ud = dev(np.zeros_like(f))
    st, res = mg.mg_run_cycles(H.h, fd.data_ptr(), ud.data_ptr(), cycles)
    u_ref = np.zeros_like(f)
    _, hist = H.oracle.solve(u_ref, f, rtol=0.0, max_cycles=cycles)
    return host(ud), res, u_ref, hist


CYCLE_CASES = [
    # dim, n, coarse, prolong, nu1, nu2, gamma
    (2, 129, 0, 3, 2, 1, 1), (2, 129, 1, 3, 2, 1, 1), (2, 129, 0, 3, 2, 1, 2),
    (2, 129, 1, 3, 2, 1, 2), (2, 129, 0, 1, 2, 1, 1), (2, 129, 1, 1, 2, 2, 1),
    (2, 257, 0, 3, 1, 1, 1), (2, 65, 0, 3, 0, 2, 1), (2, 65, 0, 3, 3, 0, 2), (2, 9, 0, 3, 2, 1, 1),
    (2, 1025, 1, 3, 2, 1, 2),
    # second-order coarse operators (section 3.1)
    (2, 257, 2, 3, 2, 1, 1), (2, 257, 3, 3, 2, 1, 1), (2, 129, 3, 1, 2, 1, 2), (2, 129, 2, 3, 2, 2, 2),
]


@pytest.mark.parametrize("dim,n,coarse,prolong,nu1,nu2,gamma", CYCLE_CASES)
def test_fixed_cycles_match_oracle(dim, n, coarse, prolong, nu1, nu2, gamma):
    H = Handle(dim, n, coarse=coarse, prolong=prolong, nu1=nu1, nu2=nu2, gamma=gamma)
    try:
        _, f, _ = inputs.manufactured_2d(n)
        cycles = 8
        u, res, u_ref, hist = _fixed_cycles(H, f, cycles)
        err = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
        assert err <= 1e-12, err
        assert res.cycles == cycles and res.history_len == cycles + 1
        gh = np.array(res.hist())
        assert np.all(np.abs(gh - hist) <= 1e-9 * hist + 5e-14)
    finally:
        H.close()


RB_CASES = [
    # dim, n, coarse, prolong, nu1, nu2, gamma: red-black Jacobi smoothing
    (2, 129, 0, 3, 2, 1, 1), (2, 129, 1, 3, 1, 1, 2), (2, 257, 3, 3, 2, 1, 1), (2, 65, 0, 1, 0, 2, 1),
    (2, 1025, 0, 3, 2, 1, 1), (2, 257, 2, 3, 1, 0, 2),
    (3, 33, 0, 3, 2, 1, 1), (3, 65, 1, 3, 2, 2, 2), (3, 65, 0, 3, 1, 1, 1), (3, 65, 3, 1, 2, 1, 1),
    (3, 129, 0, 3, 2, 1, 1), (3, 65, 0, 1, 0, 2, 2),
]


@pytest.mark.parametrize("fused", ["0", "1"])
@pytest.mark.parametrize("n,nu1,nu2,gamma", [(65, 2, 1, 1), (65, 1, 2, 2), (129, 2, 1, 1)])
def test_red_black_3d_one_pass_and_two_launch_agree(fused, n, nu1, nu2, gamma, monkeypatch):
    """3D red-black sweeps in one pass or as two partial-step launches: both equal the
    oracle's cycles."""
    monkeypatch.setenv("MG_RB3_FUSED", fused)
    H = Handle(3, n, nu1=nu1, nu2=nu2, gamma=gamma, smoother=1)
    try:
        f = inputs.smooth_sine_3d(n)
        u, res, u_ref, hist = _fixed_cycles(H, f, 3)
        assert np.linalg.norm(u - u_ref) <= 1e-12 * np.linalg.norm(u_ref)
        gh = np.array(res.hist())
        assert np.all(np.abs(gh - hist) <= 1e-9 * hist + 5e-14)
    finally:
        H.close()


@pytest.mark.parametrize("dim,n,coarse,prolong,nu1,nu2,gamma", RB_CASES)
def test_red_black_cycles_match_oracle(dim, n, coarse, prolong, nu1, nu2, gamma):
    """Cycles with red-black Jacobi smoothing (section 3.1 eq. S_rb) on every level,
    the LDS-resident tail's included."""
    H = Handle(dim, n, coarse=coarse, prolong=prolong, nu1=nu1, nu2=nu2, gamma=gamma, smoother=1)
    try:
        f = inputs.manufactured_2d(n)[1] if dim == 2 else inputs.smooth_sine_3d(n)
        cycles = 5
        u, res, u_ref, hist = _fixed_cycles(H, f, cycles)
        err = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
        assert err <= 1e-12, err
        gh = np.array(res.hist())
        assert np.all(np.abs(gh - hist) <= 1e-9 * hist + 5e-14)
    finally:
        H.close()


CUBIC_R_CYCLES = [
    # dim, n, coarse, nu1, nu2, gamma, smoother: the cubic-adjoint restriction (appendix A.4)
    (2, 129, 0, 2, 1, 1, 0), (2, 257, 2, 2, 1, 2, 0), (2, 1025, 0, 2, 1, 1, 1), (2, 257, 0, 2, 1, 1, 2),
    (3, 33, 0, 2, 1, 1, 0), (3, 65, 0, 2, 2, 2, 0), (3, 65, 2, 2, 1, 1, 1),
]


@pytest.mark.parametrize("dim,n,coarse,nu1,nu2,gamma,smoother", CUBIC_R_CYCLES)
def test_cubic_restriction_cycles_match_oracle(dim, n, coarse, nu1, nu2, gamma, smoother):
    """Cycles with cubic interpolation and its adjoint restriction against the oracle's."""
    print("cubic restriction cycles dim=%d n=%d" % (dim, n), flush=True)
    H = Handle(dim, n, coarse=coarse, nu1=nu1, nu2=nu2, gamma=gamma, smoother=smoother, restrict_op=3)
    try:
        f = inputs.manufactured_2d(n)[1] if dim == 2 else inputs.smooth_sine_3d(n)
        u, res, u_ref, hist = _fixed_cycles(H, f, 5)
        err = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
        assert err <= 1e-12, err
        gh = np.array(res.hist())
        assert np.all(np.abs(gh - hist) <= 1e-9 * hist + 5e-14)
    finally:
        H.close()


GS_CYCLES = [
    # n, order, coarse, prolong, nu1, nu2, gamma: red-black Gauss-Seidel (section 3.1 eq. S_GS)
    (129, 4, 0, 3, 2, 1, 1), (257, 4, 0, 3, 1, 1, 2), (257, 4, 2, 3, 2, 1, 1), (65, 4, 0, 1, 0, 2, 1),
    (1025, 4, 0, 3, 2, 1, 1), (257, 6, 0, 3, 2, 1, 1), (129, 6, 2, 1, 2, 2, 2), (4097, 4, 0, 3, 2, 1, 1),
]


@pytest.mark.parametrize("n,order,coarse,prolong,nu1,nu2,gamma", GS_CYCLES)
def test_gauss_seidel_cycles_match_oracle(n, order, coarse, prolong, nu1, nu2, gamma):
    """Cycles with red-black Gauss-Seidel smoothing on every level against the oracle's."""
    print("gs cycles n=%d order=%d coarse=%d" % (n, order, coarse), flush=True)
    H = Handle(2, n, coarse=coarse, prolong=prolong, nu1=nu1, nu2=nu2, gamma=gamma, order=order,
               smoother=mg.MG_SMOOTH_RBGS)
    try:
        f = inputs.fourier_rhs(n, 2, 64, seed=inputs.SEED_BASE + 2) if n == 4097 else inputs.manufactured_2d(n)[1]
        cycles = 2 if n == 4097 else 5
        u, res, u_ref, hist = _fixed_cycles(H, f, cycles)
        err = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
        assert err <= 1e-12, err
        gh = np.array(res.hist())
        assert np.all(np.abs(gh - hist) <= 1e-9 * hist + 5e-14)
    finally:
        H.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_gauss_seidel_solve_to_tolerance(precision):
    """A 1025^2 solve with red-black Gauss-Seidel (FP64, and FP32 cycles in FP64 refinement)
    reaches 1e-10 and lies within the bound 1e-10 ||f||_h / lambda_min of the exact discrete
    solution; the rate per cycle is near the LFA two-grid factor (0.017 at omega 1.16)."""
    n = 1025
    f = inputs.fourier_rhs(n, 2, 64, seed=inputs.SEED_BASE + 2)
    H = Handle(2, n, smoother=mg.MG_SMOOTH_RBGS, precision=precision, rtol=1e-10, max_cycles=30,
               inner_cycles=3)
    try:
        fd, ud = dev(f), dev(np.zeros_like(f))
        st, res = mg.mg_solve(H.h, fd.data_ptr(), ud.data_ptr())
        assert st == mg.MG_OK and res.rel_residual <= 1e-10
        if precision == 0:
            assert res.cycles <= 8
        exact = dst.solve(f)
        bound = 1e-10 * oracle.norm(f) / dst.min_eigenvalue(n, 2)
        assert oracle.norm(host(ud) - exact) <= 1.01 * bound
    finally:
        H.close()


@pytest.mark.parametrize("fused", ["0", "1"])
@pytest.mark.parametrize("nu1,nu2,gamma", [(2, 1, 1), (2, 1, 2), (1, 1, 1), (3, 2, 1), (0, 1, 1),
                                           (1, 0, 2), (2, 2, 2)])
def test_red_black_fused_cycles(fused, nu1, nu2, gamma, monkeypatch):
    """2D red-black cycles through the fused passes (one pass per red-black sweep, with
    the third sweep target when the pass count is odd) and through the separate kernels,
    against the oracle, on a grid with row-marching (1025, 513 tiles) and tail levels."""
    monkeypatch.setenv("MG_FUSED", fused)
    n = 1025
    H = Handle(2, n, nu1=nu1, nu2=nu2, gamma=gamma, smoother=1)
    try:
        _, f, _ = inputs.manufactured_2d(n)
        u, res, u_ref, hist = _fixed_cycles(H, f, 3)
        err = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
        assert err <= 1e-12, err
        gh = np.array(res.hist())
        assert np.all(np.abs(gh - hist) <= 1e-9 * hist + 5e-14)
    finally:
        H.close()


SIXTH_CYCLES = [
    # dim, n, coarse, prolong, nu1, nu2, gamma, smoother: sixth-order fine operator (section 3.3)
    (2, 129, 0, 1, 2, 1, 1, 0), (2, 129, 1, 1, 2, 1, 1, 0), (2, 129, 2, 1, 2, 1, 1, 0),
    (2, 129, 3, 1, 2, 1, 1, 0), (2, 1025, 3, 3, 2, 1, 1, 0), (2, 257, 0, 3, 1, 1, 2, 0),
    (2, 1025, 3, 1, 2, 1, 1, 1), (2, 257, 1, 3, 1, 1, 2, 1),
    (3, 33, 0, 3, 2, 1, 1, 0), (3, 65, 3, 1, 2, 1, 1, 0), (3, 65, 1, 3, 2, 2, 2, 0),
    (3, 65, 2, 1, 2, 1, 1, 1),
]


@pytest.mark.parametrize("dim,n,coarse,prolong,nu1,nu2,gamma,smoother", SIXTH_CYCLES)
def test_sixth_order_cycles_match_oracle(dim, n, coarse, prolong, nu1, nu2, gamma, smoother):
    """Cycles with the sixth-order fine operator and each coarse operator (section 3.3:
    second-order rediscretized or Galerkin coarse operators against sixth-order ones)."""
    H = Handle(dim, n, coarse=coarse, prolong=prolong, nu1=nu1, nu2=nu2, gamma=gamma, order=6,
               smoother=smoother)
    try:
        f = inputs.manufactured_2d(n)[1] if dim == 2 else inputs.smooth_sine_3d(n)
        u, res, u_ref, hist = _fixed_cycles(H, f, 4)
        err = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
        assert err <= 1e-12, err
        gh = np.array(res.hist())
        assert np.all(np.abs(gh - hist) <= 1e-9 * hist + 5e-14)
    finally:
        H.close()


@pytest.mark.parametrize("r3", ["0", "1"])
@pytest.mark.parametrize("n,coarse,smoother", [(65, 0, 0), (129, 3, 0), (65, 2, 1)])
def test_sixth_order_3d_cross_and_separable_agree(r3, n, coarse, smoother, monkeypatch):
    """3D sixth-order level 0 through the radius-3 cross sweep or the separable sweep:
    both equal the oracle's cycles."""
    monkeypatch.setenv("MG_X3_R3", r3)
    H = Handle(3, n, coarse=coarse, order=6, smoother=smoother)
    try:
        f = inputs.smooth_sine_3d(n)
        u, res, u_ref, hist = _fixed_cycles(H, f, 3)
        assert np.linalg.norm(u - u_ref) <= 1e-12 * np.linalg.norm(u_ref)
        gh = np.array(res.hist())
        assert np.all(np.abs(gh - hist) <= 1e-9 * hist + 5e-14)
    finally:
        H.close()


@pytest.mark.parametrize("dim,n,smoother", [(2, 513, 0), (3, 65, 0), (3, 65, 1)])
def test_sixth_order_mixed_precision_matches_fp64(dim, n, smoother):
    """Sixth-order solves in mixed precision reach 1e-10 and agree with the FP64 solve."""
    f = inputs.manufactured_2d(n)[1] if dim == 2 else inputs.smooth_sine_3d(n)
    out = []
    for precision in (0, 1):
        H = Handle(dim, n, coarse=3, order=6, smoother=smoother, precision=precision, inner_cycles=3)
        try:
            fd, ud = dev(f), dev(np.zeros_like(f))
            st, res = mg.mg_solve(H.h, fd.data_ptr(), ud.data_ptr())
            assert st == mg.MG_OK and res.rel_residual <= 1e-10, (precision, res.rel_residual)
            out.append(host(ud))
        finally:
            H.close()
    assert np.linalg.norm(out[1] - out[0]) <= 1e-8 * np.linalg.norm(out[0])


def test_sixth_order_solve_converges_to_discrete_solution():
    """A 2D sixth-order solve to 1e-10 lands on the exact discrete solution (sine
    transform with the sixth-order eigenvalues) within the bound its residual implies."""
    n = 513
    H = Handle(2, n, coarse=3, prolong=1, order=6, rtol=1e-10)
    try:
        ustar, f, c = inputs.manufactured_2d(n)
        fd, ud = dev(f), dev(np.zeros_like(f))
        st, res = mg.mg_solve(H.h, fd.data_ptr(), ud.data_ptr())
        assert st == mg.MG_OK and res.rel_residual <= 1e-10
        exact = dst.solve(f, order=6)
        lam_min = dst.eigenvalues(n, 2, order=6).min()
        bound = res.rel_residual * np.linalg.norm(f[1:-1, 1:-1]) / lam_min
        assert np.linalg.norm(host(ud) - exact) <= 1.01 * bound + 1e-12 * np.linalg.norm(exact)
        # the sixth-order discrete solution is far closer to u* than the fourth-order one
        assert np.abs(exact - ustar).max() < 1e-9 * np.abs(ustar).max()
    finally:
        H.close()


@pytest.mark.parametrize("dim,n,nc,order,omega", [(2, 257, 5, 2, 1.0), (2, 129, 17, 2, 0.0), (3, 65, 5, 2, 0.0),
                                                (2, 257, 33, 4, 0.0), (3, 33, 5, 4, 1.0)])
def test_red_black_other_orders_and_coarsest_sides(dim, n, nc, order, omega):
    """Red-black cycles with the second-order operator (red-black Gauss-Seidel for the
    five-point stencil at omega = 1), other coarsest sides and explicit omega."""
    H = Handle(dim, n, n_coarsest=nc, order=order, omega=omega, smoother=1)
    try:
        f = inputs.manufactured_2d(n)[1] if dim == 2 else inputs.smooth_sine_3d(n)
        u, res, u_ref, hist = _fixed_cycles(H, f, 4)
        assert np.linalg.norm(u - u_ref) <= 1e-12 * np.linalg.norm(u_ref)
        gh = np.array(res.hist())
        assert np.all(np.abs(gh - hist) <= 1e-9 * hist + 5e-14)
    finally:
        H.close()


@pytest.mark.parametrize("dim,n,tail", [(2, 257, "0"), (2, 257, "33"), (3, 33, "0"), (3, 33, "17"),
                                         (3, 33, None)])
def test_red_black_tail_variants_agree(dim, n, tail, monkeypatch):
    """Red-black smoothing inside and outside the LDS-resident tail (in 3D also the
    line-pass tail of the 17^3 and 9^3 levels, tail=None): same cycles."""
    if tail is None:
        monkeypatch.delenv("MG_TAIL_N", raising=False)
    else:
        monkeypatch.setenv("MG_TAIL_N", tail)
    H = Handle(dim, n, gamma=2, smoother=1)
    try:
        f = inputs.manufactured_2d(n)[1] if dim == 2 else inputs.smooth_sine_3d(n)
        u, res, u_ref, hist = _fixed_cycles(H, f, 4)
        assert np.linalg.norm(u - u_ref) <= 1e-12 * np.linalg.norm(u_ref)
    finally:
        H.close()


def test_red_black_mixed_precision_solves():
    """FP32 red-black cycles inside FP64 refinement reach the FP64 tolerance."""
    for dim, n in ((2, 513), (3, 65)):
        H = Handle(dim, n, smoother=1, precision=1, rtol=1e-10, inner_cycles=2)
        try:
            f = inputs.manufactured_2d(n)[1] if dim == 2 else inputs.smooth_sine_3d(n)
            fd, ud = dev(f), dev(np.zeros_like(f))
            st, res = mg.mg_solve(H.h, fd.data_ptr(), ud.data_ptr())
            assert st == mg.MG_OK and res.rel_residual <= 1e-10, (dim, res.rel_residual)
            rel = mg.mg_residual_norm(H.h, fd.data_ptr(), ud.data_ptr())
            assert rel <= 1e-10
        finally:
            H.close()


@pytest.mark.parametrize("fused,tail,dst", [("1", None, "1"), ("0", "0", "1"), ("1", "0", "1"),
                                            ("1", "17", "1"), ("0", "65", "1"), ("1", None, "0")])
@pytest.mark.parametrize("coarse,gamma", [(0, 1), (1, 2)])
def test_runtime_variants_agree(fused, tail, dst, coarse, gamma, monkeypatch):
    """Fused or separate kernels, with or without the LDS-resident tail, the tail's
    coarsest solve by sine transforms or the dense inverse: same cycles."""
    monkeypatch.setenv("MG_COARSE_DST", dst)
    monkeypatch.setenv("MG_FUSED", fused)
    if tail is None:
        monkeypatch.delenv("MG_TAIL_N", raising=False)
    else:
        monkeypatch.setenv("MG_TAIL_N", tail)
    n = 257
    H = Handle(2, n, coarse=coarse, gamma=gamma)
    try:
        _, f, _ = inputs.manufactured_2d(n)
        u, res, u_ref, hist = _fixed_cycles(H, f, 6)
        assert np.linalg.norm(u - u_ref) <= 1e-12 * np.linalg.norm(u_ref)
    finally:
        H.close()


def test_c1_solve_to_tolerance():
    """2D 129^2, manufactured solution, V(2,1), nG, FW + cubic, omega = 10/13, to 1e-10."""
    n = 129
    H = Handle(2, n, rtol=1e-10, max_cycles=60)
    try:
        ustar, f, c = inputs.manufactured_2d(n)
        fd, ud = dev(f), dev(np.zeros_like(f))
        st, res = mg.mg_solve(H.h, fd.data_ptr(), ud.data_ptr())
        assert st == mg.MG_OK and res.status == 1
        assert res.rel_residual <= 1e-10
        u = host(ud)
        u_ref = np.zeros_like(f)
        cyc, hist = H.oracle.solve(u_ref, f, rtol=1e-10, max_cycles=60)
        assert res.cycles == cyc
        assert np.linalg.norm(u - u_ref) <= 1e-12 * np.linalg.norm(u_ref)
        exact = dst.discrete_solution_of_sine_series(n, c)
        bound = res.rel_residual * oracle.norm(f) / dst.eigenvalues(n, 2).min()
        assert oracle.norm(u - exact) <= 1.01 * bound
        # the device residual check agrees with the oracle's long-double residual
        s = H.oracle.level_stencil(0)[1]
        rel_ld = oracle.residual_norm_ld(s, f, u) / oracle.norm(f)
        assert abs(res.rel_residual - rel_ld) <= 1e-3 * rel_ld
        assert abs(mg.mg_residual_norm(H.h, fd.data_ptr(), ud.data_ptr()) - rel_ld) <= 1e-3 * rel_ld
    finally:
        H.close()


@pytest.mark.parametrize("coarse,gamma", [(0, 1), (1, 1), (0, 2), (1, 2), (2, 1), (3, 1)])
def test_c2_full_size(coarse, gamma):
    """2D 4097^2, Fourier right-hand side k <= 64, V(2,1)/W(2,1), nG/Galerkin, FP64: the
    solve reaches 1e-10 or the rounding floor, and matches the exact discrete solution."""
    n = 4097
    f = inputs.fourier_rhs(n, 2, 64, seed=inputs.SEED_BASE + 2)
    H = Handle(2, n, coarse=coarse, gamma=gamma, rtol=1e-10, max_cycles=40)
    try:
        fd, ud = dev(f), dev(np.zeros_like(f))
        st, res = mg.mg_solve(H.h, fd.data_ptr(), ud.data_ptr())
        # a solve stopped at the rounding floor above rtol reports MG_ENOCONV with floor_hit
        assert st == mg.MG_OK or (st == mg.MG_ENOCONV and res.floor_hit), res.status
        assert res.rel_residual <= 1e-10 or (res.floor_hit and res.rel_residual <= 3e-10)
        assert res.cycles <= 30
        u = host(ud)
        exact = dst.solve(f)
        err = np.linalg.norm(u - exact) / np.linalg.norm(exact)
        assert err <= 1e-9, err
        # the device residual equals an independent long-double evaluation
        s = oracle.fine_stencil(2, 4, 1.0 / (n - 1))
        rel_ld = oracle.residual_norm_ld(s, f, u) / oracle.norm(f)
        assert abs(res.rel_residual - rel_ld) <= 0.05 * rel_ld
    finally:
        H.close()


def test_c2_two_cycles_match_oracle_elementwise():
    n = 4097
    f = inputs.fourier_rhs(n, 2, 64, seed=inputs.SEED_BASE + 2)
    H = Handle(2, n)
    try:
        u, res, u_ref, hist = _fixed_cycles(H, f, 2)
        assert np.linalg.norm(u - u_ref) <= 1e-12 * np.linalg.norm(u_ref)
        assert np.abs(u - u_ref).max() <= 1e-12 * np.abs(u_ref).max()
    finally:
        H.close()


@pytest.mark.parametrize("smoother,order,coarse", [(1, 4, 0), (0, 6, 3), (1, 6, 3), (1, 4, 1)])
def test_c2_4097_two_cycles_variants(smoother, order, coarse):
    """The 4097^2 launch shapes of the benchmark with red-black smoothing (fused passes with
    the third sweep target) and with the sixth-order operator: two V(2,1) cycles equal the
    oracle's element by element."""
    n = 4097
    print("4097 variant smoother=%d order=%d coarse=%d" % (smoother, order, coarse), flush=True)
    f = inputs.fourier_rhs(n, 2, 64, seed=inputs.SEED_BASE + 2)
    H = Handle(2, n, smoother=smoother, order=order, coarse=coarse)
    try:
        u, res, u_ref, hist = _fixed_cycles(H, f, 2)
        assert np.linalg.norm(u - u_ref) <= 1e-12 * np.linalg.norm(u_ref)
        assert np.abs(u - u_ref).max() <= 1e-12 * np.abs(u_ref).max()
        gh = np.array(res.hist())
        assert np.all(np.abs(gh - hist) <= 1e-9 * hist + 5e-14)
    finally:
        H.close()


def test_mixed_precision_2d():
    """FP32 cycles inside FP64 refinement reach the FP64 tolerance; final error vs FP64."""
    n = 1025
    f = inputs.fourier_rhs(n, 2, 64, seed=inputs.SEED_BASE + 2)
    H64 = Handle(2, n, rtol=1e-10)
    Hmx = Handle(2, n, precision=1, rtol=1e-10, max_cycles=20, inner_cycles=4)
    try:
        fd = dev(f)
        u64, umx = dev(np.zeros_like(f)), dev(np.zeros_like(f))
        st, r64 = mg.mg_solve(H64.h, fd.data_ptr(), u64.data_ptr())
        st2, rmx = mg.mg_solve(Hmx.h, fd.data_ptr(), umx.data_ptr())
        assert st == mg.MG_OK and st2 == mg.MG_OK
        assert rmx.rel_residual <= 1e-10 and rmx.outer_steps >= 2
        a, b = host(u64), host(umx)
        rel = np.linalg.norm(a - b) / np.linalg.norm(a)
        assert rel <= 1e-9, rel
        exact = dst.solve(f)
        assert np.linalg.norm(b - exact) / np.linalg.norm(exact) <= 1e-9
    finally:
        H64.close()
        Hmx.close()


def test_async_solve_matches_sync_and_is_deterministic():
    n = 513
    f = inputs.fourier_rhs(n, 2, 64, seed=inputs.SEED_BASE + 2)
    H = Handle(2, n, rtol=1e-10, max_cycles=40)
    try:
        fd = dev(f)
        u1, u2, u3 = (dev(np.zeros_like(f)) for _ in range(3))
        _, r1 = mg.mg_solve(H.h, fd.data_ptr(), u1.data_ptr())
        _, r2 = mg.mg_solve(H.h, fd.data_ptr(), u2.data_ptr())   # new pointers: new graph
        mg.mg_solve_async(H.h, fd.data_ptr(), u3.data_ptr())
        import time
        while True:
            st, r3 = mg.mg_query(H.h)
            if st != mg.MG_EBUSY:
                break
            time.sleep(0.001)
        a, b, c = host(u1), host(u2), host(u3)
        assert np.array_equal(a, b) and np.array_equal(a, c)
        assert r1.cycles == r2.cycles == r3.cycles
        assert r1.hist() == r3.hist()
    finally:
        H.close()


def test_warm_start_continues_the_iteration():
    """u is the whole state: k cycles then m cycles equals k+m cycles."""
    n = 257
    _, f, _ = inputs.manufactured_2d(n)
    H = Handle(2, n)
    try:
        fd = dev(f)
        a, b = dev(np.zeros_like(f)), dev(np.zeros_like(f))
        mg.mg_run_cycles(H.h, fd.data_ptr(), a.data_ptr(), 5)
        mg.mg_run_cycles(H.h, fd.data_ptr(), b.data_ptr(), 3)
        mg.mg_run_cycles(H.h, fd.data_ptr(), b.data_ptr(), 2)
        assert np.array_equal(host(a), host(b))
    finally:
        H.close()


def test_cycle_cap_reports_enoconv():
    n = 129
    _, f, _ = inputs.manufactured_2d(n)
    H = Handle(2, n, rtol=1e-14, max_cycles=3)
    try:
        fd, ud = dev(f), dev(np.zeros_like(f))
        st, res = mg.mg_solve(H.h, fd.data_ptr(), ud.data_ptr())
        assert st == mg.MG_ENOCONV and res.status == 2 and res.cycles == 3
    finally:
        H.close()


def test_rounding_floor_reports_enoconv():
    """An rtol below what FP64 can certify: the solve stops at the rounding floor before
    the cycle cap and reports MG_ENOCONV with floor_hit (rtol was not reached)."""
    n = 129
    _, f, _ = inputs.manufactured_2d(n)
    H = Handle(2, n, rtol=1e-18, max_cycles=80)
    try:
        fd, ud = dev(f), dev(np.zeros_like(f))
        st, res = mg.mg_solve(H.h, fd.data_ptr(), ud.data_ptr())
        assert st == mg.MG_ENOCONV and res.status == 3 and res.floor_hit == 1
        assert res.cycles < 80 and 1e-18 < res.rel_residual <= 1e-12
        assert "rounding floor" in mg.last_error()
    finally:
        H.close()


def test_nonfinite_rhs_reports_enumeric():
    n = 65
    f = np.zeros((n, n))
    f[10, 10] = np.nan
    H = Handle(2, n)
    try:
        fd, ud = dev(f), dev(np.zeros_like(f))
        st, res = mg.mg_solve(H.h, fd.data_ptr(), ud.data_ptr())
        assert st == mg.MG_ENUMERIC and res.status == 4
    finally:
        H.close()


CYCLE_CASES_3D = [
    # n, coarse, prolong, nu1, nu2, gamma
    (17, 0, 3, 2, 1, 1), (33, 0, 3, 2, 1, 1), (33, 1, 3, 2, 1, 1), (33, 0, 3, 2, 2, 2),
    (33, 1, 3, 2, 2, 2), (33, 0, 1, 1, 1, 1), (65, 0, 3, 2, 1, 1), (65, 1, 3, 2, 2, 2),
    (33, 1, 3, 0, 2, 1), (129, 1, 3, 2, 2, 2),
    (65, 2, 3, 2, 1, 1), (65, 3, 3, 2, 2, 2), (33, 3, 1, 2, 1, 1),
]


@pytest.mark.parametrize("n,coarse,prolong,nu1,nu2,gamma", CYCLE_CASES_3D)
def test_fixed_cycles_match_oracle_3d(n, coarse, prolong, nu1, nu2, gamma):
    H = Handle(3, n, coarse=coarse, prolong=prolong, nu1=nu1, nu2=nu2, gamma=gamma)
    try:
        f = inputs.smooth_sine_3d(n)
        cycles = 6
        u, res, u_ref, hist = _fixed_cycles(H, f, cycles)
        err = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
        assert err <= 1e-12, err
        gh = np.array(res.hist())
        assert np.all(np.abs(gh - hist) <= 1e-9 * hist + 5e-14)
    finally:
        H.close()


@pytest.mark.parametrize("tail,dst,coarse,tail3", [(None, "1", 0, "1"), (None, "0", 0, "1"), ("0", "1", 0, "1"),
                                                    (None, "1", 1, "1"), ("17", "1", 0, "1"), ("17", "0", 1, "1"),
                                                    ("33", "1", 1, "1"), (None, "1", 1, "0"), (None, "1", 2, "1"),
                                                    (None, "1", 3, "1")])
@pytest.mark.parametrize("precision", [0, 1])
def test_3d_tail_variants_agree(tail, dst, coarse, tail3, precision, monkeypatch):
    """With or without the LDS-resident tail, the line-pass tail of the 17^3 and 9^3
    levels (the default when the sine table exists; MG_TAIL3=0 or an explicit MG_TAIL_N
    turns it off), the coarsest solve by sine transforms or by the dense inverse: same
    cycles as the oracle (mixed precision: FP32 cycles inside FP64 steps, against FP64
    cycles, to the FP32 level)."""
    if tail is None:
        monkeypatch.delenv("MG_TAIL_N", raising=False)
    else:
        monkeypatch.setenv("MG_TAIL_N", tail)
    monkeypatch.setenv("MG_COARSE_DST", dst)
    monkeypatch.setenv("MG_TAIL3", tail3)
    n = 33
    if precision:
        f = inputs.smooth_sine_3d(n)
        fd = dev(f)
        out = []
        for p in (0, 1):
            H = Handle(3, n, gamma=2, coarse=coarse, precision=p, inner_cycles=1)
            try:
                ud = dev(np.zeros_like(f))
                mg.mg_run_cycles(H.h, fd.data_ptr(), ud.data_ptr(), 3)
                out.append(host(ud))
            finally:
                H.close()
        assert np.linalg.norm(out[1] - out[0]) <= 1e-5 * np.linalg.norm(out[0])
        return
    H = Handle(3, n, gamma=2, coarse=coarse)
    try:
        f = inputs.smooth_sine_3d(n)
        u, res, u_ref, hist = _fixed_cycles(H, f, 4)
        assert np.linalg.norm(u - u_ref) <= 1e-12 * np.linalg.norm(u_ref)
    finally:
        H.close()


def test_mixed_precision_3d():
    """3D noise right-hand side: FP32 cycles in FP64 refinement reach 1e-10 like FP64."""
    n = 129
    f = inputs.smoothed_noise_3d(n)
    H64 = Handle(3, n, rtol=1e-10, max_cycles=60)
    Hmx = Handle(3, n, precision=1, rtol=1e-10, max_cycles=20, inner_cycles=4)
    try:
        fd = dev(f)
        u64, umx = dev(np.zeros_like(f)), dev(np.zeros_like(f))
        st, r64 = mg.mg_solve(H64.h, fd.data_ptr(), u64.data_ptr())
        st2, rmx = mg.mg_solve(Hmx.h, fd.data_ptr(), umx.data_ptr())
        assert st == mg.MG_OK and st2 == mg.MG_OK
        assert r64.rel_residual <= 1e-10 and rmx.rel_residual <= 1e-10
        a, b = host(u64), host(umx)
        assert np.linalg.norm(a - b) / np.linalg.norm(a) <= 1e-9
        exact = dst.solve(f)
        assert np.linalg.norm(a - exact) / np.linalg.norm(exact) <= 1e-9
    finally:
        H64.close()
        Hmx.close()


def test_c3_513_fp64_solve():
    """3D 513^3, smoothed-noise right-hand side, V(2,1), FP64, to 1e-10: the device residual
    agrees with a long-double evaluation of the returned iterate."""
    n = 513
    f = inputs.smoothed_noise_3d(n)
    H = Handle(3, n, rtol=1e-10, max_cycles=60)
    try:
        fd, ud = dev(f), dev(np.zeros_like(f))
        st, res = mg.mg_solve(H.h, fd.data_ptr(), ud.data_ptr())
        assert st == mg.MG_OK and res.rel_residual <= 1e-10
        assert res.cycles <= 40
        u = host(ud)
        s = oracle.fine_stencil(3, 4, 1.0 / (n - 1))
        rel_ld = oracle.residual_norm_ld(s, f, u) / oracle.norm(f)
        assert abs(res.rel_residual - rel_ld) <= 0.05 * rel_ld
    finally:
        H.close()


def test_c3_513_cycles_match_oracle():
    """3D 513^3 (the benchmark's launch shapes: 64-wide FP64 tiles on level 0), smoothed
    noise right-hand side: two FP64 V(2,1) cycles equal the oracle's element by element."""
    n = 513
    print("C3 513^3 two FP64 cycles", flush=True)
    f = inputs.smoothed_noise_3d(n)
    H = Handle(3, n)
    try:
        u, res, u_ref, hist = _fixed_cycles(H, f, 2)
        nrm = np.linalg.norm(u_ref)
        assert np.linalg.norm(u - u_ref) <= 1e-12 * nrm
        gh = np.array(res.hist())
        assert np.all(np.abs(gh - hist) <= 1e-9 * hist + 5e-14)
    finally:
        H.close()


def _exact_error_h(u_dev, exact_dev, n):
    """||u - exact||_h on the device (boundary values are zero in both)."""
    t = torch()
    d = t.linalg.vector_norm(u_dev - exact_dev).item()
    return d * (1.0 / (n - 1)) ** 1.5


def test_c3_513_mixed_and_fp64_match_exact():
    """3D 513^3, V(2,1): the mixed-precision solve (FP32 cycles in FP64 refinement) and the
    FP64 solve both reach 1e-10 and both lie within the bound 1e-10 ||f||_h / lambda_min of
    the exact discrete solution (sine transform); mixed and FP64 agree to 1e-9."""
    n = 513
    print("C3 513^3 mixed vs FP64 vs exact", flush=True)
    f = inputs.smoothed_noise_3d(n)
    exact = dev(dst.solve(f))
    fd = dev(f)
    bound = 1e-10 * oracle.norm(f) / dst.min_eigenvalue(n, 3)
    out = {}
    for prec, inner in ((0, 4), (1, 8)):
        H = Handle(3, n, precision=prec, rtol=1e-10, max_cycles=60 if prec == 0 else 20,
                   inner_cycles=inner)
        try:
            ud = dev(np.zeros_like(f))
            st, res = mg.mg_solve(H.h, fd.data_ptr(), ud.data_ptr())
            assert st == mg.MG_OK and res.rel_residual <= 1e-10, (prec, res.status)
            if prec:
                assert res.outer_steps >= 2
            err = _exact_error_h(ud, exact, n)
            assert err <= 1.01 * bound, (prec, err, bound)
            out[prec] = ud
        finally:
            H.close()
    t = torch()
    rel = (t.linalg.vector_norm(out[1] - out[0]) / t.linalg.vector_norm(out[0])).item()
    assert rel <= 1e-9, rel


def test_c5_1025_galerkin_w22_match_exact():
    """3D 1025^3, Galerkin coarse operators, W(2,2), smooth sine-series right-hand side:
    the FP64 and the mixed-precision solves reach 1e-10 and lie within 1e-10 ||f||_h /
    lambda_min of the exact discrete solution, which for a sine series is the series with
    each coefficient divided by the operator's eigenvalue (no multigrid code); mixed and
    FP64 agree to 1e-9."""
    n = 1025
    print("C5 1025^3 Galerkin W(2,2) FP64 and mixed vs exact", flush=True)
    f, g = inputs.smooth_sine_3d(n, return_coeffs=True)
    K = g.shape[0]
    k2 = inputs.wavenumber_sq(K, 3)
    fn = oracle.norm(f)
    fd = dev(f)
    del f
    exact = dev(dst.discrete_solution_of_sine_series(n, g / (np.pi ** 2 * k2)))
    bound = 1e-10 * fn / dst.min_eigenvalue(n, 3)
    out = {}
    for prec, inner in ((0, 1), (1, 1)):
        H = mg.mg_setup(mg.make_config(dim=3, n=n, coarse=1, gamma=2, nu1=2, nu2=2, precision=prec,
                                       rtol=1e-10, max_cycles=30, inner_cycles=inner), stream())
        try:
            ud = torch().zeros_like(fd)
            st, res = mg.mg_solve(H, fd.data_ptr(), ud.data_ptr())
            print("  precision %d: status %d, %d cycles, %.3e" % (prec, res.status, res.cycles,
                                                                  res.rel_residual), flush=True)
            assert st == mg.MG_OK and res.rel_residual <= 1e-10, (prec, res.status)
            err = _exact_error_h(ud, exact, n)
            assert err <= 1.01 * bound, (prec, err, bound)
            out[prec] = ud
        finally:
            mg.mg_destroy(H)
    t = torch()
    rel = (t.linalg.vector_norm(out[1] - out[0]) / t.linalg.vector_norm(out[0])).item()
    assert rel <= 1e-9, rel


@pytest.mark.parametrize("n,coarse,order,nu1,precision", [(65, 0, 4, 2, 0), (65, 1, 4, 2, 0), (129, 1, 4, 2, 1),
                                                          (65, 0, 6, 2, 0), (65, 3, 6, 3, 1), (33, 1, 4, 3, 0)])
def test_two_sweeps_from_zero_in_one_pass(n, coarse, order, nu1, precision, monkeypatch):
    """3D levels entered with a zero iterate take their first two omega-Jacobi sweeps in
    one pass (the first sweep's omega / a0 * f formed on the fly): the same cycles, bit
    for bit, as two passes (MG_Z2=0), and the oracle's to 1e-12 in FP64."""
    f = inputs.smoothed_noise_3d(n)
    out = {}
    for z2 in ("0", "1"):
        monkeypatch.setenv("MG_Z2", z2)
        H = Handle(3, n, coarse=coarse, order=order, nu1=nu1, nu2=2, gamma=2, precision=precision,
                   inner_cycles=1)
        try:
            fd, ud = dev(f), dev(np.zeros_like(f))
            st, res = mg.mg_run_cycles(H.h, fd.data_ptr(), ud.data_ptr(), 3)
            out[z2] = host(ud)
            if z2 == "1" and precision == 0:
                u_ref = np.zeros_like(f)
                H.oracle.solve(u_ref, f, rtol=0.0, max_cycles=3)
                assert np.linalg.norm(out[z2] - u_ref) <= 1e-12 * np.linalg.norm(u_ref)
        finally:
            H.close()
    assert np.array_equal(out["0"], out["1"])


@pytest.mark.parametrize("n,coarse,nu1,nu2,gamma,precision", [(65, 0, 2, 2, 2, 0), (65, 1, 2, 1, 1, 0),
                                                             (129, 1, 2, 2, 2, 1), (65, 0, 3, 3, 1, 0),
                                                             (33, 0, 4, 2, 2, 0)])
def test_two_jacobi_sweeps_in_one_pass(n, coarse, nu1, nu2, gamma, precision, monkeypatch):
    """Pairs of omega-Jacobi sweeps on 3D cross levels run as one pass (the first sweep
    on a plane and its frame, the second two planes behind; MG_X2=1 turns it on for FP32
    too): the cycles of one sweep per pass (MG_X2=0) and the oracle's, to rounding."""
    f = inputs.smoothed_noise_3d(n)
    out = {}
    for x2 in ("0", "1"):
        monkeypatch.setenv("MG_X2", x2)
        H = Handle(3, n, coarse=coarse, nu1=nu1, nu2=nu2, gamma=gamma, precision=precision, inner_cycles=1)
        try:
            fd, ud = dev(f), dev(np.zeros_like(f))
            mg.mg_run_cycles(H.h, fd.data_ptr(), ud.data_ptr(), 3)
            out[x2] = host(ud)
            if x2 == "1" and precision == 0:
                u_ref = np.zeros_like(f)
                H.oracle.solve(u_ref, f, rtol=0.0, max_cycles=3)
                assert np.linalg.norm(out[x2] - u_ref) <= 1e-12 * np.linalg.norm(u_ref)
        finally:
            H.close()
    tol = 1e-13 if precision == 0 else 1e-6
    assert np.linalg.norm(out["1"] - out["0"]) <= tol * np.linalg.norm(out["0"])


@pytest.mark.parametrize("n,coarse,nu1,nu2,gamma,inner", [(65, 1, 2, 2, 2, 1), (65, 0, 2, 1, 1, 2), (129, 1, 2, 2, 2, 1),
                                                          (33, 0, 1, 2, 1, 3), (257, 0, 2, 1, 1, 1)])
def test_fused_correction_equals_separate(n, coarse, nu1, nu2, gamma, inner, monkeypatch):
    """Mixed-precision steps whose last level-0 FP32 sweep adds its result to the FP64
    iterate (the correction fused into the sweep) give, bit for bit, the steps with the
    sweep stored and the correction u += e as a pass of its own (MG_FUSE_CORR=0): the same
    iterate and the same residual history; and both approach the oracle's FP64 solution
    of the same problem."""
    f = inputs.smoothed_noise_3d(n)
    out = {}
    for fuse in ("0", "1"):
        monkeypatch.setenv("MG_FUSE_CORR", fuse)
        H = Handle(3, n, coarse=coarse, nu1=nu1, nu2=nu2, gamma=gamma, precision=1, inner_cycles=inner,
                   max_cycles=30)
        try:
            fd, ud = dev(f), dev(np.zeros_like(f))
            st, res = mg.mg_run_cycles(H.h, fd.data_ptr(), ud.data_ptr(), 3)
            u3 = host(ud)
            st2, res2 = mg.mg_solve(H.h, fd.data_ptr(), ud.data_ptr())
            out[fuse] = (u3, res.hist(), host(ud), res2.hist(), st2, res2.rel_residual)
        finally:
            H.close()
    assert np.array_equal(out["0"][0], out["1"][0])
    assert out["0"][1] == out["1"][1]
    assert np.array_equal(out["0"][2], out["1"][2])
    assert out["0"][3] == out["1"][3] and out["0"][4] == out["1"][4] == mg.MG_OK
    # the solve's residual bounds its error against the exact discrete solution
    rel = out["1"][5]
    assert rel <= 1e-10
    err = oracle.norm(out["1"][2] - dst.solve(f))
    assert err <= 1.01 * rel * oracle.norm(f) / dst.min_eigenvalue(n, 3) + 1e-14 * oracle.norm(out["1"][2])


@pytest.mark.parametrize("n,coarse,gamma,precision", [(65, 1, 2, 0), (129, 1, 1, 0), (65, 3, 2, 0), (129, 1, 2, 1),
                                                      (33, 1, 1, 0)])
def test_galerkin_two_pass_restriction(n, coarse, gamma, precision, monkeypatch):
    """3D Galerkin levels: the defect formed by the pencil kernel and then restricted by
    full weighting (the cycle's default) against the fused separable defect + full
    weighting (MG_GRR_2PASS=0), to rounding; in FP64 also against the oracle's cycles."""
    f = inputs.smoothed_noise_3d(n)
    out = {}
    for two in ("0", "1"):
        monkeypatch.setenv("MG_GRR_2PASS", two)
        H = Handle(3, n, coarse=coarse, nu1=2, nu2=2, gamma=gamma, precision=precision, inner_cycles=1)
        try:
            fd, ud = dev(f), dev(np.zeros_like(f))
            mg.mg_run_cycles(H.h, fd.data_ptr(), ud.data_ptr(), 3)
            out[two] = host(ud)
            if two == "1" and precision == 0:
                u_ref = np.zeros_like(f)
                H.oracle.solve(u_ref, f, rtol=0.0, max_cycles=3)
                assert np.linalg.norm(out[two] - u_ref) <= 1e-12 * np.linalg.norm(u_ref)
        finally:
            H.close()
    tol = 1e-13 if precision == 0 else 1e-6
    assert np.linalg.norm(out["1"] - out["0"]) <= tol * np.linalg.norm(out["0"])
