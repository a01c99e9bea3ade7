"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each test checks the C oracle against something independent of it: stencils and
weights printed in the paper, Fourier symbols printed in the paper, closed forms,
explicit matrices assembled on tiny grids, an exact sine-transform solve, and
manufactured solutions.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import dst, explicit, lfa
from paper_2008_03885_amd import inputs
from conftest import read_golden


# ---------------------------------------------------------------- printed stencils --

def test_fourth_order_stencil_matches_printed():
    printed, factor = read_golden("stencil_4th_order_2d.txt")
    h = 0.125
    s = oracle.fine_stencil(2, 4, h)
    np.testing.assert_allclose(s * h * h, printed * factor, rtol=0, atol=1e-15)
    # The oracle's operator applied to a unit function reproduces the same stencil.
    n = 9
    u = np.zeros((n, n))
    u[4, 4] = 1.0
    Lu = oracle.apply(s, u)
    np.testing.assert_allclose(Lu[2:7, 2:7] * h * h, (printed * factor)[::-1, ::-1], atol=1e-15)


def test_sixth_order_stencil_matches_printed():
    printed, factor = read_golden("stencil_6th_order_2d.txt")
    h = 0.125
    s = oracle.fine_stencil(2, 6, h)
    np.testing.assert_allclose(s * h * h, printed * factor, rtol=0, atol=1e-14)
    # the 3D operator is the sum of the three axis operators (the 1D one is the printed
    # middle row with half its centre)
    s3 = oracle.fine_stencil(3, 6, 1.0)
    axis = printed[3] * factor
    axis[3] /= 2
    off = [0, 1, 2, 4, 5, 6]
    for line in (s3[3, 3, :], s3[3, :, 3], s3[:, 3, 3]):
        np.testing.assert_allclose(line[off], axis[off], atol=1e-14)
    assert abs(s3[3, 3, 3] - 3 * axis[3]) < 1e-13 and abs(s3.sum()) < 1e-12
    assert np.count_nonzero(s3) == 19


def test_3d_operator_is_sum_of_axis_operators():
    s = oracle.fine_stencil(3, 4, 1.0)
    c = np.array([1, -16, 30, -16, 1]) / 12.0
    ref = np.zeros((5, 5, 5))
    ref[2, 2, :] += c
    ref[2, :, 2] += c
    ref[:, 2, 2] += c
    np.testing.assert_allclose(s, ref, atol=1e-15)
    assert np.count_nonzero(s) == 13


def _distribution_weights(prolong, dim=2):
    """Fine values produced by interpolating one interior coarse unit value."""
    nc, nf = 9, 17
    v = np.zeros((nc,) * dim)
    v[(4,) * dim] = 1.0
    u = np.zeros((nf,) * dim)
    oracle.prolong_add(v, u, prolong)
    return u


def test_interpolation_weights_match_printed():
    for name, op, r in (("bilinear_interpolation_2d.txt", oracle.PROLONG_LINEAR, 1),
                        ("cubic_interpolation_2d.txt", oracle.PROLONG_CUBIC, 3)):
        printed, factor = read_golden(name)
        u = _distribution_weights(op)
        np.testing.assert_allclose(u[8 - r:9 + r, 8 - r:9 + r], printed * factor, atol=1e-15)
        assert abs(u.sum() - (printed * factor).sum()) < 1e-14


def test_restriction_weights_match_printed():
    for name, op, r in (("full_weighting_2d.txt", oracle.RESTRICT_FW, 1),
                        ("cubic_restriction_2d.txt", oracle.RESTRICT_CUBIC, 3)):
        printed, factor = read_golden(name)
        nf = 17
        got = np.zeros((2 * r + 1, 2 * r + 1))
        for oy, ox in itertools.product(range(-r, r + 1), repeat=2):
            d = np.zeros((nf, nf))
            d[8 + oy, 8 + ox] = 1.0
            got[oy + r, ox + r] = oracle.restrict(d, op)[4, 4]
        np.testing.assert_allclose(got, printed * factor, atol=1e-15)


def test_galerkin_of_five_point_operator_matches_printed():
    printed, factor = read_golden("galerkin_order2_fw_bilinear_2d.txt")
    h = 1.0 / 16
    H = 2 * h
    sc = oracle.galerkin_stencil(oracle.fine_stencil(2, 2, h), oracle.RESTRICT_FW, oracle.PROLONG_LINEAR)
    R = (sc.shape[0] - 1) // 2
    inner = sc[R - 1:R + 2, R - 1:R + 2]
    np.testing.assert_allclose(inner * H * H, printed * factor, atol=1e-13)
    outer = sc.copy()
    outer[R - 1:R + 2, R - 1:R + 2] = 0
    assert np.abs(outer).max() < 1e-12


def test_second_order_coarse_operators_of_the_hierarchy():
    """Section 3.1: with a fourth-order fine operator, the "Galerkin" second-order coarse
    operator of the hierarchy (full weighting, bilinear interpolation) is the printed
    appendix A.2 operator at level 1, and the rediscretized one is the 5-point operator
    at H on every coarse level (eq. L_H_2d), in the printed units."""
    printed, factor = read_golden("galerkin_order2_fw_bilinear_2d.txt")
    n = 33
    mg = oracle.Multigrid(2, n, coarse=oracle.COARSE_G2, prolong=oracle.PROLONG_LINEAR, n_coarsest=9)
    n1, s1 = mg.level_stencil(1)
    H = 1.0 / (n1 - 1)
    R = (s1.shape[0] - 1) // 2
    np.testing.assert_allclose(s1[R - 1:R + 2, R - 1:R + 2] * H * H, printed * factor, atol=1e-12)
    # level 0 stays the fourth-order operator
    n0, s0 = mg.level_stencil(0)
    np.testing.assert_allclose(s0, oracle.fine_stencil(2, 4, 1.0 / (n - 1)), atol=0)
    mg2 = oracle.Multigrid(2, n, coarse=oracle.COARSE_NG2, n_coarsest=9)
    five = printed * 0
    five[1, :] = [-1, 4, -1]
    five[:, 1] += [-1, 0, -1]
    for l in (1, 2):
        nl, sl = mg2.level_stencil(l)
        Hl = 1.0 / (nl - 1)
        np.testing.assert_allclose(sl * Hl * Hl, five, atol=1e-12)


# ------------------------------------------------------------------ Fourier symbols --

@pytest.mark.parametrize("dim,order", [(2, 4), (3, 4), (2, 2), (3, 2), (2, 6), (3, 6)])
def test_operator_symbol_on_sine_modes(dim, order):
    """L_h sin-mode = symbol(theta) * sin-mode (appendix A.4 eq. L_hat_2d_4o)."""
    n = 17 if dim == 2 else 9
    h = 1.0 / (n - 1)
    s = oracle.fine_stencil(dim, order, h)
    x = np.linspace(0, 1, n)
    rng = np.random.default_rng(1)
    for _ in range(4):
        k = rng.integers(1, n - 1, dim)
        mode = np.ones((n,) * dim)
        for a in range(dim):
            shape = [1] * dim
            shape[dim - 1 - a] = n
            mode = mode * np.sin(k[a] * np.pi * x).reshape(shape)
        lam = lfa.symbol_fine(k * np.pi * h, h, order)
        Lu = oracle.apply(s, mode)
        inner = tuple(slice(1, n - 1) for _ in range(dim))
        np.testing.assert_allclose(Lu[inner], lam * mode[inner], rtol=0, atol=1e-12 * lam)


def test_transfer_symbols_on_sine_modes():
    """Restriction of a fine sine mode k is r(theta) times the coarse mode k; the
    restricted alias N-k is -r(theta_bar) times it (appendix A.2 eq. transfer_2dstd_eqn)."""
    nf = 33
    N = nf - 1
    x = np.linspace(0, 1, nf)
    X = np.linspace(0, 1, N // 2 + 1)
    for op in (oracle.RESTRICT_FW, oracle.RESTRICT_CUBIC):
        for k in (1, 3, 7, 15):
            d = np.outer(np.sin(k * np.pi * x), np.sin(k * np.pi * x))
            fc = oracle.restrict(d, op)
            th = np.array([k * np.pi / N, k * np.pi / N])
            coarse_mode = np.outer(np.sin(k * np.pi * X), np.sin(k * np.pi * X))
            np.testing.assert_allclose(fc, lfa.symbol_transfer(th, op) * coarse_mode, atol=1e-13)
    for op in (oracle.PROLONG_LINEAR, oracle.PROLONG_CUBIC):
        for k in (1, 5, 9, 15):
            v = np.outer(np.sin(k * np.pi * X), np.sin(k * np.pi * X))
            u = oracle.prolong_add(v, np.zeros((nf, nf)), op)
            th = np.array([k * np.pi / N] * 2)
            # components on the four fine modes (k or N-k per axis), by projection
            for ay, ax in itertools.product((0, 1), repeat=2):
                ky, kx = (N - k if ay else k), (N - k if ax else k)
                m = np.outer(np.sin(ky * np.pi * x), np.sin(kx * np.pi * x))
                coef = np.sum(u * m) / np.sum(m * m)
                alias = th + np.pi * np.array([ax, ay])
                sign = (-1) ** (ax + ay)
                np.testing.assert_allclose(coef, sign * lfa.symbol_transfer(alias, op), atol=1e-13)


# ------------------------------------------------------------------- Jacobi optimum --

def test_jacobi_optimum_order2_matches_paper_formula():
    """Section 5.3 eqs. mu_w_J_r / muStarfactorR at r = 2: zeta = sin^2(pi/4)/d."""
    for d in (2, 3):
        zeta = np.sin(np.pi / 4) ** 2 / d
        w, mu = lfa.jacobi_optimum(d, 2)
        assert abs(w - 1 / (1 + zeta)) < 1e-15
        assert abs(mu - (1 - zeta) / (1 + zeta)) < 1e-15


@pytest.mark.parametrize("dim,order,omega,mu", [(2, 4, 10 / 13, 25 / 39), (3, 4, 9 / 11, 41 / 55),
                                                (2, 6, 490 / 653, 435 / 653),
                                                (3, 6, 147 / 185, 707 / 925)])
def test_jacobi_optimum_fourth_order(dim, order, omega, mu):
    w, m = lfa.jacobi_optimum(dim, order)
    assert abs(w - omega) < 1e-15 and abs(m - mu) < 1e-15
    assert abs(oracle.jacobi_omega(dim, order) - omega) < 1e-15
    # The closed form is the supremum of |S| over the high frequencies ...
    sch = lfa.Scheme(dim, order=order, omega=w)
    assert abs(lfa.smoothing_factor(sch, m=32 if dim == 3 else 64) - mu) < 1e-12
    # ... and any other omega smooths worse.
    for dw in (-0.02, 0.02):
        assert lfa.smoothing_factor(lfa.Scheme(dim, order=order, omega=w + dw), m=16) > mu


def test_smoother_diagonal_from_symbol():
    """The centre coefficient recovered from the symbol's mean equals the stencil's."""
    for dim in (2, 3):
        sch = lfa.Scheme(dim, coarse=lfa.GALERKIN)
        h = 1.0 / 16
        assert abs(sch.level_diagonal(0, h) - 30 * dim / (12 * h * h)) < 1e-9
        mg = oracle.Multigrid(dim, 33 if dim == 2 else 17, coarse=oracle.COARSE_GALERKIN,
                              n_coarsest=9)
        n1, s1 = mg.level_stencil(1)
        R = (s1.shape[0] - 1) // 2
        centre = s1[(R,) * dim]
        h0 = 1.0 / (mg.n - 1)
        assert abs(sch.level_diagonal(1, h0) - centre) < 1e-9 * centre


# ------------------------------------------------------- two-grid spectrum (exact) --

def _cycle_matrix(mg, n, dim):
    q = n - 2
    m = q ** dim
    f = np.zeros((n,) * dim)
    M = np.zeros((m, m))
    for p in range(m):
        u = np.zeros((n,) * dim)
        idx = np.unravel_index(p, (q,) * dim)
        u[tuple(i + 1 for i in idx)] = 1.0
        mg.cycle(u, f)
        M[:, p] = u[tuple(slice(1, n - 1) for _ in range(dim))].ravel()
    return M


CASES_2G = [(2, 17, 9, c, p, nu, 0) for c in (0, 1, 2, 3) for p in (1, 3) for nu in ((2, 1), (1, 1))] + \
           [(3, 9, 5, c, 3, (2, 1), 0) for c in (0, 1, 2, 3)] + \
           [(2, 17, 9, c, p, nu, 1) for c in (0, 1, 2, 3) for p in (1, 3) for nu in ((2, 1), (1, 1))] + \
           [(2, 13, 7, 0, 3, (1, 1), 1), (3, 9, 5, 0, 3, (2, 1), 1), (3, 9, 5, 1, 3, (1, 1), 1),
            (3, 9, 5, 3, 1, (2, 1), 1)]


@pytest.mark.parametrize("dim,n,nc,coarse,prolong,nu,smoother", CASES_2G)
def test_two_grid_spectrum_equals_lfa(dim, n, nc, coarse, prolong, nu, smoother):
    """The computed two-grid operator has exactly the eigenvalues the LFA symbols give
    on the finite grid (section 2.2 eqs. K, M_2level; appendix A.2 eq. M_2), for
    omega-Jacobi and for red-black Jacobi (section 5.3 eqs. S_hat_F, M_2)."""
    mg = oracle.Multigrid(dim, n, coarse=coarse, prolong=prolong, nu1=nu[0], nu2=nu[1],
                          n_coarsest=nc, smoother=smoother)
    assert mg.levels == 2
    ev = np.linalg.eigvals(_cycle_matrix(mg, n, dim))
    sch = lfa.Scheme(dim, coarse=coarse, prolong=prolong, nu1=nu[0], nu2=nu[1], smoother=smoother)
    ref = lfa.finite_two_grid_spectrum(sch, n)
    assert len(ev) == len(ref)
    key = lambda z: (round(z.real, 9), round(z.imag, 9))
    a = np.array(sorted(ev, key=key))
    b = np.array(sorted(ref.astype(complex), key=key))
    # multiple eigenvalues of a non-normal matrix are only determined to ~sqrt(eps)
    np.testing.assert_allclose(a, b, atol=1e-9)


def test_two_grid_rho_values():
    """LFA two-grid factors at omega*: 2D V(2,1) close to mu*^3 for every operator/transfer."""
    for coarse in (lfa.NG, lfa.GALERKIN):
        for prolong in (lfa.LINEAR, lfa.CUBIC):
            rho = lfa.two_grid_rho(lfa.Scheme(2, coarse=coarse, prolong=prolong), m=24)
            assert 0.255 < rho < (25 / 39) ** 3 + 1e-9


@pytest.mark.parametrize("gamma", [1, 2])
@pytest.mark.parametrize("coarse", [0, 1, 2, 3])
@pytest.mark.parametrize("smoother", [0, 1])
def test_multilevel_cycle_matches_explicit_matrices(gamma, coarse, smoother):
    """Three-level V and W cycles equal the composition of explicit matrices by the
    recursion of section 2.2 (eqs. K_l, M) with appendix A.3.1 eq. L_H_approx; the
    red-black smoother as the product of masked Jacobi matrices (section 3.1 eq. S_rb)."""
    dim, n = 2, 17
    mg = oracle.Multigrid(dim, n, coarse=coarse, gamma=gamma, n_coarsest=5, smoother=smoother)
    assert mg.levels == 3
    M = _cycle_matrix(mg, n, dim)
    ns = [17, 9, 5]
    stencils = [mg.level_stencil(l)[1] for l in range(3)]
    As = [explicit.operator(s, ns[l]) for l, s in enumerate(stencils)]
    a0 = [s[((s.shape[0] - 1) // 2,) * dim] for s in stencils]
    Me = explicit.cycle_matrix(As, a0, mg.cfg.omega, 2, 1, gamma, dim, ns, rb=smoother == 1)
    np.testing.assert_allclose(M, Me, atol=1e-13)


@pytest.mark.parametrize("coarse,prolong,smoother", [(0, 1, 0), (1, 1, 0), (2, 1, 0), (3, 1, 0),
                                                    (0, 3, 0), (3, 3, 1), (0, 1, 1)])
def test_two_grid_spectrum_equals_lfa_sixth_order(coarse, prolong, smoother):
    """Sixth-order fine operator (section 3.3) with the transfers of eq. transfer_2d or cubic
    interpolation, the four coarse operators, both smoothers: exact finite-grid spectra."""
    n = 17
    mg = oracle.Multigrid(2, n, order=6, coarse=coarse, prolong=prolong, nu1=1, nu2=1,
                          n_coarsest=9, smoother=smoother)
    assert mg.levels == 2
    ev = np.linalg.eigvals(_cycle_matrix(mg, n, 2))
    sch = lfa.Scheme(2, order=6, coarse=coarse, prolong=prolong, nu1=1, nu2=1, smoother=smoother,
                     omega=mg.cfg.omega)
    ref = lfa.finite_two_grid_spectrum(sch, n)
    key = lambda z: (round(z.real, 9), round(z.imag, 9))
    a = np.array(sorted(ev, key=key))
    b = np.array(sorted(ref.astype(complex), key=key))
    np.testing.assert_allclose(a, b, atol=1e-9)


def test_sixth_order_galerkin_equals_brute_force_rap():
    """R L_h P of the sixth-order operator by the oracle's definition-based construction
    against explicit matrices; the coarse stencil keeps radius 3."""
    n = 17
    sf = oracle.fine_stencil(2, 6, 1.0 / (n - 1))
    sc = oracle.galerkin_stencil(sf, oracle.RESTRICT_FW, oracle.PROLONG_CUBIC)
    assert sc.shape == (7, 7)
    A = explicit.operator(sf, n)
    Rm = explicit.restriction(2, n, 1)
    Pm = explicit.prolongation(2, n, 3)
    Ac = explicit.galerkin(Rm, A, Pm).toarray()
    nc = (n - 1) // 2 + 1
    # interior rows far from the boundary equal the stencil
    Ae = explicit.operator(sc, nc).toarray()
    q = nc - 2
    for J in range(3, q - 3):
        for I in range(3, q - 3):
            row = J * q + I
            np.testing.assert_allclose(Ac[row], Ae[row], atol=1e-9 * np.abs(Ae).max())


# ------------------------------------------------------------ red-black smoothing --

def test_rb_symbol_matches_printed_five_point():
    """For the five-point operator the alias-mask construction of the red-black sweep
    reduces to the printed 2 x 2 symbols (section 5.3 eq. S_hat_RB_2d, with xi of eq. xi_r2)
    on span{theta, theta + (pi, pi)}, and leaves the other pair of aliases to itself."""
    rng = np.random.default_rng(11)
    for w in (1.0, 0.8, 1.2):
        sch = lfa.Scheme(2, order=2, omega=w, smoother=lfa.RBJ)
        for _ in range(5):
            th = rng.uniform(-np.pi / 2, np.pi / 2, 2)
            xi = 0.5 * (np.sin(th[0] / 2) ** 2 + np.sin(th[1] / 2) ** 2)
            D = np.diag([xi, 1 - xi])
            SR = np.eye(2) - w * np.array([[1.0, -1.0], [-1.0, 1.0]]) @ D
            SB = np.eye(2) - w * np.array([[1.0, 1.0], [1.0, 1.0]]) @ D
            S = sch.smoother_matrix(th)  # aliases (0,0), (0,1), (1,0), (1,1)
            np.testing.assert_allclose(S[np.ix_([0, 3], [0, 3])], SB @ SR, atol=1e-14)
            assert np.abs(S[np.ix_([0, 3], [1, 2])]).max() < 1e-15
            assert np.abs(S[np.ix_([1, 2], [0, 3])]).max() < 1e-15


@pytest.mark.parametrize("nu,rho", [(1, 0.250), (2, 0.074), (3, 0.053), (4, 0.041)])
def test_rb_five_point_two_grid_factors_textbook(nu, rho):
    """For the five-point operator red-black Jacobi is red-black Gauss-Seidel (no
    same-colour neighbours).  Its LFA two-grid factors with full weighting and bilinear
    interpolation at omega = 1 are the classical 0.250, 0.074, 0.053, 0.041 for nu = 1..4
    (U. Trottenberg, C. W. Oosterlee, A. Schueller, Multigrid, 2001, section 4.5), and its
    smoothing factor (section 5.3 eq. mu_2_2) is 1/4."""
    sch = lfa.Scheme(2, order=2, prolong=lfa.LINEAR, nu1=nu, nu2=0, omega=1.0, smoother=lfa.RBJ)
    assert abs(lfa.two_grid_rho(sch, m=96) - rho) < 5e-4
    assert abs(lfa.rb_smoothing_factor(sch, 1, m=32) - 0.25) < 1e-12


def _rb_gauss_seidel_five_point(f, u, h, omega):
    """In-place Gauss-Seidel over the red points (odd i+j), then the black points, for
    the five-point operator (section 5.3): each point solves its own equation given its
    neighbours' current values, over-relaxed by omega."""
    n = u.shape[0]
    u = u.copy()
    for colour in (1, 0):
        for j in range(1, n - 1):
            for i in range(1, n - 1):
                if (i + j) % 2 != colour:
                    continue
                nb = u[j, i - 1] + u[j, i + 1] + u[j - 1, i] + u[j + 1, i]
                gs = (h * h * f[j, i] + nb) / 4.0
                u[j, i] = (1 - omega) * u[j, i] + omega * gs
    return u


def test_rb_partial_steps_equal_gauss_seidel_five_point():
    """The red then black partial steps of the oracle equal in-place red-black
    Gauss-Seidel for the five-point operator, which pins the colour of every point."""
    n = 11
    h = 1.0 / (n - 1)
    rng = np.random.default_rng(5)
    f = np.zeros((n, n))
    u = np.zeros((n, n))
    f[1:-1, 1:-1] = rng.standard_normal((n - 2, n - 2))
    u[1:-1, 1:-1] = rng.standard_normal((n - 2, n - 2))
    s = oracle.fine_stencil(2, 2, h)
    for w in (1.0, 1.15):
        red = oracle.jacobi_colour(s, w, 1, f, u)
        both = oracle.jacobi_colour(s, w, 2, f, red)
        np.testing.assert_allclose(both, _rb_gauss_seidel_five_point(f, u, h, w), atol=1e-12)
        odd = (np.add.outer(np.arange(n), np.arange(n)) % 2) == 1
        assert np.array_equal(red[~odd], u[~odd])  # the red step leaves black points alone
    np.testing.assert_array_equal(oracle.jacobi_colour(s, 0.9, 0, f, u), oracle.jacobi(s, 0.9, f, u))


@pytest.mark.parametrize("dim,order,coarse", [(d, o, c) for d in (2, 3) for o in (4, 6) for c in range(4)]
                         + [(2, 2, 0), (2, 2, 1), (3, 2, 0), (3, 2, 1)])
def test_rbj_default_omega_is_lfa_optimum(dim, order, coarse):
    """The default red-black omega minimises the LFA two-grid factor of V(2,1) for each coarse
    operator (the reading that omega is chosen for rho rather than mu, section 2.2 after
    eq. mu; section 3.1 re-tunes omega per coarse operator)."""
    w, rho = lfa.rbj_optimum(dim, order, coarse=coarse)
    assert abs(w - oracle.rbj_omega(dim, order, coarse)) < 0.01
    assert lfa.RBJ_OMEGA[(dim, order, coarse)] == oracle.rbj_omega(dim, order, coarse)
    jac = lfa.two_grid_rho(lfa.Scheme(dim, order=order, coarse=coarse), m=12 if dim == 3 else 24)
    assert rho < 0.2 * jac  # red-black Jacobi beats omega-Jacobi per sweep by far here


# ------------------------------------------------- red-black Gauss-Seidel (S_GS) --

def _gs_partial_step_by_matrices(s, omega, colour, f, u):
    """Section 3.1 eq. S_GS written with explicit matrices: on the unknowns of the colour,
    (a_0/omega I + A_low) x = a_0/omega u_c + f_c - (A u)_c + A_low u_c, A the folded
    operator matrix and A_low its strictly lower part (earlier unknowns in lexicographic
    order, x fastest) between points of the colour; a triangular solve."""
    import scipy.sparse as sps
    import scipy.sparse.linalg as spla
    n = u.shape[0]
    A = explicit.operator(s, n).tocsr()
    a0 = s[(s.shape[0] // 2,) * s.ndim]
    idx = [tuple(reversed(t)) for t in itertools.product(range(1, n - 1), repeat=s.ndim)]  # x fastest
    pts = [p for p, ijk in enumerate(idx) if (sum(ijk) % 2 == 1) == (colour == 1)]
    interior = (slice(1, n - 1),) * s.ndim
    uv = u[interior].reshape(-1)
    fv = f[interior].reshape(-1)
    Acc = A[pts][:, pts]
    low = sps.tril(Acc, k=-1).tocsr()
    rhs = a0 / omega * uv[pts] + fv[pts] - (A @ uv)[pts] + low @ uv[pts]
    M = (low + (a0 / omega) * sps.identity(len(pts))).tocsr()
    x = spla.spsolve_triangular(M, rhs, lower=True)
    out = uv.copy()
    out[pts] = x
    res = u.copy()
    res[interior] = out.reshape((n - 2,) * s.ndim)
    return res


@pytest.mark.parametrize("dim,n,order", [(2, 11, 4), (2, 17, 4), (2, 13, 6), (3, 9, 4)])
def test_gs_partial_step_is_the_triangular_solve(dim, n, order):
    """The oracle's in-place lexicographic sweep of a colour equals the explicit-matrix
    form of -(L+)^{-1} L- (L+ = a_0/omega + the earlier same-colour entries), boundary
    rows included."""
    h = 1.0 / (n - 1)
    s = oracle.fine_stencil(dim, order, h)
    rng = np.random.default_rng(31)
    f = np.zeros((n,) * dim)
    u = np.zeros((n,) * dim)
    f[(slice(1, -1),) * dim] = rng.standard_normal((n - 2,) * dim) / h ** 2
    u[(slice(1, -1),) * dim] = rng.standard_normal((n - 2,) * dim)
    for w in (1.0, 1.16):
        for c in (1, 2):
            got = oracle.gs_colour(s, w, c, f, u)
            ref = _gs_partial_step_by_matrices(s, w, c, f, u)
            np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
            # the other colour is left alone
            other = (np.indices(u.shape).sum(axis=0) % 2 == 1) != (c == 1)
            assert np.array_equal(got[other], u[other])


def test_gs_equals_jacobi_partial_step_for_five_point():
    """With no same-colour neighbours (five-point operator) the Gauss-Seidel partial step
    is the Jacobi partial step, to the bit."""
    n = 17
    s = oracle.fine_stencil(2, 2, 1.0 / (n - 1))
    rng = np.random.default_rng(3)
    f, u = np.zeros((n, n)), np.zeros((n, n))
    f[1:-1, 1:-1] = rng.standard_normal((n - 2, n - 2))
    u[1:-1, 1:-1] = rng.standard_normal((n - 2, n - 2))
    for c in (1, 2):
        assert np.array_equal(oracle.gs_colour(s, 1.1, c, f, u), oracle.jacobi_colour(s, 1.1, c, f, u))


def test_gs_symbol_matches_printed():
    """The LFA's Gauss-Seidel symbol, built as 1 - L^/L+^, equals the symbol appendix A.4
    prints for eq. S_GS with the fourth-order operator:
    -(60(1 - 1/omega) - 32(cos t1 + cos t2) + e^{2 i t1} + e^{2 i t2}) /
     (60/omega + e^{-2 i t1} + e^{-2 i t2})."""
    rng = np.random.default_rng(8)
    for w in (0.9, 1.0, 1.2, 1.5):
        sch = lfa.Scheme(2, 4, omega=w, smoother=lfa.RBGS)
        for _ in range(6):
            t = rng.uniform(-np.pi, np.pi, 2)
            printed = -(60 * (1 - 1 / w) - 32 * (np.cos(t[0]) + np.cos(t[1])) + np.exp(2j * t[0])
                        + np.exp(2j * t[1])) / (60 / w + np.exp(-2j * t[0]) + np.exp(-2j * t[1]))
            assert abs(sch.gs_symbol(t) - printed) < 1e-13
    # five-point operator: the Jacobi symbol
    sch = lfa.Scheme(2, 2, omega=1.1, smoother=lfa.RBGS)
    t = np.array([0.4, -2.0])
    assert abs(sch.gs_symbol(t) - sch.smoother_symbol(t)) < 1e-14


@pytest.mark.parametrize("n,nc,w", [(65, 33, 1.0), (129, 65, 1.16)])
def test_rbgs_two_level_rate_near_lfa(n, nc, w):
    """Two-level V(2,1) cycles with red-black Gauss-Seidel: the measured asymptotic rate is
    within 15% of the LFA two-grid factor.  Unlike the Jacobi smoothers, lexicographic
    Gauss-Seidel does not map sine modes to sine modes, so the finite Dirichlet grid is
    only close to the infinite-grid analysis (measured: 0.048 vs 0.050, 0.0155 vs 0.0165)."""
    mg = oracle.Multigrid(2, n, n_coarsest=nc, nu1=2, nu2=1, smoother=oracle.SMOOTH_RBGS, omega=w)
    assert mg.levels == 2
    s = mg.level_stencil(0)[1]
    rng = np.random.default_rng(5)
    f, u = np.zeros((n, n)), np.zeros((n, n))
    u[1:-1, 1:-1] = rng.standard_normal((n - 2, n - 2))
    r = [oracle.norm(oracle.residual(s, f, u))]
    for _ in range(14):
        mg.cycle(u, f)
        r.append(oracle.norm(oracle.residual(s, f, u)))
    cr = r[-1] / r[-2]
    rho = lfa.two_grid_rho(lfa.Scheme(2, 4, nu1=2, nu2=1, omega=w, smoother=lfa.RBGS), m=32)
    assert 0.85 * rho <= cr <= 1.15 * rho, (cr, rho)


@pytest.mark.parametrize("order,coarse", [(4, 0), (4, 2), (6, 0), (6, 2)])
def test_rbgs_default_omega_is_lfa_optimum(order, coarse):
    w, rho = lfa.rbgs_optimum(order, coarse=coarse)
    assert abs(w - oracle.rbgs_omega(2, order, coarse)) < 0.01
    assert lfa.RBGS_OMEGA[(2, order, coarse)] == oracle.rbgs_omega(2, order, coarse)
    assert rho < 0.2 * lfa.two_grid_rho(lfa.Scheme(2, order=order, coarse=coarse), m=24)


# ----------------------------------------------------------------- brute-force RAP --

@pytest.mark.parametrize("dim,n,prolong", [(2, 9, 3), (2, 17, 3), (2, 33, 3), (2, 17, 1), (3, 9, 3)])
def test_galerkin_equals_brute_force_rap(dim, n, prolong):
    """The stencil-form Galerkin operator, folded at the boundary, equals R*A*P built
    from explicit matrices on the finite grid (eq. L_H_G)."""
    h = 1.0 / (n - 1)
    sf = oracle.fine_stencil(dim, 4, h)
    sc = oracle.galerkin_stencil(sf, oracle.RESTRICT_FW, prolong)
    A = explicit.operator(sf, n)
    G = explicit.galerkin(explicit.restriction(dim, n, 1), A, explicit.prolongation(dim, n, prolong))
    nc = (n - 1) // 2 + 1
    Ac = explicit.operator(sc, nc)
    scale = np.abs(G).max()
    assert np.abs(G - Ac).max() <= 1e-13 * scale
    if nc >= 9:
        # second generation: R * (R A P) * P
        sc2 = oracle.galerkin_stencil(sc, oracle.RESTRICT_FW, prolong)
        G2 = explicit.galerkin(explicit.restriction(dim, nc, 1), Ac, explicit.prolongation(dim, nc, prolong))
        Ac2 = explicit.operator(sc2, (nc - 1) // 2 + 1)
        assert np.abs(G2 - Ac2).max() <= 1e-13 * np.abs(G2).max()


@pytest.mark.parametrize("dim,n,prolong", [(2, 17, 3), (2, 33, 1), (3, 17, 3)])
def test_second_order_galerkin_equals_brute_force_rap(dim, n, prolong):
    """The hierarchy's "Galerkin" second-order coarse operators (section 3.1 eq.
    L_H_2G_2d): level 1 equals R A2 P with A2 the explicit second-order operator at the
    finest spacing, level 2 equals R A1 P, from explicit matrices."""
    mg = oracle.Multigrid(dim, n, coarse=oracle.COARSE_G2, prolong=prolong, n_coarsest=5)
    A2 = explicit.operator(oracle.fine_stencil(dim, 2, 1.0 / (n - 1)), n)
    G1 = explicit.galerkin(explicit.restriction(dim, n, 1), A2, explicit.prolongation(dim, n, prolong))
    n1, s1 = mg.level_stencil(1)
    A1 = explicit.operator(s1, n1)
    assert np.abs(G1 - A1).max() <= 1e-13 * np.abs(G1).max()
    G2 = explicit.galerkin(explicit.restriction(dim, n1, 1), A1, explicit.prolongation(dim, n1, prolong))
    n2, s2 = mg.level_stencil(2)
    assert np.abs(G2 - explicit.operator(s2, n2)).max() <= 1e-13 * np.abs(G2).max()


def test_galerkin_radius_with_cubic_interpolation():
    """FW + cubic: radius 3 at the first coarse level and it stays 3."""
    h = 1.0 / 64
    s = oracle.fine_stencil(2, 4, h)
    for _ in range(3):
        s = oracle.galerkin_stencil(s, oracle.RESTRICT_FW, oracle.PROLONG_CUBIC)
        assert s.shape == (7, 7)
        assert np.allclose(s, s.T) and np.allclose(s, s[::-1, :])
        assert abs(s.sum()) < 1e-9 * np.abs(s).max()  # annihilates constants


# -------------------------------------------------------------- exact discrete solve --

@pytest.mark.parametrize("dim,n", [(2, 17), (2, 33), (3, 9)])
def test_dst_solve_equals_dense_solve(dim, n):
    A = explicit.operator(oracle.fine_stencil(dim, 4, 1.0 / (n - 1)), n).toarray()
    rng = np.random.default_rng(7)
    f = np.zeros((n,) * dim)
    inner = tuple(slice(1, n - 1) for _ in range(dim))
    f[inner] = rng.standard_normal((n - 2,) * dim)
    u = dst.solve(f)
    ref = np.linalg.solve(A, f[inner].ravel())
    np.testing.assert_allclose(u[inner].ravel(), ref, rtol=1e-11, atol=1e-14)


def test_sine_series_closed_form_equals_dst():
    n = 65
    _, f, c = inputs.manufactured_2d(n)
    np.testing.assert_allclose(dst.discrete_solution_of_sine_series(n, c), dst.solve(f), atol=1e-12)


def test_manufactured_solution_converges_at_fourth_order():
    """Discretization error of the exact discrete solution falls by ~16 per refinement."""
    errs = []
    ns = [17, 33, 65, 129, 257]
    for n in ns:
        ustar, f, c = inputs.manufactured_2d(n)
        u = dst.discrete_solution_of_sine_series(n, c)
        errs.append(np.abs(u - ustar).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders[1:] > 3.8) and np.all(orders[1:] < 4.2), orders


def test_manufactured_solution_converges_at_sixth_order():
    """Sixth-order operator (section 3.3): the error falls by ~64 per refinement, and the
    oracle's stencil applied to the DST solution gives back f."""
    errs = []
    for n in [33, 65, 129, 257]:
        ustar, f, c = inputs.manufactured_2d(n)
        u = dst.discrete_solution_of_sine_series(n, c, order=6)
        errs.append(np.abs(u - ustar).max())
        if n == 65:
            # the sine transform with the sixth-order eigenvalues inverts the oracle's
            # stencil with its odd-reflection closure (radius 3 reaches two points out)
            g = oracle.apply(oracle.fine_stencil(2, 6, 1.0 / (n - 1)), np.ascontiguousarray(u))
            np.testing.assert_allclose(dst.solve(g, order=6), u, atol=1e-11 * np.abs(u).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 5.7) and np.all(orders < 6.3), orders


def test_multigrid_converges_to_exact_discrete_solution():
    """The oracle's V(2,1) solve reaches the DST solution within the iteration bound."""
    n = 129
    ustar, f, c = inputs.manufactured_2d(n)
    mg = oracle.Multigrid(2, n)
    u = np.zeros((n, n))
    cycles, hist = mg.solve(u, f, rtol=1e-12, max_cycles=60)
    assert hist[-1] <= 1e-12
    exact = dst.discrete_solution_of_sine_series(n, c)
    # ||u - u_h|| <= ||L^-1|| ||r||, ||L^-1|| = 1/lambda_min
    lam_min = dst.eigenvalues(n, 2).min()
    bound = hist[-1] * oracle.norm(f) / lam_min
    err = oracle.norm(u - exact)
    assert err <= 1.01 * bound + 1e-15
    # The remaining distance to u* is the discretization error of the exact discrete solution.
    disc = np.abs(exact - ustar).max()
    assert abs(np.abs(u - ustar).max() - disc) < 1e-3 * disc


def test_measured_two_grid_rate_matches_lfa():
    """CR from residual ratios (section 2.2 eq. CR) approaches the LFA two-grid factor.
    Homogeneous problem, so the iterate decays without meeting a rounding floor."""
    n = 65
    mg = oracle.Multigrid(2, n, n_coarsest=33)
    assert mg.levels == 2
    s = mg.level_stencil(0)[1]
    rng = np.random.default_rng(3)
    f = np.zeros((n, n))
    u = np.zeros((n, n))
    u[1:-1, 1:-1] = rng.standard_normal((n - 2, n - 2))
    r = [oracle.norm(oracle.residual(s, f, u))]
    for _ in range(100):
        mg.cycle(u, f)
        r.append(oracle.norm(oracle.residual(s, f, u)))
    cr = r[-1] / r[-2]
    rho = np.abs(lfa.finite_two_grid_spectrum(lfa.Scheme(2), n)).max()
    assert rho - 0.01 * rho < cr <= rho * (1 + 1e-9)


@pytest.mark.parametrize("gamma,coarse,smoother", [(1, 0, 0), (2, 0, 0), (1, 2, 0), (1, 3, 0),
                                                (2, 3, 0), (1, 0, 1), (2, 1, 1)])
def test_multilevel_rate_is_near_two_grid_rate(gamma, coarse, smoother):
    """Measured multilevel rate against the LFA two-grid factor of the same coarse
    operator (for the second-order ones, section 3.1's claim that the lower-order coarse
    operator does not slow the cycle is what the LFA quantifies)."""
    n = 129
    mg = oracle.Multigrid(2, n, gamma=gamma, coarse=coarse, smoother=smoother)
    s = mg.level_stencil(0)[1]
    rng = np.random.default_rng(4)
    f = np.zeros((n, n))
    u = np.zeros((n, n))
    u[1:-1, 1:-1] = rng.standard_normal((n - 2, n - 2))
    r = [oracle.norm(oracle.residual(s, f, u))]
    for _ in range(40):
        mg.cycle(u, f)
        r.append(oracle.norm(oracle.residual(s, f, u)))
    cr = r[-1] / r[-2]
    rho2 = lfa.two_grid_rho(lfa.Scheme(2, coarse=coarse, smoother=smoother), m=16)
    assert rho2 - 0.01 <= cr <= rho2 + 0.05


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("coarse,smoother", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_three_grid_with_exact_level1_solve_splits_into_two_grid_blocks(dim, coarse, smoother):
    """With the level-1 equation solved exactly the 4^d modes theta + (pi/2) k decouple
    into the 2^d alias sets of theta + (pi/2) b, b in {0,1}^d, so the three-level symbol's
    eigenvalues are those of the two-grid symbols at those frequencies (the mode
    bookkeeping of the three-level analysis, eq. M_3level, checked against eq. M_2level)."""
    sch = lfa.Scheme(dim, coarse=coarse, smoother=smoother)
    rng = np.random.default_rng(11)
    for theta in rng.uniform(-np.pi / 4, np.pi / 4, size=(3, dim)):
        e3 = np.linalg.eigvals(sch.three_grid_matrix(theta, gamma=None))
        e2 = np.concatenate([np.linalg.eigvals(sch.two_grid_matrix(theta + (np.pi / 2) * np.array(b)))
                             for b in itertools.product((0, 1), repeat=dim)])
        assert len(e3) == len(e2) == 4 ** dim
        assert max(np.min(np.abs(e2 - z)) for z in e3) < 1e-12
        assert max(np.min(np.abs(e3 - z)) for z in e2) < 1e-12


@pytest.mark.parametrize("dim,n,nc,m", [(2, 129, 33, 16), (3, 33, 9, 6)])
@pytest.mark.parametrize("gamma,coarse,smoother", [(1, 0, 0), (2, 0, 0), (1, 1, 0), (1, 3, 0),
                                                (1, 0, 1), (2, 1, 1)])
def test_measured_three_level_rate_matches_three_grid_lfa(dim, n, nc, m, gamma, coarse, smoother):
    """A three-level cycle's measured asymptotic rate (section 2.2 eq. CR) against the
    three-level Fourier analysis (eqs. K_l and M; the approximate level-1 solve of eq.
    L_H_approx).  For the red-black V-cycle the level-1 V-cycle's own error is visible:
    the rate is well above the two-grid factor and the three-level analysis predicts it."""
    mg = oracle.Multigrid(dim, n, n_coarsest=nc, gamma=gamma, coarse=coarse, smoother=smoother)
    assert mg.levels == 3
    s = mg.level_stencil(0)[1]
    rng = np.random.default_rng(5)
    f = np.zeros((n,) * dim)
    u = np.zeros((n,) * dim)
    u[(slice(1, -1),) * dim] = rng.standard_normal((n - 2,) * dim)
    r = [oracle.norm(oracle.residual(s, f, u))]
    for _ in range(40 if smoother == oracle.SMOOTH_JACOBI else 20):
        mg.cycle(u, f)
        r.append(oracle.norm(oracle.residual(s, f, u)))
    cr = r[-1] / r[-2]
    sch = lfa.Scheme(dim, coarse=coarse, smoother=smoother)
    rho3 = lfa.three_grid_rho(sch, m, gamma)
    assert 0.93 * rho3 <= cr <= 1.02 * rho3
    if gamma == 1 and smoother == oracle.SMOOTH_RBJ:
        assert cr > 1.2 * lfa.two_grid_rho(sch, m=2 * m)

def test_residual_norm_long_double_agrees():
    n = 65
    _, f, _ = inputs.manufactured_2d(n)
    s = oracle.fine_stencil(2, 4, 1.0 / (n - 1))
    rng = np.random.default_rng(5)
    u = np.zeros((n, n))
    u[1:-1, 1:-1] = rng.standard_normal((n - 2, n - 2))
    a = oracle.norm(oracle.residual(s, f, u))
    b = oracle.residual_norm_ld(s, f, u)
    assert abs(a - b) <= 1e-13 * b


def _sine_mode(n, k):
    """prod_a sin(k_a pi x_a) on the n-point grid, exactly zero on the boundary; k is
    (kx, ky[, kz]) and the array is indexed [z][y][x]."""
    x = np.linspace(0.0, 1.0, n)
    v = np.ones((n,) * len(k))
    for a, ka in enumerate(k):
        shape = [1] * len(k)
        shape[len(k) - 1 - a] = n
        line = np.sin(ka * np.pi * x)
        line[0] = line[-1] = 0.0
        v = v * line.reshape(shape)
    return v


@pytest.mark.parametrize("dim,n,modes", [
    (2, 33, [(1, 1), (3, 7), (31, 1), (16, 16), (31, 31)]),
    (3, 17, [(1, 1, 1), (2, 5, 15), (8, 8, 8), (15, 1, 15)]),
])
def test_norm_of_sine_modes_is_closed_form(dim, n, modes):
    """The grid norm ||v||_h = (h^dim sum over interior points of v^2)^(1/2) of a sine
    mode is 2^(-dim/2) exactly: along an axis the interior sum of sin^2(k pi i/N) is N/2
    for 1 <= k <= N-1 (N = n-1), and h^dim (N/2)^dim = 2^-dim.  Boundary values are not
    part of the norm."""
    for k in modes:
        v = _sine_mode(n, k)
        assert abs(oracle.norm(v) - 2.0 ** (-dim / 2)) <= 1e-14, k
        assert abs(oracle.norm(-3.5 * v) - 3.5 * 2.0 ** (-dim / 2)) <= 1e-13, k
        w = v.copy()
        w[0] = 7.0      # a whole boundary face (z = 0 in 3D, y = 0 in 2D)
        w[..., -1] = -2.0
        assert oracle.norm(w) == oracle.norm(v)


@pytest.mark.parametrize("dim,n,k", [(2, 33, (1, 1)), (2, 33, (5, 29)), (2, 65, (64 - 1, 2)),
                                     (3, 17, (1, 2, 3)), (3, 17, (15, 15, 15)), (3, 33, (7, 1, 30))])
def test_residual_norms_of_a_sine_mode(dim, n, k):
    """With u a sine mode and f = c u, f - L_h u = (c - lambda_k) u: the odd-reflection
    closure makes the mode an exact eigenfunction, with lambda_k the fourth-order symbol
    of appendix A.4, (4/h^2) sum_a (s_a + s_a^2/3), s_a = sin^2(k_a pi h/2).  So both
    residual norms (FP64 and long double) equal |c - lambda_k| 2^(-dim/2)."""
    h = 1.0 / (n - 1)
    s = np.sin(np.array(k) * np.pi * h / 2.0) ** 2
    lam = 4.0 / h ** 2 * np.sum(s + s * s / 3.0)
    u = _sine_mode(n, k)
    st = oracle.fine_stencil(dim, 4, h)
    for c in (0.0, 0.5 * lam, 2.0 * lam):
        f = c * u
        expect = abs(c - lam) * 2.0 ** (-dim / 2)
        tol = 1e-12 * lam
        assert abs(oracle.norm(oracle.residual(st, f, u)) - expect) <= tol, c
        assert abs(oracle.residual_norm_ld(st, f, u) - expect) <= tol, c


def test_coarsest_solve_is_exact():
    mg = oracle.Multigrid(3, 17, n_coarsest=9)
    n, s = mg.level_stencil(mg.levels - 1)
    rng = np.random.default_rng(6)
    g = np.zeros((n,) * 3)
    g[1:-1, 1:-1, 1:-1] = rng.standard_normal((n - 2,) * 3)
    v = mg.coarsest_solve(g)
    r = oracle.residual(s, g, v)
    assert oracle.norm(r) <= 1e-13 * oracle.norm(g)
