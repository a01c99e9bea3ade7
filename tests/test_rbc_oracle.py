"""Pins of the red-black coarsening oracle (section 4.3 Theorems 3 and 4, section 4.4)
against what the paper prints and what the mathematics fixes."""
import numpy as np
import pytest

from oracle import rbc
from conftest import read_golden


def _rhs(n, seed):
    f = np.zeros((n, n))
    f[1:-1, 1:-1] = np.random.default_rng(seed).standard_normal((n - 2, n - 2))
    return f


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_transfers_match_printed(level):
    """eq. transfer_r2 on every level, in that level's own axes: the F neighbours of a C
    point are its axis neighbours on an even level and its diagonal ones on an odd level
    (the rotated grid's axes)."""
    R, rf = read_golden("rbc_restriction_2d.txt")
    P, pf = read_golden("rbc_interpolation_2d.txt")
    mg = rbc.RBC(33, level + 2)
    m = mg.size(level)
    c = (m // 2, m // 2) if level % 2 == 0 else (m // 2 - (m // 2) % 2,) * 2
    assert mg.masks(level)[1][c]
    to_c = lambda c: c if level % 2 == 0 else (c[0] // 2, c[1] // 2)
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            off = (a, b) if level % 2 == 0 else (a + b, b - a)  # rotated (a, b) -> storage
            e = np.zeros((m, m))
            e[c[0] + off[0], c[1] + off[1]] = 1.0
            assert mg.restrict(level, e)[to_c(c)] == pytest.approx(rf * R[a + 1, b + 1], abs=1e-15)
    ec = np.zeros((mg.size(level + 1),) * 2)
    ec[to_c(c)] = 1.0
    fine = mg.prolong(level, ec)
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            off = (a, b) if level % 2 == 0 else (a + b, b - a)
            assert fine[c[0] + off[0], c[1] + off[1]] == pytest.approx(pf * P[a + 1, b + 1], abs=1e-15)
    assert np.count_nonzero(fine) == 5


def _galerkin(mg, l):
    act_f, act_c = mg.masks(l)[0], mg.masks(l + 1)[0]
    idx_f, idx_c = np.argwhere(act_f), np.argwhere(act_c)
    P = np.zeros((len(idx_f), len(idx_c)))
    R = np.zeros((len(idx_c), len(idx_f)))
    for k, (i, j) in enumerate(idx_c):
        e = np.zeros(act_c.shape)
        e[i, j] = 1.0
        P[:, k] = mg.prolong(l, e)[act_f]
    for k, (i, j) in enumerate(idx_f):
        e = np.zeros(act_f.shape)
        e[i, j] = 1.0
        R[:, k] = mg.restrict(l, e)[act_c]
    return R @ mg.dense_operator(l) @ P, R, P


@pytest.mark.parametrize("n", [9, 17, 33])
def test_galerkin_operator_equals_brute_force_rap(n):
    """eq. L_G1: the explicit product R A P of the bounded grid (boundary rows included)
    equals the oracle's level-1 operator with its odd-reflection closure, and an interior
    row is the printed stencil on the rotated grid (H^2 = 2 h^2)."""
    mg = rbc.RBC(n, 2, coarse=rbc.G1)
    G, R, P = _galerkin(mg, 0)
    assert np.abs(G - mg.dense_operator(1)).max() < 1e-9 * np.abs(G).max()
    assert np.abs(R - P.T / 2).max() == 0.0
    S, fac = read_golden("rbc_galerkin_2d.txt")
    h2 = (1.0 / (n - 1)) ** 2
    m = mg.size(1)
    c = (m // 2, m // 2) if (m // 2) % 2 == 0 else (m // 2 - 1, m // 2 - 1)
    e = np.zeros((m, m))
    e[c] = 1.0
    col = mg.apply(1, e)  # the stencil reaches out from c symmetrically
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            want = fac * S[a + 1, b + 1] / (2.0 * h2)
            assert col[c[0] + a + b, c[1] + b - a] == pytest.approx(want, rel=1e-12)


def test_galerkin_of_the_galerkin_operator_is_not_g1():
    """The G1 operator below level 1 is the simplification of section 4.4, not the
    Galerkin recursion of eq. L_G_l: the product R L_G1 P differs from it."""
    mg = rbc.RBC(17, 3, coarse=rbc.G1)
    G, _, _ = _galerkin(mg, 1)
    assert np.abs(G - mg.dense_operator(2)).max() > 0.1 * np.abs(G).max()


def test_coarse_symbols_match_printed():
    """The symbols printed in section 4.3: (8/h^2) xi (1 - xi) for eq. L_G1 and
    (8/h^2)(xi - sin^2(theta_1/2) sin^2(theta_2/2)) for the rotated five-point operator,
    from the oracle's level-1 operators applied to a cosine mode away from the boundary."""
    n = 65
    h = 1.0 / (n - 1)
    rng = np.random.default_rng(7)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    for coarse in (rbc.G1, rbc.NG):
        mg = rbc.RBC(n, 2, coarse=coarse)
        for theta in rng.uniform(-np.pi, np.pi, size=(4, 2)):
            phi = np.cos(theta[0] * i + theta[1] * j + 0.3)
            c = (32, 32)
            x = rbc.xi(theta)
            s = np.sin(theta / 2) ** 2
            want = 8 / h ** 2 * (x * (1 - x) if coarse == rbc.G1 else x - s[0] * s[1])
            assert mg.apply(1, phi)[c] == pytest.approx(want * phi[c], rel=1e-9, abs=1e-9 / h ** 2)


@pytest.mark.parametrize("n", [9, 17, 33, 65])
@pytest.mark.parametrize("nu1", [0, 1, 2])
@pytest.mark.parametrize("coarse", [rbc.G1, rbc.GN])
def test_two_level_cycle_is_a_direct_solver(n, nu1, coarse):
    """Theorem 3: omega = 1 red-black smoothing, red-black coarsening, the transfers of
    eq. transfer_r2 and the Galerkin coarse operator solve the problem in one cycle that
    ends with a post-smoothing step."""
    mg = rbc.RBC(n, 2, coarse=coarse, nu1=nu1, nu2=1)
    f = _rhs(n, n + nu1)
    u = mg.cycle(f, np.zeros((n, n)))
    r0 = rbc.norm(f)
    assert rbc.norm(mg.residual(0, f, u)) < 1e-13 * r0


@pytest.mark.parametrize("kw", [dict(coarse=rbc.NG), dict(nu2=0), dict(omega=1.1)])
def test_two_level_cycle_is_not_direct_without_each_condition(kw):
    """Each of Theorem 3's conditions matters: the rediscretized coarse operator, no
    post-smoothing step or omega != 1 leave a residual."""
    cfg = dict(coarse=rbc.G1, nu1=1, nu2=1, omega=1.0)
    cfg.update(kw)
    mg = rbc.RBC(33, 2, **cfg)
    f = _rhs(33, 5)
    u = mg.cycle(f, np.zeros((33, 33)))
    assert rbc.norm(mg.residual(0, f, u)) > 1e-4 * rbc.norm(f)


def test_two_level_symbol_of_the_direct_solver_vanishes():
    """Theorem 4 with omega = 1 and eq. L_G1: S^R K = 0 on every E_theta, so the symbol of
    a cycle ending with a red partial step is zero."""
    for theta in np.random.default_rng(3).uniform(-np.pi / 2, np.pi / 2, size=(20, 2)):
        M = rbc.two_level_symbol(theta, 1.0, 1.0, 1, 1, rbc.G1)
        assert np.abs(M).max() < 1e-12


@pytest.mark.parametrize("omega,nu1,nu2", [(1.0, 1, 1), (1.1, 1, 1), (1.0, 2, 1), (1.2, 1, 0)])
def test_measured_two_level_rate_matches_lfa(omega, nu1, nu2):
    """Theorem 4 eq. rho_2d_rb with the rediscretized coarse operator: the finite-grid
    asymptotic rate approaches the LFA factor from below."""
    n = 65
    mg = rbc.RBC(n, 2, coarse=rbc.NG, nu1=nu1, nu2=nu2, omega=omega)
    f = np.zeros((n, n))
    u = _rhs(n, 9)
    r = [rbc.norm(mg.residual(0, f, u))]
    for _ in range(25):
        u = mg.cycle(f, u)
        r.append(rbc.norm(mg.residual(0, f, u)))
    cr = r[-1] / r[-2]
    rho = rbc.two_level_rho(omega, nu1, nu2, rbc.NG)
    assert 0.95 * rho <= cr <= 1.001 * rho


def test_multilevel_w_cycle_with_galerkin_levels_converges_fast():
    """section 4.4: with G1 operators the W-cycle at omega = 1 keeps most of the two-level
    scheme's reduction, the V-cycle much less."""
    n = 65
    rates = {}
    for gamma in (1, 2):
        mg = rbc.RBC(n, 8, coarse=rbc.G1, gamma=gamma, nu1=1, nu2=1)
        f = _rhs(n, 4)
        u = np.zeros((n, n))
        r = [rbc.norm(f)]
        for _ in range(6):
            u = mg.cycle(f, u)
            r.append(rbc.norm(mg.residual(0, f, u)))
        rates[gamma] = (r[-1] / r[0]) ** (1 / 6)
    assert rates[2] < 0.5 * rates[1]


def test_coarsest_level_is_solved_exactly():
    mg = rbc.RBC(17, 3)
    l = 2
    f = _rhs(mg.size(l), 1)
    u = mg.coarsest_solve(f)
    assert rbc.norm(mg.residual(l, f, u)) < 1e-13 * rbc.norm(f)


def test_level_counts():
    assert rbc.max_levels(17) == 8
    assert rbc.max_levels(3) == 2
    with pytest.raises(ValueError):
        rbc.RBC(17, 9)
    with pytest.raises(ValueError):
        rbc.RBC(18, 2)


@pytest.mark.parametrize("n,k", [(33, (1, 1)), (33, (3, 30)), (65, (32, 32)), (17, (15, 1))])
def test_norm_of_a_sine_mode_is_closed_form(n, k):
    """The level-0 norm sqrt(mean of r^2 over the interior) of sin(kx pi x) sin(ky pi y) is
    N / (2 (N - 1)), N = n - 1: along an axis the interior sum of sin^2(k pi i/N) is N/2 for
    1 <= k <= N-1, over N - 1 interior points.  Boundary values are not part of it."""
    N = n - 1
    x = np.linspace(0.0, 1.0, n)
    lx, ly = np.sin(k[0] * np.pi * x), np.sin(k[1] * np.pi * x)
    for line in (lx, ly):
        line[0] = line[-1] = 0.0
    r = np.outer(ly, lx)
    assert abs(rbc.norm(r) - N / (2.0 * (N - 1))) <= 1e-14
    r[0, :] = 5.0
    r[:, -1] = -1.0
    assert abs(rbc.norm(r) - N / (2.0 * (N - 1))) <= 1e-14
