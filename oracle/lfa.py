"""Local Fourier analysis of the omega-Jacobi gamma-cycle -- TEST INFRASTRUCTURE ONLY.

Everything here is built from the Fourier symbols the paper prints, not from stencils:

* fine operator symbol, fourth order: (4/h^2) sum_a (s_a + s_a^2/3), s_a = sin^2(theta_a/2)
  (appendix A.4, eq. L_hat_2d_4o, written per axis); second order: (4/h^2) sum_a s_a
  (section 5.3, the symbol behind xi_theta); sixth order (section 3.3 eq. LhOrder6):
  (4/h^2) sum_a (s_a + s_a^2/3 + 8 s_a^3/45), the next term of the series
  theta^2 = 4 arcsin^2(sqrt(s)) that the lower orders truncate;
* full weighting: prod_a (1 - s_a) (appendix A.2, below eq. transfer_hat_2d);
* cubic transfer: prod_a (1 - s_a^2 (3 - 2 s_a)) (appendix A.4);
* linear interpolation: the transpose of full weighting (appendix A.2), same values;
* omega-Jacobi: S = 1 - omega * L/a_0 with a_0 the centre coefficient (section 5.3);
* omega red-black Jacobi (section 3.1 eq. S_rb with the Jacobi partial step, the smoother of
  appendix A.4.1): the red (odd index sum) then the black points take an omega-Jacobi
  step.  Multiplying a grid function by (-1)^(index sum) moves theta to theta + (pi,..,pi),
  so a partial step is I + (1/2)(I -+ P) (S_J - I) on the 2^d aliases, P the alias
  permutation alpha -> 1 - alpha (section 5.3 eq. S_hat_RB_2d is the 2D five-point case);
* omega red-black Gauss-Seidel (section 3.1 eqs. S_rb, S_GS): the same partial steps with
  the Jacobi symbol replaced by that of S_GS = -(L+)^{-1} L-, L+ = a_0/omega + the
  same-colour entries before the point in lexicographic order; on a cross-stencil level
  these are the entries at -2 e_a, so L+^ = a_0/omega + sum_a c_2 e^{-2 i theta_a} and
  S_GS^ = 1 - L^/L+^ (appendix A.4 prints it for the fourth-order operator; for the
  five-point operator it is the Jacobi symbol);
* two-grid operator on the 2^d aliases of theta in [-pi/2, pi/2)^d:
  M = S^nu2 (I - p L_H^{-1} r^T diag(L)) S^nu1 (section 2.2 eqs. K, M_2level; appendix
  A.2 eqs. K_hat_2, M_2); Galerkin coarse symbol L_H(2 theta) = sum_alpha r_alpha L_alpha p_alpha
  (eq. L_2h_G and the line after it); second-order coarse operators (section 3.1): the
  second-order symbol at H (eq. L_H_2d), or the Galerkin symbol of the second-order
  fine symbol (eq. L_H_2G_2d);
* smoothing factor: sup over high frequencies (section 2.2 eq. mu; section 5.3).
* three-level gamma-cycle (section 2.2 eqs. K_l, M; the appendix's eqs. L_H_approx and
  M_3level): the level-1 solve replaced by gamma level-1 two-grid cycles, on the 4^d
  fine modes theta + (pi/2) k that standard coarsening couples over two levels.

Convention: an interpolated coarse mode phi_H(2 theta) is sum_alpha p(theta_alpha) phi_h(theta_alpha)
and restriction maps phi_h(theta_alpha) to r(theta_alpha) phi_H(2 theta).

On the finite Dirichlet grid with the odd-reflection closure, sine modes are exact
eigenfunctions of every operator above, so ``finite_two_grid_spectrum`` is the exact
spectrum of the computed two-grid operator (not an approximation).
"""
import itertools

import numpy as np

FW, CUBIC = 1, 3
LINEAR = 1
NG, GALERKIN = 0, 1
NG2, G2 = 2, 3  # second-order coarse operators (section 3.1 eqs. L_H_2d, L_H_2G_2d)
JACOBI, RBJ, RBGS = 0, 1, 2  # smoothers: omega-Jacobi, omega red-black Jacobi and Gauss-Seidel


def sin2(theta):
    return np.sin(np.asarray(theta, dtype=float) / 2.0) ** 2


def symbol_fine(theta, h, order=4):
    """Symbol of -Delta_h; theta has shape (..., dim)."""
    s = sin2(theta)
    if order == 4:
        return (4.0 / h ** 2) * np.sum(s + s * s / 3.0, axis=-1)
    if order == 2:
        return (4.0 / h ** 2) * np.sum(s, axis=-1)
    if order == 6:
        return (4.0 / h ** 2) * np.sum(s + s * s / 3.0 + 8.0 * s ** 3 / 45.0, axis=-1)
    raise ValueError(order)


def symbol_transfer(theta, op):
    """Restriction / interpolation symbol (full weighting or linear: op=1; cubic: op=3)."""
    s = sin2(theta)
    if op == 1:
        return np.prod(1.0 - s, axis=-1)
    if op == 3:
        return np.prod(1.0 - s * s * (3.0 - 2.0 * s), axis=-1)
    raise ValueError(op)


def aliases(theta):
    """The 2^d frequencies theta + pi*alpha, alpha in {0,1}^d (alpha = 0 first)."""
    theta = np.asarray(theta, dtype=float)
    dim = theta.shape[-1]
    out = []
    for alpha in itertools.product((0, 1), repeat=dim):
        out.append(theta + np.pi * np.array(alpha, dtype=float))
    return np.stack(out, axis=-2)  # (..., 2^d, dim)


class Scheme:
    """Parameters of the cycle being analysed."""

    def __init__(self, dim, order=4, coarse=NG, restrict_op=FW, prolong=CUBIC, nu1=2, nu2=1,
                 omega=None, smoother=JACOBI):
        self.dim, self.order, self.coarse = dim, order, coarse
        self.restrict_op, self.prolong = restrict_op, prolong
        self.nu1, self.nu2 = nu1, nu2
        self.smoother = smoother
        if omega is None:
            if smoother == JACOBI:
                omega = jacobi_optimum(dim, order)[0]
            elif smoother == RBJ:
                omega = RBJ_OMEGA[(dim, order, coarse)]
            else:
                omega = RBGS_OMEGA[(dim, order, coarse)]
        self.omega = omega

    def level_symbol(self, level, theta, h0=1.0):
        """Symbol of the level-l operator at level-l frequency theta (spacing h0 * 2^l)."""
        h = h0 * 2 ** level
        if level == 0 or self.coarse == NG:
            return symbol_fine(theta, h, self.order)
        if self.coarse == NG2:
            return symbol_fine(theta, h, 2)
        half = aliases(np.asarray(theta, dtype=float) / 2.0)
        if self.coarse == G2 and level == 1:
            fine = symbol_fine(half, h0, 2)  # the second-order operator at the finest spacing
        else:
            fine = self.level_symbol(level - 1, half, h0)
        return np.sum(symbol_transfer(half, self.restrict_op) * fine
                      * symbol_transfer(half, self.prolong), axis=-1)

    def level_diagonal(self, level, h0=1.0, m=32):
        """Centre stencil coefficient = mean of the symbol over the frequency torus."""
        key = (level, h0, m)
        memo = self.__dict__.setdefault("_diag", {})
        if key not in memo:
            grid = -np.pi + 2 * np.pi * np.arange(m) / m
            pts = np.stack(np.meshgrid(*([grid] * self.dim), indexing="ij"), axis=-1)
            memo[key] = float(np.mean(self.level_symbol(level, pts, h0)))
        return memo[key]

    def smoother_symbol(self, theta, level=0, h0=1.0):
        return 1.0 - self.omega * self.level_symbol(level, theta, h0) / self.level_diagonal(level, h0)

    def cross_c2(self, level, h0=1.0):
        """Coefficient of the entries at +-2 e_a of a cross-stencil level (the fourth-order
        operator: 1/(12 h^2); the five-point operator: 0); None for a Galerkin level."""
        h = h0 * 2 ** level
        order = self.order if (level == 0 or self.coarse == NG) else (2 if self.coarse == NG2 else None)
        if order is None:
            return None
        return {2: 0.0, 4: 1.0 / (12.0 * h * h), 6: 27.0 / (180.0 * h * h)}[order]

    def gs_symbol(self, modes, level=0, h0=1.0):
        """Symbol of S_GS = -(L+)^{-1} L- on a cross-stencil level (complex)."""
        c2 = self.cross_c2(level, h0)
        if c2 is None:
            raise ValueError("red-black Gauss-Seidel analysis needs a cross-stencil level")
        modes = np.asarray(modes, dtype=float)
        Lh = self.level_symbol(level, modes, h0)
        lplus = self.level_diagonal(level, h0) / self.omega + c2 * np.sum(np.exp(-2j * modes), axis=-1)
        return 1.0 - Lh / lplus

    def smoother_on(self, modes, partner, level=0, h0=1.0):
        """Symbol of one smoothing sweep at level l on a set of modes closed under
        theta -> theta + (pi,..,pi); partner[i] is the index of that shift of modes[i]."""
        if self.smoother == RBGS:
            D = np.diag(self.gs_symbol(modes, level, h0) - 1.0)
        else:
            D = np.diag(-self.omega * self.level_symbol(level, modes, h0) / self.level_diagonal(level, h0))
        eye = np.eye(len(D))
        if self.smoother == JACOBI:
            return eye + D
        P = eye[:, partner]  # the colour flip (-1)^(index sum) as a permutation of the modes
        red = eye + 0.5 * (eye - P) @ D
        black = eye + 0.5 * (eye + P) @ D
        return black @ red

    def smoother_matrix(self, theta, h0=1.0, level=0):
        """2^d x 2^d symbol of one smoothing sweep on the aliases of theta."""
        th = aliases(theta)
        # alias index alpha (binary, axis 0 first) -> its complement
        return self.smoother_on(th, np.arange(len(th))[::-1], level, h0)

    def two_grid_matrix(self, theta, h0=1.0, level=0):
        """2^d x 2^d symbol of S^nu2 K S^nu1 at one low frequency theta of level l, with the
        level l+1 equation solved exactly."""
        th = aliases(theta)
        L = self.level_symbol(level, th, h0)
        S = self.smoother_matrix(theta, h0, level)
        r = symbol_transfer(th, self.restrict_op)
        p = symbol_transfer(th, self.prolong)
        LH = self.level_symbol(level + 1, 2.0 * np.asarray(theta, dtype=float), h0)
        K = np.eye(len(L)) - np.outer(p, r * L) / LH
        return np.linalg.matrix_power(S, self.nu2) @ K @ np.linalg.matrix_power(S, self.nu1)

    def three_grid_matrix(self, theta, h0=1.0, gamma=1):
        """4^d x 4^d symbol of the three-level gamma-cycle at theta in [-pi/4, pi/4)^d.

        Section 2.2 eqs. K_l and M define the multi-level operator by recursion; the
        appendix on red-black coarsening writes its three-level form (eqs. L_H_approx,
        M_3level): the level-1 solve is replaced by gamma level-1 two-grid cycles from a
        zero guess, L1~^{-1} = (I - M_1^gamma) L_1^{-1}.  Standard coarsening couples the
        4^d fine modes theta + (pi/2) k, k in {0..3}^d: fine mode k restricts to the level-1
        alias 2 theta + pi (k mod 2), and those 2^d level-1 modes are the aliases on which
        M_1 acts.  gamma=None solves level 1 exactly."""
        theta = np.asarray(theta, dtype=float)
        ks = np.array(list(itertools.product(range(4), repeat=self.dim)))
        modes = theta + (np.pi / 2) * ks
        index = {tuple(k): i for i, k in enumerate(ks)}
        partner = [index[tuple((k + 2) % 4)] for k in ks]
        coarse = [int(np.dot(k % 2, 2 ** np.arange(self.dim)[::-1])) for k in ks]  # alias order
        L0 = self.level_symbol(0, modes, h0)
        theta1 = 2.0 * theta
        L1 = self.level_symbol(1, aliases(theta1), h0)
        m1 = len(L1)
        if gamma is None:
            solve1 = np.diag(1.0 / L1)
        else:
            M1 = self.two_grid_matrix(theta1, h0, level=1)
            solve1 = (np.eye(m1) - np.linalg.matrix_power(M1, gamma)) @ np.diag(1.0 / L1)
        R = np.zeros((m1, len(ks)))
        P = np.zeros((len(ks), m1))
        R[coarse, np.arange(len(ks))] = symbol_transfer(modes, self.restrict_op)
        P[np.arange(len(ks)), coarse] = symbol_transfer(modes, self.prolong)
        K = np.eye(len(ks)) - P @ solve1 @ R @ np.diag(L0)
        S = self.smoother_on(modes, partner, 0, h0)
        return np.linalg.matrix_power(S, self.nu2) @ K @ np.linalg.matrix_power(S, self.nu1)

# Default omega of the red-black Gauss-Seidel smoother (2D), per fine order and coarse
# operator (rediscretized, or the second-order one of section 3.1): the minimiser of the
# two-grid factor of the V(2,1) cycle with cubic interpolation, to two decimals
# (rbgs_optimum recomputes it).  For the five-point operator it is red-black Jacobi.
RBGS_OMEGA = {(2, 4, NG): 1.16, (2, 4, NG2): 0.98, (2, 6, NG): 1.18, (2, 6, NG2): 1.0,
              (2, 2, NG): 1.0, (2, 2, NG2): 1.0}

# Default omega of the red-black Jacobi smoother per (dim, fine order, coarse operator): the
# value minimising the two-grid factor of the V(2,1) cycle with cubic interpolation, rounded
# to two decimals (rbj_optimum recomputes it).  For the second-order fine operator the
# second-order coarse operators are the rediscretized and Galerkin ones.
RBJ_OMEGA = {
    (2, 4, NG): 1.13, (2, 4, GALERKIN): 1.0, (2, 4, NG2): 0.98, (2, 4, G2): 0.97,
    (2, 6, NG): 1.13, (2, 6, GALERKIN): 1.02, (2, 6, NG2): 0.99, (2, 6, G2): 0.99,
    (2, 2, NG): 1.0, (2, 2, GALERKIN): 0.98, (2, 2, NG2): 1.0, (2, 2, G2): 0.98,
    (3, 4, NG): 1.17, (3, 4, GALERKIN): 1.09, (3, 4, NG2): 1.09, (3, 4, G2): 1.08,
    (3, 6, NG): 1.15, (3, 6, GALERKIN): 1.1, (3, 6, NG2): 1.09, (3, 6, G2): 1.08,
    (3, 2, NG): 1.13, (3, 2, GALERKIN): 1.09, (3, 2, NG2): 1.13, (3, 2, G2): 1.09,
}


def rbj_optimum(dim, order=4, m=None, coarse=NG):
    """omega minimising two_grid_rho for red-black Jacobi, V(2,1), cubic interpolation."""
    from scipy.optimize import minimize_scalar
    m = m or (24 if dim == 2 else 10)
    rho = lambda w: two_grid_rho(Scheme(dim, order, coarse=coarse, nu1=2, nu2=1, omega=w, smoother=RBJ), m)
    r = minimize_scalar(rho, bounds=(0.8, 1.4), method="bounded", options={"xatol": 1e-4})
    return float(r.x), float(r.fun)


def jacobi_optimum(dim, order=4):
    """Optimal omega-Jacobi parameter and smoothing factor for standard coarsening.

    The smoother symbol is 1 - omega*q(theta) with q = L/a_0.  Over the high
    frequencies q ranges over [q_lo, q_hi]; equioscillation |1 - omega q_lo| =
    |1 - omega q_hi| gives omega* = 2/(q_lo + q_hi), mu* = (q_hi - q_lo)/(q_hi + q_lo)
    (the argument of section 5.3 that yields eq. mu_w_J_r).  For order 4,
    a_0 = 30 d/(12 h^2), q_lo is reached with one s_a = 1/2 and the rest 0, q_hi with
    every s_a = 1."""
    if order == 4:
        a0 = 30.0 * dim / 12.0
        g = lambda s: 4.0 * (s + s * s / 3.0)
    elif order == 6:
        a0 = 490.0 * dim / 180.0
        g = lambda s: 4.0 * (s + s * s / 3.0 + 8.0 * s ** 3 / 45.0)
    else:
        a0 = 2.0 * dim
        g = lambda s: 4.0 * s
    q_lo = g(0.5) / a0
    q_hi = dim * g(1.0) / a0
    return 2.0 / (q_lo + q_hi), (q_hi - q_lo) / (q_hi + q_lo)


def rb_smoothing_factor(scheme, nu=1, m=32):
    """mu = sup over low theta of rho(Q S^nu)^(1/nu), Q the ideal coarse-level correction
    (zero on alias 0, identity on the others): section 5.3 eq. mu_2_2, any smoother."""
    grid = -np.pi / 2 + np.pi * np.arange(m + 1) / m
    Q = np.eye(2 ** scheme.dim)
    Q[0, 0] = 0.0
    best = 0.0
    for theta in itertools.product(grid, repeat=scheme.dim):
        S = np.linalg.matrix_power(scheme.smoother_matrix(np.array(theta)), nu)
        best = max(best, float(np.max(np.abs(np.linalg.eigvals(Q @ S)))) ** (1.0 / nu))
    return best


def smoothing_factor(scheme, m=64):
    """mu = sup over high frequencies of |S(theta)| (omega-Jacobi, section 2.2 eq. mu)."""
    assert scheme.smoother == JACOBI
    grid = -np.pi + 2 * np.pi * (np.arange(m) + 0.0) / m
    pts = np.stack(np.meshgrid(*([grid] * scheme.dim), indexing="ij"), axis=-1).reshape(-1, scheme.dim)
    high = np.any(np.abs(pts) >= np.pi / 2 - 1e-12, axis=-1)
    return float(np.max(np.abs(scheme.smoother_symbol(pts[high]))))


def two_grid_rho(scheme, m=32):
    """sup over a uniform grid of low frequencies (theta = 0 excluded) of rho(M(theta))."""
    grid = -np.pi / 2 + np.pi * np.arange(m + 1) / m
    best = 0.0
    for theta in itertools.product(grid, repeat=scheme.dim):
        theta = np.array(theta)
        if np.allclose(theta, 0.0):
            continue
        best = max(best, float(np.max(np.abs(np.linalg.eigvals(scheme.two_grid_matrix(theta))))))
    return best


def three_grid_rho(scheme, m=16, gamma=1):
    """sup over a uniform grid of theta in [-pi/4, pi/4]^d (theta = 0 excluded) of the
    spectral radius of the three-level gamma-cycle."""
    grid = -np.pi / 4 + (np.pi / 2) * np.arange(m + 1) / m
    best = 0.0
    for theta in itertools.product(grid, repeat=scheme.dim):
        theta = np.array(theta)
        if np.allclose(theta, 0.0):
            continue
        M = scheme.three_grid_matrix(theta, gamma=gamma)
        best = max(best, float(np.max(np.abs(np.linalg.eigvals(M)))))
    return best

def finite_two_grid_spectrum(scheme, n):
    """Exact eigenvalues of the two-grid operator on the Dirichlet grid of n points/axis
    (interior (n-2)^dim unknowns), from the symbols at theta_a = k_a*pi/(n-1).

    Fine sine modes k and N-k (N = n-1) alias on the coarse grid; mode N/2 on an axis
    restricts to zero and is never interpolated, so on such blocks the coarse-level
    correction is the identity and the eigenvalues are S^(nu1+nu2)."""
    N = n - 1
    h0 = 1.0 / N
    eig = []
    for k in itertools.product(range(1, N // 2 + 1), repeat=scheme.dim):
        k = np.array(k, dtype=float)
        theta = k * np.pi / N
        if np.all(k < N // 2):
            eig.extend(np.linalg.eigvals(scheme.two_grid_matrix(theta, h0)))
        else:
            # On an axis with k = N/2 the alias theta + pi is the same sine mode with the
            # sign flipped; fold the 2^d alias coefficients onto the distinct modes.
            half = k == N // 2
            idx = list(itertools.product((0, 1), repeat=scheme.dim))
            keep = [i for i, a in enumerate(idx) if not any(half & (np.array(a) == 1))]
            fold = np.zeros((len(keep), len(idx)))
            for j, a in enumerate(idx):
                a = np.array(a)
                base = tuple(np.where(half, 0, a))
                fold[keep.index(idx.index(base)), j] = (-1.0) ** int(np.sum(a[half]))
            S = fold @ scheme.smoother_matrix(theta, h0)[:, keep]
            eig.extend(np.linalg.eigvals(np.linalg.matrix_power(S, scheme.nu1 + scheme.nu2)))
    return np.array(eig)


def rbgs_optimum(order=4, m=24, coarse=NG):
    """omega minimising two_grid_rho for red-black Gauss-Seidel (2D), V(2,1), cubic
    interpolation."""
    from scipy.optimize import minimize_scalar
    rho = lambda w: two_grid_rho(Scheme(2, order, coarse=coarse, nu1=2, nu2=1, omega=w, smoother=RBGS), m)
    r = minimize_scalar(rho, bounds=(0.8, 1.4), method="bounded", options={"xatol": 1e-4})
    return float(r.x), float(r.fun)
