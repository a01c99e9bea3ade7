"""Red-black coarsening multigrid in two dimensions -- TEST INFRASTRUCTURE ONLY.

Plain FP64 numpy reference for the cycle of section 4.3 (Theorem 3) and its multi-level
form of section 4.4; only the tests, the smoke check and the benchmark's CPU baseline use
it.  Nothing here is blocked, fused or reordered beyond what those sections state.

Levels (section 4.3 eq. G_r2, section 4.4): level 0 is the grid of spacing h; the coarse
grid of a level is its black points, so level 1 is the rotated grid of spacing sqrt(2) h
made of the level-0 points with an even index sum, level 2 is the standard grid of
spacing 2h, and so on: h_l = sqrt(2)^l h.  Every level is stored on the standard grid of
spacing s = 2^(l//2) h that holds it, (N/2^(l//2) + 1)^2 points; on an odd (rotated) level
only the interior points with an even index sum are unknowns.

Within a level, the points that stay on the next level are the C points (black), the rest
the F points (red): on an even level C = even index sum, on an odd level C = both indices
even.  Each F point has four C neighbours: the axis neighbours on an even level, the
diagonal ones on an odd level (a rotated level's own axes).

Operators, written on the storage grid (coefficients of the centre, the axis neighbours
at distance s, the diagonal neighbours, the axis neighbours at distance 2s):
* level 0: the second-order five-point operator (1/h^2)[-1; -1 4 -1; -1] (eq. L_h_2);
* rediscretized ('NG'): the same five-point operator on each level's own grid, whose axes
  on an odd level are the storage diagonals and H^2 = 2 s^2 (section 4.3, the operator
  before eq. L_G1: the Laplacian keeps its form under the rotation);
* 'G1': the first-generation Galerkin stencil (1/4H^2)[-1 -2 -1; -2 12 -2; -1 -2 -1]
  (eq. L_G1) on every coarse level, in that level's own axes (section 4.4, item G1): on an
  odd level its axis neighbours are the storage diagonals and its corners the storage
  axis neighbours at distance 2s;
* 'Gn': eq. L_G1 on level 1 and the rediscretized operator below (section 4.4, item Gn).
Beyond the boundary every level takes the odd reflection of the grid function (a zero
Dirichlet value on the boundary line); for a symmetric stencil this is what the Galerkin
product R L P of the bounded grid gives, which a test checks by brute force.

Transfers (eq. transfer_r2): restriction (1/8)[. 1 .; 1 4 1; . 1 .] from the C point and
its four F neighbours; interpolation (1/4)]. 1 .; 1 4 1; . 1 .[: a C point takes the coarse
value, an F point the mean of its four C neighbours (zero on the boundary).

Smoothing: omega red-black Jacobi, the F points (red) then the C points (black) each
taking an omega-Jacobi step from the current values (section 4.3, the smoother of eq.
S_hat_2d; for the five-point operator this is red-black Gauss-Seidel).  The coarsest
level is solved exactly (dense).
"""
import numpy as np

NG, G1, GN = 0, 1, 2  # coarse operators: rediscretized, first-generation Galerkin, Gn


class RBC:
    """The (levels)-level gamma-cycle with red-black coarsening on an n x n grid."""

    def __init__(self, n, levels, coarse=G1, gamma=1, nu1=1, nu2=1, omega=1.0):
        N = n - 1
        if N < 2 or N & (N - 1):
            raise ValueError("n - 1 must be a power of two")
        if levels < 1 or self_storage(n, levels - 1) < 3:
            raise ValueError("too many levels for n = %d" % n)
        self.n, self.levels, self.coarse = n, levels, coarse
        self.gamma, self.nu1, self.nu2, self.omega = gamma, nu1, nu2, omega
        self.h = 1.0 / N
        self._dense = None

    # ---- grids -------------------------------------------------------------------------
    def size(self, l):
        return self_storage(self.n, l)

    def spacing(self, l):
        return self.h * 2 ** (l // 2)

    def masks(self, l):
        """(active, C, F) boolean masks of level l on its storage grid."""
        m = self.size(l)
        i, j = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
        interior = (i > 0) & (i < m - 1) & (j > 0) & (j < m - 1)
        if l % 2 == 0:
            active = interior
            c = active & ((i + j) % 2 == 0)
        else:
            active = interior & ((i + j) % 2 == 0)
            c = active & (i % 2 == 0) & (j % 2 == 0)
        return active, c, active & ~c

    def stencil(self, l):
        """(centre, axis-1, diagonal, axis-2) coefficients of level l on its storage grid."""
        s2 = self.spacing(l) ** 2
        kind = "5"
        if l > 0 and (self.coarse == G1 or (self.coarse == GN and l == 1)):
            kind = "G1"
        if l % 2 == 0:
            if kind == "5":
                return 4.0 / s2, -1.0 / s2, 0.0, 0.0
            H2 = s2
            return 12.0 / (4 * H2), -2.0 / (4 * H2), -1.0 / (4 * H2), 0.0
        H2 = 2.0 * s2
        if kind == "5":
            return 4.0 / H2, 0.0, -1.0 / H2, 0.0
        return 12.0 / (4 * H2), 0.0, -2.0 / (4 * H2), -1.0 / (4 * H2)

    # ---- operators ---------------------------------------------------------------------
    def apply(self, l, u):
        """L_l u at every point of the storage grid (only the unknowns are meaningful)."""
        c0, a1, d1, a2 = self.stencil(l)
        p = np.pad(u, 2, mode="reflect", reflect_type="odd")
        m = u.shape[0]
        at = lambda di, dj: p[2 + di:2 + di + m, 2 + dj:2 + dj + m]
        out = c0 * u
        if a1:
            out = out + a1 * (at(1, 0) + at(-1, 0) + at(0, 1) + at(0, -1))
        if d1:
            out = out + d1 * (at(1, 1) + at(1, -1) + at(-1, 1) + at(-1, -1))
        if a2:
            out = out + a2 * (at(2, 0) + at(-2, 0) + at(0, 2) + at(0, -2))
        return out

    def residual(self, l, f, u):
        active = self.masks(l)[0]
        return np.where(active, f - self.apply(l, u), 0.0)

    def smooth_colour(self, l, f, u, colour):
        """One omega-Jacobi partial step on the F points (colour 1) or C points (colour 2)."""
        _, c, fm = self.masks(l)
        pts = fm if colour == 1 else c
        c0 = self.stencil(l)[0]
        r = f - self.apply(l, u)
        return np.where(pts, u + self.omega * r / c0, u)

    def smooth(self, l, f, u):
        u = self.smooth_colour(l, f, u, 1)
        return self.smooth_colour(l, f, u, 2)

    def _neighbours(self, l, g):
        """Sum over the four transfer neighbours (axis on even levels, diagonal on odd)."""
        p = np.pad(g, 1)
        m = g.shape[0]
        at = lambda di, dj: p[1 + di:1 + di + m, 1 + dj:1 + dj + m]
        if l % 2 == 0:
            return at(1, 0) + at(-1, 0) + at(0, 1) + at(0, -1)
        return at(1, 1) + at(1, -1) + at(-1, 1) + at(-1, -1)

    def _to_coarse(self, l, g):
        """Values at the C points of level l on the storage grid of level l + 1."""
        if l % 2 == 0:
            return np.where(self.masks(l)[1], g, 0.0)
        return np.where(self.masks(l + 1)[0], g[::2, ::2], 0.0)

    def _from_coarse(self, l, gc):
        """A level l + 1 grid function placed at the C points of level l."""
        out = np.zeros((self.size(l),) * 2)
        if l % 2 == 0:
            out[:] = np.where(self.masks(l)[1], gc, 0.0)
        else:
            out[::2, ::2] = gc
        return out

    def restrict(self, l, r):
        """eq. transfer_r2, full weighting onto the C points."""
        return self._to_coarse(l, (4.0 * r + self._neighbours(l, r)) / 8.0)

    def prolong(self, l, ec):
        """eq. transfer_r2, interpolation: C points copy, F points average 4 C neighbours."""
        _, c, fm = self.masks(l)
        e = self._from_coarse(l, ec)
        return np.where(c, e, np.where(fm, self._neighbours(l, e) / 4.0, 0.0))

    # ---- coarsest solve ----------------------------------------------------------------
    def dense_operator(self, l):
        """Matrix of L_l over its unknowns (row-major order of the storage grid)."""
        active = self.masks(l)[0]
        idx = np.argwhere(active)
        A = np.zeros((len(idx), len(idx)))
        for k, (i, j) in enumerate(idx):
            e = np.zeros(active.shape)
            e[i, j] = 1.0
            A[:, k] = self.apply(l, e)[active]
        return A

    def coarsest_solve(self, f):
        l = self.levels - 1
        active = self.masks(l)[0]
        if self._dense is None:
            self._dense = self.dense_operator(l)
        u = np.zeros(active.shape)
        u[active] = np.linalg.solve(self._dense, f[active])
        return u

    # ---- cycle -------------------------------------------------------------------------
    def _cycle(self, l, f, u):
        if l == self.levels - 1:
            return self.coarsest_solve(f)
        for _ in range(self.nu1):
            u = self.smooth(l, f, u)
        fc = self.restrict(l, self.residual(l, f, u))
        ec = np.zeros_like(fc)
        for _ in range(self.gamma if l + 1 < self.levels - 1 else 1):
            ec = self._cycle(l + 1, fc, ec)
        u = u + self.prolong(l, ec)
        for _ in range(self.nu2):
            u = self.smooth(l, f, u)
        return u

    def cycle(self, f, u):
        """One cycle on level 0; returns the new iterate (boundary values kept)."""
        return self._cycle(0, f, u)


def self_storage(n, l):
    """Storage side of level l for an n x n fine grid."""
    return (n - 1) // 2 ** (l // 2) + 1


def max_levels(n):
    """Most levels whose coarsest level still has an unknown."""
    l = 0
    while self_storage(n, l + 1) >= 3 and (n - 1) % 2 ** ((l + 1) // 2) == 0:
        l += 1
    return l + 1


def norm(r):
    """Grid l2 norm of a level-0 residual, sqrt(mean over the interior)."""
    return float(np.sqrt(np.mean(r[1:-1, 1:-1] ** 2)))


def xi(theta):
    """section 4.2 eq. xi_r2: the mean of sin^2(theta_a / 2) over the two axes."""
    s = np.sin(np.asarray(theta, dtype=float) / 2.0) ** 2
    return 0.5 * (s[..., 0] + s[..., 1])


def two_level_symbol(theta, h, omega=1.0, nu1=1, nu2=1, coarse=G1):
    """2 x 2 symbol of S^nu2 K S^nu1 on E_theta = span{phi(theta), phi(theta + (pi, pi))}
    (section 4.3, Theorem 4): L = (8/h^2) diag(xi, 1 - xi); restriction [1 - xi, xi] and
    interpolation [1 - xi; xi] (the symbols of eq. transfer_r2 on E_theta); coarse symbol
    (8/h^2) xi (1 - xi) for eq. L_G1, (8/h^2)(xi - sin^2(theta_1/2) sin^2(theta_2/2)) for
    the rediscretized operator; smoother S^B S^R (eq. S_hat_2d) with the red points those
    of odd index sum, whose mask on E_theta is (I - Q)/2, Q swapping the two modes."""
    x = float(xi(theta))
    L = (8.0 / h ** 2) * np.diag([x, 1.0 - x])
    r = np.array([[1.0 - x, x]])
    p = r.T
    if coarse == NG:
        s = np.sin(np.asarray(theta, dtype=float) / 2.0) ** 2
        LH = (8.0 / h ** 2) * (x - s[0] * s[1])
    else:
        LH = (8.0 / h ** 2) * x * (1.0 - x)
    K = np.eye(2) - p @ r @ L / LH
    Q = np.array([[0.0, 1.0], [1.0, 0.0]])
    step = -omega * L / (4.0 / h ** 2)  # S_J - I, the centre coefficient being 4/h^2
    red = np.eye(2) + 0.5 * (np.eye(2) - Q) @ step
    black = np.eye(2) + 0.5 * (np.eye(2) + Q) @ step
    S = black @ red
    return np.linalg.matrix_power(S, nu2) @ K @ np.linalg.matrix_power(S, nu1)


def two_level_rho(omega=1.0, nu1=1, nu2=1, coarse=NG, m=64):
    """section 4.3 eq. rho_2d_rb: sup over theta != 0 in Theta_rb^low (|theta_1| + |theta_2|
    <= pi, eq. Th_L_2d_rb) of rho of the two-level symbol, sampled on a uniform grid."""
    grid = -np.pi + 2 * np.pi * np.arange(m + 1) / m
    best = 0.0
    for t1 in grid:
        for t2 in grid:
            if abs(t1) + abs(t2) > np.pi + 1e-12 or (t1 == 0 and t2 == 0):
                continue
            M = two_level_symbol(np.array([t1, t2]), 1.0, omega, nu1, nu2, coarse)
            best = max(best, float(np.max(np.abs(np.linalg.eigvals(M)))))
    return best
