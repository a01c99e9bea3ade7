"""Explicit matrices of every multigrid operator on tiny grids -- TEST INFRASTRUCTURE ONLY.

Each matrix is assembled entry by entry from the paper's printed stencils (section 2.1
stencil notation, eq. bra and its reversed-bracket form), over the interior unknowns of
a Dirichlet grid, with the odd reflection u(-i) = -u(i) folded into the entries.  They
give brute-force checks of the C oracle:

* ``galerkin(R, A, P)`` is the coarse operator R*A*P of eq. L_H_G as a matrix product;
* ``cycle_matrix`` composes the gamma-cycle error propagator from section 2.2:
  M_l = S^nu2 (I - P Ltilde_{l+1}^{-1} R A_l) S^nu1 with the exact inverse on the
  coarsest level and Ltilde^{-1} = (I - M_{l+1}^gamma) A_{l+1}^{-1} elsewhere
  (appendix A.3.1, eq. L_H_approx).  With rb=True the smoother is the red-black product
  S = S^B S^R of section 3.1 eq. S_rb, S^c = I - (omega/a_0) X_c A with X_c the diagonal
  0/1 mask of colour c (red: odd index sum).

Unknown p enumerates interior points x fastest: p = ((k-1)*q + (j-1))*q + (i-1), q = n-2.
"""
import itertools

import numpy as np
import scipy.sparse as sp

RESTRICT_W = {1: {0: 0.5, 1: 0.25}, 3: {0: 0.5, 1: 9.0 / 32.0, 3: -1.0 / 32.0}}
PROLONG_W = {1: {0: 1.0, 1: 0.5}, 3: {0: 1.0, 1: 9.0 / 16.0, 3: -1.0 / 16.0}}


def _fold(c, n):
    """Reflect index c into 0..n-1; returns (index, sign)."""
    sign = 1.0
    if c < 0:
        c, sign = -c, -sign
    if c > n - 1:
        c, sign = 2 * (n - 1) - c, -sign
    return c, sign


def _unknown(idx, n):
    q = n - 2
    p = 0
    for c in reversed(idx):  # idx = (i, j[, k]) with x first
        p = p * q + (c - 1)
    return p


def _interior(n, dim):
    return itertools.product(*([range(1, n - 1)] * dim))


def _as_xyz(t):
    return tuple(reversed(t))


def operator(s, n):
    """Matrix of the stencil s (shape (2R+1,)*dim, index [oz][oy][ox]) with odd folding."""
    dim = s.ndim
    R = (s.shape[0] - 1) // 2
    m = (n - 2) ** dim
    rows, cols, vals = [], [], []
    offs = [o for o in itertools.product(*([range(-R, R + 1)] * dim)) if s[tuple(c + R for c in o)] != 0]
    for pt_zyx in _interior(n, dim):
        pt = _as_xyz(pt_zyx)
        row = _unknown(pt, n)
        for o_zyx in offs:
            o = _as_xyz(o_zyx)
            coef = s[tuple(c + R for c in o_zyx)]
            sign, tgt = 1.0, []
            for c, d in zip(pt, o):
                ci, sg = _fold(c + d, n)
                sign *= sg
                tgt.append(ci)
            if any(c == 0 or c == n - 1 for c in tgt):
                continue  # boundary value is zero
            rows.append(row)
            cols.append(_unknown(tgt, n))
            vals.append(sign * coef)
    return sp.csr_matrix((vals, (rows, cols)), shape=(m, m))


def restriction(dim, nf, op=1):
    nc = (nf - 1) // 2 + 1
    w = RESTRICT_W[op]
    r = max(w)
    rows, cols, vals = [], [], []
    for I_zyx in _interior(nc, dim):
        I = _as_xyz(I_zyx)
        row = _unknown(I, nc)
        for o in itertools.product(*([range(-r, r + 1)] * dim)):
            wt = np.prod([w.get(abs(c), 0.0) for c in o])
            if wt == 0.0:
                continue
            sign, tgt = 1.0, []
            for c, d in zip(I, o):
                ci, sg = _fold(2 * c + d, nf)
                sign *= sg
                tgt.append(ci)
            if any(c == 0 or c == nf - 1 for c in tgt):
                continue
            rows.append(row)
            cols.append(_unknown(tgt, nf))
            vals.append(sign * wt)
    return sp.csr_matrix((vals, (rows, cols)), shape=((nc - 2) ** dim, (nf - 2) ** dim))


def prolongation(dim, nf, op=3):
    nc = (nf - 1) // 2 + 1
    w = PROLONG_W[op]
    r = max(w)
    rows, cols, vals = [], [], []
    for x_zyx in _interior(nf, dim):
        x = _as_xyz(x_zyx)
        row = _unknown(x, nf)
        ranges = [range((c - r + 1) // 2 - 1, (c + r) // 2 + 1) for c in x]
        for J in itertools.product(*ranges):
            wt = np.prod([w.get(abs(c - 2 * j), 0.0) if abs(c - 2 * j) <= r else 0.0
                          for c, j in zip(x, J)])
            if wt == 0.0:
                continue
            sign, tgt = 1.0, []
            for j in J:
                ji, sg = _fold(j, nc)
                sign *= sg
                tgt.append(ji)
            if any(c == 0 or c == nc - 1 for c in tgt):
                continue
            rows.append(row)
            cols.append(_unknown(tgt, nc))
            vals.append(sign * wt)
    return sp.csr_matrix((vals, (rows, cols)), shape=((nf - 2) ** dim, (nc - 2) ** dim))


def galerkin(R, A, P):
    return (R @ A @ P).tocsr()


def jacobi(A, omega, a0):
    m = A.shape[0]
    return (sp.identity(m) - (omega / a0) * A).tocsr()


def colour_mask(n, dim, odd):
    """Diagonal of X_c over the interior unknowns: 1 where (i+j+k) % 2 == odd."""
    x = np.zeros((n - 2) ** dim)
    for pt_zyx in _interior(n, dim):
        pt = _as_xyz(pt_zyx)
        x[_unknown(pt, n)] = 1.0 if sum(pt) % 2 == odd else 0.0
    return x


def cycle_matrix(As, a0s, omega, nu1, nu2, gamma, dim, ns, restrict_op=1, prolong=3, rb=False):
    """Dense error propagator of the gamma-cycle over levels 0..L-1 (level L-1 exact)."""
    L = len(As)

    def M(l):
        A = As[l].toarray()
        m = A.shape[0]
        if rb:
            red = np.eye(m) - (omega / a0s[l]) * colour_mask(ns[l], dim, 1)[:, None] * A
            black = np.eye(m) - (omega / a0s[l]) * colour_mask(ns[l], dim, 0)[:, None] * A
            S = black @ red
        else:
            S = np.eye(m) - (omega / a0s[l]) * A
        Rm = restriction(dim, ns[l], restrict_op).toarray()
        Pm = prolongation(dim, ns[l], prolong).toarray()
        Ac_inv = np.linalg.inv(As[l + 1].toarray())
        if l + 1 == L - 1:
            Lt_inv = Ac_inv
        else:
            Mc = M(l + 1)
            Lt_inv = (np.eye(Mc.shape[0]) - np.linalg.matrix_power(Mc, gamma)) @ Ac_inv
        K = np.eye(m) - Pm @ Lt_inv @ Rm @ A
        return np.linalg.matrix_power(S, nu2) @ K @ np.linalg.matrix_power(S, nu1)

    return M(0)
