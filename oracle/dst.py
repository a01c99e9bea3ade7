"""Exact discrete solutions by sine transforms -- TEST INFRASTRUCTURE ONLY.

With the odd-reflection Dirichlet closure, the sine modes prod_a sin(k_a pi x_a),
k_a = 1..n-2, are exact eigenfunctions of the fourth-order operator with eigenvalues
given by its Fourier symbol at theta_a = k_a pi h (appendix A.4, eq. L_hat_2d_4o):
lambda_k = (4/h^2) sum_a (s_a + s_a^2/3), s_a = sin^2(theta_a/2).  A type-I discrete
sine transform therefore solves L_h u = f exactly (up to rounding), independently of
any multigrid component.
"""
import os

import numpy as np
import scipy.fft

_WORKERS = max(1, min(16, os.cpu_count() or 1))


def _per_axis(s, h, order):
    """1D symbol of the order-2/4/6 second difference at s = sin^2(theta/2) (appendix A.4;
    sixth order: section 3.3 eq. LhOrder6, one more term of the same series)."""
    if order == 2:
        return 4.0 / h ** 2 * s
    if order == 4:
        return 4.0 / h ** 2 * (s + s * s / 3.0)
    if order == 6:
        return 4.0 / h ** 2 * (s + s * s / 3.0 + 8.0 * s ** 3 / 45.0)
    raise ValueError(order)


def eigenvalues(n, dim, order=4):
    """lambda_k on the (n-2)^dim grid of interior modes, index [kz][ky][kx]."""
    h = 1.0 / (n - 1)
    k = np.arange(1, n - 1)
    s = np.sin(k * np.pi * h / 2.0) ** 2
    per_axis = _per_axis(s, h, order)
    lam = np.zeros((n - 2,) * dim)
    for a in range(dim):
        shape = [1] * dim
        shape[a] = n - 2
        lam = lam + per_axis.reshape(shape)
    return lam


def min_eigenvalue(n, dim, order=4):
    """The smallest eigenvalue, mode k = (1, ..., 1): dim times the 1D symbol at theta = pi h."""
    h = 1.0 / (n - 1)
    return dim * float(_per_axis(np.sin(np.pi * h / 2.0) ** 2, h, order))


def solve(f, order=4, dtype=np.float64):
    """Exact solution of L_h u = f (interior values of f used; zero boundary)."""
    dim, n = f.ndim, f.shape[0]
    inner = tuple(slice(1, n - 1) for _ in range(dim))
    fh = scipy.fft.dstn(np.asarray(f[inner], dtype=dtype), type=1, norm="ortho", workers=_WORKERS)
    fh /= eigenvalues(n, dim, order).astype(dtype)
    u = np.zeros(f.shape, dtype=dtype)
    u[inner] = scipy.fft.idstn(fh, type=1, norm="ortho", workers=_WORKERS)
    return u


def sine_series(n, coeffs):
    """Evaluate sum_k c_k prod_a sin(k_a pi x_a) on the n-point grid, coeffs indexed
    [kz-1][ky-1][kx-1] (2D: [ky-1][kx-1])."""
    dim = coeffs.ndim
    x = np.linspace(0.0, 1.0, n)
    out = np.asarray(coeffs, dtype=float)
    for a in range(dim):
        K = out.shape[dim - 1 - a]
        basis = np.sin(np.outer(np.arange(1, K + 1), np.pi * x))  # (K, n)
        out = np.tensordot(out, basis, axes=([dim - 1 - a], [0]))
        out = np.moveaxis(out, -1, dim - 1 - a)
    return out


def discrete_solution_of_sine_series(n, coeffs, order=4):
    """For u* = sum_k a_k prod sin(k_a pi x) and f = -Delta u* (continuous), the discrete
    solution is exactly sum_k a_k pi^2 |k|^2 / lambda_k prod sin(...)."""
    dim = coeffs.ndim
    K = coeffs.shape[0]
    h = 1.0 / (n - 1)
    k = np.arange(1, K + 1)
    s = np.sin(k * np.pi * h / 2.0) ** 2
    per_axis = _per_axis(s, h, order)
    lam = np.zeros((K,) * dim)
    ksq = np.zeros((K,) * dim)
    for a in range(dim):
        shape = [1] * dim
        shape[a] = K
        lam = lam + per_axis.reshape(shape)
        ksq = ksq + (k.astype(float) ** 2).reshape(shape)
    return sine_series(n, coeffs * np.pi ** 2 * ksq / lam)
