"""Seeded synthetic inputs (right-hand sides, manufactured solutions, request streams).

This module holds no multigrid arithmetic: it only draws seeded random numbers and
evaluates sine series and simple neighbour averages, so both the GPU path and the
CPU oracle can be fed identical inputs.  Grids have n points per axis including the
boundary, x_i = i/(n-1); arrays are float64 with index [z][y][x] (x fastest) and zero
boundary values.  Random numbers come from numpy's PCG64 generator.
"""
import numpy as np

SEED_BASE = 20080385


def generator(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _sine_basis(n, K):
    x = np.linspace(0.0, 1.0, n)
    b = np.sin(np.outer(np.arange(1, K + 1), np.pi * x))
    b[:, 0] = 0.0
    b[:, -1] = 0.0
    return b  # (K, n)


def sine_series(n, coeffs):
    """sum_k c_k prod_a sin(k_a pi x_a); coeffs shape (K,)*dim indexed [kz-1][ky-1][kx-1]."""
    coeffs = np.asarray(coeffs, dtype=np.float64)
    b = _sine_basis(n, coeffs.shape[0])
    if coeffs.ndim == 2:
        return b.T @ coeffs @ b  # [y][x]
    t = np.tensordot(coeffs, b, axes=([2], [0]))        # [kz][ky][x]
    t = np.tensordot(t, b, axes=([1], [0]))             # [kz][x][y]
    t = np.tensordot(t, b, axes=([0], [0]))             # [x][y][z]
    return np.ascontiguousarray(np.transpose(t, (2, 1, 0)))


def _wavenumber_sq(K, dim):
    k = np.arange(1, K + 1, dtype=np.float64) ** 2
    out = np.zeros((K,) * dim)
    for a in range(dim):
        shape = [1] * dim
        shape[a] = K
        out = out + k.reshape(shape)
    return out


def manufactured_2d(n, seed=SEED_BASE + 1, kmax=8):
    """u* = sin(pi x) sin(2 pi y) + sum_{kx,ky<=kmax} a_k sin(kx pi x) sin(ky pi y), a_k ~ N(0,1);
    f = -Laplace(u*) analytically.  Returns (u_star, f, coeffs)."""
    c = generator(seed).standard_normal((kmax, kmax))
    c[1, 0] += 1.0  # ky = 2, kx = 1
    u = sine_series(n, c)
    f = sine_series(n, c * np.pi ** 2 * _wavenumber_sq(kmax, 2))
    return u, f, c


def fourier_rhs(n, dim=2, kmax=64, seed=SEED_BASE + 2):
    """f = sum_{k_a <= kmax} g_k/|k| prod sin(k_a pi x_a), g_k ~ N(0,1), |k| Euclidean."""
    kmax = min(kmax, n - 2)
    g = generator(seed).standard_normal((kmax,) * dim)
    return sine_series(n, g / np.sqrt(_wavenumber_sq(kmax, dim)))


def smoothed_noise_3d(n, seed=SEED_BASE + 3, passes=3):
    """Uniform[-1,1] interior values with a zero boundary, then `passes` neighbour-average
    passes (each interior value replaced by the mean of its six face neighbours)."""
    f = np.zeros((n, n, n))
    f[1:-1, 1:-1, 1:-1] = generator(seed).uniform(-1.0, 1.0, (n - 2,) * 3)
    for _ in range(passes):
        g = np.zeros_like(f)
        g[1:-1, 1:-1, 1:-1] = (f[:-2, 1:-1, 1:-1] + f[2:, 1:-1, 1:-1] + f[1:-1, :-2, 1:-1]
                               + f[1:-1, 2:, 1:-1] + f[1:-1, 1:-1, :-2] + f[1:-1, 1:-1, 2:]) / 6.0
        f = g
    return f


def smooth_sine_3d(n, seed=SEED_BASE + 5, kmax=8, return_coeffs=False):
    """Continuous smooth right-hand side sum_{k_a <= kmax} g_k prod sin(k_a pi x_a), g_k ~ N(0,1):
    the same function at every resolution.  With return_coeffs, also g (indexed [kz][ky][kx])."""
    g = generator(seed).standard_normal((kmax,) * 3)
    f = sine_series(n, g)
    return (f, g) if return_coeffs else f


def wavenumber_sq(kmax, dim):
    """|k|^2 = sum_a k_a^2 on the grid of modes 1..kmax per axis (indexed like the coefficients)."""
    return _wavenumber_sq(kmax, dim)


def request_stream(count, rate, seed=SEED_BASE + 104, kmin=6, kmax=11):
    """Poisson arrivals: exponential gaps of mean 1/rate seconds; side n = 2^k+1 with k
    uniform on kmin..kmax; per-request right-hand-side seeds.  Returns a list of
    (arrival_time, n, rhs_seed)."""
    rng = generator(seed)
    gaps = rng.exponential(1.0 / rate, count)
    ks = rng.integers(kmin, kmax + 1, count)
    t = np.cumsum(gaps)
    return [(float(t[i]), int(2 ** ks[i] + 1), SEED_BASE + 1000 + i) for i in range(count)]
