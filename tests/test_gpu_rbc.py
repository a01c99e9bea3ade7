"""Red-black coarsening (section 4.3, 4.4) on the GPU against the oracle, through the C ABI.

Bar (FP64): every single step element by element within 1e-12 of the oracle's values
(relative to the largest magnitude); whole cycles within 1e-12 ||u|| after a fixed number
of cycles; the two-level cycle of Theorem 3 is a direct solver on the GPU too.
"""
import numpy as np
import pytest

from gpu_util import dev, host, stream, torch
from oracle import rbc as orbc
from paper_2008_03885_amd import mg, rbc

pytestmark = pytest.mark.gpu

CFG = {"NG": rbc.MG_RBC_NG, "G1": rbc.MG_RBC_G1, "GN": rbc.MG_RBC_GN}


class Pair:
    """A handle and the oracle cycle of the same configuration."""

    def __init__(self, n, levels, coarse="G1", gamma=1, nu1=1, nu2=1, omega=1.0, max_cycles=100,
                 rtol=1e-10):
        self.cfg = rbc.make_config(n=n, levels=levels, coarse=CFG[coarse], gamma=gamma, nu1=nu1,
                                   nu2=nu2, omega=omega, rtol=rtol, max_cycles=max_cycles)
        self.h = rbc.setup(self.cfg, stream())
        self.o = orbc.RBC(n, levels, coarse=CFG[coarse], gamma=gamma, nu1=nu1, nu2=nu2, omega=omega)
        for l in range(levels):
            assert rbc.level_size(self.h, l) == self.o.size(l)
            pitch = (self.o.size(l) + 1) // 2 if l % 2 else self.o.size(l)
            assert rbc.level_pitch(self.h, l) == pitch

    def close(self):
        rbc.destroy(self.h)


def _grid(m, seed, mask=None):
    a = np.zeros((m, m))
    a[1:-1, 1:-1] = np.random.default_rng(seed).standard_normal((m - 2, m - 2))
    return a if mask is None else np.where(mask, a, 0.0)


def pack(a, l):
    """A level's full storage array in the library's layout: rotated (odd) levels keep
    row i's points (i, j), i + j even, at column j // 2."""
    if l % 2 == 0:
        return a
    m = a.shape[0]
    out = np.zeros((m, (m + 1) // 2))
    out[0::2, :] = a[0::2, 0::2]
    out[1::2, :(m - 1) // 2] = a[1::2, 1::2]
    return out


def unpack(p, l):
    if l % 2 == 0:
        return p
    m = p.shape[0]
    out = np.zeros((m, m))
    out[0::2, 0::2] = p[0::2, :]
    out[1::2, 1::2] = p[1::2, :(m - 1) // 2]
    assert not p[1::2, -1].any(), "padding of an odd row must stay zero"
    return out


def _close(got, ref, what):
    scale = max(np.abs(ref).max(), 1e-300)
    err = np.abs(got - ref).max() / scale
    assert err <= 1e-12, "%s: relative error %.3e" % (what, err)


KERNEL_CASES = [(17, 8, "G1"), (65, 8, "GN"), (129, 10, "NG"), (129, 9, "G1"), (33, 6, "G1"),
                # coarsest levels of 225 (17^2) and 113 (rotated 17^2) unknowns
                (129, 7, "G1"), (129, 8, "NG")]


@pytest.mark.parametrize("n,levels,coarse", KERNEL_CASES)
def test_every_step_on_every_level(n, levels, coarse):
    print("rbc steps", n, levels, coarse, flush=True)
    P = Pair(n, levels, coarse)
    try:
        for l in range(levels):
            m = P.o.size(l)
            act, _, _ = P.o.masks(l)
            scale = 1.0 / P.o.spacing(l) ** 2
            mask = act if l % 2 else None  # a rotated level holds only its own points
            f = _grid(m, 10 * l + 1, mask) * scale
            u = _grid(m, 10 * l + 2, mask)
            fd, ud = dev(pack(f, l)), dev(pack(u, l))
            out = torch().zeros_like(ud)
            for colour in (1, 2):
                rbc.kernel_smooth(P.h, l, colour, fd.data_ptr(), ud.data_ptr(), out.data_ptr())
                _close(unpack(host(out), l), P.o.smooth_colour(l, f, u, colour),
                       "smooth l=%d c=%d" % (l, colour))
            if l == levels - 1:
                rbc.kernel_coarsest(P.h, fd.data_ptr(), out.data_ptr())
                _close(unpack(host(out), l), P.o.coarsest_solve(f), "coarsest l=%d" % l)
                inplace = fd.clone()  # f and u the same array
                rbc.kernel_coarsest(P.h, inplace.data_ptr(), inplace.data_ptr())
                _close(unpack(host(inplace), l), P.o.coarsest_solve(f), "coarsest in place l=%d" % l)
                continue
            mc = P.o.size(l + 1)
            fc = dev(pack(np.zeros((mc, mc)), l + 1))
            rbc.kernel_restrict(P.h, l, fd.data_ptr(), ud.data_ptr(), fc.data_ptr())
            _close(unpack(host(fc), l + 1), P.o.restrict(l, P.o.residual(l, f, u)), "restrict l=%d" % l)
            ec = _grid(mc, 10 * l + 3, P.o.masks(l + 1)[0])
            ecd = dev(pack(ec, l + 1))
            rbc.kernel_prolong(P.h, l, ecd.data_ptr(), ud.data_ptr(), out.data_ptr())
            _close(unpack(host(out), l), u + P.o.prolong(l, ec), "prolong l=%d" % l)
            rbc.kernel_prolong(P.h, l, ecd.data_ptr(), ud.data_ptr(), ud.data_ptr())  # in place
            _close(unpack(host(ud), l), u + P.o.prolong(l, ec), "prolong in place l=%d" % l)
    finally:
        P.close()


def test_full_size_level0_steps():
    """The 4097^2 fine level in the launch shape the solve uses."""
    n = 4097
    print("rbc full-size steps", n, flush=True)
    P = Pair(n, 20, "G1")
    try:
        f = _grid(n, 31) * (n - 1) ** 2
        u = _grid(n, 32)
        fd, ud, out = dev(f), dev(u), dev(np.zeros((n, n)))
        for colour in (1, 2):
            rbc.kernel_smooth(P.h, 0, colour, fd.data_ptr(), ud.data_ptr(), out.data_ptr())
            _close(host(out), P.o.smooth_colour(0, f, u, colour), "smooth c=%d" % colour)
        fc = dev(pack(np.zeros((n, n)), 1))
        rbc.kernel_restrict(P.h, 0, fd.data_ptr(), ud.data_ptr(), fc.data_ptr())
        _close(unpack(host(fc), 1), P.o.restrict(0, P.o.residual(0, f, u)), "restrict")
        ec = _grid(n, 33, P.o.masks(1)[0])
        rbc.kernel_prolong(P.h, 0, dev(pack(ec, 1)).data_ptr(), ud.data_ptr(), out.data_ptr())
        _close(host(out), u + P.o.prolong(0, ec), "prolong")
    finally:
        P.close()


CYCLE_CASES = [
    # n, levels, coarse, gamma, nu1, nu2, omega, cycles
    (9, 2, "G1", 1, 1, 1, 1.0, 2), (65, 8, "G1", 1, 1, 1, 1.0, 3), (65, 8, "GN", 2, 1, 1, 1.0, 3),
    (129, 10, "NG", 1, 2, 1, 1.1, 3), (129, 9, "G1", 2, 1, 1, 1.0, 2), (257, 12, "G1", 1, 0, 2, 1.2, 3),
    (1025, 16, "GN", 1, 1, 1, 1.0, 2), (17, 3, "NG", 2, 2, 2, 0.9, 3),
    (1025, 16, "G1", 1, 2, 2, 1.1, 2), (1025, 15, "NG", 1, 1, 0, 1.0, 2), (513, 14, "G1", 1, 0, 3, 1.0, 2),
    (257, 9, "GN", 1, 1, 1, 1.0, 3), (4097, 20, "G1", 1, 1, 1, 1.0, 1),
]


@pytest.mark.parametrize("n,levels,coarse,gamma,nu1,nu2,omega,cycles", CYCLE_CASES)
def test_cycles_match_oracle(n, levels, coarse, gamma, nu1, nu2, omega, cycles):
    print("rbc cycles", n, levels, coarse, gamma, nu1, nu2, omega, flush=True)
    P = Pair(n, levels, coarse, gamma, nu1, nu2, omega)
    try:
        f = _grid(n, n + levels) * (n - 1) ** 2
        fd, ud = dev(f), dev(np.zeros((n, n)))
        rbc.cycles(P.h, fd.data_ptr(), ud.data_ptr(), cycles)
        u = np.zeros((n, n))
        for _ in range(cycles):
            u = P.o.cycle(f, u)
        _close(host(ud), u, "u after %d cycles" % cycles)
        r_gpu = rbc.residual_norm(P.h, fd.data_ptr(), ud.data_ptr())
        r_or = orbc.norm(P.o.residual(0, f, u))
        assert abs(r_gpu - r_or) <= 1e-9 * r_or + 1e-12 * orbc.norm(f)
    finally:
        P.close()


TAIL_CASES = [
    # n, levels, coarse, gamma, nu1, nu2, omega, cycles
    (65, 8, "G1", 1, 1, 1, 1.0, 2), (65, 8, "GN", 2, 1, 1, 1.0, 2), (129, 10, "NG", 2, 2, 1, 1.1, 2),
    (257, 12, "G1", 1, 0, 2, 1.2, 2), (1025, 16, "GN", 2, 1, 1, 1.0, 1), (33, 6, "G1", 2, 2, 2, 0.9, 2),
    (129, 7, "G1", 1, 1, 0, 1.0, 2),
]


@pytest.mark.parametrize("side", ["17", "33", "65", "129"])
@pytest.mark.parametrize("n,levels,coarse,gamma,nu1,nu2,omega,cycles", TAIL_CASES)
def test_tail_equals_per_level_kernels(n, levels, coarse, gamma, nu1, nu2, omega, cycles, side,
                                       monkeypatch):
    """The one-workgroup tail (the levels of side <= MG_RBC_TAIL down to the coarsest in
    one launch; a side reaching level 0 runs the whole cycle there) against the cycle of
    per-level kernels, V- and W-cycles: the partial steps, interpolation and coarsest
    solve are the same device functions and the restriction sums in the same order, so
    the two agree to rounding (bit for bit where the compiler fuses the same multiply-adds:
    on the levels without distance-2 taps)."""
    print("rbc tail", n, levels, coarse, gamma, nu1, nu2, omega, side, flush=True)
    f = _grid(n, 700 + n + levels) * (n - 1) ** 2
    out = []
    for env in ("0", side):
        monkeypatch.setenv("MG_RBC_TAIL", env)
        P = Pair(n, levels, coarse, gamma, nu1, nu2, omega)
        try:
            fd, ud = dev(f), dev(np.zeros((n, n)))
            rbc.cycles(P.h, fd.data_ptr(), ud.data_ptr(), cycles)
            out.append(host(ud))
        finally:
            P.close()
    _close(out[1], out[0], "tail against per-level kernels")
    print("  bit-identical:", np.array_equal(out[0], out[1]), flush=True)


def test_full_size_cycle_matches_oracle():
    """One G1 V(1,1) cycle at 4097^2 with the 17 levels the benchmark times, from the
    benchmark's right-hand side, against the oracle's cycle."""
    from paper_2008_03885_amd import inputs
    n = 4097
    print("rbc full-size cycle", n, flush=True)
    P = Pair(n, 17, "G1", 1, 1, 1, 1.0)
    try:
        f = inputs.fourier_rhs(n)
        fd, ud = dev(f), dev(np.zeros((n, n)))
        rbc.cycles(P.h, fd.data_ptr(), ud.data_ptr(), 1)
        _close(host(ud), P.o.cycle(f, np.zeros((n, n))), "u after one 4097^2 cycle")
    finally:
        P.close()


@pytest.mark.parametrize("n", [3, 5, 9])
@pytest.mark.parametrize("nu1", [0, 1])
def test_two_level_cycle_is_a_direct_solver(n, nu1):
    """Theorem 3 on the GPU: one two-level cycle with omega = 1, eq. L_G1 and a final
    post-smoothing step leaves only rounding."""
    print("rbc theorem 3", n, nu1, flush=True)
    P = Pair(n, 2, "G1", 1, nu1, 1, 1.0)
    try:
        f = _grid(n, 5 + n) * (n - 1) ** 2
        fd, ud = dev(f), dev(np.zeros((n, n)))
        r0 = rbc.residual_norm(P.h, fd.data_ptr(), ud.data_ptr())
        rbc.cycles(P.h, fd.data_ptr(), ud.data_ptr(), 1)
        assert rbc.residual_norm(P.h, fd.data_ptr(), ud.data_ptr()) < 1e-13 * r0
    finally:
        P.close()


def test_boundary_values_are_kept_and_solve_converges_at_full_size():
    """4097^2, G1 V(1,1): the Dirichlet values in u's boundary are the solution's, the solve
    reaches 1e-10 and every cycle reduces the residual by at least the paper's two-level
    factor's order (section 4.4: V-cycles lose the direct-solver property)."""
    n = 4097
    print("rbc solve", n, flush=True)
    P = Pair(n, 20, "G1", 1, 1, 1, 1.0, max_cycles=40)
    try:
        x = np.linspace(0.0, 1.0, n)
        X, Y = np.meshgrid(x, x, indexing="ij")
        exact = np.exp(X) * np.sin(Y)  # harmonic, so f = 0 and the discrete solution is near it
        u0 = np.zeros((n, n))
        u0[0, :], u0[-1, :], u0[:, 0], u0[:, -1] = exact[0, :], exact[-1, :], exact[:, 0], exact[:, -1]
        fd, ud = dev(np.zeros((n, n))), dev(u0)
        st, k, hist = rbc.solve(P.h, fd.data_ptr(), ud.data_ptr(), 40)
        assert st == mg.MG_OK, (st, k, hist)
        u = host(ud)
        assert np.array_equal(u[0, :], u0[0, :]) and np.array_equal(u[:, -1], u0[:, -1])
        assert hist[-1] <= 1e-10 * hist[0]
        rates = np.array(hist[1:]) / np.array(hist[:-1])
        assert rates.max() < 0.5, rates
        # second-order accurate: the discrete solution is within O(h^2) of the harmonic one
        assert np.abs(u - exact).max() < 1e-6
    finally:
        P.close()


def test_errors_are_reported():
    P = Pair(17, 4, "G1")
    try:
        with pytest.raises(mg.MGError):
            rbc.kernel_smooth(P.h, 4, 1, 1, 2, 3)  # level out of range: rejected on the host
        with pytest.raises(mg.MGError):
            rbc.kernel_smooth(P.h, 0, 3, 1, 2, 3)
        with pytest.raises(mg.MGError):
            rbc.kernel_restrict(P.h, 3, 1, 2, 3)
        with pytest.raises(mg.MGError):
            rbc.kernel_smooth(P.h, 0, 1, 1, 2, 2)  # in place is not allowed  # the last level has no next level
    finally:
        P.close()
