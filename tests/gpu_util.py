"""Helpers shared by the GPU tests: device arrays, handles and oracle counterparts."""
import numpy as np

import oracle
from paper_2008_03885_amd import mg

DEV = "cuda:0"


def torch():
    import torch as _t
    return _t


def rand_grid(n, dim, seed):
    """N(0,1) interior values, zero boundary."""
    rng = np.random.default_rng(seed)
    a = np.zeros((n,) * dim)
    a[(slice(1, n - 1),) * dim] = rng.standard_normal((n - 2,) * dim)
    return a


def dev(a, fp32=False):
    t = torch()
    return t.from_numpy(np.ascontiguousarray(a)).to(DEV, t.float32 if fp32 else t.float64)


def host(t):
    torch().cuda.synchronize()
    return t.double().cpu().numpy()


def stream():
    return torch().cuda.current_stream().cuda_stream


class Handle:
    """An mg handle and the oracle hierarchy built from the same configuration."""

    def __init__(self, dim, n, coarse=0, prolong=3, n_coarsest=9, nu1=2, nu2=1, gamma=1,
                 precision=0, rtol=1e-10, max_cycles=100, inner_cycles=4, order=4, omega=0.0,
                 smoother=0, restrict_op=1):
        self.cfg = mg.make_config(dim=dim, n=n, coarse=coarse, prolong=prolong,
                                  n_coarsest=n_coarsest, nu1=nu1, nu2=nu2, gamma=gamma,
                                  precision=precision, rtol=rtol, max_cycles=max_cycles,
                                  inner_cycles=inner_cycles, order=order, omega=omega,
                                  smoother=smoother, restrict_op=restrict_op)
        self.h = mg.mg_setup(self.cfg, stream())
        self.dim, self.n = dim, n
        if omega > 0:
            self.omega = omega
        elif smoother == oracle.SMOOTH_RBJ:
            self.omega = oracle.rbj_omega(dim, order, coarse)
        elif smoother == oracle.SMOOTH_RBGS:
            self.omega = oracle.rbgs_omega(dim, order, coarse)
        else:
            self.omega = oracle.jacobi_omega(dim, order)
        self.oracle = oracle.Multigrid(dim, n, order=order, coarse=coarse, prolong=prolong,
                                       nu1=nu1, nu2=nu2, gamma=gamma, n_coarsest=n_coarsest,
                                       omega=self.omega, smoother=smoother, restrict_op=restrict_op)

    def level(self, l):
        n_l, s = self.oracle.level_stencil(l)
        assert mg.mg_level_size(self.h, l) == n_l
        return n_l, s

    def close(self):
        mg.mg_destroy(self.h)
        self.oracle.close()


def assert_close(got, ref, tol, what=""):
    err = np.abs(got - ref).max()
    assert err <= tol, "%s: max abs error %.3e > %.3e" % (what, err, tol)
    return err
