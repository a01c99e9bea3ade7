"""The residual-norm entry point that allocates nothing (mg_residual_norm_noalloc),
through the C ABI, against the handle-based mg_residual_norm on the same inputs: two calls
in a row on the shared scratch, the second with a smaller grid.  The same kernels and
summation order make the two equal bit for bit; both also match the oracle's long-double
residual norm."""
import numpy as np
import pytest

import oracle
from gpu_util import Handle, dev, rand_grid, stream, torch
from paper_2008_03885_amd import mg

pytestmark = pytest.mark.gpu


def _pair(dim, n, order, seed):
    f = rand_grid(n, dim, seed)
    u = rand_grid(n, dim, seed + 1) * 1e-3
    return f, u


@pytest.mark.parametrize("dim,sizes,order", [(2, (1025, 257), 4), (3, (129, 65), 4), (2, (513, 65), 6),
                                             (3, (65, 33), 2)])
def test_noalloc_norm_equals_handle_norm(dim, sizes, order):
    t = torch()
    rel = t.full((2,), float("nan"), dtype=t.float64, device="cuda")
    got = []
    for k, n in enumerate(sizes):
        print("noalloc dim=%d n=%d order=%d" % (dim, n, order), flush=True)
        f, u = _pair(dim, n, order, 10 * k + dim)
        fd, ud = dev(f), dev(u)
        assert mg.mg_residual_norm_noalloc(dim, n, order, fd.data_ptr(), ud.data_ptr(),
                                           rel[k:].data_ptr(), stream()) == mg.MG_OK
        t.cuda.synchronize()
        H = Handle(dim, n, order=order)
        try:
            ref = mg.mg_residual_norm(H.h, fd.data_ptr(), ud.data_ptr())
        finally:
            H.close()
        val = rel[k].item()
        assert val == ref, (n, val, ref)
        s = oracle.fine_stencil(dim, order, 1.0 / (n - 1))
        ld = oracle.residual_norm_ld(s, f, u) / oracle.norm(f)
        assert abs(val - ld) <= 1e-12 * ld, (n, val, ld)
        got.append(val)
    assert got[0] != got[1]


def test_noalloc_rejects_sizes_beyond_the_scratch():
    t = torch()
    buf = t.zeros(8, dtype=t.float64, device="cuda")
    p = buf.data_ptr()
    lib = mg.lib()
    assert lib.mg_residual_norm_noalloc(2, 32769, 4, p, p, p, None) == mg.MG_EINVAL
    assert "MG_NOALLOC_SCRATCH_BYTES" in mg.last_error()
    assert lib.mg_residual_norm_noalloc(3, 2049, 4, p, p, p, None) == mg.MG_EINVAL
    assert lib.mg_residual_norm_noalloc(3, 100, 4, p, p, p, None) == mg.MG_EINVAL
    assert lib.mg_residual_norm_noalloc(2, 129, 4, p, p, None, None) == mg.MG_EINVAL
