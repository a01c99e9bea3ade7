"""The C-ABI library loads, exports every declared entry point, and rejects bad
configurations before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

from conftest import ROOT
from paper_2008_03885_amd import mg, rbc, serve


def _declared_functions():
    names = []
    inc = os.path.join(ROOT, "include")
    for hdr in sorted(os.listdir(inc)):
        if not hdr.endswith(".h"):
            continue
        with open(os.path.join(inc, hdr)) as fh:
            text = fh.read()
        for m in re.finditer(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*(mg_[a-z0-9_]+)\s*\(", text, re.M):
            names.append(m.group(1))
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("mg_setup", "mg_solve", "mg_destroy", "mg_footprint_bytes", "mg_solve_async",
                     "mg_query", "mg_last_error", "mg_run_cycles"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(mg.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the bindings cover the same names
    assert set(_declared_functions()) <= set(mg._SIGS) | set(serve._SIGS) | set(rbc._SIGS)


@pytest.mark.parametrize("kwargs", [
    dict(dim=4), dict(order=8), dict(order=3), dict(n=100), dict(smoother=3), dict(n=129, n_coarsest=7), dict(gamma=3),
    # red-black Gauss-Seidel: 2D with cross-stencil (rediscretized) coarse operators only
    dict(smoother=2, dim=3), dict(smoother=2, coarse=1), dict(smoother=2, coarse=3),
    dict(prolong=2), dict(restrict_op=2), dict(nu1=0, nu2=0), dict(omega=2.5),
    # the cubic-adjoint restriction: rediscretized coarse operators only
    dict(restrict_op=3, coarse=1), dict(restrict_op=3, coarse=3),
    dict(max_cycles=0), dict(precision=1, inner_cycles=0), dict(coarse=5),
])
def test_invalid_configs_rejected(kwargs):
    cfg = mg.make_config(**kwargs)
    assert mg.mg_footprint_bytes(cfg) == 0
    h = ctypes.c_void_p()
    st = mg.lib().mg_setup(ctypes.byref(cfg), None, ctypes.byref(h))
    assert st == mg.MG_EINVAL
    assert h.value is None
    assert mg.last_error() != ""


def test_footprint_counts_hierarchy():
    cfg = mg.make_config(dim=2, n=4097)
    fp = mg.mg_footprint_bytes(cfg)
    # level-0 Jacobi target, three arrays per intermediate level, u and f on the coarsest
    n, total = 4097, 4097 ** 2 * 8
    n = (n - 1) // 2 + 1
    while n > 9:
        total += 3 * n * n * 8
        n = (n - 1) // 2 + 1
    total += 2 * 9 * 9 * 8
    assert total <= fp <= total + 2 * 1024 * 1024
    mixed = mg.mg_footprint_bytes(mg.make_config(dim=2, n=4097, precision=mg.MG_PREC_MIXED))
    assert mixed > 0


def test_null_arguments_rejected():
    lib = mg.lib()
    assert lib.mg_solve(None, None, None, None) == mg.MG_EINVAL
    assert lib.mg_destroy(None) == mg.MG_OK
    assert lib.mg_level_size(None, 0) == -1


def test_batch_footprint_is_linear_in_slots():
    """A batch holds per-problem arrays (level-0 f and u included) once per slot and the
    shared tables once."""
    base = mg.make_config(dim=2, n=65, precision=mg.MG_PREC_MIXED)
    for n in (65, 129, 1025):
        one, two, five = (serve.mg_serve_batch_bytes(base, n, k) for k in (1, 2, 5))
        per = two - one
        assert five == one + 4 * per
        # at least the FP64 f, u and the FP32 u, f, r of the top level per slot
        assert per >= n * n * (2 * 8 + 3 * 4)
        assert per < n * n * (2 * 8 + 3 * 4) * 4 / 3 + 64 * 1024
    assert serve.mg_serve_batch_bytes(base, 100, 1) == 0   # not 2^k + 1
    assert serve.mg_serve_batch_bytes(base, 65, 0) == 0


@pytest.mark.parametrize("change", [
    dict(max_slots=0), dict(max_slots=2000), dict(chunk_steps=0), dict(hbm_budget=0),
    dict(dim=3), dict(gamma=5),
])
def test_server_rejects_bad_configs(change):
    """Configuration errors are found before any device call."""
    kw = dict(hbm_budget=1 << 30, max_slots=8, chunk_steps=2)
    base = dict(dim=2, n=65)
    for k, v in change.items():
        (kw if k in kw else base)[k] = v
    cfg = serve.make_server_config(kw["hbm_budget"], kw["max_slots"], kw["chunk_steps"], **base)
    h = ctypes.c_void_p()
    assert serve.lib().mg_server_create(ctypes.byref(cfg), ctypes.byref(h)) == mg.MG_EINVAL
    assert h.value is None
    assert serve.lib().mg_server_submit(None, 0, 65, None, None) == mg.MG_EINVAL
    assert serve.lib().mg_server_poll(None, None, 0, 0.0) == -1
    assert serve.lib().mg_server_destroy(None) == mg.MG_OK


def test_enum_values_match_the_binding():
    """Every `MG_NAME = value` the header declares has the same value in mg.py."""
    with open(os.path.join(ROOT, "include", "mg.h")) as fh:
        text = fh.read()
    found = dict((k, int(v)) for k, v in re.findall(r"\b(MG_[A-Z0-9_]+)\s*=\s*(\d+)", text))
    for name in ("MG_COARSE_NG", "MG_COARSE_GALERKIN", "MG_COARSE_NG2", "MG_COARSE_G2",
                 "MG_SMOOTH_JACOBI", "MG_SMOOTH_RBJ", "MG_PREC_FP64", "MG_PREC_MIXED", "MG_OK",
                 "MG_EINVAL", "MG_EBUSY"):
        assert found[name] == getattr(mg, name), name


@pytest.mark.parametrize("nu1,nu2,extra", [(2, 1, True), (1, 1, False), (2, 2, False), (3, 0, False),
                                          (1, 2, True), (0, 1, False)])
def test_red_black_footprint_counts_the_third_sweep_target(nu1, nu2, extra):
    """Fused 2D red-black cycles run max(1, nu1) + max(1, nu2) passes per level; with an odd
    count they need a third sweep array on every level above the coarsest, and the
    footprint says so (host arithmetic)."""
    n, nc = 1025, 9
    base = mg.mg_footprint_bytes(mg.make_config(dim=2, n=n, nu1=nu1, nu2=nu2, n_coarsest=nc))
    rb = mg.mg_footprint_bytes(mg.make_config(dim=2, n=n, nu1=nu1, nu2=nu2, n_coarsest=nc,
                                              smoother=mg.MG_SMOOTH_RBJ))
    sides = []
    m = n
    while m > nc:
        sides.append(m)
        m = (m - 1) // 2 + 1
    t2 = sum(s * s * 8 for s in sides)
    passes = max(1, nu1) + max(1, nu2)
    assert rb - base == (t2 if passes % 2 == 1 else 0)
    assert (rb > base) == extra


@pytest.mark.parametrize("kwargs", [
    dict(n=100), dict(n=2), dict(levels=1), dict(n=17, levels=9), dict(n=129, levels=2),
    dict(coarse=3), dict(gamma=3), dict(nu1=0, nu2=0), dict(nu1=9), dict(omega=2.0),
    dict(omega=-1.0), dict(max_cycles=0), dict(rtol=-1.0),
])
def test_red_black_coarsening_invalid_configs_rejected(kwargs):
    """mg_rbc_setup validates before touching the device: too many levels for n, a
    coarsest level above MG_RBC_MAX_COARSEST unknowns (129 with two levels), bad enums."""
    cfg = rbc.make_config(**{**dict(n=17, levels=4), **kwargs})
    h = ctypes.c_void_p()
    st = rbc.lib().mg_rbc_setup(ctypes.byref(cfg), None, ctypes.byref(h))
    assert st == mg.MG_EINVAL
    assert h.value is None
    assert mg.last_error() != ""


def test_red_black_coarsening_enums_match_the_header():
    with open(os.path.join(ROOT, "include", "mg_rbc.h")) as fh:
        text = fh.read()
    m = re.search(r"enum \{ MG_RBC_NG = (\d), MG_RBC_G1 = (\d), MG_RBC_GN = (\d) \}", text)
    assert tuple(int(v) for v in m.groups()) == (rbc.MG_RBC_NG, rbc.MG_RBC_G1, rbc.MG_RBC_GN)
    assert "#define MG_RBC_MAX_COARSEST %d" % rbc.MG_RBC_MAX_COARSEST in text
    assert rbc.lib().mg_rbc_level_size(None, 0) == -1
    assert rbc.lib().mg_rbc_level_pitch(None, 0) == -1


def test_red_black_coarsening_null_arguments_rejected():
    """Every mg_rbc entry point checks its handle and pointers on the host first."""
    lib = rbc.lib()
    assert lib.mg_rbc_setup(None, None, None) == mg.MG_EINVAL
    assert lib.mg_rbc_cycles(None, None, None, 1) == mg.MG_EINVAL
    assert lib.mg_rbc_solve(None, None, None, None, None) == mg.MG_EINVAL
    assert lib.mg_rbc_residual_norm(None, None, None, None) == mg.MG_EINVAL
    assert lib.mg_rbc_kernel_smooth(None, 0, 1, None, None, None) == mg.MG_EINVAL
    assert lib.mg_rbc_kernel_restrict(None, 0, None, None, None) == mg.MG_EINVAL
    assert lib.mg_rbc_kernel_prolong(None, 0, None, None, None) == mg.MG_EINVAL
    assert lib.mg_rbc_kernel_coarsest(None, None, None) == mg.MG_EINVAL
    lib.mg_rbc_destroy(None)
    assert mg.last_error() != ""
