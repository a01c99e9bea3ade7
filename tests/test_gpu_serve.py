"""The solve server on the GPU: continuous batching of mixed-size 2D solves.

Each request must come out exactly as a standalone handle solves it (same kernels, same
per-slot reduction order), whatever else shares its batch or the device, and must
reach the 1e-10 relative residual in FP64.  Every served result is also checked against
the exact discrete solution L_h^{-1} f from the sine transform (no multigrid code): the
oracle's long-double residual of the served u is at most 1e-10 relative, and the error
is within the bound ||L_h^{-1}|| ||f - L_h u||_h = ||f - L_h u||_h / lambda_min that this
residual implies.
"""
import numpy as np
import pytest

import oracle
from gpu_util import dev, host, torch
from oracle import dst
from paper_2008_03885_amd import inputs, mg, serve

pytestmark = pytest.mark.gpu

BASE = dict(dim=2, coarse=0, gamma=1, nu1=2, nu2=1, precision=mg.MG_PREC_MIXED, rtol=1e-10,
            max_cycles=30, inner_cycles=4)


def _rhs(n, seed):
    return inputs.fourier_rhs(n, 2, min(64, (n - 1) // 4), seed=seed)


def _check_exact(u, f, what=""):
    """u against the exact discrete solution, within the bound its residual implies."""
    n = f.shape[0]
    st = oracle.fine_stencil(2, 4, 1.0 / (n - 1))
    fn = oracle.norm(f)
    rel = oracle.residual_norm_ld(st, f, u) / fn
    assert rel <= 1.01e-10, "%s: residual %.3e" % (what, rel)
    exact = dst.solve(f)
    bound = rel * fn / dst.eigenvalues(n, 2).min()
    err = oracle.norm(u - exact)
    assert err <= 1.01 * bound + 1e-14 * oracle.norm(exact), "%s: %.3e > %.3e" % (what, err, bound)


def _solo(n, f, **over):
    """u and result of a standalone handle (mg_solve) for the same configuration."""
    cfg = dict(BASE, **over)
    h = mg.mg_setup(mg.make_config(n=n, **cfg), torch().cuda.current_stream().cuda_stream)
    try:
        fd, ud = dev(f), dev(np.zeros_like(f))
        st, res = mg.mg_solve(h, fd.data_ptr(), ud.data_ptr())
        return host(ud), st, res.hist()
    finally:
        mg.mg_destroy(h)


def _serve(reqs, budget=8 << 30, max_slots=8, chunk_steps=2, stagger=None, stream_groups=0, **over):
    """Runs (tag, n, f) requests through one server; returns {tag: (u, completion)}."""
    import time
    cfg = dict(BASE, **over)
    S = serve.Server(budget, max_slots, chunk_steps, stream_groups, n=65, **cfg)
    try:
        bufs = {tag: (dev(f), dev(np.full_like(f, np.nan))) for tag, n, f in reqs}
        torch().cuda.synchronize()  # the server reads f on its own streams
        for i, (tag, n, f) in enumerate(reqs):
            st = S.submit(tag, *bufs[tag])
            assert st == mg.MG_OK, (st, mg.last_error())
            if stagger:
                time.sleep(stagger[i])
        done = S.wait_all(len(reqs), 300.0)
        stats = S.stats()
        out = {c.tag: (host(bufs[c.tag][1]), c) for c in done}
        return out, stats
    finally:
        S.close()


@pytest.mark.parametrize("precision", [mg.MG_PREC_MIXED, mg.MG_PREC_FP64])
def test_single_request_equals_standalone_solve(precision):
    n = 129
    f = _rhs(n, inputs.SEED_BASE + 1000)
    out, stats = _serve([(7, n, f)], precision=precision,
                        max_cycles=30 if precision else 60)
    u, c = out[7]
    ref, st, hist = _solo(n, f, precision=precision, max_cycles=30 if precision else 60)
    assert c.status == st == mg.MG_OK
    assert np.array_equal(u, ref)
    assert c.result.hist() == hist
    assert c.result.rel_residual <= 1e-10
    assert stats["completed"] == 1 and stats["batches_created"] == 1
    _check_exact(u, f, "single")


@pytest.mark.parametrize("stream_groups,inflight", [(0, "1"), (3, "1"), (3, "2")])
def test_results_identical_alone_and_in_the_mix(stream_groups, inflight, monkeypatch):
    """A stream of mixed sizes arriving while others run; the probe request (same n and
    f) appears three times at different points of the stream.  Every request equals its
    standalone solve bit for bit and reaches 1e-10, with batches on streams of their own
    or sharing streams by size group, and with one or two replay chunks in flight per
    batch (MG_SERVE_INFLIGHT, read when the server is created)."""
    monkeypatch.setenv("MG_SERVE_INFLIGHT", inflight)
    rng = np.random.default_rng(5)
    sizes = [65, 129, 257, 513, 1025]
    probe_n, probe_f = 257, _rhs(257, inputs.SEED_BASE + 1001)
    reqs = []
    for i in range(24):
        if i in (0, 9, 20):
            reqs.append((i, probe_n, probe_f))
        else:
            n = int(rng.choice(sizes))
            reqs.append((i, n, _rhs(n, inputs.SEED_BASE + 1100 + i)))
    stagger = list(rng.exponential(0.002, len(reqs)))
    out, stats = _serve(reqs, stagger=stagger, stream_groups=stream_groups)
    assert stats["completed"] == len(reqs)
    assert stats["peak_active"] > 1          # requests overlapped on the device
    solo = {}
    for tag, n, f in reqs:
        key = (n, tag) if tag not in (0, 9, 20) else (n, "probe")
        if key not in solo:
            solo[key] = _solo(n, f)
        ref, st, hist = solo[key]
        u, c = out[tag]
        assert c.status == mg.MG_OK and st == mg.MG_OK, tag
        assert np.array_equal(u, ref), tag
        assert c.result.hist() == hist, tag
        assert c.result.rel_residual <= 1e-10
        assert c.t_submit <= c.t_admit <= c.t_done
        _check_exact(u, f, "mix %d" % tag)
    a, b, d = out[0][0], out[9][0], out[20][0]
    assert np.array_equal(a, b) and np.array_equal(a, d)


@pytest.mark.parametrize("precision", [mg.MG_PREC_FP64, mg.MG_PREC_MIXED])
def test_red_black_requests_equal_standalone_solves(precision):
    """Red-black smoothing in batched slots (fused passes with the third sweep target,
    the LDS tail) gives each request its standalone result bit for bit."""
    rng = np.random.default_rng(9)
    reqs = []
    for i in range(10):
        n = int(rng.choice([65, 129, 257, 1025]))
        reqs.append((i, n, _rhs(n, inputs.SEED_BASE + 1200 + i)))
    over = dict(smoother=mg.MG_SMOOTH_RBJ, precision=precision, max_cycles=30)
    out, stats = _serve(reqs, **over)
    assert stats["completed"] == len(reqs)
    for tag, n, f in reqs:
        ref, st, hist = _solo(n, f, **over)
        u, c = out[tag]
        assert c.status == mg.MG_OK and st == mg.MG_OK, tag
        assert np.array_equal(u, ref), tag
        assert c.result.hist() == hist, tag
        assert c.result.rel_residual <= 1e-10
        _check_exact(u, f, "red-black %d" % tag)


def test_admission_by_footprint():
    """A budget that holds one slot of 513^2: three such requests run one after another,
    and a later 257^2 request gets memory by releasing the idle 513 batch."""
    base = mg.make_config(n=65, **BASE)
    one513 = serve.mg_serve_batch_bytes(base, 513, 1)
    one257 = serve.mg_serve_batch_bytes(base, 257, 1)
    budget = one513 + one257 // 2   # not a second 513 slot, nor a 257 batch beside it
    assert budget < serve.mg_serve_batch_bytes(base, 513, 2)
    reqs = [(i, 513, _rhs(513, inputs.SEED_BASE + 1200 + i)) for i in range(3)]
    out, stats = _serve(reqs, budget=budget)
    assert stats["peak_active"] == 1 and stats["completed"] == 3
    assert stats["peak_bytes_held"] <= budget
    for tag, n, f in reqs:
        ref, _, _ = _solo(n, f)
        assert np.array_equal(out[tag][0], ref)
        _check_exact(out[tag][0], f, "admission %d" % tag)
    # second server: a 513 request, then a 257 request that needs the 513 batch released
    reqs2 = [(0, 513, reqs[0][2]), (1, 257, _rhs(257, inputs.SEED_BASE + 1300))]
    out2, stats2 = _serve(reqs2, budget=budget, stagger=[0.05, 0.0])
    assert stats2["completed"] == 2
    assert stats2["batches_created"] == 2 and stats2["batches_released"] >= 1
    assert np.array_equal(out2[0][0], out[0][0])
    _check_exact(out2[1][0], reqs2[1][2], "admission 257")


def test_many_small_requests_fill_the_slots():
    reqs = [(i, 65, _rhs(65, inputs.SEED_BASE + 1400 + i)) for i in range(40)]
    out, stats = _serve(reqs, max_slots=16)
    assert stats["completed"] == 40 and stats["peak_active"] == 16
    for tag, n, f in reqs[:6]:
        ref, _, hist = _solo(n, f)
        assert np.array_equal(out[tag][0], ref)
        assert out[tag][1].result.hist() == hist
    for tag, n, f in reqs:
        _check_exact(out[tag][0], f, "small %d" % tag)


def test_oversized_request_is_rejected():
    base = mg.make_config(n=65, **BASE)
    budget = serve.mg_serve_batch_bytes(base, 257, 1)
    S = serve.Server(budget, 4, 2, n=65, **BASE)
    try:
        f, u = dev(np.zeros((513, 513))), dev(np.zeros((513, 513)))
        assert S.submit(1, f, u) == mg.MG_ENOMEM
        assert S.submit(2, dev(np.zeros((100, 100))), dev(np.zeros((100, 100)))) == mg.MG_EINVAL
        assert S.stats()["rejected"] == 1
    finally:
        S.close()
