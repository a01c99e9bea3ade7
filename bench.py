"""Benchmark: fourth-order Poisson multigrid solves on one MI355X.

One step is one whole solve from a zero initial guess to a 1e-10 relative residual, with
f and u resident in HBM.  The default workload is the largest configuration:

  poisson3d-1025-galerkin-w22 (default)  3D, n = 1025 (1,070,599,167 unknowns), smooth
      sine-series right-hand side (k <= 8, N(0,1) amplitudes, seeded), fourth-order
      13-point cross on the finest level, Galerkin coarse operators R L P down to 9^3
      with an exact coarsest solve, W(2,2) omega-Jacobi (omega = 9/11), full weighting,
      cubic interpolation.  Timed in mixed precision (FP32 cycles inside FP64 iterative
      refinement: `value`) and in plain FP64 (`precision_compare`), plus the error of the
      1025^3 solution against the oracle's 129^3 solve of the same continuous problem.

The same JSON line carries, as extra keys, the other configurations:
  `poisson3d_513`   3D, n = 513, uniform[-1,1] noise smoothed by three neighbour-average
                    passes, V(2,1), mixed (eight FP32 cycles per step) against FP64;
  `poisson2d_4097`  2D, n = 4097, Fourier right-hand side k <= 64 with N(0,1)/|k|
                    amplitudes, V(2,1), FP64, with the level-0 fused-kernel roofline and the
                    Galerkin, W-cycle, second-order, red-black and sixth-order variants;
  `serving`         the continuous-batching server on a Poisson stream of 2D solves
                    (n = 2^k + 1, k uniform on 6..11) at 0.5, 0.8 and 0.95 of saturation;
  `red_black_coarsening`  section 4's rotated-grid cycles on the 4097^2 second-order
                    problem.
Other workloads can be run alone with --workload.  --gpus N with N > 1 exits: the
library runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DEFAULT_WORKLOAD = "poisson3d-1025-galerkin-w22"

WORKLOADS = {
    "poisson2d-4097": dict(dim=2, n=4097, rhs="fourier", coarse=0, gamma=1, nu1=2, nu2=1,
                           precision=0, compare=False, inner=4),
    "poisson3d-513": dict(dim=3, n=513, rhs="noise", coarse=0, gamma=1, nu1=2, nu2=1,
                          precision=1, compare=True, inner=8),
    # inner = 1: measured fastest of 1, 2, 3 FP32 W-cycles per refinement step (651, 696, 723 ms)
    "poisson3d-1025-galerkin-w22": dict(dim=3, n=1025, rhs="sine", coarse=1, gamma=2, nu1=2,
                                        nu2=2, precision=1, compare=True, inner=1, check129=True),
}

# HBM traffic of the dominant kernels from rocprofv3 --pmc (FETCH_SIZE and WRITE_SIZE per
# dispatch, scaled by the counters of a plain copy of known size), valid only for the
# kernel source they were taken on.
MEASURED_TRAFFIC = {
    # 4097^2 level 0, two sweeps + defect + full weighting: 172,251.9 KiB fetched x 2.0000
    # + 169,196.7 KiB written x 1.0000 (a 2 GiB copy reads 1,048,595 KiB / writes 2,097,152)
    "k_pre2d/f64/fused2d.hip/4097": {"bytes": 526022929, "source": "80797142e6561bc3"},
    # the same pass with red-black smoothing (one red-black sweep + defect + full weighting):
    # 156,850.3 KiB x 2.0000 + 168,329.4 KiB x 1.0000
    "k_pre2d/f64/fused2d.hip/4097/rb": {"bytes": 493592759, "source": "80797142e6561bc3"},
    # 513^3 level 0 FP32 sweep (128 x 16 tiles from point 1, two rows per thread):
    # 596,214.4 KiB x 2.0000 + 550,147.5 KiB x 1.0000
    "k_xsweep3d/f32/kernels3d.hip/513": {"bytes": 1784398131, "source": "fbab958a857d17c1"},
    # 1025^3 level 0 FP32 sweep (128 x 16 tiles from point 1, two rows per thread):
    # 4,696,404.6 KiB x 2.0000 + 4,433,740.2 KiB x 1.0000
    "k_xsweep3d/f32/kernels3d.hip/1025": {"bytes": 14158386586, "source": "fbab958a857d17c1"},
    # red-black coarsening, 4097^2 level-0 partial step (XCD-remapped 64 x 4 tiles):
    # 131,353.0 KiB x 2.0000 + 131,137.3 KiB x 1.0000 (f is read whole: 24 B a point)
    "k_rbc_smooth/f64/rbc.hip/4097": {"bytes": 403291537, "source": "b03ea673ddfdb24d"},
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    p.add_argument("--no-extras", action="store_true",
                   help="only the chosen workload (no 513^3, 4097^2, serving, red-black coarsening keys)")
    p.add_argument("--n", type=int, default=None)
    p.add_argument("--coarse", type=int, default=None,
                   help="0 rediscretized, 1 Galerkin, 2 second-order rediscretized, 3 second-order Galerkin")
    p.add_argument("--gamma", type=int, default=None)
    p.add_argument("--smoother", type=int, default=None,
                   help="0 omega-Jacobi (default), 1 red-black Jacobi, 2 red-black Gauss-Seidel (2D)")
    p.add_argument("--order", type=int, default=None, help="fine operator order: 4 (default), 2 or 6")
    p.add_argument("--restrict", type=int, default=None,
                   help="restriction: 1 full weighting (default), 3 cubic adjoint (rediscretized coarse operators)")
    p.add_argument("--omega", type=float, default=None, help="relaxation (default: the LFA optimum)")
    p.add_argument("--precision", type=int, default=None)
    p.add_argument("--compare", type=int, default=None, help="also run the other precision")
    p.add_argument("--inner", type=int, default=None, help="FP32 cycles per refinement step")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-levels", action="store_true", help="skip the per-level kernel table")
    p.add_argument("--no-variants", action="store_true",
                   help="skip the Galerkin and W-cycle runs of the 2D workload")
    p.add_argument("--kernel-reps", type=int, default=30)
    p.add_argument("--pmc-probe", action="store_true",
                   help="run a plain copy of known size, then the dominant kernel (for counters)")
    p.add_argument("--pmc-level", type=int, default=0, help="--pmc-probe: the level whose kernels run")
    p.add_argument("--serve-requests", type=int, default=1000,
                   help="requests per serving run (0: skip the serving measurement)")
    p.add_argument("--serve-only", action="store_true", help="only the serving measurement")
    p.add_argument("--stream-groups", type=int, default=3,
                   help="serving: streams shared by size groups (0: one stream per batch)")
    p.add_argument("--rbc-only", action="store_true", help="only the red-black coarsening runs")
    return p.parse_args()


def source_hash(*names):
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2008_03885_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def make_rhs(w):
    from paper_2008_03885_amd import inputs
    n = w["n"]
    if w["rhs"] == "fourier":
        return inputs.fourier_rhs(n, 2, 64, seed=inputs.SEED_BASE + 2), None
    if w["rhs"] == "noise":
        return inputs.smoothed_noise_3d(n), None
    return inputs.smooth_sine_3d(n, return_coeffs=True)


def describe(w):
    kind = {0: "rediscretized", 1: "Galerkin", 2: "second-order rediscretized",
            3: "second-order Galerkin"}[w["coarse"]]
    cyc = "%s(%d,%d)" % ("W" if w["gamma"] == 2 else "V", w["nu1"], w["nu2"])
    rhs = {"fourier": "Fourier RHS k<=64 amplitudes N(0,1)/|k|",
           "noise": "uniform[-1,1] noise smoothed by 3 neighbour-average passes",
           "sine": "smooth sine-series RHS k<=8"}[w["rhs"]]
    prec = "FP64" if w["precision"] == 0 else "FP32 cycles in FP64 refinement"
    d = w["dim"]
    sm = {0: "omega-Jacobi", 1: "red-black Jacobi", 2: "red-black Gauss-Seidel"}[w.get("smoother", 0)]
    tr = "cubic-adjoint restriction + cubic" if w.get("restrict", 1) == 3 else "FW + cubic"
    return "%dD %dth-order Poisson %s, %s, %s %s, %s, %s coarse ops to 9^%d, %s, to 1e-10" % (
        d, w.get("order", 4), "x".join([str(w["n"])] * d), rhs, cyc, sm, tr, kind, d, prec)


class Run:
    """One handle of the workload at a given precision, solving from zero."""

    def __init__(self, w, precision, fd, stream):
        import torch
        from paper_2008_03885_amd import mg
        self.mg = mg
        self.cfg = mg.make_config(dim=w["dim"], n=w["n"], coarse=w["coarse"], gamma=w["gamma"],
                                  nu1=w["nu1"], nu2=w["nu2"], precision=precision, rtol=1e-10,
                                  max_cycles=60 if precision == 0 else 30,
                                  inner_cycles=w["inner"], smoother=w.get("smoother", 0),
                                  order=w.get("order", 4), omega=w.get("omega", 0.0),
                                  restrict_op=w.get("restrict", 1))
        self.h = mg.mg_setup(self.cfg, stream.cuda_stream)
        self.fd = fd
        self.ud = torch.zeros_like(fd)
        self.precision = precision

    def step(self):
        self.ud.zero_()
        return self.mg.mg_solve(self.h, self.fd.data_ptr(), self.ud.data_ptr())

    def timed(self, steps, warmup):
        import torch
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        results = [self.step() for _ in range(steps)]
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, results[-1]

    def close(self):
        self.mg.mg_destroy(self.h)


def event_time(stream, fn, reps):
    """Average duration of fn() over reps launches, HIP events on the handle's stream."""
    import torch
    for _ in range(3):
        fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def copy_rate(stream, reps=10):
    """Bytes read + written per second by a plain 2 GiB device copy (torch) on the handle's
    stream: the rate a streaming kernel reaches on this device, beside the published peak."""
    import torch
    a = torch.ones(256 * 1024 * 1024, device="cuda", dtype=torch.float64)
    b = torch.empty_like(a)
    def fn():
        with torch.cuda.stream(stream):
            b.copy_(a)
    sec = event_time(stream, fn, reps)
    nbytes = 2 * a.numel() * 8
    del a, b
    torch.cuda.empty_cache()
    return nbytes / sec / 1e9


def in_cycle_time(run, w, stream, reps):
    """Average duration of the dominant level-0 kernel in the order the cycle runs it, each
    launch bracketed by HIP events on the handle's stream: 2D, the fused pre kernel right
    after the fused post kernel that writes its input u (untimed); 3D, sweeps in a
    ping-pong, each reading what the previous one wrote."""
    import torch
    mg = run.mg
    fp32 = 1 if run.precision == 1 else 0
    dt = torch.float32 if fp32 else torch.float64
    d, n = w["dim"], mg.mg_level_size(run.h, 0)
    nc = mg.mg_level_size(run.h, 1)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    f = torch.randn((n,) * d, generator=gen, device="cuda", dtype=torch.float64).to(dt)
    u = torch.randn((n,) * d, generator=gen, device="cuda", dtype=torch.float64).to(dt)
    t = torch.empty_like(u)
    fc = torch.empty((nc,) * d, device="cuda", dtype=dt)
    v = torch.randn((nc,) * d, generator=gen, device="cuda", dtype=torch.float64).to(dt)
    if w.get("restrict", 1) == 3 and d == 2 and w.get("smoother", 0) != 2:
        bufs = [u, t]
        def one():
            e0.record(stream)
            mg.mg_kernel_smooth(run.h, 0, fp32, f.data_ptr(), bufs[0].data_ptr(), bufs[1].data_ptr())
            e1.record(stream)
            bufs.reverse()
    elif w.get("smoother", 0) == 2 or (w.get("smoother", 0) and d == 3):
        # red then black partial steps in a ping-pong, as the cycle runs them
        bufs = [u, t]
        col = [1]
        def one():
            e0.record(stream)
            mg.mg_kernel_smooth_colour(run.h, 0, fp32, col[0], f.data_ptr(), bufs[0].data_ptr(),
                                       bufs[1].data_ptr())
            e1.record(stream)
            bufs.reverse()
            col[0] = 3 - col[0]
    elif d == 2:
        def one():
            mg.mg_kernel_prolong_postsmooth(run.h, 0, fp32, v.data_ptr(), t.data_ptr(), f.data_ptr(), u.data_ptr())
            e0.record(stream)
            mg.mg_kernel_presmooth_restrict(run.h, 0, fp32, f.data_ptr(), u.data_ptr(), t.data_ptr(), fc.data_ptr())
            e1.record(stream)
    else:
        bufs = [u, t]
        def one():
            e0.record(stream)
            mg.mg_kernel_smooth(run.h, 0, fp32, f.data_ptr(), bufs[0].data_ptr(), bufs[1].data_ptr())
            e1.record(stream)
            bufs.reverse()
    total, events = 0.0, []
    for i in range(reps + 3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        one()
        if i >= 3:
            events.append((e0, e1))
    torch.cuda.synchronize()
    for e0, e1 in events:
        total += e0.elapsed_time(e1) / 1e3
    return total / len(events)


def level_kernels(run, w, stream, reps, only_level=None):
    """Per-level launches of the kernels the cycle runs on that level, each timed with HIP
    events, with their algorithmic bytes.  2D: the fused pre-smoothing + defect + full
    weighting and the fused interpolation + correction + post-smoothing; 3D: the sweep, the
    fused defect + full weighting (on Galerkin levels also the defect pass followed by full
    weighting, which the cycle runs) and the interpolation + correction."""
    import torch
    mg = run.mg
    fp32 = 1 if run.precision == 1 else 0
    dt = torch.float32 if fp32 else torch.float64
    b = 4 if fp32 else 8
    d = w["dim"]
    rows = []
    L = 0
    while mg.mg_level_size(run.h, L) > 0:
        L += 1
    tail_cap = 65 if d == 2 else 17
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    for l in range(L - 1):
        n, nc = mg.mg_level_size(run.h, l), mg.mg_level_size(run.h, l + 1)
        if n <= tail_cap or (only_level is not None and l > only_level):
            break
        if only_level is not None and l < only_level:
            continue
        shp, cshp = (n,) * d, (nc,) * d
        f = torch.randn(shp, generator=gen, device="cuda", dtype=torch.float64).to(dt)
        u = torch.randn(shp, generator=gen, device="cuda", dtype=torch.float64).to(dt)
        t = torch.empty_like(u)
        fc = torch.empty(cshp, device="cuda", dtype=dt)
        v = torch.randn(cshp, generator=gen, device="cuda", dtype=torch.float64).to(dt)
        P, Pc = n ** d, nc ** d
        rb = w.get("smoother", 0)
        if d == 2 and (rb == 2 or w.get("restrict", 1) == 3):
            # 2D separate kernels (red-black Gauss-Seidel, or the cubic-adjoint restriction):
            # a smoothing launch (a Gauss-Seidel partial step or an omega-Jacobi sweep), the
            # defect + restriction and the interpolation + correction
            if rb == 2:
                sk = ("k_gs2d", "Gauss-Seidel partial step",
                      lambda: mg.mg_kernel_smooth_colour(run.h, l, fp32, 1, f.data_ptr(), u.data_ptr(),
                                                         t.data_ptr()))
            else:
                sk = ("k_pre2d", "omega-Jacobi sweep",
                      lambda: mg.mg_kernel_smooth(run.h, l, fp32, f.data_ptr(), u.data_ptr(), t.data_ptr()))
            cubic = w.get("restrict", 1) == 3
            ks = [
                (sk[0], sk[1], 3 * P * b, sk[2]),
                ("k_restrict_cubic" if cubic else "k_pre2d",
                 "defect, then cubic-adjoint restriction" if cubic else "defect+FW",
                 ((2 * P + P) + (P + Pc)) * b if cubic else (2 * P + Pc) * b,
                 lambda: mg.mg_kernel_residual_restrict(run.h, l, fp32, f.data_ptr(), u.data_ptr(),
                                                        fc.data_ptr())),
                ("k_post2d", "interp+correct", (2 * P + Pc) * b,
                 lambda: mg.mg_kernel_prolong_correct(run.h, l, fp32, v.data_ptr(), u.data_ptr(),
                                                      t.data_ptr())),
            ]
        elif rb and d == 3:
            # 3D red-black smoothing: two partial-step launches per sweep
            sep = l > 0 and w["coarse"] in (1, 3)
            ks = [
                ("k_gpen3d" if sep else "k_xsweep3d", "red-black partial step", 3 * P * b,
                 lambda: mg.mg_kernel_smooth_colour(run.h, l, fp32, 1, f.data_ptr(), u.data_ptr(),
                                                    t.data_ptr())),
                ("k_grr3d" if sep else "k_xrr3d", "defect+FW", (2 * P + Pc) * b,
                 lambda: mg.mg_kernel_residual_restrict(run.h, l, fp32, f.data_ptr(), u.data_ptr(),
                                                        fc.data_ptr())),
                ("k_prolong%dd" % d, "interp+correct", (2 * P + Pc) * b,
                 lambda: mg.mg_kernel_prolong_correct(run.h, l, fp32, v.data_ptr(), u.data_ptr(),
                                                      t.data_ptr())),
            ]
        elif d == 2:
            # red-black: the passes hold one red-black sweep each (the cycle runs max(1, nu))
            pre = "red-black sweep" if rb else "presmooth(%d)" % w["nu1"]
            post = "red-black sweep" if rb else "postsmooth(%d)" % w["nu2"]
            ks = [
                ("k_pre2d", "%s+defect+FW" % pre, (3 * P + Pc) * b,
                 lambda: mg.mg_kernel_presmooth_restrict(run.h, l, fp32, f.data_ptr(), u.data_ptr(),
                                                         t.data_ptr(), fc.data_ptr())),
                ("k_post2d", "interp+correct+%s" % post, (3 * P + Pc) * b,
                 lambda: mg.mg_kernel_prolong_postsmooth(run.h, l, fp32, v.data_ptr(), u.data_ptr(),
                                                         f.data_ptr(), t.data_ptr())),
            ]
        else:
            # level 0 and rediscretized levels: the cross kernels; Galerkin levels: the
            # pencil sweep and the separable defect kernel
            sep = l > 0 and w["coarse"] in (1, 3)
            ks = [
                ("k_gpen3d" if sep else "k_xsweep3d", "omega-Jacobi sweep", 3 * P * b,
                 lambda: mg.mg_kernel_smooth(run.h, l, fp32, f.data_ptr(), u.data_ptr(), t.data_ptr())),
                ("k_grr3d" if sep else "k_xrr3d", "defect+FW", (2 * P + Pc) * b,
                 lambda: mg.mg_kernel_residual_restrict(run.h, l, fp32, f.data_ptr(), u.data_ptr(),
                                                        fc.data_ptr())),
                ("k_prolong3d", "interp+correct", (2 * P + Pc) * b,
                 lambda: mg.mg_kernel_prolong_correct(run.h, l, fp32, v.data_ptr(), u.data_ptr(),
                                                      t.data_ptr())),
            ]
            if sep:
                # what the cycle runs there: the pencil kernel's defect, then full weighting
                def two_pass():
                    mg.mg_kernel_residual(run.h, l, fp32, f.data_ptr(), u.data_ptr(), t.data_ptr())
                    mg.mg_kernel_residual_restrict(run.h, l, fp32, t.data_ptr(), 0, fc.data_ptr())
                ks.insert(2, ("k_gpen3d+k_xrr3d", "defect, then FW (the cycle's pass)",
                              (3 * P + P + Pc) * b, two_pass))
        for name, what, nbytes, fn in ks:
            s = event_time(stream, fn, reps)
            rows.append({"level": l, "n": n, "kernel": name, "op": what, "us": s * 1e6,
                         "bytes": nbytes, "GB/s": nbytes / s / 1e9})
        del f, u, t, fc, v
    return rows


def cpu_baseline(w, gpu_cycles, sample_n=None):
    """The oracle (plain C, FP64; OpenMP splits the outermost loop of 3D grids, 2D loops run
    on one thread) timed on the host on a bounded sample of the same configuration.
    3D: whole solves to 1e-10 of the same problem at side sample_n on all host cores, and
    a cycle on one thread scaled to that solve's cycle count.  2D: a cycle of the
    full-size problem on one thread, scaled to the cycles the GPU solve needed.  Each time
    is the median of three runs.
    Returns (baseline dict, oracle solution or None, oracle cycles, oracle final residual)."""
    import numpy as np

    import oracle
    d = w["dim"]
    n = sample_n or w["n"]
    f, _ = make_rhs(dict(w, n=n))
    all_cores = oracle.num_threads()

    def make():
        return oracle.Multigrid(d, n, coarse=w["coarse"], gamma=w["gamma"], nu1=w["nu1"], nu2=w["nu2"],
                                smoother=w.get("smoother", 0), order=w.get("order", 4),
                                omega=w.get("omega") or None)
    unknowns = (n - 2) ** d
    cyc = "%s(%d,%d)" % ("W" if w["gamma"] == 2 else "V", w["nu1"], w["nu2"])
    grid = "x".join([str(n)] * d)
    u_all, cycles, final = None, gpu_cycles, None
    out = {"unit": "unknowns/s", "kind": "oracle"}
    reps = 3  # timings: the median of three
    if d == 3:
        times = []
        for _ in range(reps):
            m = make()
            u_all = np.zeros_like(f)
            t0 = time.perf_counter()
            cycles, hist = m.solve(u_all, f, rtol=1e-10, max_cycles=60)
            times.append(time.perf_counter() - t0)
            m.close()
        t_all = float(np.median(times))
        final = float(hist[-1])
        out.update(value=unknowns / t_all, cores=all_cores,
                   sample="whole FP64 %s solves of the same problem at %s to %.1e on %d threads "
                          "(%d cycles), median of %d: %.2f s" % (cyc, grid, final, all_cores, cycles, reps, t_all))
    oracle.set_num_threads(1)
    try:
        times = []
        for _ in range(reps):
            m = make()
            u1 = np.zeros_like(f)
            t0 = time.perf_counter()
            m.cycle(u1, f)
            times.append(time.perf_counter() - t0)
            m.close()
        t1 = float(np.median(times))
    finally:
        oracle.set_num_threads(all_cores)
    one = {"value": unknowns / (t1 * cycles), "cores": 1,
           "sample": "FP64 %s cycles at %s on one thread, median of %d: %.2f s, scaled to the %d cycles of %s"
                     % (cyc, grid, reps, t1, cycles, "that solve" if d == 3 else "the GPU FP64 solve")}
    if d == 3:
        out["single_thread"] = one
    else:
        out.update(one)
    return out, u_all, cycles, final


def error_vs_129(u_inj, coeffs, u129, cycles, final):
    """The 1025^3 GPU solution injected onto the 129^3 grid against the oracle's 129^3 solve
    of the same continuous right-hand side, and both against the continuous solution."""
    import numpy as np

    from paper_2008_03885_amd import inputs
    nco = u129.shape[0]
    k2 = inputs.wavenumber_sq(coeffs.shape[0], 3)
    exact = inputs.sine_series(nco, coeffs / (np.pi ** 2 * k2))
    nrm = np.linalg.norm(u129)
    return {
        "oracle_129_cycles": int(cycles), "oracle_129_rel_residual": final,
        "rel_diff_gpu1025_vs_oracle129": float(np.linalg.norm(u_inj - u129) / nrm),
        "rel_err_oracle129_vs_continuous": float(np.linalg.norm(u129 - exact) / nrm),
        "rel_err_gpu1025_vs_continuous": float(np.linalg.norm(u_inj - exact) / nrm),
    }


def pmc_probe(w, run, stream, level=0):
    """A plain copy of known size, then the kernels of one level (level 0: the dominant
    kernel), five launches each, for hardware counters."""
    import torch
    a = torch.ones(256 * 1024 * 1024, device="cuda", dtype=torch.float64)  # 2 GiB
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    rows = level_kernels(run, w, stream, 5, only_level=level)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": a.numel() * 8,
                      "kernels": rows}), flush=True)



def rbc_pmc_probe(fd, stream, n):
    """A plain copy of known size, then five level-0 red-black coarsening partial steps
    (k_rbc_smooth), for hardware counters."""
    import torch
    from paper_2008_03885_amd import rbc
    a = torch.ones(256 * 1024 * 1024, device="cuda", dtype=torch.float64)  # 2 GiB
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    h = rbc.setup(rbc.make_config(n=n, levels=20), stream.cuda_stream)
    u = torch.rand_like(fd)
    out = torch.empty_like(fd)
    for _ in range(5):
        rbc.kernel_smooth(h, 0, 1, fd.data_ptr(), u.data_ptr(), out.data_ptr())
    torch.cuda.synchronize()
    rbc.destroy(h)
    print(json.dumps({"copy_bytes_read": 2 << 30, "copy_bytes_written": 2 << 30,
                      "kernel": "k_rbc_smooth", "launches": 5, "algorithmic_bytes": 20 * n * n}), flush=True)


SERVE_BUDGET = 32 << 30
# Serving: solve steps per replay chunk (one chunk in flight per batch).  Measured at half
# load: p50 / p99 7.5 / 11.3 ms with one step, 8.0 / 12.3 ms with two.
SERVE_CHUNK_STEPS = 1


def serve_bench(count, loads=(0.5, 0.8, 0.95), smoother=0, inner=4, stream_groups=3):
    """Continuous-batching server on a Poisson stream of 2D solves, n = 2^k + 1 with k
    uniform on 6..11, Fourier right-hand sides (k <= min(64, (n-1)/4)), mixed precision
    V(2,1) to 1e-10.  First all requests at once (saturated throughput), then open-loop
    Poisson arrivals at fractions of that rate; latency = completion - scheduled arrival."""
    import numpy as np
    import torch

    from paper_2008_03885_amd import inputs, mg, serve
    base = dict(dim=2, coarse=0, gamma=1, nu1=2, nu2=1, precision=mg.MG_PREC_MIXED, rtol=1e-10,
                max_cycles=30, inner_cycles=inner, smoother=smoother)
    stream = inputs.request_stream(count, 1.0)
    fs = {}
    reqs = []
    for i, (t, n, seed) in enumerate(stream):
        f = torch.from_numpy(inputs.fourier_rhs(n, 2, min(64, (n - 1) // 4), seed=seed)).cuda()
        reqs.append((i, n, f, torch.empty_like(f), t))
        fs.setdefault(n, f)
    torch.cuda.synchronize()
    unknowns = sum((n - 2) ** 2 for _, n, _, _, _ in reqs)
    S = serve.Server(SERVE_BUDGET, 16, SERVE_CHUNK_STEPS, stream_groups, n=65, **base)
    try:
        # warm-up: one request per size creates every batch and captures its graph
        warm = [(10 ** 6 + n, f, torch.empty_like(f)) for n, f in sorted(fs.items())]
        for tag, f, u in warm:
            S.submit(tag, f, u)
        S.wait_all(len(warm), 120.0)

        def run(arrivals):
            t0 = time.monotonic()
            got, i = [], 0
            while len(got) < len(reqs):
                now = time.monotonic() - t0
                while i < len(reqs) and arrivals[i] <= now:
                    tag, n, f, u, _ = reqs[i]
                    if S.submit(tag, f, u) != mg.MG_OK:
                        raise RuntimeError("submit failed")
                    i += 1
                wait = (arrivals[i] - now) if i < len(reqs) else 0.01
                got += S.poll(256, max(0.0, min(wait, 0.002)))
            end = max(c.t_done for c in got)
            lat = np.array([c.t_done - (t0 + arrivals[c.tag]) for c in got])
            sizes = np.array([c.n for c in got])
            bad = [c.tag for c in got if c.status != mg.MG_OK or c.result.rel_residual > 1e-10]
            return end - t0, lat, bad, sizes

        def per_size(lat, sizes):
            return {str(int(n)): {"count": int((sizes == n).sum()),
                                  "p50_ms": float(np.percentile(lat[sizes == n], 50) * 1e3),
                                  "p99_ms": float(np.percentile(lat[sizes == n], 99) * 1e3)}
                    for n in sorted(set(sizes.tolist()))}

        # one request at a time: the latency of each size on an idle device
        alone = {}
        for n, f in sorted(fs.items()):
            u = torch.empty_like(f)
            t1 = time.monotonic()
            S.submit(2 * 10 ** 6 + n, f, u)
            c = S.wait_all(1, 60.0)[0]
            alone[str(n)] = {"ms": (time.monotonic() - t1) * 1e3,
                             "solve_ms": (c.t_done - c.t_admit) * 1e3, "cycles": c.result.cycles}

        span, lat_sat, bad, _ = run([0.0] * len(reqs))
        rate_sat = len(reqs) / span
        out = {
            "requests": len(reqs), "sizes": "2^k+1, k~U{6..11}", "precision": "mixed",
            "chunk_steps": SERVE_CHUNK_STEPS,
            "stream_groups": stream_groups,
            "saturated": {"requests_per_s": rate_sat, "unknowns_per_s": unknowns / span,
                          "makespan_s": span, "p50_ms": float(np.percentile(lat_sat, 50) * 1e3),
                          "p99_ms": float(np.percentile(lat_sat, 99) * 1e3)},
            "not_converged": bad,
            "alone": alone,
        }
        gaps = np.array([t for *_, t in reqs])
        for load in loads:
            arrivals = list(gaps / (load * rate_sat))
            span, lat, bad2, sizes = run(arrivals)
            out["load_%.2f" % load] = {
                "offered_requests_per_s": load * rate_sat, "requests_per_s": len(reqs) / span,
                "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "per_size": per_size(lat, sizes)}
            out["not_converged"] += bad2
        st = S.stats()
        out["peak_active"] = st["peak_active"]
        out["batches"] = st["batches_created"]
        out["peak_hbm_bytes"] = st["peak_bytes_held"]
        out["hbm_budget"] = SERVE_BUDGET
        return out
    finally:
        S.close()


RBC_VARIANTS = (  # coarse, nu1, nu2, omega: section 4.4's G1 and Gn and the rediscretized operator
    ("G1", 1, 1, 1.0), ("G1", 2, 1, 1.0), ("G1", 2, 1, 1.2), ("GN", 1, 1, 1.0), ("NG", 1, 1, 1.0))


def rbc_bench(fd, stream, n, reps, cpu=True):
    """Red-black coarsening (section 4.3, 4.4) on the second-order five-point problem with
    the same right-hand side: V-cycles down to the first level of at most
    MG_RBC_MAX_COARSEST unknowns (17 levels at n = 4097, the last a 17x17 grid with 225
    unknowns), solved from zero to 1e-10.  Also the level-0 partial step's
    HBM rate (20 algorithmic bytes a point: u read and written, f read at half the points)
    and the CPU oracle on a bounded sample."""
    import numpy as np
    import torch
    from paper_2008_03885_amd import rbc
    def unknowns_of(l):  # of level l: interior points, only the even-index-sum ones if rotated
        side = (n - 1) // 2 ** (l // 2) + 1
        inner = (side - 2) ** 2
        return inner if l % 2 == 0 else (inner + 1) // 2
    levels = 2  # the fewest levels whose last one the coarsest solve takes
    while unknowns_of(levels - 1) > rbc.MG_RBC_MAX_COARSEST:
        levels += 1
    unknowns = (n - 2) ** 2
    out = {"levels": levels, "problem": "second-order five-point operator, same right-hand side",
           "variants": {}}
    s = stream.cuda_stream
    ud = torch.zeros_like(fd)
    for coarse, nu1, nu2, om in RBC_VARIANTS:
        cfg = rbc.make_config(n=n, levels=levels, coarse=getattr(rbc, "MG_RBC_" + coarse), gamma=1,
                              nu1=nu1, nu2=nu2, omega=om, rtol=1e-10, max_cycles=60)
        h = rbc.setup(cfg, s)
        times, cyc, hist = [], 0, []
        for k in range(reps + 1):
            ud.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, cyc, hist = rbc.solve(h, fd.data_ptr(), ud.data_ptr(), 60)
            torch.cuda.synchronize()
            if k:
                times.append(time.perf_counter() - t0)
        sec = min(times)
        name = "%s-V(%d,%d)-omega%g" % (coarse, nu1, nu2, om)
        out["variants"][name] = {"ms": 1e3 * sec, "unknowns_per_s": unknowns / sec, "cycles": cyc,
                                 "rel_residual": hist[-1] / hist[0], "status": st}
        if (coarse, nu1, nu2, om) == RBC_VARIANTS[0]:
            # cycles alone, HIP events on the handle's stream (the solve adds one norm a cycle)
            t = event_time(stream, lambda: rbc.cycles(h, fd.data_ptr(), ud.data_ptr(), 1), 10)
            out["cycle_ms"] = 1e3 * t
            tmp = torch.empty_like(fd)
            ps = event_time(stream, lambda: rbc.kernel_smooth(h, 0, 1, fd.data_ptr(), ud.data_ptr(),
                                                              tmp.data_ptr()), 50)
            byts = 20.0 * n * n
            tr = MEASURED_TRAFFIC.get("k_rbc_smooth/f64/rbc.hip/%d" % n)
            traffic = tr["bytes"] if tr and tr["source"] == source_hash("rbc.hip") else None
            out["roofline"] = {"bound": "hbm", "kernel": "k_rbc_smooth level 0 (one partial step, FP64)",
                               "achieved": byts / ps / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": byts / ps / 1e9 / HBM_PEAK_GBS, "traffic": traffic,
                               "avg_launch_us": ps * 1e6, "algorithmic_bytes_per_launch": byts}
            del tmp
        rbc.destroy(h)
    if cpu:
        from oracle import rbc as orbc
        nc = 1025
        lv = 1
        while (nc - 1) // 2 ** (lv // 2) + 1 >= 9:
            lv += 1
        o = orbc.RBC(nc, lv, coarse=orbc.G1, nu1=1, nu2=1, omega=1.0)
        fs = np.zeros((nc, nc))
        fs[1:-1, 1:-1] = np.random.default_rng(1).standard_normal((nc - 2, nc - 2))
        u = np.zeros((nc, nc))
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < 10.0 or k < 1:
            u = o.cycle(fs, u)
            k += 1
        per_cycle = (time.perf_counter() - t0) / k
        cyc = out["variants"]["G1-V(1,1)-omega1"]["cycles"]
        out["cpu_baseline"] = {"value": (nc - 2) ** 2 / (per_cycle * cyc), "unit": "unknowns/s",
                               "cores": 1, "kind": "oracle",
                               "sample": "%d G1 V(1,1) cycles of the numpy oracle at 1025^2 (%d levels), "
                                         "scaled to the %d cycles of the GPU solve" % (k, lv, cyc)}
    return out


def time_workload(w, args, stream, fd, label, variants_2d=False):
    """Solves of workload w from zero (its precision, and the other one when w["compare"]),
    the roofline of its dominant level-0 kernel, per-level kernel rates and, in 2D, the
    other coarse-operator / cycle / smoother / order combinations.  Returns (dict, main
    Run still open, its last result)."""
    import torch
    d, n = w["dim"], w["n"]
    unknowns = (n - 2) ** d
    main_run = Run(w, w["precision"], fd, stream)
    steps = args.steps if label == "primary" else max(2, args.steps // 3)
    sec, (status, res) = main_run.timed(steps, args.warmup if label == "primary" else 1)
    out = {"workload": describe(w), "ms_per_solve": 1e3 * sec, "unknowns_per_s": unknowns / sec,
           "steps": steps, "cycles": res.cycles, "outer_steps": res.outer_steps,
           "final_rel_residual": res.rel_residual, "reached_rtol": bool(res.rel_residual <= 1e-10),
           "floor_hit": bool(res.floor_hit), "status": status}
    if w["compare"]:
        other = Run(w, 1 - w["precision"], fd, stream)
        osec, (ostatus, ores) = other.timed(max(1, steps // 2), 1)
        u64, umx = (main_run.ud, other.ud) if w["precision"] == 0 else (other.ud, main_run.ud)
        rel = float(torch.linalg.vector_norm(umx - u64) / torch.linalg.vector_norm(u64))
        r64, rmx = (res, ores) if w["precision"] == 0 else (ores, res)
        s64, smx = (sec, osec) if w["precision"] == 0 else (osec, sec)
        out["precision_compare"] = {
            "fp64": {"ms": s64 * 1e3, "unknowns_per_s": unknowns / s64, "cycles": r64.cycles,
                     "rel_residual": r64.rel_residual, "reached_rtol": bool(r64.rel_residual <= 1e-10),
                     "floor_hit": bool(r64.floor_hit)},
            "mixed": {"ms": smx * 1e3, "unknowns_per_s": unknowns / smx, "outer_steps": rmx.outer_steps,
                      "fp32_cycles": rmx.cycles, "inner_cycles": w["inner"],
                      "rel_residual": rmx.rel_residual, "reached_rtol": bool(rmx.rel_residual <= 1e-10),
                      "floor_hit": bool(rmx.floor_hit)},
            "mixed_speedup": s64 / smx,
            "rel_diff_mixed_vs_fp64": rel,
        }
        other.close()
        del other
    if variants_2d:
        out["config_variants"] = config_variants_2d(w, fd, stream, sec, res)
    rows = [] if args.no_levels else level_kernels(main_run, w, stream, args.kernel_reps)
    rb = bool(w.get("smoother", 0))
    dom_name = ("k_gs2d" if w.get("smoother", 0) == 2 else "k_pre2d") if d == 2 else "k_xsweep3d"
    dom = [r for r in rows if r["level"] == 0 and r["kernel"] == dom_name]
    if not dom:
        dom = [r for r in level_kernels(main_run, w, stream, args.kernel_reps, only_level=0)
               if r["kernel"] == dom_name]
    dom = dom[0]  # with separate 2D kernels the first listed (smoothing) launch
    cyc_s = in_cycle_time(main_run, w, stream, args.kernel_reps)
    src = "fused2d.hip" if d == 2 else "kernels3d.hip"
    key = "%s/%s/%s/%d%s%s" % (dom_name, "f32" if w["precision"] else "f64", src, n, "/rb" if rb else "",
                               "/o%d" % w.get("order", 4) if w.get("order", 4) != 4 else "")
    tr = MEASURED_TRAFFIC.get(key)
    copy_gbs = copy_rate(stream)
    out["roofline"] = {
        "bound": "hbm",
        "kernel": "%s level 0 (%s, %s)" % (dom_name, dom["op"], "FP32" if w["precision"] else "FP64"),
        "achieved": dom["GB/s"],
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": dom["GB/s"] / HBM_PEAK_GBS,
        "traffic": tr["bytes"] if tr and tr["source"] == source_hash(src) else None,
        "avg_launch_us": dom["us"],
        "timing": "HIP events around back-to-back launches on the handle's stream",
        "algorithmic_bytes_per_launch": dom["bytes"],
        "in_cycle_us": cyc_s * 1e6,
        "in_cycle_GBs": dom["bytes"] / cyc_s / 1e9,
        "copy_GBs": copy_gbs,
        "frac_of_copy": dom["GB/s"] / copy_gbs,
    }
    if rows:
        out["levels"] = [{k: (round(v, 2) if isinstance(v, float) else v) for k, v in r.items()}
                         for r in rows]
    return out, main_run, res


VARIANTS_2D = (  # coarse, gamma, smoother, order, omega
    (0, 1, 0, 4, 0.0), (1, 1, 0, 4, 0.0), (0, 2, 0, 4, 0.0), (1, 2, 0, 4, 0.0),
    (2, 1, 0, 4, 0.0), (3, 1, 0, 4, 0.0),
    (0, 1, 1, 4, 0.0), (1, 1, 1, 4, 0.0), (3, 1, 1, 4, 0.0), (0, 2, 1, 4, 0.0),
    (0, 1, 1, 4, 1.17),  # the measured multilevel optimum, above the two-grid one
    (0, 1, 0, 6, 0.0), (3, 1, 0, 6, 0.0), (3, 1, 1, 6, 0.0))


def config_variants_2d(w, fd, stream, sec, res):
    """The other coarse-operator / cycle / smoother / order combinations of the 2D problem."""
    unknowns = (w["n"] - 2) ** 2
    kinds = {0: "rediscretized", 1: "galerkin", 2: "rediscretized-order2", 3: "galerkin-order2"}
    variants = {}
    for coarse, gamma, sm, order, om in VARIANTS_2D:
        name = "%s-%s(%d,%d)" % (kinds[coarse], "W" if gamma == 2 else "V", w["nu1"], w["nu2"])
        if sm:
            name = "redblack-" + name
        if order != 4:
            name = "order%d-%s" % (order, name)
        if om:
            name += "-omega%g" % om
        if (coarse == w["coarse"] and gamma == w["gamma"] and sm == w.get("smoother", 0)
                and order == w.get("order", 4) and not om and not w.get("omega")):
            vs, vres = sec, res
        else:
            vr = Run(dict(w, coarse=coarse, gamma=gamma, smoother=sm, order=order, omega=om),
                     w["precision"], fd, stream)
            vs, (vst, vres) = vr.timed(2, 1)
            vr.close()
        variants[name] = {"ms": 1e3 * vs, "unknowns_per_s": unknowns / vs, "cycles": vres.cycles,
                          "rel_residual": vres.rel_residual}
    return variants


def setup_workload(args, name):
    w = dict(WORKLOADS[name])
    if name == args.workload:
        for k in ("n", "coarse", "gamma", "precision", "compare", "inner", "smoother", "order", "omega",
                  "restrict"):
            if getattr(args, k) is not None:
                w[k] = getattr(args, k)
    return w


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    w = setup_workload(args, args.workload)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.serve_only:
        print(json.dumps({"serving": serve_bench(max(args.serve_requests, 1), smoother=w.get("smoother", 0),
                                                 inner=args.inner or 4, stream_groups=args.stream_groups)}),
              flush=True)
        return
    served = {}
    if (not args.no_extras and args.workload == DEFAULT_WORKLOAD and args.serve_requests > 0
            and not (args.rbc_only or args.pmc_probe)):
        # the serving runs first, on a quiet host: the CPU baselines below leave thread
        # pools (OpenMP, BLAS) behind that compete with the server's host thread
        print("bench: serving", file=sys.stderr, flush=True)
        served["serving"] = serve_bench(args.serve_requests, stream_groups=args.stream_groups)
        # the same stream with red-black Jacobi smoothing (2 FP32 cycles per refinement step)
        served["serving_redblack"] = serve_bench(args.serve_requests, smoother=1, inner=2,
                                                 stream_groups=args.stream_groups)
        torch.cuda.empty_cache()
    f, coeffs = make_rhs(w)
    fd = torch.from_numpy(f).cuda()
    del f
    if args.rbc_only and args.pmc_probe:
        rbc_pmc_probe(fd, stream, w["n"])
        return
    if args.rbc_only:
        print(json.dumps({"red_black_coarsening": rbc_bench(fd, stream, w["n"], args.steps,
                                                            cpu=not args.no_cpu)}), flush=True)
        return
    if args.pmc_probe:
        run = Run(w, w["precision"], fd, stream)
        pmc_probe(w, run, stream, args.pmc_level)
        run.close()
        return
    d, n = w["dim"], w["n"]
    unknowns = (n - 2) ** d
    print("bench: %s" % describe(w), file=sys.stderr, flush=True)
    prim, main_run, res = time_workload(w, args, stream, fd, "primary",
                                        variants_2d=(d == 2 and not args.no_variants))
    inj = None
    if w.get("check129"):
        stride = (n - 1) // 128
        inj = main_run.ud[::stride, ::stride, ::stride].cpu().numpy()
    main_run.close()
    del main_run, fd
    torch.cuda.empty_cache()

    cyc = "%s(%d,%d)" % ("W" if w["gamma"] == 2 else "V", w["nu1"], w["nu2"])
    cfg = {
        "workload": prim["workload"], "name": args.workload, "dim": d, "n": n, "unknowns": unknowns,
        "cycle": cyc, "coarse": ["rediscretized", "galerkin", "rediscretized-order2",
                                 "galerkin-order2"][w["coarse"]],
        "precision": "fp64" if w["precision"] == 0 else "mixed",
        "inner_cycles": w["inner"] if w["precision"] else None,
        "smoother": {0: "jacobi", 1: "red-black-jacobi", 2: "red-black-gauss-seidel"}[w.get("smoother", 0)],
        "order": w.get("order", 4),
        "cycles": prim["cycles"], "outer_steps": prim["outer_steps"],
        "final_rel_residual": prim["final_rel_residual"], "reached_rtol": prim["reached_rtol"],
        "floor_hit": prim["floor_hit"], "status": prim["status"],
    }
    out = {
        "metric": "unknowns/s to 1e-10 rel. residual (mixed vs FP64) + smoother HBM GB/s; p99 lat",
        "value": prim["unknowns_per_s"],
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": prim["steps"],
        "warmup": args.warmup,
        "ms_per_step": prim["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if w["precision"] == 0 else "f32-in-f64",
        "data": "synthetic",
        "config": cfg,
        "roofline": prim["roofline"],
    }
    for k in ("precision_compare", "config_variants", "levels"):
        if k in prim:
            out[k] = prim[k]
    fp64_cycles = (prim["precision_compare"]["fp64"]["cycles"] if "precision_compare" in prim
                   else prim["cycles"])
    if not args.no_cpu:
        sample = 129 if (d == 3 and n > 129) else None
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        base, u129, ocyc, ofinal = cpu_baseline(w, max(fp64_cycles, 1), sample)
        out["cpu_baseline"] = base
        if inj is not None and u129 is not None:
            out["error_vs_oracle_129"] = error_vs_129(inj, coeffs, u129, ocyc, ofinal)

    if not args.no_extras and args.workload == DEFAULT_WORKLOAD:
        # the 3D 513^3 configuration: mixed (eight FP32 cycles per step) against FP64
        print("bench: extra poisson3d-513", file=sys.stderr, flush=True)
        w3 = setup_workload(args, "poisson3d-513")
        f3, _ = make_rhs(w3)
        fd3 = torch.from_numpy(f3).cuda()
        del f3
        e3, r3, _ = time_workload(w3, args, stream, fd3, "extra")
        r3.close()
        e3.pop("levels", None)
        out["poisson3d_513"] = e3
        del fd3, r3
        torch.cuda.empty_cache()
        # the 2D 4097^2 configuration (FP64) and its variants
        print("bench: extra poisson2d-4097", file=sys.stderr, flush=True)
        w2 = setup_workload(args, "poisson2d-4097")
        f2, _ = make_rhs(w2)
        fd2 = torch.from_numpy(f2).cuda()
        del f2
        e2, r2, _ = time_workload(w2, args, stream, fd2, "extra", variants_2d=not args.no_variants)
        r2.close()
        out["poisson2d_4097"] = e2
        if not args.no_variants:
            print("bench: red-black coarsening", file=sys.stderr, flush=True)
            out["red_black_coarsening"] = rbc_bench(fd2, stream, w2["n"], 3, cpu=not args.no_cpu)
        del fd2, r2
        torch.cuda.empty_cache()
        out.update(served)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
