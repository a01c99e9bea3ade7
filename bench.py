"""Benchmark: 2D fourth-order Poisson multigrid solve on one MI355X.

Workload (one step = one whole solve from a zero initial guess to a 1e-10 relative
residual, or the FP64 rounding floor): n = 4097 points per side (16,769,025 unknowns),
right-hand side sum_{kx,ky<=64} g_k/|k| sin(kx pi x) sin(ky pi y), g_k ~ N(0,1) (seeded),
fourth-order width-5 operator, homogeneous Dirichlet boundary, V(2,1) cycles with
omega-Jacobi (omega = 10/13), full weighting, cubic interpolation, rediscretized coarse
operators down to 9x9 with an exact coarsest solve, all in FP64.

Prints one JSON line: throughput in unknowns/s, the roofline of the level-0 Jacobi sweep
(HIP-event timed here), and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--n", type=int, default=4097)
    p.add_argument("--coarse", type=int, default=0)
    p.add_argument("--gamma", type=int, default=1)
    p.add_argument("--precision", type=int, default=0)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--kernel-reps", type=int, default=50)
    return p.parse_args()


def cpu_baseline(n, cycles_needed, budget_s=20.0):
    """The oracle (plain C, FP64, OpenMP over rows) on a bounded sample: whole cycles of
    the same problem, timed, scaled to the cycles the GPU solve needed."""
    import numpy as np

    import oracle
    from paper_2008_03885_amd import inputs

    f = inputs.fourier_rhs(n, 2, 64, seed=inputs.SEED_BASE + 2)
    m = oracle.Multigrid(2, n)
    u = np.zeros_like(f)
    t0 = time.perf_counter()
    m.cycle(u, f)
    t_cycle = time.perf_counter() - t0
    done = 1
    while done * t_cycle < budget_s and done < 4:
        t0 = time.perf_counter()
        m.cycle(u, f)
        t_cycle = min(t_cycle, time.perf_counter() - t0)
        done += 1
    unknowns = (n - 2) ** 2
    return {
        "value": unknowns / (t_cycle * cycles_needed),
        "unit": "unknowns/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": "%d V(2,1) cycles of the %dx%d problem (best cycle %.2f s), scaled to the %d "
                  "cycles the solve needs" % (done, n, n, t_cycle, cycles_needed),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2008_03885_amd import inputs, mg

    torch.cuda.set_device(0)
    n = args.n
    f = inputs.fourier_rhs(n, 2, 64, seed=inputs.SEED_BASE + 2)
    fd = torch.from_numpy(f).cuda()
    ud = torch.zeros_like(fd)
    stream = torch.cuda.current_stream()
    cfg = mg.make_config(dim=2, n=n, coarse=args.coarse, gamma=args.gamma, nu1=2, nu2=1,
                         precision=args.precision, rtol=1e-10, max_cycles=60, inner_cycles=4)
    h = mg.mg_setup(cfg, stream.cuda_stream)

    def step():
        ud.zero_()
        return mg.mg_solve(h, fd.data_ptr(), ud.data_ptr())

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    status, res = results[-1]
    ms = 1e3 * elapsed / args.steps
    unknowns = (n - 2) ** 2

    # Dominant kernel: the level-0 omega-Jacobi sweep, same launch as inside the cycle.
    tmp = torch.empty_like(fd)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(5):
        mg.mg_kernel_smooth(h, 0, 0, fd.data_ptr(), ud.data_ptr(), tmp.data_ptr())
    ev0.record(stream)
    for _ in range(args.kernel_reps):
        mg.mg_kernel_smooth(h, 0, 0, fd.data_ptr(), ud.data_ptr(), tmp.data_ptr())
    ev1.record(stream)
    ev1.synchronize()
    sweep_s = ev0.elapsed_time(ev1) / 1e3 / args.kernel_reps
    sweep_bytes = 3 * n * n * 8  # read u, f; write u' (FP64)
    achieved = sweep_bytes / sweep_s / 1e9

    out = {
        "metric": "unknowns/s to 1e-10 rel. residual (mixed vs FP64) + smoother HBM GB/s; p99 lat",
        "value": unknowns / (ms / 1e3),
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 0 else "f32-in-f64",
        "data": "synthetic",
        "config": {
            "workload": "2D 4th-order Poisson %dx%d, Fourier RHS k<=64, V(2,1) omega-Jacobi, FW + cubic, "
                        "%s coarse ops to 9x9, FP64, to 1e-10" % (n, n, "Galerkin" if args.coarse else "rediscretized"),
            "n": n, "unknowns": unknowns, "cycle": "W(2,1)" if args.gamma == 2 else "V(2,1)",
            "coarse": "galerkin" if args.coarse else "rediscretized",
            "precision": "fp64" if args.precision == 0 else "mixed",
            "cycles": res.cycles, "outer_steps": res.outer_steps,
            "final_rel_residual": res.rel_residual, "floor_hit": bool(res.floor_hit),
            "status": status,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_sweep2d (level-0 omega-Jacobi, FP64)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "avg_launch_us": sweep_s * 1e6,
            "algorithmic_bytes_per_launch": sweep_bytes,
        },
    }
    mg.mg_destroy(h)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(n, max(res.cycles, 1))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
