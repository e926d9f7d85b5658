#!/usr/bin/env python3
"""Benchmark of the RIDC hot path on one MI355X.

Workload: 1D reaction-diffusion u_t = nu u_xx + u(1-u), Dirichlet 0 on [0,1], N = 8192 interior
points, nu = 1e-3, eight seeded Gaussian bumps, RIDC order 4 (predictor + 3 correctors), T = 1,
Nt = 2000 uniform steps, FP64.  One bench step is one whole integration (all Nt time steps of
all four levels, i.e. Nt + 6 pipeline steps) with the data already resident in HBM.

Prints one JSON line: grid-point-steps/s (unknowns x Nt / wall time), the roofline of the
dominant kernel (the fused 1D level-step) from per-launch HIP events, and the FP64 CPU oracle
timed on the host on the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E datasheet peak


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--profile-launches", type=int, default=400,
                    help="steady-state launches timed one by one for the roofline")
    return ap.parse_args()


def kernel_roofline(torch, ridc, solver, x0, nt, launches):
    """Average duration of the fused level-step kernel, from HIP events around single launches.

    The launches are queued behind a sleep so that the host never starves the GPU; each one is
    a steady-state pipeline step (all four levels active) on the solver's stream.
    """
    P = solver.order
    first = P * (P - 1) // 2 + 1            # first step with every level active
    solver.begin(x0, nt)
    ridc.advance([solver], first - 1)
    launches = min(launches, nt - first)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(launches)]
    torch.cuda.synchronize()
    torch.cuda._sleep(int(2e8))             # let the host queue every launch first
    stream = torch.cuda.current_stream()
    for a, b in evs:
        a.record(stream)
        ridc.advance([solver], 1)
        b.record(stream)
    torch.cuda.synchronize()
    times_ms = np.array([a.elapsed_time(b) for a, b in evs])
    return float(np.mean(times_ms)) * 1e-3, float(np.median(times_ms)) * 1e-3


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: every box here has a single MI355X, and this "
              "build measures the one-GPU hot path (see DESIGN.md for how it would shard).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads
    from paper_1209_4297_amd import ridc

    prob, u0 = workloads.config_reacdiff_1d()
    n, nt, P = prob["n"], prob["nt"], prob["order"]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    solver = ridc.Ridc(prob)
    tile = solver.autotune()                 # result-neutral tiling choice, measured
    x0 = torch.tensor(u0, dtype=torch.float64, device="cuda")
    uT = torch.empty_like(x0)

    for _ in range(args.warmup):
        solver.integrate(x0, nt, uT, sync=False)
    torch.cuda.synchronize()
    solver.sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solver.integrate(x0, nt, uT, sync=False)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    solver.sync()
    gps = n * nt * args.steps / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    result = uT.cpu().numpy()

    # roofline of the dominant kernel
    bytes_per_launch, _ = solver.step_cost()
    mean_s, median_s = kernel_roofline(torch, ridc, solver, x0, nt, args.profile_launches)
    achieved = bytes_per_launch / mean_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                "kernel": "k_step1d", "launch_us_mean": round(mean_s * 1e6, 3),
                "launch_us_median": round(median_s * 1e6, 3),
                "bytes_per_launch": bytes_per_launch}

    cpu = None
    rel = None
    if not args.no_cpu:
        from oracle import Problem, rel_l2, ridc_pipelined
        try:
            from threadpoolctl import threadpool_limits
            limiter = threadpool_limits(limits=1)
        except Exception:  # noqa: BLE001
            limiter = None
        p = Problem.from_dict(prob)
        t1 = time.perf_counter()
        ref = ridc_pipelined(p, u0, nt, P)[-1]
        cpu_s = time.perf_counter() - t1
        if limiter is not None:
            limiter.unregister()
        rel = rel_l2(result, ref)
        cpu = {"value": round(n * nt / cpu_s, 1), "unit": "grid-point-steps/s", "cores": 1,
               "kind": "oracle",
               "sample": f"the full workload once (N={n}, Nt={nt}, order {P}), {cpu_s:.2f} s, "
                         f"one thread; host has {os.cpu_count()} logical CPUs"}

    line = {
        "metric": "RIDC4 grid-point-steps/s at matched L2 error vs FP64",
        "value": round(gps, 1),
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "1D reaction-diffusion u_t = nu u_xx + u(1-u), Dirichlet [0,1], "
                               "N=8192, nu=1e-3, 8 seeded Gaussians, RIDC order 4, T=1, "
                               "Nt=2000, FP64",
                   "n": n, "nt": nt, "order": P, "pipeline_steps": nt + P * (P - 1) // 2,
                   "tile": {"threads": tile[0], "rows": tile[1]},
                   "parallelism": "single GPU"},
        "rel_l2_vs_oracle": rel,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    solver.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
