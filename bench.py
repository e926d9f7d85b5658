#!/usr/bin/env python3
"""Benchmark of the RIDC hot path on one MI355X.

Default workload (``--workload reacdiff2d``): 2D reaction-diffusion u_t = nu Lap u + u(1-u),
Dirichlet 0 on [0,1]^2, 1024 x 1024 interior points, nu = 1e-4, eight seeded radial Gaussian
bumps, RIDC order 4 (predictor + 3 correctors), T = 1, Nt = 500.  One bench step is one whole
integration (all Nt time steps of all four levels, Nt + 6 pipeline steps) with the data already
resident in HBM.  ``value`` is the FP64 rate; the ``matched`` block times the same integration
with split-BF16 (and FP32) transforms plus one FP64 refinement and states its relative L2
distance to the FP64 result against the RIDC4 discretisation error (Richardson with an FP64 run
at 2 Nt): a reduced-precision run is matched when that distance is at most 0.1 of it.

Other workloads: ``reacdiff1d`` (N = 8192 Dirichlet, Nt = 2000), ``advdiff1d`` (N = 128
periodic), ``batched1d`` (256 ragged periodic instances, Nt = 1000, T = 0.25, one grouped launch
per step), ``serving`` (Poisson 2D request stream) and the paper's own 1D cases.

Prints one JSON line: grid-point-steps/s (unknowns x Nt / wall time), the roofline of the
dominant kernel (HIP events around back-to-back launches on the library's stream), and the FP64
CPU oracle timed on the host on a bounded sample of the same workload.
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

HBM_PEAK_GBS = 8000.0                                    # MI355X HBM3E
MFMA_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}   # dense matrix peaks
METRIC = "RIDC4 grid-point-steps/s at matched L2 error vs FP64"

# HBM bytes per launch of the dominant kernels, from two hardware-counter runs of the same
# workload and tiling (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads for a
# plain copy of known size: x2.0 and x1.0).  Reported only while the kernel's source hashes to
# the one that was profiled; otherwise the traffic is unknown and reported as null.
KERNEL_SOURCE = {
    "1d": os.path.join(ROOT, "paper_1209_4297_amd", "csrc", "kernels_1d.hip"),
    "2d": os.path.join(ROOT, "paper_1209_4297_amd", "csrc", "kernels_2d.hip"),
}
MEASURED_TRAFFIC = {
    ("reacdiff1d", (1024, 128, 1)): ("1d", "7487c6781845e08d", 4530176),
    ("reacdiff1d", (1024, 128, 0)): ("1d", "7487c6781845e08d", 4530176),
    ("batched1d", (256, 1536)): ("1d", "7487c6781845e08d", 72678016),
    ("batched1d", (512, 1536)): ("1d", "7487c6781845e08d", 72604672),
    ("reacdiff2d_rhs", "fp64"): ("2d", "1f1d915c37f8735f", 148586752),
    ("reacdiff2d_rhs", "fp32"): ("2d", "1f1d915c37f8735f", 167388416),
    ("reacdiff2d_rhs", "bf16x3"): ("2d", "1f1d915c37f8735f", 167307008),
    # the timed transform pass (the second of a step) per (precision, pass-shape bits)
    ("reacdiff2d", ("fp64", 0)): ("2d", "1f1d915c37f8735f", 100898304),
    ("reacdiff2d", ("fp64", 4)): ("2d", "1f1d915c37f8735f", 100911360),
    ("reacdiff2d", ("fp32", 0)): ("2d", "1f1d915c37f8735f", 50555648),
    ("reacdiff2d", ("fp32", 4)): ("2d", "1f1d915c37f8735f", 50574080),
    ("reacdiff2d", ("bf16x3", 0)): ("2d", "1f1d915c37f8735f", 50544384),
    # bit 2 reshapes only the first pass of each solve: the timed pass is the same kernel
    ("reacdiff2d", ("bf16x3", 2)): ("2d", "1f1d915c37f8735f", 50544384),
    ("reacdiff2d", ("bf16x3", 4)): ("2d", "1f1d915c37f8735f", 50552576),
}


def hbm_roofline(kernel, us, own, method):
    """HBM roofline of one launch: `own` is what the kernel must move at this step (every stored
    value it reads, once, and every vector it writes; it recomputes f instead of storing it),
    `method` the count for the method with stored f windows (method_step_bytes).  The kernel
    does not move the difference, so only `own` is a fraction of the HBM peak; the method's
    rate is a labelled extra and can exceed the peak."""
    ach = own / (us * 1e-6) / 1e9
    return {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": None, "kernel": kernel,
            "launch_us": round(us, 3), "bytes_per_launch": own,
            "method_bytes_per_launch": method,
            "method_equivalent_gbs": round(method / (us * 1e-6) / 1e9, 2),
            "note": "achieved counts the bytes the kernel must move (stored values read once, "
                    "vectors written; f recomputed); method_equivalent_gbs counts the method's "
                    "stored-window bytes per unknown-step, which are not moved"}


def method_step_bytes(P, unknowns):
    """Algorithmic HBM bytes of one pipeline step with every level active, counted for the
    method's level windows kept as stored vectors (FP64): level 0 reads its value and writes its
    value, F = f(eta) and C = L eta + f_E(eta of the previous node); a middle level j reads its
    value, the j+1 F of its window and one C, and writes value, F and C; the top level reads P+2
    vectors and writes its value.  That is 2, 9, 17, 26 vectors per unknown for orders 1-4
    (16, 72, 136, 208 B).  The kernels keep only the values and recompute f from them, so they
    move fewer bytes than this count (hbm_roofline)."""
    if P == 1:
        vectors = 2
    else:
        vectors = 4 + sum(j + 6 for j in range(1, P - 1)) + (P + 3)
    return 8 * vectors * unknowns


def code_hash(path):
    """First 16 hex digits of the SHA-256 of a C++/HIP source with its comments and blank space
    removed: the code the counters were taken on (a comment edit keeps the hash)."""
    import hashlib
    import re
    with open(path) as f:
        text = f.read()
    text = re.sub(r"//[^\n]*", "", re.sub(r"/\*.*?\*/", "", text, flags=re.S))
    return hashlib.sha256("".join(text.split()).encode()).hexdigest()[:16]


def measured_traffic(workload, key):
    """Counter-measured HBM bytes per launch of this workload's dominant kernel, if the kernel
    code is the one the counters were taken on, else None."""
    entry = MEASURED_TRAFFIC.get((workload, tuple(key) if isinstance(key, (list, tuple)) else key))
    if entry is None or not os.path.exists(KERNEL_SOURCE[entry[0]]):
        return None
    if code_hash(KERNEL_SOURCE[entry[0]]) != entry[1]:
        return None
    return entry[2]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="reacdiff2d",
                    choices=["reacdiff1d", "advdiff1d", "reacdiff2d", "batched1d", "serving",
                             "paper_advdiff", "paper_burgers", "stiff1d", "ark1d",
                             "order_sweep"])
    ap.add_argument("--rate", type=float, default=200.0,
                    help="serving: Poisson arrival rate in requests/s (the configured load is 200)")
    ap.add_argument("--horizon", type=float, default=60.0,
                    help="serving: seconds of Poisson arrivals admitted")
    ap.add_argument("--max-wall", type=float, default=90.0,
                    help="serving: wall-clock cap; work still queued then is reported unserved")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16x3"],
                    help="2D: transform precision of the value line (the matched block always "
                         "times the reduced-precision transforms)")
    ap.add_argument("--no-matched", action="store_true",
                    help="2D: skip the reduced-precision (matched) integrations")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-check", action="store_true",
                    help="2D: skip the FP64 reference integrations (error checks), e.g. when "
                         "profiling")
    ap.add_argument("--reps", type=int, default=200, help="launches timed for the roofline")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first copy a float64 tensor of this many MiB three times (a plain "
                         "copy kernel of known size, to scale hardware byte counters)")
    ap.add_argument("--nt", type=int, default=None,
                    help="override the number of time steps (short runs for counter profiling)")
    ap.add_argument("--tile", default=None,
                    help="1D tiling 'threads,rows,flags' instead of autotuning (rows 0 = whole cycle)")
    ap.add_argument("--pass-shape", type=int, default=None, metavar="BITS",
                    help="2D: transform-pass shape bits (1: 64-column waves, 2: 32-wide split-BF16 "
                         "slices, 4: row-major intermediates instead of prefolded planes) instead "
                         "of autotuning")
    ap.add_argument("--batch-tile", default=None,
                    help="batched 1D: grouped-launch tiling 'threads,rows' instead of autotuning "
                         "(rows 0 = whole cycles)")
    return ap.parse_args()


CPU_SAMPLE_S = 10.0      # seconds of oracle work timed for the CPU baseline


def oracle_time(fn, min_s=CPU_SAMPLE_S):
    """Run fn() on one core -- BLAS threads limited to one and scipy.fft's workers set to one
    (the oracle's transforms follow scipy.fft.set_workers) -- again and again until min_s
    seconds have passed (at least once); returns (first result, repetitions, seconds)."""
    import scipy.fft
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(limits=1)
    except Exception:  # noqa: BLE001
        limiter = None
    with scipy.fft.set_workers(1):
        t = time.perf_counter()
        out = fn()
        reps = 1
        while time.perf_counter() - t < min_s:
            fn()
            reps += 1
        dt = time.perf_counter() - t
    if limiter is not None:
        limiter.unregister()
    return out, reps, dt


def run_single(args, torch, ridc, prob, u0, prec, steps, warmup, tune=True, segments=1):
    """Whole integrations of one instance (split into `segments` restarted RIDC runs when above
    one); returns (seconds per integration, result, solver, initial data, tile)."""
    s = ridc.Ridc(prob, prec=prec)
    tile = None
    if prob["dim"] == 1 and args.tile:
        tile = tuple(int(x) for x in args.tile.split(",")) + (0,)
        tile = tile[:3]
        s.set_tile(*tile)
    elif prob["dim"] == 2 and args.pass_shape is not None:
        s.set_tile(0, 0, args.pass_shape)
        tile = (256 if args.pass_shape & 1 else 512, 0, args.pass_shape)
    elif tune:
        tile = s.autotune()     # 1D tiling, or the 2D transform-pass shape (cached per n, prec)
    x0 = torch.tensor(np.asarray(u0).reshape(-1), dtype=torch.float64, device="cuda")
    uT = torch.empty_like(x0)
    def run():
        if segments > 1:
            s.integrate_restarts(x0, prob["nt"], segments, uT, sync=False)
        else:
            s.integrate(x0, prob["nt"], uT, sync=False)
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    s.sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    s.sync()
    return el, uT.cpu().numpy(), s, x0, tile


def roofline_single(ridc, s, x0, nt, reps, bound, prec):
    P = s.order
    s.begin(x0, nt)
    ridc.advance([s], P * (P - 1) // 2)            # next step has every level active
    us, work = s.kernel_time(reps)
    s.sync()
    if bound == "hbm":
        return hbm_roofline("k_step1d", us, work, method_step_bytes(P, s.side))
    return roofline_pass(us, work, s.side, prec)


def roofline_pass(us, dense, n, prec):
    """Roofline of one transform pass over every level: `dense` is the plain product's 2 n^3
    flops per level.  The pass folds the symmetric sine matrix by its reflection symmetry when n
    is a multiple of 64, so its contraction has half that length: n^3 flops per level are the
    work of the folded product, which is what the matrix cores must issue (three BF16 products
    per folded product in the split-BF16 pass).  achieved/frac count that issued work against
    the dtype's dense MFMA peak; the dense count is kept as a labelled extra."""
    fold = 0.5 if n % 64 == 0 else 1.0
    products = 3.0 if prec == "bf16x3" else 1.0
    issued = dense * fold * products
    peak = MFMA_PEAK_TFLOPS[prec]
    ach = issued / (us * 1e-6) / 1e12
    return {"bound": "mfma", "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(ach / peak, 5), "traffic": None,
            "kernel": f"k_pass2d<{prec}>", "launch_us": round(us, 3),
            "flops_per_launch": issued,
            "dense_flops_per_launch": dense,
            "dense_equivalent_tflops": round(dense / (us * 1e-6) / 1e12, 3),
            "note": ("flops_per_launch is the folded contraction's n^3 per level"
                     + (" times 3 BF16 products" if prec == "bf16x3" else "")
                     + "; dense_flops_per_launch is the plain product's 2 n^3 per level, which "
                       "the folded kernel does not issue")}


def bench_1d(args, torch, ridc, which):
    import workloads
    segments = 1                                        # restarted RIDC segments (section III-E)
    if which == "reacdiff1d":
        prob, u0 = workloads.config_reacdiff_1d()
        if args.nt:
            prob = dict(prob, nt=args.nt, T=prob["T"] * args.nt / prob["nt"])
        desc = ("1D reaction-diffusion u_t = nu u_xx + u(1-u), Dirichlet [0,1], N=8192, "
                "nu=1e-3, 8 seeded Gaussians, RIDC order 4, T=1, Nt=2000, FP64")
        steps, warmup = args.steps or 20, args.warmup if args.warmup is not None else 3
    elif which == "paper_advdiff":
        prob, u0 = workloads.config_paper_advdiff()
        desc = ("paper section IV-A: u_t = 0.1 u_x + 1e-3 u_xx, periodic [0,1], dx=1/1000, "
                "first-order upwind advection, u0=2+sin 2pi x, RIDC order 4, T=40, Nt=4000 in "
                "10 restarted segments, FP64")
        segments = 10
        steps, warmup = args.steps or 10, args.warmup if args.warmup is not None else 2
    elif which == "paper_burgers":
        prob, u0 = workloads.config_paper_burgers()
        desc = ("paper section IV-B: u_t + (u^2/2)_x = 1e-3 u_xx, Dirichlet [0,1], dx=1/1000, "
                "flux F=(u_{i+1}^2+u_i^2)/2, u0=sin 2pi x + sin(pi x)/2, RIDC order 4, T=1, "
                "Nt=1000, FP64")
        steps, warmup = args.steps or 20, args.warmup if args.warmup is not None else 3
    else:
        prob, u0 = workloads.config_advdiff_1d()
        desc = ("1D advection-diffusion u_t + u_x = 0.1 u_xx, periodic [0,2pi), N=128, "
                "u0=sin x, RIDC order 4, T=1, Nt=200, FP64")
        steps, warmup = args.steps or 200, args.warmup if args.warmup is not None else 10
    n, nt, P = prob["n"], prob["nt"], prob["order"]
    el, out, s, x0, tile = run_single(args, torch, ridc, prob, u0, "fp64", steps, warmup,
                                      segments=segments)
    roof = roofline_single(ridc, s, x0, nt, args.reps, "hbm", "fp64")
    s.close()
    traffic = measured_traffic(which, tile)
    if traffic is not None:
        roof["traffic"] = traffic
        roof["traffic_note"] = ("HBM bytes per launch from FETCH_SIZE/WRITE_SIZE counters, "
                                "copy-calibrated; the chunk halos are re-read")
    cpu = rel = None
    if not args.no_cpu:
        from oracle import Problem, rel_l2, ridc_pipelined, ridc_restarted
        if segments > 1:
            ref, reps, sec = oracle_time(lambda: ridc_restarted(Problem.from_dict(prob), u0, nt,
                                                                P, segments))
        else:
            ref, reps, sec = oracle_time(lambda: ridc_pipelined(Problem.from_dict(prob), u0, nt,
                                                                P)[-1])
        rel = rel_l2(out, ref)
        cpu = {"value": round(n * nt * reps / sec, 1), "unit": "grid-point-steps/s", "cores": 1,
               "kind": "oracle",
               "sample": f"the full workload {reps}x (N={n}, Nt={nt}, order {P}), {sec:.2f} s, "
                         f"one thread; host has {os.cpu_count()} logical CPUs"}
    return dict(value=n * nt / el, ms=1e3 * el, steps=steps, warmup=warmup, dtype="f64",
                config={"workload": desc, "n": n, "nt": nt, "order": P, "segments": segments,
                        "pipeline_steps": nt + segments * (P * (P - 1) // 2),
                        "tile": {"threads": tile[0], "rows": tile[1], "flags": tile[2]}},
                roofline=roof, cpu=cpu, check={"rel_l2_vs_oracle": rel})


def imex_delays(pairs):
    """Pipeline start of each IMEX level: d_0 = 0, d_j = d_{j-1} + S_j - 1 with S_j the order
    p_0 + .. + p_j of level j (the library's schedule for ARK-based RIDC)."""
    order = {"fbe": 1, "ark3": 3, "ark4": 4}
    S, acc, d = [], 0, [0]
    for x in pairs:
        acc += order[x]
        S.append(acc)
    for j in range(1, len(S)):
        d.append(d[-1] + S[j] - 1)
    return S, d


def bench_imex(args, torch, ridc, which):
    """1D IMEX levels: ``stiff1d`` (RIDC4-FBE with the cubic reaction in the stiff part, Newton
    per stage) and ``ark1d`` (an ARK3 predictor and a forward-backward Euler corrector, order 4,
    on the N = 8192 reaction-diffusion workload)."""
    import workloads
    if which == "stiff1d":
        prob, u0 = workloads.config_stiff_1d()
        desc = ("1D u_t = 1e-3 u_xx + 1e3 (u - u^3), Dirichlet [0,1], N=8192, the reaction in "
                "the stiff part (Newton per stage), 8 seeded Gaussians, RIDC-FBE order 4, "
                "T=0.2, Nt=400, FP64")
    else:
        prob, u0 = workloads.config_reacdiff_1d()
        prob = dict(prob, order=2, pairs=["ark3", "fbe"])
        desc = ("1D reaction-diffusion u_t = 1e-3 u_xx + u(1-u), Dirichlet [0,1], N=8192, 8 "
                "seeded Gaussians, ARK-based RIDC: ARK3 predictor + FBE corrector (order 4), "
                "T=1, Nt=2000, FP64")
    if args.nt:
        prob = dict(prob, nt=args.nt, T=prob["T"] * args.nt / prob["nt"])
    pairs = prob.get("pairs", ["fbe"] * prob["order"])
    S, d = imex_delays(pairs)
    steps, warmup = args.steps or 10, args.warmup if args.warmup is not None else 2
    n, nt, P = prob["n"], prob["nt"], prob["order"]
    el, out, s, x0, _ = run_single(args, torch, ridc, prob, u0, "fp64", steps, warmup,
                                   tune=False)
    s.begin(x0, nt)
    if d[-1] > 0:
        ridc.advance([s], d[-1])              # next step has every level active
    us, alg = s.kernel_time(args.reps)
    s.sync()
    s.close()
    ach = alg / (us * 1e-6) / 1e9
    roof = {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": None, "kernel": "k_imex1d",
            "launch_us": round(us, 3), "bytes_per_launch": alg,
            "note": "one workgroup per level; a level reads its value and its window's values "
                    "and stored f, and writes its value and f; latency-bound (stage solves and "
                    "Newton iterates inside one workgroup)"}
    cpu = rel = None
    if not args.no_cpu:
        from oracle import Problem, rel_l2
        from oracle import ridc_ext as X
        ref, reps, sec = oracle_time(lambda: X.ridc_ark_pipelined(Problem.from_dict(prob), u0,
                                                                  nt, pairs)[-1])
        rel = rel_l2(out, ref)
        cpu = {"value": round(n * nt * reps / sec, 1), "unit": "grid-point-steps/s", "cores": 1,
               "kind": "oracle",
               "sample": f"the full workload {reps}x (N={n}, Nt={nt}, pairs {pairs}), "
                         f"{sec:.2f} s, one thread; host has {os.cpu_count()} logical CPUs"}
    return dict(value=n * nt / el, ms=1e3 * el, steps=steps, warmup=warmup, dtype="f64",
                config={"workload": desc, "n": n, "nt": nt, "levels": P, "pairs": pairs,
                        "order": S[-1], "pipeline_steps": nt + d[-1]},
                roofline=roof, cpu=cpu, check={"rel_l2_vs_oracle": rel})


def bench_order_sweep(args, torch, ridc):
    """Order against wall clock on one GPU (the paper's claim, section IV: a fourth-order RIDC
    solution in about the wall clock of a first-order one): whole integrations of the 1D
    N = 8192 reaction-diffusion workload (Nt = 2000) and of the 2D 1024^2 one (Nt = 100) for
    RIDC-FBE of orders 1-4 and two ARK-based RIDC schemes (Thm 2); the error is against an FP64
    RIDC4 run with 4x the steps.  The value is the RIDC4 1D rate."""
    import workloads
    steps, warmup = args.steps or 5, args.warmup if args.warmup is not None else 1
    rows = []

    def timed(prob, u0, prec="fp64"):
        s = ridc.Ridc(prob, prec=prec)
        if not prob.get("pairs"):
            s.autotune()     # the measured launch shape (cached per key), as elsewhere
        x0 = torch.tensor(np.asarray(u0).reshape(-1), dtype=torch.float64, device="cuda")
        uT = torch.empty_like(x0)
        for _ in range(warmup):
            s.integrate(x0, prob["nt"], uT, sync=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.integrate(x0, prob["nt"], uT, sync=False)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        s.sync()
        s.close()
        return el, uT.cpu().numpy()

    base1, v1 = workloads.config_reacdiff_1d()
    fine = dict(base1, nt=4 * base1["nt"])
    _, ref1 = timed(fine, v1)
    schemes1 = [("FBE (order 1)", dict(base1, order=1)),
                ("RIDC2-FBE", dict(base1, order=2)),
                ("RIDC3-FBE", dict(base1, order=3)),
                ("RIDC4-FBE", dict(base1, order=4)),
                ("RIDC: ARK3 + FBE (order 4)", dict(base1, order=2, pairs=["ark3", "fbe"])),
                ("RIDC: ARK4 + ARK3 (order 7)", dict(base1, order=2, pairs=["ark4", "ark3"]))]
    value = None
    for name, prob in schemes1:
        el, out = timed(prob, v1)
        err = float(np.linalg.norm(out - ref1) / np.linalg.norm(ref1))
        rows.append({"grid": "1D N=8192, Nt=2000", "scheme": name, "ms": round(1e3 * el, 3),
                     "rel_l2_vs_ridc4_4x_steps": err})
        if name == "RIDC4-FBE":
            value = base1["n"] * base1["nt"] / el
    base2, v2 = workloads.config_reacdiff_2d(nt=100, T=0.2)
    _, ref2 = timed(dict(base2, nt=400), v2)
    for name, order in (("FBE (order 1)", 1), ("RIDC2-FBE", 2), ("RIDC4-FBE", 4)):
        el, out = timed(dict(base2, order=order), v2)
        err = float(np.linalg.norm(out - ref2.reshape(out.shape)) / np.linalg.norm(ref2))
        rows.append({"grid": "2D 1024^2, Nt=100, T=0.2, FP64", "scheme": name,
                     "ms": round(1e3 * el, 3), "rel_l2_vs_ridc4_4x_steps": err})
    desc = ("order against wall clock: 1D reaction-diffusion N=8192 (Nt=2000, T=1) and 2D "
            "1024^2 (Nt=100, T=0.2), FBE, RIDC2-4 and ARK-based RIDC, FP64; value = RIDC4-FBE "
            "1D rate")
    return dict(value=value, ms=None, steps=steps, warmup=warmup, dtype="f64",
                config={"workload": desc, "sweep": rows}, roofline=None, cpu=None, check={})


def shape_name(shape):
    """The 2D transform-pass shape ridc_autotune chose: (threads, 0, shape bits)."""
    if shape is None:
        return None
    bits = shape[2]
    return {"bits": bits, "threads": shape[0], "wave_columns": 64 if bits & 1 else 32,
            "k_slice": "32 (two LDS stages)" if bits & 2 else "default",
            "intermediates": "row-major, folded while staging" if bits & 4
            else "prefolded planes (n a multiple of 256)"}


def stencil_roofline(ridc, s, x0, nt, reps):
    """HBM roofline of the right-hand-side kernel (stencils and quadrature of every level) at a
    steady-state step of the same integration."""
    P, n = s.order, s.side
    s.begin(x0, nt)
    ridc.advance([s], P * (P - 1) // 2)
    us, kbytes = s.stencil_time(reps)
    s.sync()
    return hbm_roofline("k_rhs2d", us, kbytes, method_step_bytes(P, n * n))


def bench_2d(args, torch, ridc):
    import workloads
    prob, u0 = workloads.config_reacdiff_2d()
    if args.nt:
        prob = dict(prob, nt=args.nt, T=prob["T"] * args.nt / prob["nt"])
    n, nt, P = prob["n"], prob["nt"], prob["order"]
    steps, warmup = args.steps or 3, args.warmup if args.warmup is not None else 1
    reps = max(10, args.reps // 10)
    el, out, s, x0, shape = run_single(args, torch, ridc, prob, u0, args.prec, steps, warmup)
    roof = roofline_single(ridc, s, x0, nt, reps, "mfma", args.prec)
    roof["pass_shape"] = shape_name(shape)
    roof_rhs = stencil_roofline(ridc, s, x0, nt, reps)
    if args.nt is None:
        roof["traffic"] = measured_traffic("reacdiff2d", (args.prec, shape[2] if shape else 0))
        roof_rhs["traffic"] = measured_traffic("reacdiff2d_rhs", args.prec)
    s.close()
    check = {}
    golden = os.path.join(ROOT, "tests", "golden", "reacdiff2d_n1024_nt500.npz")
    if os.path.exists(golden) and nt == 500:
        ref = np.load(golden)
        flat = out.reshape(-1)
        samp = ref["samples"][-1]
        check["rel_l2_vs_oracle_samples"] = float(np.linalg.norm(flat[ref["idx"]] - samp)
                                                  / np.linalg.norm(samp))
        check["rel_l2_vs_oracle_subgrid"] = float(
            np.linalg.norm(out.reshape(n, n)[::8, ::8] - ref["top_sub8"])
            / np.linalg.norm(ref["top_sub8"]))
    matched = {}
    if not args.no_check:
        # discretisation error of RIDC4 at this Nt: Richardson with an FP64 run at 2 Nt
        s2 = ridc.Ridc(dict(prob, nt=2 * nt), prec="fp64")
        u2 = s2.integrate(x0, 2 * nt).cpu().numpy()
        s2.close()
        u64 = out
        if args.prec != "fp64":
            s3 = ridc.Ridc(prob, prec="fp64")
            u64 = s3.integrate(x0, nt).cpu().numpy()
            s3.close()
            check["rel_l2_vs_fp64_gpu"] = float(np.linalg.norm(out - u64) / np.linalg.norm(u64))
        err_disc = 16.0 / 15.0 * float(np.linalg.norm(u64 - u2) / np.linalg.norm(u2))
        check["err_disc_ridc4"] = err_disc
        if args.prec != "fp64":
            check["matched"] = bool(check["rel_l2_vs_fp64_gpu"] <= 0.1 * err_disc)
        if not args.no_matched and args.prec == "fp64":
            for prec in ("bf16x3", "fp32"):
                el_m, out_m, sm, _, shape_m = run_single(args, torch, ridc, prob, u0, prec,
                                                         steps, warmup)
                roof_m = roofline_single(ridc, sm, x0, nt, reps, "mfma", prec)
                roof_m["pass_shape"] = shape_name(shape_m)
                if args.nt is None:
                    roof_m["traffic"] = measured_traffic("reacdiff2d",
                                                         (prec, shape_m[2] if shape_m else 0))
                sm.close()
                dist = float(np.linalg.norm(out_m - u64) / np.linalg.norm(u64))
                matched[prec] = {
                    "value": round(n * n * nt / el_m, 1), "unit": "grid-point-steps/s",
                    "ms_per_step": round(1e3 * el_m, 4), "speedup_vs_fp64": round(el / el_m, 4),
                    "transforms": {"bf16x3": "split-BF16 (hi/lo, 3 products, FP32 accumulation)",
                                   "fp32": "FP32"}[prec] + " + one FP64 residual refinement; "
                                                          "FP64 sums and level differences",
                    "rel_l2_vs_fp64": dist, "err_disc": err_disc,
                    "matched": bool(dist <= 0.1 * err_disc),
                    "roofline": {k: roof_m[k] for k in ("bound", "achieved", "peak", "unit",
                                                        "frac", "traffic", "kernel", "launch_us",
                                                        "flops_per_launch", "pass_shape")}}
    cpu = None
    if not args.no_cpu:
        from oracle import Problem, ridc_pipelined
        nts = 6
        _, creps, sec = oracle_time(lambda: ridc_pipelined(Problem.from_dict(prob), u0, nts, P))
        cpu = {"value": round(n * n * nts * creps / sec, 1), "unit": "grid-point-steps/s",
               "cores": 1, "kind": "oracle",
               "sample": f"the full {n}^2 grid for the first {nts} time steps of all {P} levels, "
                         f"{creps}x ({P * nts * creps} level steps, {sec:.1f} s) on one core "
                         f"(one BLAS thread, one FFT worker); host has {os.cpu_count()} logical "
                         "CPUs"}
    desc = ("2D reaction-diffusion u_t = nu Lap u + u(1-u), Dirichlet [0,1]^2, 1024x1024, "
            f"nu=1e-4, 8 seeded bumps, RIDC order 4, T={prob['T']:g}, Nt={nt}, "
            f"transforms {args.prec}")
    line = dict(value=n * n * nt / el, ms=1e3 * el, steps=steps, warmup=warmup,
                dtype={"fp64": "f64", "fp32": "f32 transforms, f64 sums",
                       "bf16x3": "bf16x3 transforms, f64 sums"}[args.prec],
                config={"workload": desc, "n": n, "nt": nt, "order": P, "prec": args.prec,
                        "pipeline_steps": nt + P * (P - 1) // 2},
                roofline=roof, roofline_stencil=roof_rhs, cpu=cpu, check=check)
    if matched:
        line["matched"] = matched
    return line


def bench_batched(args, torch, ridc):
    import workloads
    cases = workloads.config_batched_1d(**({"nt": args.nt, "T": 0.25 * args.nt / 1000}
                                          if args.nt else {}))
    steps, warmup = args.steps or 3, args.warmup if args.warmup is not None else 1
    solvers, u0s, uTs = [], [], []
    for prob, u0 in cases:
        s = ridc.Ridc(prob)
        solvers.append(s)
        u0s.append(torch.tensor(u0, dtype=torch.float64, device="cuda"))
        uTs.append(torch.empty_like(u0s[-1]))
    if args.batch_tile:
        batch_tile = tuple(int(x) for x in args.batch_tile.split(","))
        ridc.set_batch_tile(*batch_tile)
    else:
        batch_tile = ridc.autotune_batch(solvers)       # measured grouped-launch tiling
    nts = [p["nt"] for p, _ in cases]
    for _ in range(warmup):
        ridc.integrate_batch(solvers, u0s, nts, uTs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ridc.integrate_batch(solvers, u0s, nts, uTs)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    total = sum(p["n"] for p, _ in cases) * cases[0][0]["nt"]
    # roofline: back-to-back grouped launches of one steady-state step (HIP events, library)
    for s, x0, nt in zip(solvers, u0s, nts):
        s.begin(x0, nt)
    ridc.advance(solvers, 6)
    us, bytes_per = ridc.batch_kernel_time(solvers, args.reps)
    alg = sum(method_step_bytes(p["order"], p["n"]) for p, _ in cases)
    roof = hbm_roofline("k_step1d (grouped)", us, bytes_per, alg)
    traffic = measured_traffic("batched1d", batch_tile)
    if traffic is not None and args.nt is None:
        roof["traffic"] = traffic
        roof["traffic_note"] = ("HBM bytes per launch from FETCH_SIZE/WRITE_SIZE counters, "
                                "copy-calibrated; chunk halos of the long systems are re-read")
    outs = [u.cpu().numpy() for u in uTs]
    for s in solvers:
        s.close()
    cpu = None
    check = {}
    if not args.no_cpu:
        from oracle import Problem, rel_l2, ridc_pipelined
        idx = [0, 1, 2, 3]
        def run():
            return [ridc_pipelined(Problem.from_dict(cases[i][0]), cases[i][1], nts[i], 4)[-1]
                    for i in idx]
        refs, reps, sec = oracle_time(run)
        check["rel_l2_vs_oracle_max_of_sample"] = max(rel_l2(outs[i], r) for i, r in zip(idx, refs))
        pts = sum(cases[i][0]["n"] * nts[i] for i in idx) * reps
        cpu = {"value": round(pts / sec, 1), "unit": "grid-point-steps/s", "cores": 1,
               "kind": "oracle",
               "sample": f"instances 0-3 of 256 (n = {[cases[i][0]['n'] for i in idx]}), full "
                         f"Nt=1000, {reps}x, {sec:.1f} s, one thread"}
    desc = ("256 periodic advection-diffusion instances, N ~ U{256..4096}, a ~ U(0.5,2), "
            "nu ~ logU(1e-3,1e-1), 8 Fourier modes, RIDC order 4, Nt=1000, T=0.25, FP64")
    return dict(value=total / el, ms=1e3 * el, steps=steps, warmup=warmup, dtype="f64",
                config={"workload": desc, "instances": len(cases),
                        "unknowns": sum(p["n"] for p, _ in cases), "nt": nts[0], "order": 4,
                        "batch_tile": {"threads": batch_tile[0], "rows": batch_tile[1]}},
                roofline=roof, cpu=cpu, check=check)


def bench_serving(args, torch, ridc):
    """Poisson stream of 2D reaction-diffusion requests (200 req/s; side 128..1024, order 2..4,
    Nt 100..500, split-BF16 or FP32 transforms with FP64 refinement), continuous batching."""
    import workloads
    from paper_1209_4297_amd.serve import GpuExecutor, Request, Server
    arrivals = workloads.serving_requests(rate=args.rate, duration=args.horizon)
    reqs = []
    for i, a in enumerate(arrivals):
        n = a["prob"]["n"]
        u0 = workloads.bumps_2d(n, a["bump_seed"]).reshape(-1)
        reqs.append(Request(rid=i, prob=a["prob"], u0=u0, nsteps=a["prob"]["nt"],
                            prec=args.prec if args.prec != "fp64" else "bf16x3",
                            t_arrival=a["t_arrival"]))
    free, total = torch.cuda.mem_get_info()
    srv = Server(GpuExecutor(), hbm_budget=int(min(free * 0.5, 64 * 2**30)), max_slots=96,
                 tick_steps=8)
    # warm the transform caches and kernels before the clock starts
    for n in (128, 256, 512, 1024):
        prob, u0 = workloads.config_reacdiff_2d(n=n, nt=3, order=4)
        sv = ridc.Ridc(prob, prec=reqs[0].prec)
        sv.integrate(torch.tensor(u0.reshape(-1), dtype=torch.float64, device="cuda"), 3)
        sv.close()
    torch.cuda.synchronize()
    stats = srv.run(reqs, horizon=args.horizon, max_wall=args.max_wall)
    # one finished request of each size checked against its solo integration (bitwise)
    check = {"solo_bitwise_equal": True, "checked": 0}
    seen = set()
    for r in srv.done:
        if r.status != "done" or r.prob["n"] in seen:
            continue
        seen.add(r.prob["n"])
        sv = ridc.Ridc(r.prob, prec=r.prec)
        alone = sv.integrate(torch.tensor(r.u0, dtype=torch.float64, device="cuda"), r.nsteps)
        sv.close()
        check["checked"] += 1
        check["solo_bitwise_equal"] &= bool(torch.equal(alone, r.result))
    desc = (f"serving: Poisson {args.rate:g} req/s 2D reaction-diffusion, side "
            "U{128,256,512,1024}, order U{2,3,4}, nu logU(1e-5,1e-3), Nt U{100..500}, T=1, "
            "seeded bumps, transforms "
            f"{reqs[0].prec} + FP64 refinement; arrivals for {args.horizon:.0f} s")
    roof = None
    return dict(value=stats["completed_grid_point_steps_per_s"], ms=1e3 * stats["wall_s"],
                steps=1, warmup=0, dtype=f"{reqs[0].prec} transforms, f64 sums",
                config={"workload": desc, "offered": len(reqs), **{k: stats[k] for k in (
                    "completed", "status_counts", "p50_latency_s", "p99_latency_s",
                    "completed_requests_per_s", "peak_resident", "peak_hbm_bytes", "ticks")}},
                roofline=roof, cpu=None, check=check)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only (--gpus 1): the hot path runs on a single MI355X; "
              "independent instances and requests would shard one process per GPU with no "
              "exchange between them.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1209_4297_amd import ridc
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        if args.calibrate_copy:
            src = torch.ones(args.calibrate_copy * 2**17, dtype=torch.float64, device="cuda")
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            del src, dst
        line = run_workload(args, torch, ridc)
    print(json.dumps(line), flush=True)


def run_workload(args, torch, ridc):
    if args.workload in ("reacdiff1d", "advdiff1d", "paper_advdiff", "paper_burgers"):
        r = bench_1d(args, torch, ridc, args.workload)
    elif args.workload == "reacdiff2d":
        r = bench_2d(args, torch, ridc)
    elif args.workload == "serving":
        r = bench_serving(args, torch, ridc)
    elif args.workload in ("stiff1d", "ark1d"):
        r = bench_imex(args, torch, ridc, args.workload)
    elif args.workload == "order_sweep":
        r = bench_order_sweep(args, torch, ridc)
    else:
        r = bench_batched(args, torch, ridc)
    cfg = dict(r["config"], parallelism="single GPU")
    line = {
        "metric": METRIC,
        "value": round(r["value"], 1),
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": r["steps"],
        "warmup": r["warmup"],
        "ms_per_step": round(r["ms"], 4) if r["ms"] is not None else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": r["dtype"],
        "data": "synthetic",
        "config": cfg,
        "check": r["check"],
        "roofline": r["roofline"],
        "cpu_baseline": r["cpu"],
    }
    if r.get("roofline_stencil"):
        line["roofline_stencil"] = r["roofline_stencil"]
    if r.get("matched"):
        line["matched"] = r["matched"]
    return line


if __name__ == "__main__":
    main()
