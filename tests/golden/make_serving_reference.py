"""Write the oracle's reference samples for served 2D requests of every side.

The serving workload is a Poisson stream of 2D reaction-diffusion requests (side uniform in
{128, 256, 512, 1024}, order in {2, 3, 4}, nu log-uniform in [1e-5, 1e-3], Nt in 100..500,
T = 1, seeded Gaussian bumps) at 200 requests/s for 60 s.  This script takes, for each side,
the first request of that side in the stream (``workloads.serving_requests``) and integrates it
with the FP64 oracle (``oracle.ridc_pipelined``); the GPU path is never involved.  Stored per
request: its index in the stream, the top level at 4096 seeded points (every point when the
grid has fewer), the top level's L2 norm and sum, and the top level on the every-8th-point
sub-grid.

    python tests/golden/make_serving_reference.py [out.npz]
"""
import os
import sys
import time

import numpy as np
import scipy.fft

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import Problem, ridc_pipelined  # noqa: E402

SIDES = (128, 256, 512, 1024)


def first_of_each_side(stream):
    picked = {}
    for i, a in enumerate(stream):
        n = a["prob"]["n"]
        if n in SIDES and n not in picked:
            picked[n] = i
        if len(picked) == len(SIDES):
            break
    return [picked[n] for n in SIDES]


def main(path):
    stream = workloads.serving_requests(rate=200.0, duration=60.0)
    out = {}
    t0 = time.time()
    for n, i in zip(SIDES, first_of_each_side(stream)):
        a = stream[i]
        prob = a["prob"]
        u0 = workloads.bumps_2d(n, a["bump_seed"])
        with scipy.fft.set_workers(os.cpu_count() or 1):   # the values do not depend on it
            top = ridc_pipelined(Problem.from_dict(prob), u0, prob["nt"], prob["order"])[-1]
        rng = np.random.default_rng(7000 + n)
        idx = (np.arange(n * n) if n * n <= 4096
               else np.sort(rng.choice(n * n, size=4096, replace=False)))
        out[f"n{n}_request"] = i
        out[f"n{n}_idx"] = idx
        out[f"n{n}_samples"] = top.reshape(-1)[idx]
        out[f"n{n}_norm"] = np.linalg.norm(top)
        out[f"n{n}_sum"] = top.sum()
        out[f"n{n}_sub8"] = top[::8, ::8].copy()
        print(f"request {i}: n={n} order {prob['order']} nt={prob['nt']} done, "
              f"{time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(path, **out)
    print(f"wrote {path} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(HERE, "serving_first_per_side.npz"))
