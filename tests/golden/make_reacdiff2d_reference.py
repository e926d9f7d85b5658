"""Write the oracle's reference samples for the full 2D reaction-diffusion workload.

u_t = nu Lap u + u(1-u), Dirichlet 0 on [0,1]^2, 1024 x 1024 interior points, nu = 1e-4,
eight seeded radial Gaussians, RIDC order 4, T = 1, Nt = 500.  Calls only the FP64 oracle
(``oracle.ridc_pipelined``) and the seeded input generator (``workloads``); the GPU path is
never involved.  The full run takes several minutes on a multi-core host, so the test suite
compares the GPU result with the samples stored here: every level's value at 4096 seeded
points, every level's L2 norm and sum, and the top level on the every-8th-point sub-grid.

    python tests/golden/make_reacdiff2d_reference.py [out.npz]
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


def main(path):
    prob, u0 = workloads.config_reacdiff_2d()
    p = Problem.from_dict(prob)
    n, nt, order = prob["n"], prob["nt"], prob["order"]
    t0 = time.time()
    steps = [0]

    def trace(sigma, j, m):
        if j == 0 and m % 25 == 0:
            print(f"oracle step {sigma} (level 0 at t_{m}), {time.time() - t0:.0f} s", flush=True)

    with scipy.fft.set_workers(os.cpu_count() or 1):     # the values do not depend on it
        levels = ridc_pipelined(p, u0, nt, order, trace=trace)
    rng = np.random.default_rng(20240)
    idx = rng.choice(n * n, size=4096, replace=False)
    np.savez_compressed(
        path,
        idx=idx,
        samples=np.stack([lv.reshape(-1)[idx] for lv in levels]),
        norms=np.array([np.linalg.norm(lv) for lv in levels]),
        sums=np.array([lv.sum() for lv in levels]),
        top_sub8=levels[-1][::8, ::8].copy(),
        n=n, nt=nt, order=order, seconds=time.time() - t0)
    print(f"wrote {path} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(HERE, "reacdiff2d_n1024_nt500.npz"))
