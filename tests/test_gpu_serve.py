"""Serving on the GPU: requests of mixed sizes, orders, dimensions and precisions admitted while
others run produce, bit for bit, the result of the same request integrated alone, and the
reduced-precision ones stay within their tolerance of the FP64 oracle."""
import os
import sys

import numpy as np
import pytest

import workloads
from oracle import Problem, rel_l2, ridc_pipelined

pytestmark = pytest.mark.gpu

# FP64: the spec bar.  Reduced precision: the bound of the result's level index,
# test_gpu_2d.tol_of (about 100 x the measured errors; the RIDC4 top level at the matched bar).
from tolerances import tol_of  # noqa: E402


def _mix():
    reqs = []
    rid = 0
    for n, order, nt, prec in [(64, 4, 12, "fp32"), (96, 2, 9, "bf16x3"), (32, 3, 15, "fp64"),
                               (64, 3, 7, "fp32"), (128, 4, 5, "fp64"), (64, 4, 12, "fp32"),
                               (32, 2, 30, "bf16x3")]:
        prob, u0 = workloads.config_reacdiff_2d(n=n, nt=nt, order=order, T=nt * 2e-3, nu=1e-3,
                                                seed=500 + rid)
        reqs.append(dict(rid=rid, prob=prob, u0=u0.reshape(-1), nsteps=nt, prec=prec))
        rid += 1
    for n, order, nt in [(300, 4, 40), (2048, 3, 25)]:
        prob, u0 = workloads.config_reacdiff_1d(n=n, nt=nt, order=order, T=nt * 5e-4)
        reqs.append(dict(rid=rid, prob=prob, u0=u0, nsteps=nt, prec="fp64"))
        rid += 1
    return reqs


def test_served_results_equal_solo_results():
    import torch
    from paper_1209_4297_amd import ridc
    from paper_1209_4297_amd.serve import GpuExecutor, Request, Server

    specs = _mix()
    solo = {}
    for sp in specs:
        s = ridc.Ridc(sp["prob"], prec=sp["prec"])
        x0 = torch.tensor(sp["u0"], dtype=torch.float64, device="cuda")
        solo[sp["rid"]] = s.integrate(x0, sp["nsteps"]).cpu().numpy()
        s.close()
    srv = Server(GpuExecutor(), hbm_budget=2**30, max_slots=5, tick_steps=3)
    reqs = [Request(**sp) for sp in specs]
    # staggered arrivals: two at first, then one more per tick
    srv.submit(reqs[0])
    srv.submit(reqs[1])
    i = 2
    while not srv.idle() or i < len(reqs):
        if i < len(reqs):
            srv.submit(reqs[i])
            i += 1
        srv.tick()
    assert srv.peak_running >= 3
    for r in reqs:
        print(f"request {r.rid}: {r.status} n={r.prob['n']} dim={r.prob['dim']} {r.prec}",
              flush=True)
        assert r.status == "done", r.error
        np.testing.assert_array_equal(r.result.cpu().numpy(), solo[r.rid])
        if r.prec != "fp64" and r.rid % 2 == 0:
            ref = ridc_pipelined(Problem.from_dict(r.prob), np.asarray(r.u0).reshape(
                r.prob["n"], r.prob["n"]), r.nsteps, r.prob["order"])[-1]
            err = rel_l2(r.result.cpu().numpy().reshape(ref.shape), ref)
            assert err <= tol_of(r.prec, r.prob["order"] - 1), err


SERVING_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "serving_first_per_side.npz")


@pytest.mark.skipif(not os.path.exists(SERVING_GOLDEN), reason="serving samples not generated")
@pytest.mark.parametrize("prec", ["fp64", "bf16x3", "fp32"])
def test_served_requests_of_every_side_against_oracle(prec):
    """The first request of each side (128, 256, 512, 1024) of the 200 req/s serving stream,
    served together through the continuous-batching server, against the FP64 oracle's values
    stored in tests/golden (every point of the sampled set, the norm, the sum and the
    every-8th-point sub-grid)."""
    import torch
    from paper_1209_4297_amd.serve import GpuExecutor, Request, Server

    ref = np.load(SERVING_GOLDEN)
    stream = workloads.serving_requests(rate=200.0, duration=60.0)
    reqs = []
    for n in (128, 256, 512, 1024):
        i = int(ref[f"n{n}_request"])
        a = stream[i]
        assert a["prob"]["n"] == n
        u0 = workloads.bumps_2d(n, a["bump_seed"]).reshape(-1)
        reqs.append(Request(rid=i, prob=a["prob"], u0=u0, nsteps=a["prob"]["nt"], prec=prec))
    srv = Server(GpuExecutor(), hbm_budget=8 * 2**30, max_slots=8, tick_steps=16)
    for r in reqs:
        srv.submit(r)
    while not srv.idle():
        srv.tick()
    for r in reqs:
        n = r.prob["n"]
        tol = tol_of(prec, r.prob["order"] - 1)
        assert r.status == "done", r.error
        got = r.result.cpu().numpy()
        samp = ref[f"n{n}_samples"]
        g = got[ref[f"n{n}_idx"]]
        err = np.linalg.norm(g - samp) / np.linalg.norm(samp)
        emax = float(np.max(np.abs(g - samp)) / np.max(np.abs(samp)))
        nerr = abs(np.linalg.norm(got) - ref[f"n{n}_norm"]) / ref[f"n{n}_norm"]
        sub = got.reshape(n, n)[::8, ::8]
        serr = np.linalg.norm(sub - ref[f"n{n}_sub8"]) / np.linalg.norm(ref[f"n{n}_sub8"])
        print(f"request {r.rid} n={n} P={r.prob['order']} nt={r.nsteps} {prec}: sampled rel L2 "
              f"{err:.3e}, max {emax:.3e}, norm {nerr:.3e}, sub-grid {serr:.3e}", flush=True)
        assert err <= tol and emax <= tol and nerr <= tol and serr <= tol, (n, err, emax, nerr,
                                                                           serr)
