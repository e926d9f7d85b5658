"""GPU parity of grouped 1D launches against the FP64 oracle.

* The 256-instance batch (periodic advection-diffusion, N ~ U{256..4096}, Nt = 1000, T = 0.25)
  at full shape, in the tiling the benchmark measures (autotuned), every instance checked in
  full against the oracle's mode-by-mode evaluation of the same linear periodic problem
  (``oracle.ridc_linear_periodic``, pinned against the vector oracle on the CPU).
* A small ragged batch (periodic and Dirichlet, orders 3 and 4) against the vector oracle.
* Batches of different handles on two streams, called alternately without waiting: every
  result bitwise equals the instance integrated alone (the launch tables shared by grouped
  calls must not be rewritten while another stream's kernels still read them).

Bar: relative L2 <= 1e-12 per instance and max |gpu - oracle| <= 1e-12 max |oracle|.
"""
import sys

import numpy as np
import pytest

import workloads
from oracle import Problem, rel_l2, ridc_linear_periodic, ridc_pipelined

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1209_4297_amd import ridc
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, ridc


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _check(got, ref, what):
    err = rel_l2(got, ref)
    emax = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    assert err <= TOL and emax <= TOL, (what, err, emax)
    return err, emax


def _batch(env, cases, tune=False):
    torch, ridc = env
    solvers = [ridc.Ridc(p) for p, _ in cases]
    u0s = [torch.tensor(u, dtype=torch.float64, device="cuda") for _, u in cases]
    uTs = [torch.empty_like(x) for x in u0s]
    try:
        if tune:
            t, r = ridc.autotune_batch(solvers)
            _say(f"batch tiling: threads {t}, rows {r}")
        ridc.integrate_batch(solvers, u0s, [p["nt"] for p, _ in cases], uTs)
        for s in solvers:
            s.sync()
        return [u.cpu().numpy() for u in uTs]
    finally:
        for s in solvers:
            s.close()
        ridc.set_batch_tile(256, 0)


def test_full_batch_against_fourier_oracle(env):
    cases = workloads.config_batched_1d()
    _say(f"case: {len(cases)} instances, nt={cases[0][0]['nt']}, T={cases[0][0]['T']}, "
         f"unknowns {sum(p['n'] for p, _ in cases)}")
    outs = _batch(env, cases, tune=True)
    worst = (0.0, 0.0)
    for i, ((prob, u0), got) in enumerate(zip(cases, outs)):
        ref = ridc_linear_periodic(Problem.from_dict(prob), u0, prob["nt"], prob["order"])[-1]
        e = _check(got, ref, (i, prob["n"]))
        worst = (max(worst[0], e[0]), max(worst[1], e[1]))
    _say(f"  worst instance: rel L2 {worst[0]:.3e}, max abs / max {worst[1]:.3e}")


def test_small_ragged_batch_against_vector_oracle(env):
    cases = workloads.config_batched_1d(count=12, nt=120, T=0.03)
    cases.append(workloads.config_reacdiff_1d(n=2500, nt=90, order=3, T=0.05))
    _say(f"case: 13 instances, sizes {[p['n'] for p, _ in cases]}")
    outs = _batch(env, cases)
    for i, ((prob, u0), got) in enumerate(zip(cases, outs)):
        ref = ridc_pipelined(Problem.from_dict(prob), u0, prob["nt"], prob["order"])[-1]
        err, emax = _check(got, ref, (i, prob["n"]))
        _say(f"  instance {i} n={prob['n']} P={prob['order']}: rel L2 {err:.3e}, "
             f"max {emax:.3e}")


def test_batches_on_two_streams_called_alternately(env):
    torch, ridc = env
    cases_a = workloads.config_batched_1d(count=9, nt=80, T=0.02, seed=41)
    cases_b = workloads.config_batched_1d(count=7, nt=60, T=0.015, seed=42)
    cases_b.append(workloads.config_reacdiff_1d(n=3000, nt=50, order=4, T=0.02))
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    groups = []
    for cases, st in ((cases_a, sa), (cases_b, sb)):
        solvers = [ridc.Ridc(p, stream=st) for p, _ in cases]
        u0s = [torch.tensor(u, dtype=torch.float64, device="cuda") for _, u in cases]
        groups.append((cases, st, solvers, u0s))
    torch.cuda.synchronize()
    solo = []
    for cases, _, _, u0s in groups:
        ref = []
        for (p, _), x0 in zip(cases, u0s):
            s = ridc.Ridc(p)
            ref.append(s.integrate(x0, p["nt"]).cpu().numpy())
            s.close()
        solo.append(ref)
    try:
        for rnd in range(3):
            outs = []
            for cases, st, solvers, u0s in groups:
                uTs = [torch.empty_like(x) for x in u0s]
                ridc.integrate_batch(solvers, u0s, [p["nt"] for p, _ in cases], uTs)
                outs.append(uTs)
            # stepping interface on both streams, interleaved
            for cases, st, solvers, u0s in groups:
                for s, x0, (p, _) in zip(solvers, u0s, cases):
                    s.begin(x0, p["nt"])
            while any(s.remaining() > 0 for g in groups for s in g[2]):
                for cases, st, solvers, u0s in groups:
                    if any(s.remaining() > 0 for s in solvers):
                        ridc.advance(solvers, 11)
            torch.cuda.synchronize()
            for g, (cases, st, solvers, u0s) in enumerate(groups):
                for i, s in enumerate(solvers):
                    np.testing.assert_array_equal(outs[g][i].cpu().numpy(), solo[g][i])
                    out = torch.empty_like(u0s[i])
                    s.read(out)
                    s.sync()
                    np.testing.assert_array_equal(out.cpu().numpy(), solo[g][i])
            _say(f"round {rnd}: both streams bitwise equal to solo runs")
    finally:
        for g in groups:
            for s in g[2]:
                s.close()
