"""GPU parity of the IMEX level step (ARK-based RIDC, Thm 2; Newton for a stiff reaction,
section III-B) against the FP64 extension oracle.

Bar: relative L2 <= 1e-12 per level against ``oracle.ridc_ext.ridc_ark_pipelined`` on the same
seeded inputs, and the largest pointwise difference <= 1e-12 of the largest value.  Both sides
solve every implicit stage to rounding (the GPU by a partition tridiagonal solver, the oracle by
FFT or banded LU; Newton iterates on both until the update reaches rounding), so only rounding
differs.  Grouped launches must not change a single bit.
"""
import sys

import numpy as np
import pytest

import workloads
from oracle import Problem, rel_l2, ridc_pipelined
from oracle import ridc_ext as X

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


def run_gpu(env, prob, u0, nt, newton_maxit=0):
    torch, ridc = env
    s = ridc.Ridc(prob, newton_maxit=newton_maxit)
    x0 = torch.tensor(np.asarray(u0), dtype=torch.float64, device="cuda")
    uT = torch.empty_like(x0)
    lv = torch.empty(prob["order"] * x0.numel(), dtype=torch.float64, device="cuda")
    s.integrate(x0, nt, uT, lv)
    out = uT.cpu().numpy(), lv.cpu().numpy().reshape(prob["order"], -1)
    s.close()
    return out


def schemes_of(prob):
    return prob.get("pairs", ["fbe"] * prob["order"])


def check(env, prob, u0, nt, tol=TOL):
    _say(f"case: {prob['bc']} n={prob['n']} pairs={schemes_of(prob)} fi={prob.get('fi')} "
         f"kappa={prob.get('kappa', 0)} fe={prob['fe']} nt={nt}")
    p = Problem.from_dict(prob)
    ref = X.ridc_ark_pipelined(p, np.asarray(u0), nt, schemes_of(prob))
    top, lvs = run_gpu(env, prob, u0, nt)
    assert np.array_equal(top, lvs[-1])
    errs = []
    for j in range(prob["order"]):
        err = rel_l2(lvs[j], ref[j])
        mx = np.abs(lvs[j] - ref[j]).max() / np.abs(ref[j]).max()
        errs.append((err, mx))
        assert err <= tol and mx <= tol, (j, err, mx)
    _say("  rel L2 / max per level: " + ", ".join(f"{a:.2e}/{b:.2e}" for a, b in errs))
    return top


ADV = [("fbe",) * 4, ("ark3",), ("ark4",), ("ark3", "fbe"), ("fbe", "ark3"),
       ("ark3", "ark3"), ("ark4", "fbe", "fbe"), ("fbe", "fbe", "ark3")]


@pytest.mark.parametrize("pairs", ADV, ids=["-".join(p) for p in ADV])
def test_ark_ridc_periodic_advection_diffusion(env, pairs):
    prob, u0 = workloads.config_advdiff_1d(n=128, nt=200, order=len(pairs))
    prob["pairs"] = list(pairs)
    check(env, prob, u0, 60)


@pytest.mark.parametrize("pairs", [("ark3", "fbe"), ("ark4", "ark3"), ("fbe",) * 3],
                         ids=["ark3-fbe", "ark4-ark3", "fbe3"])
@pytest.mark.parametrize("n", [1000, 4097, 8192])
def test_ark_ridc_dirichlet_reaction_diffusion(env, pairs, n):
    # explicit logistic term, diffusion implicit; n = 4097 leaves a ragged last block
    prob, u0 = workloads.config_reacdiff_1d(n=n, nt=2000, order=len(pairs))
    prob["pairs"] = list(pairs)
    check(env, prob, u0, 30)


def test_ark_ridc_paper_upwind_case(env):
    # the paper's advection-diffusion workload (section IV-A, periodic, upwind) with an ARK3
    # predictor and a forward-backward Euler corrector (order 4)
    prob, u0 = workloads.config_paper_advdiff(n=1000, nt=4000, order=2)
    prob["pairs"] = ["ark3", "fbe"]
    check(env, prob, u0, 40)


def test_euler_pairs_equal_ridc_fbe(env):
    # forward-backward Euler levels through the IMEX kernel are RIDC-FBE: compare with the base
    # oracle and with the library's own RIDC-FBE kernel
    torch, ridc = env
    prob, u0 = workloads.config_reacdiff_1d(n=8192, nt=2000, order=4)
    ref = ridc_pipelined(Problem.from_dict(prob), u0, 100, 4)[-1]
    imex = dict(prob, pairs=["fbe"] * 4)
    top, _ = run_gpu(env, imex, u0, 100)
    s = ridc.Ridc(prob)
    base = s.integrate(torch.tensor(u0, device="cuda"), 100).cpu().numpy()
    s.close()
    _say(f"fbe via IMEX kernel: vs oracle {rel_l2(top, ref):.2e}, vs PCR kernel "
         f"{rel_l2(top, base):.2e}")
    assert rel_l2(top, ref) <= TOL and rel_l2(top, base) <= TOL


# (reaction, kappa, pairs, steps over T = 0.2).  Every case keeps tau kappa max g' < 1 (tau =
# dt times the largest diagonal entry of the stiff tableau), so that each stage equation has
# one root near the solution and Newton's method converges to rounding on both sides.
NEWTON = [("cubic", 1e3, ("fbe",) * 4, 400), ("logistic", 50.0, ("fbe",) * 4, 400),
          ("cubic", 1e3, ("ark3", "fbe"), 400), ("cubic", 1e4, ("fbe", "fbe"), 4000)]


@pytest.mark.parametrize("fi,kappa,pairs,nt", NEWTON,
                         ids=[f"{a}-{b:g}-{'-'.join(c)}" for a, b, c, _ in NEWTON])
@pytest.mark.parametrize("n", [999, 8192])
def test_newton_stiff_reaction(env, fi, kappa, pairs, nt, n):
    prob, u0 = workloads.config_stiff_1d(n=n, nt=nt, order=len(pairs), fi=fi, kappa=kappa,
                                         pairs=pairs)
    check(env, prob, u0, 40)


def test_newton_with_explicit_advection(env):
    # Burgers flux explicit (section IV-B) next to an implicit cubic reaction
    prob, u0 = workloads.config_stiff_1d(n=999, order=3, fi="cubic", kappa=200.0,
                                         fe="burgers")
    check(env, prob, u0, 40)


def test_newton_iteration_cap_reports_nonfinite(env):
    # one Newton iterate cannot reach rounding on a stiff reaction: the stage result is NaN and
    # the library reports it on sync (the limit is forced from the host; every kernel exits)
    torch, ridc = env
    prob, u0 = workloads.config_stiff_1d(n=999, order=2, fi="cubic", kappa=1e3)
    s = ridc.Ridc(prob, newton_maxit=1)
    x0 = torch.tensor(u0, device="cuda")
    with pytest.raises(ridc.RidcError) as e:
        s.integrate(x0, 10)
    assert e.value.code == ridc.RIDC_E_NONFINITE
    s.close()


def test_grouped_imex_launches_are_bitwise_solo(env):
    torch, ridc = env
    cases = [
        workloads.config_stiff_1d(n=999, order=2, fi="cubic", kappa=1e3, pairs=("ark3", "fbe")),
        workloads.config_stiff_1d(n=2000, order=4, fi="logistic", kappa=50.0),
        workloads.config_reacdiff_1d(n=1000, nt=2000, order=2),
        workloads.config_reacdiff_1d(n=3000, nt=2000, order=3),
    ]
    cases[2][0]["pairs"] = ["ark4", "fbe"]
    cases[3][0]["pairs"] = ["fbe", "ark3", "fbe"]
    nts = [30, 40, 25, 35]
    solo = [run_gpu(env, p, u, nt)[0] for (p, u), nt in zip(cases, nts)]
    hs = [ridc.Ridc(p) for p, _ in cases]
    x0 = [torch.tensor(u, device="cuda") for _, u in cases]
    uT = [torch.empty_like(x) for x in x0]
    _say("case: grouped IMEX batch of 4")
    ridc.integrate_batch(hs, x0, nts, uT)
    for h in hs:
        h.sync()
    for a, b in zip(uT, solo):
        assert np.array_equal(a.cpu().numpy(), b)
    for h in hs:
        h.close()
    ref = X.ridc_ark_pipelined(Problem.from_dict(cases[0][0]), cases[0][1], 30,
                               ["ark3", "fbe"])[-1]
    assert rel_l2(solo[0], ref) <= TOL


@pytest.mark.parametrize("which", ["ark3-fbe N=8192 Nt=2000", "stiff N=8192 Nt=400"])
def test_full_length_workloads(env, which):
    # the two benchmarked IMEX workloads at their full length: rounding must not accumulate
    # past the bar (each linear stage is refined once, each Newton stage solved to rounding)
    if which.startswith("ark3"):
        prob, u0 = workloads.config_reacdiff_1d()
        prob = dict(prob, order=2, pairs=["ark3", "fbe"])
    else:
        prob, u0 = workloads.config_stiff_1d()
    check(env, prob, u0, prob["nt"])
