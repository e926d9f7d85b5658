"""GPU parity on the paper's own workloads (section IV): first-order upwind advection-diffusion
with restarts (section III-E) and viscous Burgers with the numerical flux of section IV-B, at
the paper's resolution dx = 1/1000."""
import numpy as np
import pytest

import workloads
from oracle import Problem, rel_l2, ridc_pipelined, ridc_restarted

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1209_4297_amd import ridc
    return torch, ridc


@pytest.mark.parametrize("segments", [1, 10])
def test_paper_advection_diffusion(env, segments):
    torch, ridc = env
    prob, u0 = workloads.config_paper_advdiff()            # N=1000, T=40, 4000 steps
    print(f"case: upwind advection-diffusion N=1000 Nt=4000 segments={segments}", flush=True)
    s = ridc.Ridc(prob)
    out = s.integrate_restarts(torch.tensor(u0, dtype=torch.float64, device="cuda"),
                               prob["nt"], segments).cpu().numpy()
    s.close()
    ref = ridc_restarted(Problem.from_dict(prob), u0, prob["nt"], 4, segments)
    err = rel_l2(out, ref)
    print(f"  rel L2 vs oracle {err:.3e}", flush=True)
    assert err <= 1e-12
    # mass (the mean, 2) is conserved by upwind and centred diffusion stencils
    assert abs(out.mean() - 2.0) < 1e-12


@pytest.mark.parametrize("nt", [1000, 2000])
def test_paper_burgers(env, nt):
    torch, ridc = env
    prob, u0 = workloads.config_paper_burgers(nt=nt)       # N=999 interior, eps=1e-3, T=1
    print(f"case: Burgers N=999 Nt={nt}", flush=True)
    s = ridc.Ridc(prob)
    lv = torch.empty(4 * prob["n"], dtype=torch.float64, device="cuda")
    out = s.integrate(torch.tensor(u0, dtype=torch.float64, device="cuda"), nt,
                      levels=lv).cpu().numpy()
    s.close()
    ref = ridc_pipelined(Problem.from_dict(prob), u0, nt, 4)
    lvs = lv.cpu().numpy().reshape(4, -1)
    for j in range(4):
        err = rel_l2(lvs[j], ref[j])
        print(f"  level {j}: rel L2 {err:.3e}", flush=True)
        assert err <= 1e-12
    np.testing.assert_array_equal(out, lvs[-1])


def test_paper_burgers_beyond_cfl_is_reported(env):
    """dt = 5e-3 with dx = 1e-3 puts the explicit flux far beyond its stability limit: the
    integration blows up, and the library reports it instead of returning garbage."""
    torch, ridc = env
    prob, u0 = workloads.config_paper_burgers(nt=200)
    s = ridc.Ridc(prob)
    with pytest.raises(ridc.RidcError) as ei:
        s.integrate(torch.tensor(u0, dtype=torch.float64, device="cuda"), 200)
    assert ei.value.code == ridc.RIDC_E_NONFINITE
    s.close()
