"""The allocation-free 1D entry point (ridc_integrate_noalloc) against ridc_integrate.

ridc_integrate_noalloc runs the same level-step kernels as a handle's integration, with its
rings and tables in the library's fixed per-GPU array instead of a handle's device pool, so its
result must be bitwise the handle's.  Two calls in a row, the second on a smaller system, check
that nothing of the first call's contents of the shared array leaks into the second.  The
second call is also held to the FP64 oracle at the parity bar (rel. L2 <= 1e-12).
"""
import ctypes
import sys

import numpy as np
import pytest

import workloads
from oracle import Problem, rel_l2, ridc_pipelined

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1209_4297_amd import ridc
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, ridc


def _noalloc(env, prob, x0, nt):
    """One call through the C ABI, with a non-finite flag; returns (result, flag)."""
    torch, ridc = env
    uT = torch.full_like(x0, float("nan"))
    flag = torch.zeros(1, dtype=torch.int32, device=x0.device)
    p = ridc.make_problem(prob)
    stream = torch.cuda.current_stream()
    rc = ridc.lib().ridc_integrate_noalloc(ctypes.byref(p), ctypes.c_void_p(stream.cuda_stream),
                                           ctypes.c_void_p(x0.data_ptr()), int(nt),
                                           ctypes.c_void_p(uT.data_ptr()),
                                           ctypes.c_void_p(flag.data_ptr()))
    assert rc == 0, ridc.lib().ridc_last_error().decode()
    torch.cuda.synchronize()
    return uT.cpu().numpy(), int(flag.item())


def _handle(env, prob, x0, nt):
    torch, ridc = env
    s = ridc.Ridc(prob)
    out = s.integrate(x0, nt).cpu().numpy()
    s.close()
    return out


def test_two_calls_match_the_handle_path(env):
    torch, ridc = env
    # first call: the N = 8192 Dirichlet reaction-diffusion system, RIDC4, 300 steps
    prob1, u1 = workloads.config_reacdiff_1d(nt=2000)
    x1 = torch.tensor(u1, dtype=torch.float64, device="cuda")
    _say("case: noalloc call 1, 1D dirichlet n=8192 P=4 nt=300 logistic")
    a1, f1 = _noalloc(env, prob1, x1, 300)
    b1 = _handle(env, prob1, x1, 300)
    assert f1 == 0
    assert np.isfinite(a1).all()
    assert np.array_equal(a1, b1), f"max diff {np.abs(a1 - b1).max():.3e}"
    # second call, smaller: the paper's upwind advection-diffusion on 1000 periodic points,
    # order 3, 120 steps
    prob2, u2 = workloads.config_paper_advdiff(n=1000, nt=4000, order=3)
    x2 = torch.tensor(u2, dtype=torch.float64, device="cuda")
    _say("case: noalloc call 2, 1D periodic n=1000 P=3 nt=120 upwind")
    a2, f2 = _noalloc(env, prob2, x2, 120)
    b2 = _handle(env, prob2, x2, 120)
    assert f2 == 0
    assert np.array_equal(a2, b2), f"max diff {np.abs(a2 - b2).max():.3e}"
    p2 = Problem.from_dict(prob2)
    ref = ridc_pipelined(p2, u2, 120, 3)[-1]
    err = rel_l2(a2, ref)
    _say(f"noalloc call 2 vs oracle: rel L2 {err:.3e}")
    assert err <= 1e-12


def test_zero_steps_and_rejections(env):
    torch, ridc = env
    prob, u0 = workloads.config_advdiff_1d(n=128, nt=200, order=4)
    x0 = torch.tensor(u0, dtype=torch.float64, device="cuda")
    _say("case: noalloc nsteps=0 and oversize rejection")
    out, flag = _noalloc(env, prob, x0, 0)
    assert flag == 0 and np.array_equal(out, u0)
    big = dict(prob, n=1 << 20)          # 17 ring slots of 8 MiB: above the 32 MiB array
    xb = torch.zeros(1 << 20, dtype=torch.float64, device="cuda")
    with pytest.raises(ridc.RidcError) as e:
        ridc.integrate_noalloc(big, xb, 10)
    assert e.value.code == ridc.RIDC_E_UNSUPPORTED
