"""GPU parity of the 2D RIDC path (FP64 right-hand side + fast-diagonalisation transforms on
the matrix cores) against the FP64 oracle.

FP64: relative L2 <= 1e-12 per level.  Reduced precision (FP32 or split-BF16 transforms with
one FP64 residual refinement): a bound per level index (TOL), about 100 x the largest error
measured for that level over these cases, the full-size case and the served requests (FP32:
4.2e-15, 7.4e-16, 7.0e-16, 5.1e-16 for levels 0-3; split BF16: 1.5e-11, 2.7e-12, 3.2e-14,
3.1e-15), with the RIDC4 top level capped at 1.5e-13 = 0.1 x the discretisation error of the
1024^2 workload (1.5e-12, Richardson), the bar at which a reduced-precision result counts as
matched.  The lower levels of the split-BF16 path sit far above the top level: each level's
increment is solved to about 1e-11 of itself, and a level's error against the oracle is small
next to its own discretisation error (level 0 is first order).  Every bound holds for the
relative L2 error and for the largest pointwise error relative to the largest value.
"""
import math
import os
import sys

import numpy as np
import pytest

import workloads
from oracle import Problem, rel_l2, ridc_pipelined

pytestmark = pytest.mark.gpu

from tolerances import TOL64, tol_of  # noqa: E402  (per-level bounds, derivation above)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "reacdiff2d_n1024_nt500.npz")


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1209_4297_amd import ridc
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, ridc


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run2d(env, prob, u0, prec="fp64", nt=None, levels=True):
    torch, ridc = env
    nt = prob["nt"] if nt is None else nt
    s = ridc.Ridc(prob, dt=prob["T"] / prob["nt"], prec=prec)
    x0 = torch.tensor(np.asarray(u0), dtype=torch.float64, device="cuda").reshape(-1)
    uT = torch.empty_like(x0)
    lv = (torch.empty(prob["order"] * x0.numel(), dtype=torch.float64, device="cuda")
          if levels else None)
    s.integrate(x0, nt, uT, lv)
    n = prob["n"]
    out = uT.cpu().numpy().reshape(n, n)
    lvs = lv.cpu().numpy().reshape(prob["order"], n, n) if levels else None
    s.close()
    return out, lvs


def errs(got, ref):
    """(relative L2, largest pointwise difference over the largest reference value)."""
    return rel_l2(got, ref), float(np.abs(got - ref).max() / np.abs(ref).max())


def oracle2d(prob, u0, nt=None):
    nt = prob["nt"] if nt is None else nt
    return ridc_pipelined(Problem.from_dict(prob), u0, nt, prob["order"])


# n = 256 and 768 (multiples of 256) run the passes that exchange prefolded planes; 768 also
# has a contraction (n/2 = 384) that is not a power of two
@pytest.mark.parametrize("n,nt,order", [(64, 40, 4), (96, 30, 4), (256, 20, 4), (160, 12, 3),
                                        (32, 8, 1), (64, 6, 6), (32, 20, 8),
                                        (192, 10, 4), (768, 6, 4)])
def test_fp64_parity(env, n, nt, order):
    prob, u0 = workloads.config_reacdiff_2d(n=n, nt=nt, order=order, T=nt * 2e-3, nu=1e-3)
    _say(f"case: 2D fp64 n={n} nt={nt} P={order}")
    ref = oracle2d(prob, u0)
    top, lvs = run2d(env, prob, u0)
    for j in range(order):
        err, emax = errs(lvs[j], ref[j])
        _say(f"  level {j}: rel L2 {err:.3e}, max {emax:.3e}")
        assert err <= TOL64 and emax <= TOL64, (j, err, emax)
    np.testing.assert_array_equal(top, lvs[-1])


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("n,nt", [(128, 40), (96, 20), (192, 10), (256, 12), (768, 6)])
def test_mixed_precision_parity(env, prec, n, nt):
    prob, u0 = workloads.config_reacdiff_2d(n=n, nt=nt, order=4, T=nt * 2e-3, nu=1e-3)
    _say(f"case: 2D {prec} n={n} nt={nt}")
    ref = oracle2d(prob, u0)
    top, lvs = run2d(env, prob, u0, prec=prec)
    for j in range(4):
        err, emax = errs(lvs[j], ref[j])
        _say(f"  level {j}: rel L2 {err:.3e}, max {emax:.3e}")
        assert err <= tol_of(prec, j) and emax <= tol_of(prec, j), (j, err, emax)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_kernel_time_leaves_the_integration_unchanged(env, prec):
    """ridc_kernel_time runs the next step's stages again and again around its timed pass; the
    level rings and the handle's position must come out as they went in, so an integration
    timed half-way ends bitwise where an untimed one does."""
    torch, ridc = env
    prob, u0 = workloads.config_reacdiff_2d(n=256, nt=12, order=4, T=0.024, nu=1e-3)
    _say(f"case: 2D {prec} kernel_time mid-integration")
    x0 = torch.tensor(u0.reshape(-1), device="cuda")

    def run(timed):
        s = ridc.Ridc(prob, prec=prec)
        s.begin(x0, prob["nt"])
        ridc.advance([s], 8)
        if timed:
            us, flops = s.kernel_time(3)
            assert us > 0 and flops > 0
        ridc.advance([s], s.remaining())
        uT = torch.empty_like(x0)
        s.read(uT)
        s.sync()
        s.close()
        return uT.cpu().numpy()

    assert np.array_equal(run(True), run(False))


def test_largest_side_sine_mode_closed_form(env):
    """n = 16384, the largest 2D side (a vector is 2 GiB, so every address is 64-bit).  With no
    explicit term a discrete sine mode is an eigenvector of the 5-point Laplacian, and order 1
    (IMEX Euler, section II) divides it by 1 + dt nu mu each step, mu = (4/h^2)(sin^2(p pi h/2)
    + sin^2(q pi h/2)).  Sampled against that closed form.  Rounding bound: four passes of FP64
    sums of n/2 products, about 4 (n/2) eps = 3.6e-12 of the unit amplitude; checked at 1e-11.
    p != q, so a transposed axis would fail."""
    torch, ridc = env
    n, nt, p, q, nu, T = 16384, 2, 3, 5, 0.1, 0.02
    _say(f"case: 2D fp64 sine mode ({p},{q}) n={n} nt={nt} order 1")
    prob = dict(dim=2, bc="dirichlet", n=n, length=1.0, fe="none", a=0.0, nu=nu, T=T, nt=nt,
                order=1)
    h = 1.0 / (n + 1)
    idx = torch.arange(1, n + 1, dtype=torch.float64, device="cuda")
    x0 = torch.outer(torch.sin(math.pi * q * h * idx), torch.sin(math.pi * p * h * idx))
    x0 = x0.reshape(-1)                                   # row iy (mode q), column ix (mode p)
    uT = torch.empty_like(x0)
    s = ridc.Ridc(prob, dt=T / nt)
    s.integrate(x0, nt, uT)
    s.close()
    mu = 4.0 / h**2 * (math.sin(p * math.pi * h / 2) ** 2 + math.sin(q * math.pi * h / 2) ** 2)
    amp = (1.0 + (T / nt) * nu * mu) ** (-nt)
    rng = np.random.default_rng(16384)
    iy = np.concatenate([rng.integers(0, n, 2000), [0, 0, n - 1, n - 1, n // 2]])
    ix = np.concatenate([rng.integers(0, n, 2000), [0, n - 1, 0, n - 1, n // 2]])
    sel = torch.tensor(iy * n + ix, dtype=torch.int64, device="cuda")
    got = uT[sel].cpu().numpy()
    del x0, uT
    want = amp * np.sin(math.pi * q * h * (iy + 1)) * np.sin(math.pi * p * h * (ix + 1))
    err = float(np.max(np.abs(got - want)))
    _say(f"  amplitude {amp:.6f}, max abs error {err:.3e}")
    assert err <= 1e-11


def test_zero_steps_and_fixed_point(env):
    torch, ridc = env
    prob, u0 = workloads.config_reacdiff_2d(n=64, nt=10, order=4)
    top, _ = run2d(env, prob, u0, nt=0)
    np.testing.assert_array_equal(top, u0)
    # u = 0 is a fixed point of u(1-u) with zero Dirichlet data
    z = np.zeros((64, 64))
    top, lvs = run2d(env, prob, z)
    assert np.all(top == 0.0) and np.all(lvs == 0.0)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_batch_bitwise_equals_solo_2d(env, prec):
    torch, ridc = env
    cases = [workloads.config_reacdiff_2d(n=n, nt=nt, order=o, T=nt * 2e-3, nu=1e-3, seed=100 + n)
             for n, nt, o in [(64, 12, 4), (128, 9, 2), (64, 7, 3)]]
    solvers, u0s, uTs, solo = [], [], [], []
    for prob, u0 in cases:
        s = ridc.Ridc(prob, prec=prec)
        x0 = torch.tensor(u0.reshape(-1), dtype=torch.float64, device="cuda")
        solo.append(s.integrate(x0, prob["nt"]).cpu().numpy())
        solvers.append(s)
        u0s.append(x0)
        uTs.append(torch.empty_like(x0))
    ridc.integrate_batch(solvers, u0s, [p["nt"] for p, _ in cases], uTs)
    torch.cuda.synchronize()
    for i in range(len(cases)):
        np.testing.assert_array_equal(uTs[i].cpu().numpy(), solo[i])
    for s in solvers:
        s.close()


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="reference samples not generated")
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_full_size_against_reference_samples(env, prec):
    """1024^2, Nt=500, order 4: the launch configuration of the full workload, checked at the
    oracle's 4096 stored sample points, norms and sums (tests/golden)."""
    ref = np.load(GOLDEN)
    prob, u0 = workloads.config_reacdiff_2d()
    _say(f"case: 2D {prec} full n=1024 nt=500")
    top, lvs = run2d(env, prob, u0, prec=prec)
    idx = ref["idx"]
    for j in range(4):
        tol = tol_of(prec, j)
        flat = lvs[j].reshape(-1)
        err, emax = errs(flat[idx], ref["samples"][j])
        nerr = abs(np.linalg.norm(flat) - ref["norms"][j]) / ref["norms"][j]
        _say(f"  level {j}: sampled rel L2 {err:.3e}, max {emax:.3e}, norm rel diff {nerr:.3e}")
        assert err <= tol and emax <= tol and nerr <= tol, (j, err, emax, nerr)
    # the result (top level): matched when within 0.1 x the RIDC4 discretisation error
    tol = tol_of(prec, 3)
    err, emax = errs(top[::8, ::8], ref["top_sub8"])
    _say(f"  top level on the 128^2 sub-grid: rel L2 {err:.3e}, max {emax:.3e}")
    assert err <= tol and emax <= tol


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_stencil_time_bytes(env, prec):
    """The right-hand-side kernel's algorithmic bytes: every level reads its value and (j > 0)
    its j+1 window vectors, and writes the FP64 right-hand side plus a 4-byte copy in the
    reduced-precision paths."""
    torch, ridc = env
    n, P = 128, 4
    prob, u0 = workloads.config_reacdiff_2d(n=n, nt=12, order=P, T=0.02)
    s = ridc.Ridc(prob, prec=prec)
    s.begin(torch.tensor(u0.reshape(-1), dtype=torch.float64, device="cuda"), 12)
    with pytest.raises(ridc.RidcError):                    # start-up step
        s.stencil_time(3)
    ridc.advance([s], P * (P - 1) // 2)
    us, nbytes = s.stencil_time(5)
    lo = 0 if prec == "fp64" else 4
    want = sum(8 * (1 if j == 0 else j + 2) + 8 + lo for j in range(P)) * n * n
    assert us > 0 and nbytes == want
    s.sync()
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_graph_and_direct_launch_agree_2d(env, prec, monkeypatch):
    torch, _ = env
    prob, u0 = workloads.config_reacdiff_2d(n=128, nt=20, order=4, T=0.04, nu=1e-3)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        a, _ = run2d(env, prob, u0, prec, levels=False)       # captured and replayed
    direct, _ = run2d(env, prob, u0, prec, levels=False)      # null stream
    monkeypatch.setenv("RIDC_GRAPH", "0")
    with torch.cuda.stream(side):
        c, _ = run2d(env, prob, u0, prec, levels=False)
    np.testing.assert_array_equal(a, direct)
    np.testing.assert_array_equal(a, c)


def test_batch_mixing_1d_and_2d(env):
    """One batched integration over 1D and 2D instances (and two precisions) gives every
    instance the bits of its solo integration."""
    torch, ridc = env
    cases = [(workloads.config_reacdiff_2d(n=128, nt=16, order=3, T=0.03, nu=1e-3), "fp64"),
             (workloads.config_reacdiff_2d(n=96, nt=12, order=4, T=0.02, nu=1e-3), "fp32"),
             (workloads.config_reacdiff_1d(n=700, nt=30, order=4, T=0.02), "fp64"),
             (workloads.config_advdiff_1d(n=300, nt=25, order=2), "fp64")]
    solvers, u0s, uTs, solo = [], [], [], []
    for (prob, u0), prec in cases:
        s = ridc.Ridc(prob, prec=prec)
        x0 = torch.tensor(np.asarray(u0).reshape(-1), dtype=torch.float64, device="cuda")
        solo.append(s.integrate(x0, prob["nt"]).cpu().numpy())
        solvers.append(s)
        u0s.append(x0)
        uTs.append(torch.empty_like(x0))
    ridc.integrate_batch(solvers, u0s, [p["nt"] for (p, _), _ in cases], uTs)
    torch.cuda.synchronize()
    for s, uT, ref in zip(solvers, uTs, solo):
        s.sync()
        np.testing.assert_array_equal(uT.cpu().numpy(), ref)
        s.close()
