"""GPU parity of the 1D RIDC path (fused level-step + PCR in LDS) against the FP64 oracle.

Bar: relative L2 <= 1e-12 per level against the oracle on the same seeded inputs, and the largest
pointwise difference <= 1e-12 of the largest value (both FP64; the GPU contracts to FMA and solves
by PCR, the oracle solves by FFT or banded LU, so only rounding differs).  Tiling, batching, graph replay and repetition must not change a single bit.
"""
import math
import sys

import numpy as np
import pytest

import workloads
from oracle import Problem, rel_l2, ridc_pipelined

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


def run_gpu(env, prob, u0, nt=None, levels=True, prec="fp64", tile=None):
    torch, ridc = env
    nt = prob["nt"] if nt is None else nt
    dt = prob["T"] / prob["nt"]
    s = ridc.Ridc(prob, dt=dt, prec=prec)
    if tile is not None:
        s.set_tile(*tile)
    x0 = torch.tensor(np.asarray(u0), dtype=torch.float64, device="cuda").reshape(-1)
    uT = torch.empty_like(x0)
    lv = torch.empty(prob["order"] * x0.numel(), dtype=torch.float64, device="cuda") if levels else None
    s.integrate(x0, nt, uT, lv)
    out = uT.cpu().numpy()
    lvs = lv.cpu().numpy().reshape(prob["order"], -1) if levels else None
    s.close()
    return out, lvs


def check_against_oracle(env, prob, u0, nt=None, tol=TOL):
    nt = prob["nt"] if nt is None else nt
    _say(f"case: {prob['dim']}D {prob['bc']} n={prob['n']} P={prob['order']} nt={nt} fe={prob['fe']}")
    p = Problem(dim=prob["dim"], bc=prob["bc"], n=prob["n"], length=prob["length"], fe=prob["fe"],
                a=prob.get("a", 0.0), nu=prob["nu"], dt=prob["T"] / prob["nt"])
    ref = ridc_pipelined(p, np.asarray(u0), nt, prob["order"])
    top, lvs = run_gpu(env, prob, u0, nt)
    for j in range(prob["order"]):
        scale = np.abs(ref[j]).max()
        err = rel_l2(lvs[j], ref[j]) if scale > 0 else np.abs(lvs[j]).max()
        emax = np.abs(lvs[j] - ref[j]).max() / (scale if scale > 0 else 1.0)
        assert err <= tol and emax <= tol, (j, err, emax)
    np.testing.assert_array_equal(top, lvs[-1])
    return ref, top


def test_advdiff_n128_full(env):
    prob, u0 = workloads.config_advdiff_1d()
    ref, top = check_against_oracle(env, prob, u0)
    # and it is a fourth-order accurate answer to the semi-discrete problem (sanity)
    h = 2 * math.pi / 128
    lam = -1j * math.sin(h) / h - (4 * 0.1 / h**2) * math.sin(h / 2) ** 2
    x = np.arange(128) * h
    exact = np.imag(np.exp(lam) * np.exp(1j * x))
    assert rel_l2(top, exact) < 1e-9


def test_reacdiff_n8192_full(env):
    prob, u0 = workloads.config_reacdiff_1d()
    check_against_oracle(env, prob, u0)


def test_reacdiff_chunked_ragged(env):
    # n = 3000 with r = 4.5: few PCR stages, so the default tiling cuts it into chunks (128
    # rows, the last one ragged)
    prob, u0 = workloads.config_reacdiff_1d(n=3000, nt=400, T=0.2)
    check_against_oracle(env, prob, u0)


@pytest.mark.parametrize("order", [6, 8])
def test_long_system_default_tiling_high_orders(env, order):
    # orders 6 and 8 on a chunked system: the default tiling takes 1024 threads up to order 6
    # and 256 above, with chunks of at least 128 rows
    prob, u0 = workloads.config_reacdiff_1d(n=2304, nt=24, order=order, T=0.012)
    check_against_oracle(env, prob, u0)


@pytest.mark.parametrize("order", [1, 2, 3, 5, 6])
def test_orders(env, order):
    prob, u0 = workloads.config_advdiff_1d(n=96, nt=40, order=order, T=0.4)
    check_against_oracle(env, prob, u0)


@pytest.mark.parametrize("order", [2, 4])
def test_minimum_steps(env, order):
    prob, u0 = workloads.config_reacdiff_1d(n=64, nt=order - 1, order=order, T=0.01)
    check_against_oracle(env, prob, u0)


def test_zero_steps_returns_u0(env):
    prob, u0 = workloads.config_advdiff_1d(n=32, nt=10)
    top, lvs = run_gpu(env, prob, u0, nt=0)
    np.testing.assert_array_equal(top, u0)
    for j in range(prob["order"]):
        np.testing.assert_array_equal(lvs[j], u0)


@pytest.mark.parametrize("bc,n,fe,nu,T,nt", [
    ("periodic", 2, "advect", 0.5, 1.0, 20),      # smallest periodic cycle
    ("dirichlet", 2, "logistic", 0.1, 1.0, 20),
    ("periodic", 100, "advect", 0.05, 1.0, 50),   # non-power-of-two cycle, threshold plan
    ("periodic", 64, "none", 5.0, 1.0, 10),       # huge r: exact plan down to the 2x2 end
    ("dirichlet", 777, "advect", 1e-2, 0.5, 60),  # advection with zero ghosts
    ("dirichlet", 5000, "none", 1e-3, 1.0, 20),   # r = 1250, wrap mode on the odd extension
    ("periodic", 4096, "advect", 1e-3, 0.25, 200),
])
def test_edge_grids(env, bc, n, fe, nu, T, nt):
    length = 2 * math.pi if bc == "periodic" else 1.0
    x = workloads.grid_points(bc, n, length)
    u0 = np.sin(x) + 0.5 * np.cos(3 * x) + (0.3 if bc == "periodic" else 0.0)
    if bc == "dirichlet":
        u0 = np.clip(x * (length - x) * 3, 0, 1) + 0.1 * np.sin(7 * x)
    prob = dict(dim=1, bc=bc, n=n, length=length, fe=fe, a=0.8, nu=nu, T=T, nt=nt, order=4)
    check_against_oracle(env, prob, u0)


def test_largest_system_sine_mode_closed_form(env):
    """n = 2^28, the largest 1D system (a vector is 2 GiB; 2^21 chunks per level).  Periodic,
    no explicit term: sin(k x) is an eigenvector of the second difference, and order 1 (IMEX
    Euler, section II) divides it by 1 + 4 r sin^2(kh/2) each step, r = nu dt / h^2.  k = n/8,
    so kh = pi/4 and the mode repeats every 8 rows (built from i mod 8, exact at any i).
    Sampled against the closed form; the solve's rounding does not grow with n (a few PCR
    stages), checked at 1e-12."""
    torch, ridc = env
    n, nt, r, T = 1 << 28, 2, 0.5, 0.02
    L = 2 * math.pi
    h, dt = L / n, T / nt
    prob = dict(dim=1, bc="periodic", n=n, length=L, fe="none", a=0.0, nu=r * h * h / dt, T=T,
                nt=nt, order=1)
    _say(f"case: 1D sine mode n=2^28 nt={nt} order 1 r={r}")
    i8 = torch.arange(n, dtype=torch.int64, device="cuda") % 8
    x0 = torch.sin((math.pi / 4) * i8.to(torch.float64))
    del i8
    uT = torch.empty_like(x0)
    s = ridc.Ridc(prob, dt=dt)
    s.integrate(x0, nt, uT)
    s.close()
    amp = (1.0 + 4.0 * r * math.sin(math.pi / 8) ** 2) ** (-nt)
    rng = np.random.default_rng(1 << 28)
    idx = np.concatenate([rng.integers(0, n, 4000), [0, 1, n // 2, n - 2, n - 1]])
    got = uT[torch.tensor(idx, dtype=torch.int64, device="cuda")].cpu().numpy()
    del x0, uT
    want = amp * np.sin((math.pi / 4) * (idx % 8))
    err = float(np.max(np.abs(got - want)))
    _say(f"  amplitude {amp:.6f}, max abs error {err:.3e}")
    assert err <= 1e-12


def test_batch_bitwise_equals_solo(env):
    torch, ridc = env
    cases = workloads.config_batched_1d(count=12, nt=120, T=0.03)
    solvers, u0s, uTs, solo = [], [], [], []
    for prob, u0 in cases:
        s = ridc.Ridc(prob)
        x0 = torch.tensor(u0, dtype=torch.float64, device="cuda")
        solo.append(s.integrate(x0, prob["nt"]).cpu().numpy())
        solvers.append(s)
        u0s.append(x0)
        uTs.append(torch.empty_like(x0))
    # mix in a Dirichlet reaction-diffusion instance of another order
    prob2, u02 = workloads.config_reacdiff_1d(n=2500, nt=90, order=3, T=0.05)
    s2 = ridc.Ridc(prob2)
    x2 = torch.tensor(u02, dtype=torch.float64, device="cuda")
    solo.append(s2.integrate(x2, prob2["nt"]).cpu().numpy())
    solvers.append(s2)
    u0s.append(x2)
    uTs.append(torch.empty_like(x2))
    nts = [p["nt"] for p, _ in cases] + [prob2["nt"]]
    ridc.integrate_batch(solvers, u0s, nts, uTs)
    torch.cuda.synchronize()
    for i, uT in enumerate(uTs):
        np.testing.assert_array_equal(uT.cpu().numpy(), solo[i])
    # stepping interface with uneven chunks gives the same bits too
    for s, x0, prob_nt in zip(solvers, u0s, nts):
        s.begin(x0, prob_nt)
    while any(s.remaining() > 0 for s in solvers):
        ridc.advance(solvers, 37)
    for i, s in enumerate(solvers):
        out = torch.empty_like(u0s[i])
        s.read(out)
        s.sync()
        np.testing.assert_array_equal(out.cpu().numpy(), solo[i])
    for s in solvers:
        s.close()


@pytest.mark.parametrize("policy", [(256, 0), (512, 512), (1024, 768), (256, 1024), (1024, 0),
                                    "tuned"])
def test_batch_tilings_are_bitwise_identical(env, policy):
    """Grouped launches cut long cycles into chunks, change the thread count, and use the
    kernels specialised for the batch's highest order; none of it may change a bit."""
    torch, ridc = env
    cases = workloads.config_batched_1d(count=10, nt=60, T=0.015)
    prob2, u02 = workloads.config_reacdiff_1d(n=2500, nt=50, order=3, T=0.03)
    prob3, _ = workloads.config_advdiff_1d(n=512, nt=40, order=7, T=0.05)   # levels up to 6
    u03 = workloads.fourier_modes_1d(512, np.random.default_rng(7))
    cases = cases + [(prob2, u02), (prob3, u03)]
    solvers, u0s, uTs, solo = [], [], [], []
    for prob, u0 in cases:
        s = ridc.Ridc(prob)
        x0 = torch.tensor(u0, dtype=torch.float64, device="cuda")
        solo.append(s.integrate(x0, prob["nt"]).cpu().numpy())
        solvers.append(s)
        u0s.append(x0)
        uTs.append(torch.empty_like(x0))
    nts = [p["nt"] for p, _ in cases]
    try:
        if policy == "tuned":
            t, r = ridc.autotune_batch(solvers)
            _say(f"batch tiling chosen: threads {t}, rows {r}")
        else:
            ridc.set_batch_tile(*policy)
        ridc.integrate_batch(solvers, u0s, nts, uTs)
        torch.cuda.synchronize()
        for i, uT in enumerate(uTs):
            np.testing.assert_array_equal(uT.cpu().numpy(), solo[i])
    finally:
        ridc.set_batch_tile(256, 0)
        for s in solvers:
            s.close()


def test_graph_and_direct_launch_agree(env, monkeypatch):
    """On a stream of its own an integration is captured in a HIP graph and replayed (a second
    call replays the cached graph); it must give the bits of direct launches, on that stream
    with capture switched off and on the null stream."""
    torch, _ = env
    prob, u0 = workloads.config_reacdiff_1d(n=2048, nt=300, T=0.15)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        a, _ = run_gpu(env, prob, u0, levels=False)          # captured
        b, _ = run_gpu(env, prob, u0, levels=False)
    direct, _ = run_gpu(env, prob, u0, levels=False)          # null stream: direct launches
    monkeypatch.setenv("RIDC_GRAPH", "0")
    with torch.cuda.stream(side):
        c, _ = run_gpu(env, prob, u0, levels=False)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(a, c)
    np.testing.assert_array_equal(a, direct)


def test_graph_replay_of_one_handle(env):
    """One handle integrating twice on its own stream replays its cached graph."""
    torch, ridc = env
    prob, u0 = workloads.config_advdiff_1d(n=256, nt=60)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        s = ridc.Ridc(prob)
        x0 = torch.tensor(u0, dtype=torch.float64, device="cuda")
        first = s.integrate(x0, 60).clone()
        second = s.integrate(x0, 60)
        side.synchronize()
        s.close()
    alone, _ = run_gpu(env, prob, u0, levels=False)
    np.testing.assert_array_equal(first.cpu().numpy(), alone)
    np.testing.assert_array_equal(second.cpu().numpy(), alone)


def test_nonfinite_is_reported(env):
    torch, ridc = env
    prob, u0 = workloads.config_advdiff_1d(n=64, nt=20)
    u0 = u0.copy()
    u0[5] = np.nan
    s = ridc.Ridc(prob)
    x0 = torch.tensor(u0, dtype=torch.float64, device="cuda")
    with pytest.raises(ridc.RidcError) as ei:
        s.integrate(x0, 20)
    assert ei.value.code == ridc.RIDC_E_NONFINITE
    # the handle stays usable
    out = s.integrate(torch.tensor(workloads.config_advdiff_1d(n=64, nt=20)[1], dtype=torch.float64,
                                   device="cuda"), 20)
    assert torch.isfinite(out).all()
    s.close()


def test_batch_reports_nonfinite_per_instance(env):
    """A batched integration flags the instance whose result is not finite, and only it."""
    torch, ridc = env
    cases = [workloads.config_advdiff_1d(n=n, nt=20) for n in (64, 256, 100)]
    solvers = [ridc.Ridc(p) for p, _ in cases]
    u0s = [torch.tensor(u, dtype=torch.float64, device="cuda") for _, u in cases]
    u0s[1][17] = float("nan")
    uTs = [torch.empty_like(x) for x in u0s]
    ridc.integrate_batch(solvers, u0s, [20, 20, 20], uTs)
    solvers[0].sync()
    solvers[2].sync()
    with pytest.raises(ridc.RidcError) as ei:
        solvers[1].sync()
    assert ei.value.code == ridc.RIDC_E_NONFINITE
    for i in (0, 2):
        alone = solvers[i].integrate(u0s[i], 20)
        assert torch.equal(alone, uTs[i])
    for s in solvers:
        s.close()


def test_state_errors(env):
    torch, ridc = env
    prob, u0 = workloads.config_advdiff_1d(n=64, nt=20)
    s = ridc.Ridc(prob)
    x0 = torch.tensor(u0, dtype=torch.float64, device="cuda")
    out = torch.empty_like(x0)
    with pytest.raises(ridc.RidcError) as ei:
        s.read(out)
    assert ei.value.code == ridc.RIDC_E_STATE
    s.begin(x0, 20)
    assert s.remaining() == 20 + 6
    with pytest.raises(ridc.RidcError):
        s.read(out)
    with pytest.raises(ridc.RidcError) as ei:
        s.begin(x0, 2)                      # below order - 1
    assert ei.value.code == ridc.RIDC_E_INVAL
    s.close()


def test_tilings_are_bitwise_identical(env):
    torch, ridc = env
    prob, u0 = workloads.config_reacdiff_1d(n=2048, nt=120, T=0.06)
    x0 = torch.tensor(u0, dtype=torch.float64, device="cuda")
    s = ridc.Ridc(prob)
    outs = []
    tiles = [(256, 0, 0), (1024, 0, 1), (256, 1024, 0), (512, 512, 1), (128, 2048, 0),
             (1024, 256, 1), (512, 0, 2), (1024, 0, 2)]
    for threads, rows, flags in tiles:
        try:
            s.set_tile(threads, rows, flags)
        except ridc.RidcError:
            continue
        _say(f"tile threads={threads} rows={rows} flags={flags}")
        outs.append(s.integrate(x0, prob["nt"]).cpu().numpy())
    assert len(outs) >= 6
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])
    t, r, f = s.autotune()
    _say(f"autotuned: threads={t} rows={r} flags={f}")
    np.testing.assert_array_equal(s.integrate(x0, prob["nt"]).cpu().numpy(), outs[0])
    s.close()


@pytest.mark.parametrize("bc,n,order,nt", [("periodic", 1000, 4, 50), ("dirichlet", 999, 4, 40),
                                           ("periodic", 2048, 4, 30), ("dirichlet", 3000, 3, 30),
                                           ("periodic", 128, 1, 20), ("dirichlet", 64, 6, 25),
                                           ("periodic", 4096, 2, 40), ("periodic", 128, 4, 60),
                                           ("dirichlet", 200, 4, 30)])
def test_fused_integration_equals_per_step_kernel(env, bc, n, order, nt):
    """Systems that fit one CU run their whole integration in one workgroup; the result is
    bitwise that of one launch per pipeline step."""
    torch, ridc = env
    length = 2 * math.pi if bc == "periodic" else 1.0
    x = workloads.grid_points(bc, n, length)
    u0 = np.sin(x) + 0.25 * np.cos(5 * x) if bc == "periodic" else x * (length - x) * 4
    prob = dict(dim=1, bc=bc, n=n, length=length, fe="advect" if bc == "periodic" else "logistic",
                a=0.6, nu=2e-3, T=0.05, nt=nt, order=order)
    _say(f"case: fused vs per-step {bc} n={n} P={order} nt={nt}")
    step, lv_s = run_gpu(env, prob, u0)
    fused, lv_f = run_gpu(env, prob, u0, tile=(512, 0, 2))
    if order <= 4:
        fused2, _ = run_gpu(env, prob, u0, tile=(1024, 0, 2))
        np.testing.assert_array_equal(fused2, step)
    else:                                   # the 1024-thread workgroup covers orders <= 4
        with pytest.raises(ridc.RidcError) as ei:
            run_gpu(env, prob, u0, tile=(1024, 0, 2))
        assert ei.value.code == ridc.RIDC_E_INVAL
    np.testing.assert_array_equal(fused, step)
    np.testing.assert_array_equal(lv_f, lv_s)
    p = Problem(dim=1, bc=bc, n=n, length=length, fe=prob["fe"], a=0.6, nu=2e-3, dt=0.05 / nt)
    ref = ridc_pipelined(p, u0, nt, order)[-1]
    assert rel_l2(fused, ref) <= TOL


def test_batch_kernel_time_and_its_errors(env):
    torch, ridc = env
    cases = workloads.config_batched_1d(count=6, nt=40, T=0.01)
    solvers = [ridc.Ridc(p) for p, _ in cases]
    x0s = [torch.tensor(u, dtype=torch.float64, device="cuda") for _, u in cases]
    try:
        with pytest.raises(ridc.RidcError) as ei:          # not armed
            ridc.batch_kernel_time(solvers, 5)
        assert ei.value.code == ridc.RIDC_E_STATE
        for s, x0, (p, _) in zip(solvers, x0s, cases):
            s.begin(x0, p["nt"])
        with pytest.raises(ridc.RidcError) as ei:          # start-up step: not every level active
            ridc.batch_kernel_time(solvers, 5)
        assert ei.value.code == ridc.RIDC_E_STATE
        ridc.advance(solvers, 6)
        us, nbytes = ridc.batch_kernel_time(solvers, 10)
        assert us > 0
        assert nbytes == sum(s.step_cost()[0] for s in solvers)
        # the handles did not advance: the integration finishes with the solo bits
        while any(s.remaining() > 0 for s in solvers):
            ridc.advance(solvers, 64)
        for s, x0, (p, _) in zip(solvers, x0s, cases):
            out = torch.empty_like(x0)
            s.read(out)
            s.sync()
            solo = ridc.Ridc(p)
            np.testing.assert_array_equal(out.cpu().numpy(), solo.integrate(x0, p["nt"]).cpu().numpy())
            solo.close()
    finally:
        for s in solvers:
            s.close()


def test_stencil_time_is_2d_only(env):
    torch, ridc = env
    prob, u0 = workloads.config_advdiff_1d(n=64, nt=20)
    s = ridc.Ridc(prob)
    s.begin(torch.tensor(u0, dtype=torch.float64, device="cuda"), 20)
    with pytest.raises(ridc.RidcError) as ei:
        s.stencil_time(5)
    assert ei.value.code == ridc.RIDC_E_UNSUPPORTED
    s.close()
