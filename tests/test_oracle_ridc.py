"""Pins for the full RIDC oracle against mathematics it must obey.

* order 1 is forward-backward Euler, whose Fourier-mode amplification is a closed form;
* linear periodic problems decouple into Fourier modes, so the vector oracle must equal the
  scalar RIDC recurrence of each mode;
* Theorem 1 (section III-D): level j (j+1 nodes, j corrections) is order j+1 -- measured
  against the exact semi-discrete solution, the exact logistic ODE solution, and by
  self-convergence for the nonlinear PDEs;
* centred periodic stencils conserve the grid sum;
* the pipelined schedule (section III-E) is a schedule only: it equals the level-sequential
  evaluation bit for bit, starts level j after j(j+1)/2 steps, and never reads an evicted value.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import Problem, fbe, rel_l2, ridc_pipelined, ridc_sequential


def _advdiff(n=128, nt=200, T=1.0, a=1.0, nu=0.1):
    return Problem(dim=1, bc="periodic", n=n, length=2 * math.pi, fe="advect", a=a, nu=nu,
                   dt=T / nt)


def _mode_eigs(p, k):
    lam_e = -1j * p.a * math.sin(k * p.h) / p.h
    lam_i = -(4 * p.nu / p.h**2) * math.sin(k * p.h / 2) ** 2
    return lam_e, lam_i


def test_order1_is_fbe_closed_form():
    p = _advdiff(n=64, nt=40)
    x = np.arange(p.n) * p.h
    k = 3
    u0 = np.sin(k * x)
    lam_e, lam_i = _mode_eigs(p, k)
    g = ((1 + p.dt * lam_e) / (1 - p.dt * lam_i)) ** 40
    expect = np.imag(g * np.exp(1j * k * x))
    out = ridc_sequential(p, u0, 40, 1)
    assert len(out) == 1
    np.testing.assert_allclose(out[0], expect, atol=1e-13)
    np.testing.assert_array_equal(fbe(p, u0, 40), out[0])


def _scalar_ridc(lam_e, lam_i, dt, nt, order):
    """Scalar complex RIDC-FBE of y' = (lam_e + lam_i) y, y(0) = 1, all levels' final values.

    Weights from a least-squares-free construction: solve the Vandermonde system for the
    rule exact on 1, t, ..., t^j over the interval (a different route than Lagrange products).
    """
    def weights(nodes, lo, hi):
        v = np.vander(np.asarray(nodes, float), increasing=True).T
        rhs = np.array([(hi ** (d + 1) - lo ** (d + 1)) / (d + 1) for d in range(len(nodes))])
        return np.linalg.solve(v, rhs)

    lam = lam_e + lam_i
    prev = [1.0 + 0j]
    for _ in range(nt):
        prev.append(prev[-1] * (1 + dt * lam_e) / (1 - dt * lam_i))
    finals = [prev[-1]]
    for j in range(1, order):
        cur = [1.0 + 0j]
        for n in range(nt):
            nodes = list(range(n + 1 - j, n + 2)) if n >= j - 1 else list(range(j + 1))
            w = weights(nodes, n, n + 1)
            quad = sum(wk * lam * prev[m] for wk, m in zip(w, nodes))
            rhs = cur[n] + dt * lam_e * cur[n] - dt * (lam_i * prev[n + 1] + lam_e * prev[n]) \
                + dt * quad
            cur.append(rhs / (1 - dt * lam_i))
        prev = cur
        finals.append(cur[-1])
    return finals


@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_vector_oracle_equals_scalar_mode_recurrence(order):
    p = _advdiff(n=48, nt=30, T=0.6, a=1.3, nu=0.05)
    x = np.arange(p.n) * p.h
    k = 2
    u0 = np.cos(k * x)
    lam_e, lam_i = _mode_eigs(p, k)
    g = _scalar_ridc(lam_e, lam_i, p.dt, 30, order)
    out = ridc_sequential(p, u0, 30, order)
    for j in range(order):
        np.testing.assert_allclose(out[j], np.real(g[j] * np.exp(1j * k * x)), atol=1e-12)


def test_levels_converge_at_orders_1_to_4_advdiff():
    """Theorem 1 on the N=128 advection-diffusion case: errors against exp((lam_e+lam_i) T)."""
    nts = [25, 50, 100, 200]
    errs = []
    for nt in nts:
        p = _advdiff(n=128, nt=nt)
        x = np.arange(p.n) * p.h
        lam_e, lam_i = _mode_eigs(p, 1)
        exact = np.imag(np.exp((lam_e + lam_i) * 1.0) * np.exp(1j * x))
        out = ridc_sequential(p, np.sin(x), nt, 4)
        errs.append([rel_l2(o, exact) for o in out])
    errs = np.array(errs)
    slopes = np.log2(errs[-2] / errs[-1])
    for j in range(4):
        assert abs(slopes[j] - (j + 1)) < 0.25, (j, slopes)
    # the fourth-order level is far more accurate than the predictor
    assert errs[-1, 3] < 1e-9 * errs[-1, 0] / 1e-4


def test_logistic_ode_limit_orders():
    """nu = 0: every point is u' = u(1-u), exact solution u0 e^t / (1 - u0 + u0 e^t)."""
    n = 16
    u0 = np.random.default_rng(11).uniform(0.05, 0.95, n)
    T = 1.0
    exact = u0 * math.e / (1 - u0 + u0 * math.e)
    errs = []
    nts = [20, 40, 80]
    for nt in nts:
        p = Problem(dim=1, bc="dirichlet", n=n, length=1.0, fe="logistic", a=0.0, nu=0.0,
                    dt=T / nt)
        out = ridc_sequential(p, u0, nt, 4)
        errs.append([rel_l2(o, exact) for o in out])
    errs = np.array(errs)
    slopes = np.log2(errs[-2] / errs[-1])
    for j in range(4):
        assert abs(slopes[j] - (j + 1)) < 0.3, slopes
    # u0 = 0 is a fixed point at every level
    p = Problem(dim=1, bc="dirichlet", n=4, length=1.0, fe="logistic", a=0.0, nu=0.0, dt=0.1)
    for o in ridc_sequential(p, np.zeros(4), 10, 4):
        np.testing.assert_array_equal(o, 0.0)


def _self_convergence_slopes(prob_fn, u0, nts, order):
    """Level-j error ~ C dt^(j+1): slopes of successive differences of the level's values."""
    vals = []
    for nt in nts:
        vals.append(ridc_sequential(prob_fn(nt), u0, nt, order))
    slopes = []
    for j in range(order):
        d1 = np.linalg.norm(vals[0][j] - vals[1][j])
        d2 = np.linalg.norm(vals[1][j] - vals[2][j])
        slopes.append(math.log2(d1 / d2))
    return slopes


def test_reaction_diffusion_1d_orders():
    # stiff diffusion delays the asymptotic regime (r = dt nu / h^2 must be small), so the
    # grid is coarse and the steps fine
    prob, u0 = workloads.config_reacdiff_1d(n=32, nt=1, order=4, nu=1e-3)

    def mk(nt):
        return Problem.from_dict(prob, nt=nt)

    slopes = _self_convergence_slopes(mk, u0, [40, 80, 160], 4)
    for j in range(4):
        assert abs(slopes[j] - (j + 1)) < 0.3, slopes


def test_reaction_diffusion_2d_orders():
    prob, u0 = workloads.config_reacdiff_2d(n=12, nt=1, order=3, nu=1e-2)

    def mk(nt):
        return Problem.from_dict(prob, nt=nt)

    slopes = _self_convergence_slopes(mk, u0, [32, 64, 128], 3)
    for j in range(3):
        assert abs(slopes[j] - (j + 1)) < 0.3, slopes


def test_periodic_mass_conservation():
    p = _advdiff(n=96, nt=50, a=0.7, nu=0.2)
    x = np.arange(p.n) * p.h
    u0 = 2 + np.sin(x) + 0.3 * np.cos(3 * x)          # nonzero mean, as in section IV-A
    mass0 = u0.sum()
    for o in ridc_sequential(p, u0, 50, 4):
        assert abs(o.sum() - mass0) < 1e-12 * abs(mass0)


@pytest.mark.parametrize("order,nt", [(1, 7), (2, 1), (3, 2), (4, 3), (4, 17), (5, 9), (6, 12)])
def test_pipelined_equals_sequential_bitwise(order, nt):
    prob, u0 = workloads.config_reacdiff_1d(n=32, nt=nt, order=order, nu=5e-3)
    p = Problem.from_dict(prob)
    seq = ridc_sequential(p, u0, nt, order)
    pipe = ridc_pipelined(p, u0, nt, order)
    for a, b in zip(seq, pipe):
        np.testing.assert_array_equal(a, b)


def test_pipeline_schedule_start_up_and_drain():
    order, nt = 4, 9
    prob, u0 = workloads.config_advdiff_1d(n=16, nt=nt, order=order)
    p = Problem.from_dict(prob)
    events = []
    ridc_pipelined(p, u0, nt, order, trace=lambda s, j, m: events.append((s, j, m)))
    first = {}
    for s, j, m in events:
        first.setdefault(j, s)
    # level j waits j(j+1)/2 steps, then computes t_1 (section III-E: node 2 waits 3 steps)
    assert [first[j] - 1 for j in range(order)] == [j * (j + 1) // 2 for j in range(order)]
    # every level computes every time step exactly once, in order
    for j in range(order):
        ms = [m for s, jj, m in events if jj == j]
        assert ms == list(range(1, nt + 1))
    # total pipeline steps: nt + P(P-1)/2 (the drain leaves lower levels idle at the end)
    assert max(s for s, _, _ in events) == nt + order * (order - 1) // 2
    # at steady state, level j-1 is one time step ahead plus j (Fig. 1: core 0 at t_{n+2}
    # while core 1 is at t_{n+1})
    by_step = {}
    for s, j, m in events:
        by_step.setdefault(s, {})[j] = m
    s = 8
    assert by_step[s][0] - by_step[s][1] == 1
    assert by_step[s][1] - by_step[s][2] == 2


def test_degenerate_cases():
    prob, u0 = workloads.config_advdiff_1d(n=16, nt=1)
    p = Problem.from_dict(prob)
    for o in ridc_pipelined(p, u0, 0, 4):                  # zero steps returns the data
        np.testing.assert_array_equal(o, u0)
    with pytest.raises(ValueError):
        ridc_pipelined(p, u0, 2, 4)                        # start-up needs nt >= order - 1
    with pytest.raises(ValueError):
        ridc_pipelined(p, u0, 5, 0)


@pytest.mark.parametrize("fe,a", [("advect", 1.3), ("upwind", 0.7), ("upwind", -0.9),
                                  ("none", 0.0)])
@pytest.mark.parametrize("order", [1, 2, 4, 5])
def test_fourier_space_evaluation_equals_vector_oracle(fe, a, order):
    """The mode-by-mode evaluation of a linear periodic problem (scalar steps in Fourier space)
    and the vector oracle (stencils, FFT solve with refinement) compute the same RIDC values by
    different routes; a dropped term, a wrong sign or a misplaced node in either would split
    them."""
    from oracle import ridc_linear_periodic
    p = Problem(dim=1, bc="periodic", n=40, length=2 * math.pi, fe=fe, a=a, nu=0.07, dt=0.02)
    u0 = workloads.fourier_modes_1d(40, np.random.default_rng(3)) + 0.4
    nt = 23
    vec = ridc_sequential(p, u0, nt, order)
    modal = ridc_linear_periodic(p, u0, nt, order)
    for j in range(order):
        assert rel_l2(modal[j], vec[j]) < 1e-13, (j, rel_l2(modal[j], vec[j]))


def test_fourier_space_evaluation_closed_forms():
    """Order 1 on one mode is the forward-backward Euler amplification; the zero mode (the grid
    sum) is conserved by every level."""
    from oracle import periodic_mode_symbols, ridc_linear_periodic
    p = _advdiff(n=64, nt=40)
    x = np.arange(p.n) * p.h
    out = ridc_linear_periodic(p, np.sin(3 * x), 40, 1)[0]
    lam_e, lam_i = _mode_eigs(p, 3)
    g = ((1 + p.dt * lam_e) / (1 - p.dt * lam_i)) ** 40
    np.testing.assert_allclose(out, np.imag(g * np.exp(3j * x)), atol=1e-13)
    le, li = periodic_mode_symbols(p)
    assert abs(le[3] - lam_e) < 1e-12 and abs(li[3] - lam_i) < 1e-12
    u0 = 2 + np.cos(2 * x)
    for o in ridc_linear_periodic(p, u0, 40, 4):
        assert abs(o.sum() - u0.sum()) < 1e-12 * u0.sum()
    with pytest.raises(ValueError):
        periodic_mode_symbols(Problem(dim=1, bc="periodic", n=8, length=1.0, fe="burgers",
                                      a=0.0, nu=0.1, dt=0.1))
