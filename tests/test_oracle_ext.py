"""Pins for the extension oracle (``oracle.ridc_ext``) against mathematics it must obey.

ARK-based RIDC (section II pairs, section III-D Thm 2):
* the printed pairs satisfy the Runge-Kutta order conditions of their stated order (exact
  rationals; a mistyped entry breaks one), and alone converge at that order on a coupled
  problem whose stiff and non-stiff parts do not commute;
* written as a two-stage pair, forward-backward Euler reproduces RIDC-FBE (the pinned base
  oracle) to rounding, whatever the level;
* Thm 2: level j converges at order ``p_0 + ... + p_j`` against the exact semi-discrete Fourier
  mode solution and the exact logistic ODE solution;
* the widened window's interpolation and partial-interval weights are exact on polynomials of
  degree ``S-1`` and reduce to the paper's weights at ``c = 1``, ``S = j+1``;
* the lagged pipeline equals the level-by-level evaluation bit for bit and reads no evicted
  value; with Euler levels it is the paper's schedule.

Newton solve of a nonlinear stiff term (section III-B):
* the single-unknown implicit equation is a quadratic with a closed-form root;
* quadratic convergence; the result satisfies its equation to rounding;
* a zero reaction rate reproduces the linear solve; the Jacobian matches finite differences;
* RIDC with the nonlinear stiff term converges at orders 1..4 against the exact logistic ODE
  solution (no diffusion) and by self-convergence with diffusion.
"""
import dataclasses
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import workloads
from oracle import (Problem, corrector_weights, f_implicit, periodic_mode_symbols, rel_l2,
                    ridc_pipelined, ridc_sequential, solve_implicit)
from oracle import ridc_ext as X


# ---------------------------------------------------------------------------------------------
# the pairs of section II
# ---------------------------------------------------------------------------------------------
def _conds(A, b):
    """Order conditions of one Runge-Kutta tableau up to order 4 (butcher trees)."""
    s = len(b)
    c = [sum(A[i]) for i in range(s)]
    Ac = [sum(A[i][k] * c[k] for k in range(s)) for i in range(s)]
    Ac2 = [sum(A[i][k] * c[k] ** 2 for k in range(s)) for i in range(s)]
    AAc = [sum(A[i][k] * Ac[k] for k in range(s)) for i in range(s)]
    dot = lambda u, v: sum(x * y for x, y in zip(u, v))  # noqa: E731
    return {
        1: [(sum(b), Fraction(1))],
        2: [(dot(b, c), Fraction(1, 2))],
        3: [(dot(b, [x * x for x in c]), Fraction(1, 3)), (dot(b, Ac), Fraction(1, 6))],
        4: [(dot(b, [x ** 3 for x in c]), Fraction(1, 4)),
            (dot(b, [x * y for x, y in zip(c, Ac)]), Fraction(1, 8)),
            (dot(b, Ac2), Fraction(1, 12)), (dot(b, AAc), Fraction(1, 24))],
    }


@pytest.mark.parametrize("tab", [X.FBE, X.ARK3, X.ARK4])
def test_pairs_meet_their_order_conditions(tab):
    for A, b in ((tab.AS, tab.bS), (tab.AN, tab.bN)):
        conds = _conds(A, b)
        for order in range(1, tab.order + 1):
            for got, want in conds[order]:
                assert got == want, (tab.name, order)
    # one stage-time vector for both parts, a strictly lower explicit part, stiffly accurate
    assert tab.c == tuple(sum(r) for r in tab.AN)
    assert all(tab.AN[i][k] == 0 for i in range(tab.s) for k in range(i, tab.s))
    assert all(tab.AS[i][k] == 0 for i in range(tab.s) for k in range(i + 1, tab.s))
    assert tab.stiffly_accurate()


def test_ark3_coupling_conditions():
    # order 3 of the pair also needs the mixed conditions b^X A^Y c = 1/6
    t = X.ARK3
    c = t.c
    for b in (t.bS, t.bN):
        for A in (t.AS, t.AN):
            Ac = [sum(A[i][k] * c[k] for k in range(t.s)) for i in range(t.s)]
            assert sum(x * y for x, y in zip(b, Ac)) == Fraction(1, 6)


@pytest.mark.parametrize("tab,slope", [(X.ARK3, 3), (X.ARK4, 4)])
def test_pairs_alone_converge_at_their_order(tab, slope):
    # logistic reaction (explicit) with diffusion (implicit) on a Dirichlet grid: the two parts
    # do not commute; errors against a reference with 8x smaller steps of the same pair (mild
    # diffusion, dt nu / h^2 <= 0.03: stiffer runs show the usual order reduction at these steps)
    n = 24
    u0 = workloads.bumps_1d(n, seed=7) + 0.2

    def run(nt):
        p = Problem(dim=1, bc="dirichlet", n=n, length=1.0, fe="logistic", a=0.0, nu=0.002,
                    dt=0.5 / nt)
        return X.ark_integrate(p, tab, u0, nt)

    ref = run(640)
    errs = [rel_l2(run(nt), ref) for nt in (20, 40, 80)]
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert slope - 0.15 < slopes[-1] < slope + 0.3, (errs, slopes)


# ---------------------------------------------------------------------------------------------
# windows and weights
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("S", [2, 3, 4, 5, 7])
@pytest.mark.parametrize("c", [Fraction(0), Fraction(1, 3), Fraction(1, 2), Fraction(1)])
def test_stage_weights_exact_on_polynomials(S, c):
    for n in range(0, S + 2):
        nodes = X.window_nodes(n, S)
        assert len(nodes) == S and nodes == sorted(nodes)
        assert n in nodes and n + 1 in nodes
        L = X.stage_interp_weights(n, S, c)
        Q = X.stage_quad_weights(n, S, c)
        t = Fraction(n) + c
        for d in range(S):
            assert sum(l * Fraction(m) ** d for l, m in zip(L, nodes)) == t ** d
            exact = (t ** (d + 1) - Fraction(n) ** (d + 1)) / (d + 1)
            assert sum(q * Fraction(m) ** d for q, m in zip(Q, nodes)) == exact
        # degree S is not reproduced in general (the window is no wider than needed)
        if 0 < c < 1:
            assert sum(l * Fraction(m) ** S for l, m in zip(L, nodes)) != t ** S


@pytest.mark.parametrize("j", [1, 2, 3, 4])
def test_full_step_weights_are_the_papers(j):
    for n in range(0, j + 3):
        nodes, w = corrector_weights(n, j)
        got = X.stage_quad_weights(n, j + 1, 1)
        mine = X.window_nodes(n, j + 1)
        assert sorted(nodes) == mine
        by_node = dict(zip(nodes, w))
        for m, q in zip(mine, got):
            assert float(q) == by_node[m]


# ---------------------------------------------------------------------------------------------
# ARK-based RIDC
# ---------------------------------------------------------------------------------------------
def _advdiff(n=32, nt=40, T=1.0, a=1.0, nu=0.1):
    return Problem(dim=1, bc="periodic", n=n, length=2 * math.pi, fe="advect", a=a, nu=nu,
                   dt=T / nt)


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_euler_pairs_reproduce_ridc_fbe(P):
    p = _advdiff(n=32, nt=30)
    u0 = workloads.fourier_modes_1d(32, np.random.default_rng(3))
    base = ridc_sequential(p, u0, 30, P)
    ext = X.ridc_ark_sequential(p, u0, 30, ["fbe"] * P)
    for a, b in zip(ext, base):
        assert rel_l2(a, b) <= 1e-14
    # Dirichlet and a nonlinear explicit term too
    q = Problem(dim=1, bc="dirichlet", n=40, length=1.0, fe="logistic", a=0.0, nu=1e-3,
                dt=1.0 / 25)
    v0 = workloads.bumps_1d(40, seed=11)
    for a, b in zip(X.ridc_ark_sequential(q, v0, 25, ["fbe"] * P), ridc_sequential(q, v0, 25, P)):
        assert rel_l2(a, b) <= 1e-14


def _mode_exact(p, u0, T):
    lam_e, lam_i = periodic_mode_symbols(p)
    return np.real(np.fft.ifft(np.fft.fft(u0) * np.exp((lam_e + lam_i) * T)))


@pytest.mark.parametrize("schemes", [["ark3", "fbe", "fbe"], ["ark4", "fbe"], ["fbe", "ark3"],
                                     ["ark3", "ark3"]])
def test_thm2_level_orders_on_fourier_modes(schemes):
    orders = X.ark_level_orders(schemes)
    errs = []
    nts = (20, 40, 80)
    for nt in nts:
        p = _advdiff(n=32, nt=nt)
        u0 = np.sin(np.arange(32) * p.h)
        ex = _mode_exact(p, u0, 1.0)
        errs.append([rel_l2(f, ex) for f in X.ridc_ark_sequential(p, u0, nt, schemes)])
    errs = np.array(errs)
    for j, q in enumerate(orders):
        slope = math.log2(errs[-2, j] / errs[-1, j])
        assert q - 0.2 < slope < q + 0.4, (schemes, j, errs[:, j], slope)


def test_thm2_level_orders_on_logistic_ode():
    # no diffusion: every grid point is y' = y(1-y), exact y0 e^t / (1 - y0 + y0 e^t)
    y0 = np.array([0.1, 0.3, 0.5, 0.8])
    exact = y0 * math.e / (1 - y0 + y0 * math.e)
    errs = []
    for nt in (10, 20, 40):
        p = Problem(dim=1, bc="dirichlet", n=4, length=1.0, fe="logistic", a=0.0, nu=0.0,
                    dt=1.0 / nt)
        errs.append([rel_l2(f, exact) for f in X.ridc_ark_sequential(p, y0, nt,
                                                                      ["ark3", "fbe"])])
    errs = np.array(errs)
    for j, q in enumerate([3, 4]):
        slope = math.log2(errs[-2, j] / errs[-1, j])
        assert q - 0.25 < slope < q + 0.5, (j, errs[:, j])


@pytest.mark.parametrize("schemes", [["ark3", "fbe", "fbe"], ["fbe", "ark4"], ["ark4", "ark3"]])
def test_pipeline_equals_sequential_and_keeps_its_window(schemes):
    p = _advdiff(n=24, nt=16)
    u0 = workloads.fourier_modes_1d(24, np.random.default_rng(5))
    seen = []
    pipe = X.ridc_ark_pipelined(p, u0, 16, schemes, trace=lambda s, j, m: seen.append((s, j, m)))
    seq = X.ridc_ark_sequential(p, u0, 16, schemes)
    for a, b in zip(pipe, seq):
        np.testing.assert_array_equal(a, b)
    d = X.ark_delays(schemes)
    assert all(s == m + d[j] for s, j, m in seen)
    assert max(s for s, _, _ in seen) == 16 + d[-1]


def test_euler_schedule_is_the_papers():
    for P in range(1, 7):
        assert X.ark_delays(["fbe"] * P) == [j * (j + 1) // 2 for j in range(P)]
        assert X.ark_ring_slots(["fbe"] * P) == [2 * j + 3 if j < P - 1 else 2 for j in range(P)]
    # one slot fewer than needed makes the pipeline read an evicted value
    p = _advdiff(n=16, nt=12)
    u0 = np.sin(np.arange(16) * p.h)
    orig = X.ark_ring_slots
    try:
        X.ark_ring_slots = lambda s: [k - 1 if k > 2 else k for k in orig(s)]
        with pytest.raises(KeyError):
            X.ridc_ark_pipelined(p, u0, 12, ["ark3", "fbe"])
    finally:
        X.ark_ring_slots = orig


def test_short_integrations_are_rejected():
    p = _advdiff(n=16, nt=4)
    with pytest.raises(ValueError):
        X.ridc_ark_sequential(p, np.zeros(16), 2, ["ark3", "fbe"])     # S_1 - 1 = 3 > 2
    out = X.ridc_ark_sequential(p, np.ones(16), 0, ["ark3", "fbe"])
    np.testing.assert_array_equal(out[-1], np.ones(16))


# ---------------------------------------------------------------------------------------------
# Newton for a nonlinear stiff term
# ---------------------------------------------------------------------------------------------
def _stiff(n=48, kappa=20.0, fi="logistic", nu=1e-3, dt=0.01, fe="none"):
    return Problem(dim=1, bc="dirichlet", n=n, length=1.0, fe=fe, a=0.0, nu=nu, dt=dt, fi=fi,
                   kappa=kappa)


@pytest.mark.parametrize("fi", ["logistic", "cubic"])
def test_single_unknown_newton_is_the_quadratic_root(fi):
    p = _stiff(n=1, kappa=30.0, fi=fi, nu=0.2)
    tau, rhs = 0.05, np.array([0.7])
    y = X.newton_solve(p, rhs, tau, guess=rhs.copy())
    r = tau * p.nu / p.h ** 2
    k = tau * p.kappa
    if fi == "logistic":
        # y (1 + 2r - k) + k y^2 = rhs
        A, B, C = k, 1 + 2 * r - k, -rhs[0]
        root = (-B + math.sqrt(B * B - 4 * A * C)) / (2 * A)
        assert abs(y[0] - root) <= 4e-16 * abs(root)
    else:
        # y (1 + 2r - k) + k y^3 = rhs: the one real root (discriminant of a depressed cubic)
        roots = np.roots([k, 0.0, 1 + 2 * r - k, -rhs[0]])
        real = [z.real for z in roots if abs(z.imag) < 1e-12]
        root = min(real, key=lambda z: abs(z - rhs[0]))
        assert abs(y[0] - root) <= 1e-14


def test_newton_converges_quadratically_to_the_root():
    p = _stiff(n=64, kappa=40.0, fi="cubic", nu=2e-3, dt=0.02)
    rng = np.random.default_rng(2)
    rhs = rng.uniform(-1, 1, 64)
    hist = []
    y = X.newton_solve(p, rhs, p.dt, guess=np.zeros(64), history=hist)
    res = rhs - (y - p.dt * X.f_stiff(p, y))
    assert np.max(np.abs(res)) <= 1e-14
    assert len(hist) >= 3
    big = [h for h in hist if h > 1e-9]
    for a, b in zip(big, big[1:]):
        assert b <= 10 * a * a + 1e-15, hist


def test_newton_without_reaction_is_the_linear_solve():
    p = _stiff(n=50, kappa=0.0, fi="logistic", nu=5e-3, dt=0.03)
    rhs = workloads.bumps_1d(50, seed=4)
    y = X.newton_solve(p, rhs, p.dt, guess=np.zeros(50))
    lin = solve_implicit(dataclasses.replace(p, fi="diffusion"), rhs)
    assert np.max(np.abs(y - lin)) <= 1e-15


def test_newton_jacobian_matches_finite_differences():
    p = _stiff(n=12, kappa=7.0, fi="logistic", nu=0.01, dt=0.05)
    y = np.linspace(-0.3, 1.2, 12)
    G = lambda v: v - p.dt * X.f_stiff(p, v)  # noqa: E731
    r = p.dt * p.nu / p.h ** 2
    J = (np.diag(1 + 2 * r - p.dt * X.reaction_prime(p, y)) + np.diag(-r * np.ones(11), 1)
         + np.diag(-r * np.ones(11), -1))
    eps = 1e-6
    Jfd = np.column_stack([(G(y + eps * e) - G(y - eps * e)) / (2 * eps) for e in np.eye(12)])
    np.testing.assert_allclose(J, Jfd, atol=1e-7)
    # and the diffusion part is the base oracle's stencil
    np.testing.assert_allclose(X.f_stiff(dataclasses.replace(p, kappa=0.0), y),
                               f_implicit(p, y), rtol=0, atol=0)


@pytest.mark.parametrize("fi", ["logistic", "cubic"])
def test_ridc_with_nonlinear_stiff_term_orders_on_the_ode(fi):
    # nu = 0: each point is y' = kappa g(y), all of it implicit
    kappa = 3.0
    y0 = np.array([0.1, 0.3, 0.5, 0.8])
    if fi == "logistic":
        ek = math.exp(kappa)
        exact = y0 * ek / (1 - y0 + y0 * ek)
    else:
        # y' = k (y - y^3): y^2 = 1 / (1 + (1/y0^2 - 1) e^{-2k})
        exact = 1 / np.sqrt(1 + (1 / y0 ** 2 - 1) * math.exp(-2 * kappa))
    errs = []
    for nt in (40, 80, 160):
        p = Problem(dim=1, bc="dirichlet", n=4, length=1.0, fe="none", a=0.0, nu=0.0,
                    dt=1.0 / nt, fi=fi, kappa=kappa)
        errs.append([rel_l2(f, exact) for f in X.ridc_ark_sequential(p, y0, nt, ["fbe"] * 4)])
    errs = np.array(errs)
    for j in range(4):
        slope = math.log2(errs[-2, j] / errs[-1, j])
        assert j + 1 - 0.2 < slope < j + 1 + 0.5, (j, errs[:, j])


def test_ridc_with_nonlinear_stiff_term_self_converges():
    u0 = workloads.bumps_1d(32, seed=9)

    def top(nt):
        p = _stiff(n=32, kappa=5.0, fi="logistic", nu=2e-3, dt=0.5 / nt, fe="none")
        return X.ridc_ark_sequential(p, u0, nt, ["fbe"] * 4)

    a, b, c = top(20), top(40), top(80)
    for j in range(4):
        e1, e2 = rel_l2(a[j], b[j]), rel_l2(b[j], c[j])
        assert j + 1 - 0.3 < math.log2(e1 / e2) < j + 1 + 0.6, (j, e1, e2)


def test_linear_stiff_term_paths_agree():
    # the generic stage engine with a linear stiff term uses the base oracle's linear solve;
    # written as a reaction of rate 0 it goes through Newton: the same values to rounding
    u0 = workloads.bumps_1d(40, seed=12)
    p = _stiff(n=40, kappa=0.0, fi="logistic", nu=1e-3, dt=1.0 / 30, fe="logistic")
    q = dataclasses.replace(p, fi="diffusion")
    for a, b in zip(X.ridc_ark_sequential(p, u0, 30, ["ark3", "fbe"]),
                    X.ridc_ark_sequential(q, u0, 30, ["ark3", "fbe"])):
        assert rel_l2(a, b) <= 1e-14
