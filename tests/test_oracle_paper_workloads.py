"""Pins for the oracle parts that reproduce the paper's own workloads (section IV):
first-order upwind advection, the Burgers numerical flux, and restarts (section III-E)."""
import math

import numpy as np
import pytest

import workloads
from oracle import (Problem, f_explicit, rel_l2, ridc_pipelined, ridc_restarted,
                    ridc_sequential)


def _p(fe, n, a=0.0, bc="periodic", length=2 * math.pi, nu=0.0, dt=0.01):
    return Problem(dim=1, bc=bc, n=n, length=length, fe=fe, a=a, nu=nu, dt=dt)


@pytest.mark.parametrize("a", [0.7, -0.3])
@pytest.mark.parametrize("k", [1, 5])
def test_upwind_on_fourier_modes(a, k):
    p = _p("upwind", 40, a=a)
    x = np.arange(p.n) * p.h
    v = np.exp(1j * k * x)
    # backward difference for a >= 0, forward difference for a < 0
    lam = -a * (1 - np.exp(-1j * k * p.h)) / p.h if a >= 0 else -a * (np.exp(1j * k * p.h) - 1) / p.h
    np.testing.assert_allclose(f_explicit(p, np.real(v)), np.real(lam * v), atol=1e-12)
    np.testing.assert_allclose(f_explicit(p, np.imag(v)), np.imag(lam * v), atol=1e-12)


def test_burgers_flux_consistency_and_conservation():
    errs = []
    for n in (64, 128, 256):
        p = _p("burgers", n)
        x = np.arange(n) * p.h
        u = np.sin(x) + 0.5
        # -(u^2/2)_x = -u u_x
        errs.append(np.abs(f_explicit(p, u) + u * np.cos(x)).max())
        assert abs(f_explicit(p, u).sum()) < 1e-12 * n      # telescoping flux differences
    assert abs(math.log2(errs[0] / errs[1]) - 2) < 0.1
    assert abs(math.log2(errs[1] / errs[2]) - 2) < 0.1
    # Dirichlet: zero ghosts, u = 0 gives zero flux; a constant state has zero interior flux
    pd = _p("burgers", 10, bc="dirichlet", length=1.0)
    np.testing.assert_array_equal(f_explicit(pd, np.zeros(10)), 0.0)
    f = f_explicit(pd, np.ones(10))
    np.testing.assert_array_equal(f[1:-1], 0.0)


def test_upwind_ridc_orders_against_semi_discrete_solution():
    prob, _ = workloads.config_paper_advdiff(n=64, nt=1, T=2.0)
    errs = []
    for nt in (40, 80, 160):
        p = Problem.from_dict(prob, nt=nt)
        x = np.arange(p.n) * p.h
        k = 2 * math.pi
        lam = -p.a * (np.exp(1j * k * p.h) - 1) / p.h - (4 * p.nu / p.h**2) * math.sin(k * p.h / 2) ** 2
        exact = 2 + np.imag(np.exp(lam * prob["T"]) * np.exp(1j * k * x))
        u0 = 2 + np.sin(k * x)
        errs.append([rel_l2(o, exact) for o in ridc_sequential(p, u0, nt, 4)])
    errs = np.array(errs)
    slopes = np.log2(errs[-2] / errs[-1])
    for j in range(4):
        assert abs(slopes[j] - (j + 1)) < 0.3, slopes


def test_burgers_ridc_self_convergence():
    prob, u0 = workloads.config_paper_burgers(n=63, T=0.1)
    prob["nu"] = 1e-2
    vals = [ridc_sequential(Problem.from_dict(prob, nt=nt), u0, nt, 4) for nt in (40, 80, 160)]
    for j in range(4):
        d1 = np.linalg.norm(vals[0][j] - vals[1][j])
        d2 = np.linalg.norm(vals[1][j] - vals[2][j])
        assert abs(math.log2(d1 / d2) - (j + 1)) < 0.35, (j, math.log2(d1 / d2))


def test_restarts():
    prob, u0 = workloads.config_paper_advdiff(n=200, nt=1000, T=10.0)
    p = Problem.from_dict(prob)
    # one segment is plain RIDC
    np.testing.assert_array_equal(ridc_restarted(p, u0, 1000, 4, 1),
                                  ridc_pipelined(p, u0, 1000, 4)[-1])
    # section III-E / the restart figure: the error falls as the number of restarts grows
    x = np.arange(p.n) * p.h
    k = 2 * math.pi
    lam = -p.a * (np.exp(1j * k * p.h) - 1) / p.h - (4 * p.nu / p.h**2) * math.sin(k * p.h / 2) ** 2
    exact = 2 + np.imag(np.exp(lam * 10.0) * np.exp(1j * k * x))
    errs = [rel_l2(ridc_restarted(p, u0, 1000, 4, s), exact) for s in (1, 2, 5, 10)]
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    with pytest.raises(ValueError):
        ridc_restarted(p, u0, 1000, 4, 3)
