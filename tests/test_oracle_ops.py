"""Pins for the oracle's operators and implicit solvers against closed forms and dense algebra.

Fourier and sine modes are eigenvectors of the centred difference operators with known
eigenvalues; the solvers are checked against ``numpy.linalg.solve`` on matrices assembled here
entry by entry from the textbook stencils (section IV: centred differences for the diffusion).
"""
import math

import numpy as np
import pytest

from oracle import Problem, f_explicit, f_implicit, solve_implicit


def _prob(dim, bc, n, fe="none", a=0.0, nu=0.3, dt=0.01, length=None):
    if length is None:
        length = 2 * math.pi if bc == "periodic" else 1.0
    return Problem(dim=dim, bc=bc, n=n, length=length, fe=fe, a=a, nu=nu, dt=dt)


@pytest.mark.parametrize("k", [1, 3, 7])
def test_periodic_operators_on_fourier_modes(k):
    p = _prob(1, "periodic", 32, fe="advect", a=1.7, nu=0.3)
    x = np.arange(p.n) * p.h
    c, s = np.cos(k * x), np.sin(k * x)
    lam_i = -(4 * p.nu / p.h**2) * math.sin(k * p.h / 2) ** 2
    np.testing.assert_allclose(f_implicit(p, c), lam_i * c, atol=1e-12)
    # -a D0 e^{ikx} = -i a sin(kh)/h e^{ikx}: cos -> a sin(kh)/h sin, sin -> -a sin(kh)/h cos
    g = p.a * math.sin(k * p.h) / p.h
    np.testing.assert_allclose(f_explicit(p, c), g * s, atol=1e-12)
    np.testing.assert_allclose(f_explicit(p, s), -g * c, atol=1e-12)


@pytest.mark.parametrize("k", [1, 2, 5])
def test_dirichlet_operators_on_sine_modes(k):
    p = _prob(1, "dirichlet", 24, nu=0.02)
    x = np.arange(1, p.n + 1) * p.h
    v = np.sin(k * math.pi * x)
    lam = -(4 * p.nu / p.h**2) * math.sin(k * math.pi * p.h / 2) ** 2
    np.testing.assert_allclose(f_implicit(p, v), lam * v, atol=1e-11)
    # 2D: product of sine modes, eigenvalue is the sum
    p2 = _prob(2, "dirichlet", 12, nu=0.05)
    x2 = np.arange(1, p2.n + 1) * p2.h
    v2 = np.outer(np.sin(2 * math.pi * x2), np.sin(k * math.pi * x2))     # [iy, ix]
    lam2 = -(4 * p2.nu / p2.h**2) * (math.sin(2 * math.pi * p2.h / 2) ** 2
                                     + math.sin(k * math.pi * p2.h / 2) ** 2)
    np.testing.assert_allclose(f_implicit(p2, v2), lam2 * v2, atol=1e-11)


def test_logistic_is_pointwise():
    p = _prob(1, "dirichlet", 5, fe="logistic")
    u = np.array([0.0, 1.0, 0.5, 2.0, -1.0])
    np.testing.assert_array_equal(f_explicit(p, u), [0.0, 0.0, 0.25, -2.0, -2.0])


def _dense_1d(n, r, periodic):
    m = np.zeros((n, n))
    for i in range(n):
        m[i, i] = 1 + 2 * r
        for d in (-1, 1):
            k = i + d
            if periodic:
                m[i, k % n] += -r
            elif 0 <= k < n:
                m[i, k] += -r
    return m


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("dt", [1e-3, 0.37, 50.0])
def test_1d_solve_matches_dense(bc, dt):
    p = _prob(1, bc, 8, nu=0.11, dt=dt)
    r = p.dt * p.nu / p.h**2
    rhs = np.random.default_rng(3).standard_normal(8)
    x = solve_implicit(p, rhs)
    ref = np.linalg.solve(_dense_1d(8, r, bc == "periodic"), rhs)
    np.testing.assert_allclose(x, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("dt", [1e-3, 0.9, 40.0])
def test_2d_solve_matches_dense_kronecker(dt):
    n = 8
    p = _prob(2, "dirichlet", n, nu=0.07, dt=dt)
    r = p.dt * p.nu / p.h**2
    # 64 x 64 matrix of I - dt nu (Dxx + Dyy), assembled point by point (row-major [iy, ix])
    m = np.zeros((n * n, n * n))
    for iy in range(n):
        for ix in range(n):
            row = iy * n + ix
            m[row, row] = 1 + 4 * r
            for dy, dx in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                jy, jx = iy + dy, ix + dx
                if 0 <= jy < n and 0 <= jx < n:
                    m[row, jy * n + jx] = -r
    rhs = np.random.default_rng(5).standard_normal((n, n))
    x = solve_implicit(p, rhs)
    ref = np.linalg.solve(m, rhs.reshape(-1)).reshape(n, n)
    np.testing.assert_allclose(x, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


def test_solve_on_modes_closed_form():
    p = _prob(1, "periodic", 64, nu=0.2, dt=0.05)
    x = np.arange(p.n) * p.h
    for k in (0, 1, 9, 32):
        v = np.cos(k * x)
        eig = 1 + p.dt * (4 * p.nu / p.h**2) * math.sin(k * p.h / 2) ** 2
        np.testing.assert_allclose(solve_implicit(p, v), v / eig, atol=1e-13)
    p2 = _prob(2, "dirichlet", 16, nu=0.01, dt=0.3)
    x2 = np.arange(1, 17) * p2.h
    v2 = np.outer(np.sin(3 * math.pi * x2), np.sin(5 * math.pi * x2))
    eig2 = 1 + p2.dt * (4 * p2.nu / p2.h**2) * (math.sin(3 * math.pi * p2.h / 2) ** 2
                                                + math.sin(5 * math.pi * p2.h / 2) ** 2)
    np.testing.assert_allclose(solve_implicit(p2, v2), v2 / eig2, atol=1e-13)


def _thomas_longdouble(r, rhs):
    """Tridiagonal (Dirichlet) solve of (1+2r) x_i - r x_{i-1} - r x_{i+1} = rhs_i in long
    double (64-bit mantissa), by the Thomas algorithm."""
    n = len(rhs)
    ld = np.longdouble
    b = ld(1) + 2 * ld(r)
    a = -ld(r)
    cp = [ld(0)] * n
    dp = [ld(0)] * n
    cp[0] = a / b
    dp[0] = ld(rhs[0]) / b
    for i in range(1, n):
        den = b - a * cp[i - 1]
        cp[i] = a / den
        dp[i] = (ld(rhs[i]) - a * dp[i - 1]) / den
    x = [ld(0)] * n
    x[-1] = dp[-1]
    for i in range(n - 2, -1, -1):
        x[i] = dp[i] - cp[i] * x[i + 1]
    return np.array(x, dtype=np.longdouble)


@pytest.mark.parametrize("r,bound", [(0.3, 1e-15), (33.6, 1.5e-15), (2.5e3, 5e-15)])
def test_dirichlet_solve_is_accurate_to_rounding(r, bound):
    """The refined oracle solve sits within a few ulps (growing slowly with the condition
    number 1 + 4r) of a long-double Thomas solve."""
    n = 1024
    p = _prob(1, "dirichlet", n, nu=1.0, dt=r / (n + 1) ** 2)
    assert abs(p.dt * p.nu / p.h**2 - r) < 1e-9 * r
    rhs = np.random.default_rng(7).uniform(0.0, 1.0, n)
    x = solve_implicit(p, rhs)
    ref = _thomas_longdouble(p.dt * p.nu / p.h**2, rhs)
    err = np.max(np.abs(x - ref.astype(np.float64))) / np.max(np.abs(ref.astype(np.float64)))
    assert err < bound, err
