"""Seeded synthetic workloads for semi-implicit RIDC.

This module only describes problems and draws their initial data.  It holds none of the
integrator's arithmetic (no operators, weights, solves or time stepping), so that the CPU
oracle and the HIP path can both take their inputs from here without sharing any of the
method.  Every draw uses ``numpy.random.default_rng(seed)`` and takes its values in the order
written below, so a workload is fixed by its seed.

Problem dictionaries use these keys:

``dim``      1 or 2
``bc``       ``"periodic"`` or ``"dirichlet"``
``n``        unknowns per axis (periodic: points ``x_i = i*h``, ``h = length/n``;
             Dirichlet: interior points ``x_i = i*h``, ``i = 1..n``, ``h = length/(n+1)``)
``length``   domain length per axis
``fe``       explicit term: ``"none"``, ``"advect"`` (``-a u_x``, centred), ``"upwind"``
             (``-a u_x``, first-order upwind), ``"burgers"`` (``-(u^2/2)_x``, flux form) or
             ``"logistic"`` (``u(1-u)``)
``a``        advection speed (``fe == "advect"``)
``nu``       diffusion coefficient of the implicit term ``nu * Laplacian``
``T``        final time
``nt``       number of uniform time steps
``order``    RIDC order P (number of levels)
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "grid_points",
    "bumps_1d",
    "bumps_2d",
    "fourier_modes_1d",
    "config_advdiff_1d",
    "config_reacdiff_1d",
    "config_stiff_1d",
    "config_reacdiff_2d",
    "config_batched_1d",
    "serving_requests",
    "config_paper_advdiff",
    "config_paper_burgers",
    "SEED_BASE",
]

SEED_BASE = 1209


def grid_points(bc: str, n: int, length: float) -> np.ndarray:
    """Coordinates of the unknowns on one axis (see the module docstring)."""
    if bc == "periodic":
        h = length / n
        return np.arange(n, dtype=np.float64) * h
    if bc == "dirichlet":
        h = length / (n + 1)
        return np.arange(1, n + 1, dtype=np.float64) * h
    raise ValueError(f"unknown boundary condition {bc!r}")


def _bump_params(rng: np.random.Generator, count: int, dim: int):
    amp = rng.uniform(0.0, 1.0, count)
    width = rng.uniform(0.01, 0.05, count)
    centres = [rng.uniform(0.2, 0.8, count) for _ in range(dim)]
    return amp, width, centres


def bumps_1d(n: int, seed: int, count: int = 8, length: float = 1.0) -> np.ndarray:
    """Sum of ``count`` Gaussians ``A exp(-((x-c)/w)^2)`` on a Dirichlet grid of [0, length].

    Draws, in order: amplitudes A ~ U(0,1), widths w ~ U(0.01,0.05), centres c ~ U(0.2,0.8).
    """
    rng = np.random.default_rng(seed)
    amp, width, (cx,) = _bump_params(rng, count, 1)
    x = grid_points("dirichlet", n, length)
    u = np.zeros(n)
    for k in range(count):
        u += amp[k] * np.exp(-(((x - cx[k]) / width[k]) ** 2))
    return u


def bumps_2d(n: int, seed: int, count: int = 8, length: float = 1.0) -> np.ndarray:
    """Sum of ``count`` radial Gaussians on an n x n Dirichlet grid of [0, length]^2.

    Draws, in order: amplitudes, widths, x-centres, y-centres (ranges as in ``bumps_1d``).
    Returned row-major with the first index along y: ``u[iy, ix]``.
    """
    rng = np.random.default_rng(seed)
    amp, width, (cx, cy) = _bump_params(rng, count, 2)
    x = grid_points("dirichlet", n, length)
    u = np.zeros((n, n))
    for k in range(count):
        gx = np.exp(-(((x - cx[k]) / width[k]) ** 2))
        gy = np.exp(-(((x - cy[k]) / width[k]) ** 2))
        u += amp[k] * np.outer(gy, gx)
    return u


def fourier_modes_1d(n: int, rng: np.random.Generator, modes: int = 8) -> np.ndarray:
    """``sum_k (alpha_k cos kx + beta_k sin kx)``, k = 1..modes, on the periodic grid of [0, 2 pi).

    Draws, in order: alpha_1..alpha_modes, then beta_1..beta_modes, each N(0,1)/k^2.
    """
    k = np.arange(1, modes + 1, dtype=np.float64)
    alpha = rng.standard_normal(modes) / k**2
    beta = rng.standard_normal(modes) / k**2
    x = grid_points("periodic", n, 2.0 * math.pi)
    u = np.zeros(n)
    for i in range(modes):
        u += alpha[i] * np.cos(k[i] * x) + beta[i] * np.sin(k[i] * x)
    return u


def config_advdiff_1d(n: int = 128, nt: int = 200, order: int = 4, T: float = 1.0):
    """u_t + a u_x = nu u_xx on periodic [0, 2 pi), a = 1, nu = 0.1, u0 = sin x."""
    prob = dict(dim=1, bc="periodic", n=n, length=2.0 * math.pi, fe="advect", a=1.0, nu=0.1,
                T=T, nt=nt, order=order)
    u0 = np.sin(grid_points("periodic", n, 2.0 * math.pi))
    return prob, u0


def config_reacdiff_1d(n: int = 8192, nt: int = 2000, order: int = 4, T: float = 1.0,
                       nu: float = 1e-3, seed: int = SEED_BASE + 2):
    """u_t = nu u_xx + u(1-u), Dirichlet 0 on [0, 1], u0 = 8 seeded Gaussians."""
    prob = dict(dim=1, bc="dirichlet", n=n, length=1.0, fe="logistic", a=0.0, nu=nu,
                T=T, nt=nt, order=order)
    return prob, bumps_1d(n, seed)


def config_stiff_1d(n: int = 8192, nt: int = 400, order: int = 4, T: float = 0.2,
                    nu: float = 1e-3, kappa: float = 1e3, fi: str = "cubic", fe: str = "none",
                    pairs=None, seed: int = SEED_BASE + 2):
    """u_t = nu u_xx + kappa g(u) + f_E(u), Dirichlet 0 on [0, 1], with the reaction g
    (``cubic``: u - u^3, ``logistic``: u(1-u)) in the stiff part, solved implicitly by Newton's
    method; u0 = the 8 seeded Gaussians of ``config_reacdiff_1d``.  ``pairs`` (optional): the
    IMEX pair of each level."""
    prob = dict(dim=1, bc="dirichlet", n=n, length=1.0, fe=fe, a=0.0, nu=nu, T=T, nt=nt,
                order=order, fi=fi, kappa=kappa)
    if pairs is not None:
        prob["pairs"] = list(pairs)
    return prob, bumps_1d(n, seed)


def config_reacdiff_2d(n: int = 1024, nt: int = 500, order: int = 4, T: float = 1.0,
                       nu: float = 1e-4, seed: int = SEED_BASE + 3):
    """u_t = nu Lap u + u(1-u), Dirichlet 0 on [0, 1]^2, u0 = 8 seeded radial Gaussians."""
    prob = dict(dim=2, bc="dirichlet", n=n, length=1.0, fe="logistic", a=0.0, nu=nu,
                T=T, nt=nt, order=order)
    return prob, bumps_2d(n, seed)


def config_batched_1d(count: int = 256, nt: int = 1000, order: int = 4, T: float = 0.25,
                      sizes=(256, 512, 1024, 2048, 4096), seed: int = SEED_BASE + 4):
    """Independent periodic advection-diffusion instances with ragged sizes.

    Per instance, draws in order: n ~ U(sizes), a ~ U(0.5, 2), log10(nu) ~ U(-3, -1), then the
    Fourier-mode initial data (``fourier_modes_1d``).
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice(np.asarray(sizes)))
        a = float(rng.uniform(0.5, 2.0))
        nu = float(10.0 ** rng.uniform(-3.0, -1.0))
        u0 = fourier_modes_1d(n, rng)
        prob = dict(dim=1, bc="periodic", n=n, length=2.0 * math.pi, fe="advect", a=a, nu=nu,
                    T=T, nt=nt, order=order)
        out.append((prob, u0))
    return out


def serving_requests(rate: float = 200.0, duration: float = 60.0,
                     sides=(128, 256, 512, 1024), orders=(2, 3, 4), nt_range=(100, 500),
                     seed: int = SEED_BASE + 5, max_requests: int | None = None):
    """Poisson stream of 2D reaction-diffusion requests.

    Per request, draws in order: the inter-arrival gap ~ Exp(rate), side n ~ U(sides),
    order ~ U(orders), log10(nu) ~ U(-5, -3), nt ~ U{nt_range}, and a bump seed.  The initial
    data is produced lazily by ``bumps_2d(n, bump_seed)``.  Returns a list of dicts with keys
    ``t_arrival``, ``prob`` and ``bump_seed``.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        n = int(rng.choice(np.asarray(sides)))
        order = int(rng.choice(np.asarray(orders)))
        nu = float(10.0 ** rng.uniform(-5.0, -3.0))
        nt = int(rng.integers(nt_range[0], nt_range[1] + 1))
        bump_seed = int(rng.integers(0, 2**31 - 1))
        prob = dict(dim=2, bc="dirichlet", n=n, length=1.0, fe="logistic", a=0.0, nu=nu,
                    T=1.0, nt=nt, order=order)
        out.append(dict(t_arrival=t, prob=prob, bump_seed=bump_seed))
        if max_requests is not None and len(out) >= max_requests:
            break
    return out


def config_paper_advdiff(n: int = 1000, nt: int = 4000, order: int = 4, T: float = 40.0):
    """The paper's advection-diffusion case: u_t = c u_x + d u_xx, c = 0.1, d = 1e-3, periodic
    on [0, 1], dx = 1/1000, u0 = 2 + sin(2 pi x), first-order upwind advection (a = -c)."""
    prob = dict(dim=1, bc="periodic", n=n, length=1.0, fe="upwind", a=-0.1, nu=1e-3,
                T=T, nt=nt, order=order)
    x = grid_points("periodic", n, 1.0)
    return prob, 2.0 + np.sin(2.0 * math.pi * x)


def config_paper_burgers(n: int = 999, nt: int = 1000, order: int = 4, T: float = 1.0):
    """The paper's viscous Burgers case: u_t + (u^2/2)_x = eps u_xx, eps = 1e-3, u = 0 at
    x = 0, 1, dx = 1/1000 (999 interior points), u0 = sin(2 pi x) + sin(pi x)/2."""
    prob = dict(dim=1, bc="dirichlet", n=n, length=1.0, fe="burgers", a=0.0, nu=1e-3,
                T=T, nt=nt, order=order)
    x = grid_points("dirichlet", n, 1.0)
    return prob, np.sin(2.0 * math.pi * x) + 0.5 * np.sin(math.pi * x)
