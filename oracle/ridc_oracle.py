"""Plain FP64 CPU oracle for semi-implicit RIDC-FBE.

Ong, Melfi and Christlieb, "Parallel Semi-Implicit Time Integrators" (arXiv:1209.4297).

TEST INFRASTRUCTURE ONLY.  This module exists to check the HIP implementation.  Only the test
suite, the package smoke check and the CPU-baseline leg of the benchmark import it; the product
path never calls, links or imports anything here, and nothing here imports the product package.
It shares no code with the HIP path: only the seeded initial data (``workloads``) is common.

What it computes (every step written out in plain NumPy/SciPy, FP64, no blocking or fusion):

* The IVP ``y' = f^S(y) + f^N(y)`` (section II, eq. ode) with the stiff part linear,
  ``f^S(y) = nu * Lap_h y`` (the diffusion operator, section IV), and the non-stiff part
  ``f^N`` one of: none, centred or first-order upwind advection ``-a u_x`` (section IV-A),
  the Burgers numerical flux (section IV-B), or the logistic reaction ``u(1-u)``.
* Level 0, the predictor: first-order IMEX (forward-backward) Euler, section II
  eq. (imex_diffusion) and section III-B eq. (pred):
  ``(I - dt D) eta[0]_{n+1} = eta[0]_n + dt f^N(eta[0]_n)``.
* Level j >= 1, the corrector, section III-C eq. (corr): an IMEX Euler step on the error
  equation plus the integral of ``f = f^S + f^N`` along the previous level,
  ``eta[j]_{n+1} = eta[j]_n + dt[f^S(eta[j]_{n+1}) + f^N(eta[j]_n)]
                   - dt[f^S(eta[j-1]_{n+1}) + f^N(eta[j-1]_n)]
                   + int_{t_n}^{t_{n+1}} f(eta[j-1])``.
  The second bracket carries ``dt`` on both terms (the printed bracket puts ``dt`` on the
  first term only; the equation is an IMEX Euler discretisation of eq. (error_eqn), so both
  terms are rates times ``dt``).
* The integral is the (j+1)-node Lagrange quadrature of section III-C: nodes
  ``t_{n+1-k}, k = 0..j`` when ``n >= j-1`` and ``t_0..t_j`` otherwise, weights the exact
  integrals of the Lagrange basis over ``[t_n, t_{n+1}]``.  The printed index range of the
  weights (``k = 0..j-1``) is read as ``k = 0..j``, matching the sums they enter.
* Every level starts from the initial data (section III-E, Fig. 2 caption).
* Output: the final value of every level; the top level is the most accurate (section III-E).
* Restarts (section III-E): equal segments, each restarted from the top level of the previous.

Solvers for ``(I - dt nu Lap_h) x = b`` (the paper pre-factors this matrix by QR; any exact
solver gives the same values up to rounding): FFT diagonalisation of the circulant (periodic
1D), a banded LU (Dirichlet 1D), an orthonormal type-I sine transform (Dirichlet 2D), each
followed by one step of iterative refinement so that every step's linear system is solved to
rounding.

Linear periodic 1D problems can also be evaluated mode by mode in Fourier space
(``ridc_linear_periodic``): the same steps on the scalar equation of each discrete mode.

Grids: periodic ``x_i = i h``, ``h = L/n``; Dirichlet ``x_i = i h``, ``i = 1..n``,
``h = L/(n+1)``, with zero ghost values.  2D arrays are ``u[iy, ix]``.
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction

import numpy as np
import scipy.fft
import scipy.linalg

__all__ = [
    "Problem",
    "lagrange_integral_weights",
    "corrector_nodes",
    "corrector_weights",
    "f_explicit",
    "f_implicit",
    "solve_implicit",
    "ridc_sequential",
    "ridc_pipelined",
    "ridc",
    "ridc_restarted",
    "fbe",
    "rel_l2",
    "periodic_mode_symbols",
    "ridc_linear_periodic",
]


# ---------------------------------------------------------------------------------------------
# Problem description
# ---------------------------------------------------------------------------------------------
@dataclass(frozen=True)
class Problem:
    dim: int
    bc: str
    n: int
    length: float
    fe: str
    a: float
    nu: float
    dt: float
    # stiff term f^S: "diffusion" (nu Lap_h, linear) or, for the Newton path of
    # ``oracle.ridc_ext``, diffusion plus a pointwise reaction of rate kappa
    fi: str = "diffusion"
    kappa: float = 0.0

    @staticmethod
    def from_dict(d: dict, nt: int | None = None) -> "Problem":
        nt = d["nt"] if nt is None else nt
        return Problem(dim=int(d["dim"]), bc=d["bc"], n=int(d["n"]), length=float(d["length"]),
                       fe=d["fe"], a=float(d.get("a", 0.0)), nu=float(d["nu"]),
                       dt=float(d["T"]) / nt, fi=d.get("fi", "diffusion"),
                       kappa=float(d.get("kappa", 0.0)))

    @property
    def h(self) -> float:
        return self.length / self.n if self.bc == "periodic" else self.length / (self.n + 1)


# ---------------------------------------------------------------------------------------------
# Quadrature weights (section III-C)
# ---------------------------------------------------------------------------------------------
def _poly_mul(p: list, q: list) -> list:
    out = [Fraction(0)] * (len(p) + len(q) - 1)
    for i, pi in enumerate(p):
        for k, qk in enumerate(q):
            out[i + k] += pi * qk
    return out


def lagrange_integral_weights(nodes, lo, hi) -> list:
    """Exact ``int_lo^hi l_k(t) dt`` for the Lagrange basis ``l_k`` on ``nodes`` (rationals)."""
    nodes = [Fraction(x) for x in nodes]
    lo, hi = Fraction(lo), Fraction(hi)
    weights = []
    for k, tk in enumerate(nodes):
        poly = [Fraction(1)]          # coefficients, lowest degree first
        denom = Fraction(1)
        for i, ti in enumerate(nodes):
            if i == k:
                continue
            poly = _poly_mul(poly, [-ti, Fraction(1)])
            denom *= tk - ti
        integral = sum(c * (hi ** (d + 1) - lo ** (d + 1)) / (d + 1) for d, c in enumerate(poly))
        weights.append(integral / denom)
    return weights


def corrector_nodes(n: int, j: int) -> list:
    """Time indices of the j+1 quadrature nodes used by corrector j on ``[t_n, t_{n+1}]``.

    Section III-C: ``t_{n+1-k}, k = 0..j`` when ``n >= j-1``, else ``t_0..t_j``.
    """
    if n >= j - 1:
        return [n + 1 - k for k in range(j + 1)]
    return list(range(j + 1))


_WEIGHT_CACHE: dict = {}


def corrector_weights(n: int, j: int):
    """(nodes, weights) with weights in units of dt: ``alpha_{nk} = dt * w_k``."""
    nodes = corrector_nodes(n, j)
    lo = nodes[-1] if n >= j - 1 else 0
    key = (j, n - lo)                # uniform steps: weights depend only on the offset
    if key not in _WEIGHT_CACHE:
        rel = [x - lo for x in nodes]
        _WEIGHT_CACHE[key] = [float(w) for w in lagrange_integral_weights(rel, n - lo, n - lo + 1)]
    return nodes, _WEIGHT_CACHE[key]


# ---------------------------------------------------------------------------------------------
# Operators (section IV: diffusion is the stiff term, centred differences)
# ---------------------------------------------------------------------------------------------
def _shift(p: Problem, u: np.ndarray, offset: int, axis: int) -> np.ndarray:
    """``v[i] = u[i + offset]`` along ``axis`` (periodic wrap, or zero ghosts for Dirichlet)."""
    if p.bc == "periodic":
        return np.roll(u, -offset, axis=axis)
    v = np.zeros_like(u)
    src = [slice(None)] * u.ndim
    dst = [slice(None)] * u.ndim
    if offset > 0:
        src[axis] = slice(offset, None)
        dst[axis] = slice(None, -offset)
    else:
        src[axis] = slice(None, offset)
        dst[axis] = slice(-offset, None)
    v[tuple(dst)] = u[tuple(src)]
    return v


def f_implicit(p: Problem, u: np.ndarray) -> np.ndarray:
    """``f^S(u) = nu * Lap_h u`` (3-point in 1D, 5-point in 2D)."""
    h2 = p.h * p.h
    lap = np.zeros_like(u)
    for axis in range(p.dim):
        lap += (_shift(p, u, 1, axis) - 2.0 * u + _shift(p, u, -1, axis)) / h2
    return p.nu * lap


def f_explicit(p: Problem, u: np.ndarray) -> np.ndarray:
    """``f^N(u)`` for ``u_t + a u_x = ...`` and friends:

    * ``none``: 0;
    * ``logistic``: ``u(1-u)``;
    * ``advect`` (1D): centred ``-a (u_{i+1} - u_{i-1}) / (2h)``;
    * ``upwind`` (1D, section IV-A): first-order upwind ``-a (u_i - u_{i-1}) / h`` for
      ``a >= 0`` and ``-a (u_{i+1} - u_i) / h`` for ``a < 0`` (the paper's ``u_t = c u_x`` is
      ``a = -c``);
    * ``burgers`` (1D, section IV-B): ``-(1/2)(f_{i+1/2} - f_{i-1/2}) / h`` with the flux
      ``f_{i+1/2} = (u_{i+1}^2 + u_i^2) / 2``.
    """
    if p.fe == "none":
        return np.zeros_like(u)
    if p.fe == "logistic":
        return u * (1.0 - u)
    if p.fe in ("advect", "upwind", "burgers") and p.dim != 1:
        raise ValueError(f"{p.fe} is defined for 1D problems")
    up = _shift(p, u, 1, 0)
    um = _shift(p, u, -1, 0)
    if p.fe == "advect":
        return -p.a * (up - um) / (2.0 * p.h)
    if p.fe == "upwind":
        if p.a >= 0:
            return -p.a * (u - um) / p.h
        return -p.a * (up - u) / p.h
    if p.fe == "burgers":
        flux_right = 0.5 * (up * up + u * u)        # f_{i+1/2}
        flux_left = 0.5 * (u * u + um * um)         # f_{i-1/2}
        return -0.5 * (flux_right - flux_left) / p.h
    raise ValueError(f"unknown explicit term {p.fe!r}")


def f_total(p: Problem, u: np.ndarray) -> np.ndarray:
    return f_explicit(p, u) + f_implicit(p, u)


def _solve_direct(p: Problem, rhs: np.ndarray) -> np.ndarray:
    """One direct solve of ``(I - dt nu Lap_h) x = rhs``."""
    r = p.dt * p.nu / (p.h * p.h)
    n = p.n
    if p.dim == 1 and p.bc == "periodic":
        k = np.arange(n)
        eig = 1.0 + 4.0 * r * np.sin(np.pi * k / n) ** 2
        return np.real(np.fft.ifft(np.fft.fft(rhs) / eig))
    if p.dim == 1 and p.bc == "dirichlet":
        ab = np.empty((3, n))
        ab[0, :] = -r
        ab[1, :] = 1.0 + 2.0 * r
        ab[2, :] = -r
        return scipy.linalg.solve_banded((1, 1), ab, rhs)
    if p.dim == 2 and p.bc == "dirichlet":
        k = np.arange(1, n + 1)
        s = np.sin(np.pi * k / (2.0 * (n + 1))) ** 2
        eig = 1.0 + 4.0 * r * (s[:, None] + s[None, :])
        # the FFT worker count follows scipy.fft.set_workers (one thread unless a caller asks
        # for more); the values do not depend on it
        bh = scipy.fft.dstn(rhs, type=1, norm="ortho")
        return scipy.fft.idstn(bh / eig, type=1, norm="ortho")
    raise ValueError(f"unsupported grid dim={p.dim} bc={p.bc}")


def solve_implicit(p: Problem, rhs: np.ndarray) -> np.ndarray:
    """Solve ``(I - dt nu Lap_h) x = rhs`` to rounding: a direct solve, then one correction by
    the solve of the residual ``rhs - (x - dt f^S(x))`` (plain iterative refinement; the direct
    solvers alone lose up to a few units in the last place per step, which adds up over
    thousands of steps)."""
    if p.fi != "diffusion":
        raise ValueError("a nonlinear stiff term needs the Newton solve of oracle.ridc_ext")
    x = _solve_direct(p, rhs)
    res = rhs - (x - p.dt * f_implicit(p, x))
    return x + _solve_direct(p, res)


# ---------------------------------------------------------------------------------------------
# RIDC-FBE
# ---------------------------------------------------------------------------------------------
def _check(nt: int, order: int):
    if order < 1:
        raise ValueError("order must be >= 1")
    if nt < 0:
        raise ValueError("nt must be >= 0")
    if 0 < nt < order - 1:
        raise ValueError("the start-up quadrature of the top corrector needs nt >= order - 1")


def _predictor_step(p: Problem, u: np.ndarray) -> np.ndarray:
    """Eq. (imex_diffusion): ``(I - dt D) y_{n+1} = y_n + dt f^N(y_n)``."""
    return solve_implicit(p, u + p.dt * f_explicit(p, u))


def _corrector_step(p: Problem, j: int, n: int, cur_n: np.ndarray, prev) -> np.ndarray:
    """Eq. (corr) for level j from ``t_n`` to ``t_{n+1}``; ``prev(m)`` returns ``eta[j-1]_m``."""
    dt = p.dt
    nodes, w = corrector_weights(n, j)
    quad = np.zeros_like(cur_n)
    for node, wk in zip(nodes, w):
        quad += wk * f_total(p, prev(node))
    rhs = (cur_n + dt * f_explicit(p, cur_n)
           - dt * (f_implicit(p, prev(n + 1)) + f_explicit(p, prev(n)))
           + dt * quad)
    return solve_implicit(p, rhs)


def ridc_sequential(p: Problem, u0: np.ndarray, nt: int, order: int) -> list:
    """Level-by-level RIDC: each level's whole trajectory before the next level starts.

    Stores every level's trajectory, so it suits small cases.  Returns the final value of
    every level, ``[eta[0]_nt, ..., eta[order-1]_nt]``.
    """
    _check(nt, order)
    u0 = np.asarray(u0, dtype=np.float64)
    traj = [u0.copy()]
    for _ in range(nt):
        traj.append(_predictor_step(p, traj[-1]))
    finals = [traj[-1]]
    for j in range(1, order):
        prev_traj = traj
        traj = [u0.copy()]
        for n in range(nt):
            traj.append(_corrector_step(p, j, n, traj[n], lambda m: prev_traj[m]))
        finals.append(traj[-1])
    return finals


def ridc_pipelined(p: Problem, u0: np.ndarray, nt: int, order: int, trace=None) -> list:
    """RIDC run as the lagged pipeline of section III (Fig. 1, Fig. 2).

    At pipeline step ``sigma`` level j computes ``t_m`` with ``m = sigma - j(j+1)/2`` (level j
    starts after waiting ``j(j+1)/2`` steps, section III-E), so all active levels of one step
    are independent.  Each level keeps only the values a later step still reads; an evicted
    value is deleted, so a read of it raises ``KeyError`` instead of returning stale data.
    ``trace``, if given, is called with ``(sigma, j, m)`` for every level-step.
    """
    _check(nt, order)
    u0 = np.asarray(u0, dtype=np.float64)
    hist = [{0: u0.copy()} for _ in range(order)]
    latest = [0] * order
    total = nt + order * (order - 1) // 2 if nt > 0 else 0
    for sigma in range(1, total + 1):
        produced = []
        for j in range(order):
            m = sigma - j * (j + 1) // 2
            if not 1 <= m <= nt:
                continue
            if trace is not None:
                trace(sigma, j, m)
            if j == 0:
                val = _predictor_step(p, hist[0][m - 1])
            else:
                prev_hist = hist[j - 1]
                val = _corrector_step(p, j, m - 1, hist[j][m - 1], lambda k: prev_hist[k])
            produced.append((j, m, val))
        for j, m, val in produced:
            hist[j][m] = val
            latest[j] = m
        # evict what no later step reads: level j keeps its own latest value and the nodes
        # that level j+1 still needs for its next step (its window starts at
        # max(0, latest[j+1] + 1 - (j+1)) = max(0, latest[j+1] - j)).
        for j in range(order):
            keep_from = latest[j]
            if j + 1 < order and latest[j + 1] < nt:
                keep_from = min(keep_from, max(0, latest[j + 1] - j))
            for k in [k for k in hist[j] if k < keep_from]:
                del hist[j][k]
    return [hist[j][nt] for j in range(order)]


def ridc(p: Problem, u0: np.ndarray, nt: int, order: int) -> np.ndarray:
    """Top-level (most accurate) RIDC solution at ``t = nt * dt``."""
    return ridc_pipelined(p, u0, nt, order)[-1]


def ridc_restarted(p: Problem, u0: np.ndarray, nt: int, order: int, segments: int) -> np.ndarray:
    """RIDC with restarts (section III-E): the nt steps are split into ``segments`` equal
    intervals; each is a full RIDC integration started from the most accurate (top) level of
    the previous one."""
    if segments < 1 or nt % segments:
        raise ValueError("nt must be a positive multiple of segments")
    u = np.asarray(u0, dtype=np.float64)
    for _ in range(segments):
        u = ridc_pipelined(p, u, nt // segments, order)[-1]
    return u


def fbe(p: Problem, u0: np.ndarray, nt: int) -> np.ndarray:
    """First-order IMEX Euler alone (the order-1 case)."""
    u = np.asarray(u0, dtype=np.float64).copy()
    for _ in range(nt):
        u = _predictor_step(p, u)
    return u


# ---------------------------------------------------------------------------------------------
# Linear periodic 1D problems, mode by mode
# ---------------------------------------------------------------------------------------------
def periodic_mode_symbols(p: Problem):
    """Eigenvalues ``(lam_e, lam_i)`` of ``f^N`` and ``f^S`` on the discrete Fourier modes of a
    periodic 1D grid, ordered like ``numpy.fft.fft``: mode m is ``exp(i theta_m l)`` with
    ``theta_m = 2 pi m / n``, an eigenvector of every translation-invariant stencil.

    * diffusion ``nu (u_{l+1} - 2 u_l + u_{l-1}) / h^2``: ``-(4 nu / h^2) sin^2(theta / 2)``;
    * centred advection ``-a (u_{l+1} - u_{l-1}) / (2h)``: ``-i a sin(theta) / h``;
    * first-order upwind (section IV-A): ``-a (1 - exp(-i theta)) / h`` for ``a >= 0``,
      ``-a (exp(i theta) - 1) / h`` for ``a < 0``;
    * none: 0.  Nonlinear explicit terms have no symbol and raise.
    """
    if p.dim != 1 or p.bc != "periodic":
        raise ValueError("Fourier modes diagonalise periodic 1D problems only")
    theta = 2.0 * np.pi * np.arange(p.n) / p.n
    lam_i = -(4.0 * p.nu / (p.h * p.h)) * np.sin(theta / 2.0) ** 2
    if p.fe == "none":
        lam_e = np.zeros(p.n, dtype=complex)
    elif p.fe == "advect":
        lam_e = -1j * p.a * np.sin(theta) / p.h
    elif p.fe == "upwind":
        if p.a >= 0:
            lam_e = -p.a * (1.0 - np.exp(-1j * theta)) / p.h
        else:
            lam_e = -p.a * (np.exp(1j * theta) - 1.0) / p.h
    else:
        raise ValueError(f"{p.fe!r} is not linear: no Fourier symbol")
    return lam_e, lam_i


def ridc_linear_periodic(p: Problem, u0: np.ndarray, nt: int, order: int) -> list:
    """RIDC-FBE of a linear periodic 1D problem evaluated in Fourier space.

    Both operators are circulant, so the discrete Fourier transform decouples the system into
    scalar equations ``y' = lam_e y + lam_i y``, one per mode.  Every mode takes the steps of the
    vector method -- eq. (pred) for level 0, eq. (corr) with the (j+1)-node quadrature of
    section III-C for level j -- with ``f^N(y) = lam_e y``, ``f^S(y) = lam_i y`` and the solve a
    division by ``1 - dt lam_i``.  Level by level, whole trajectories, like
    ``ridc_sequential``.  Returns every level's final value (real).
    """
    _check(nt, order)
    dt = p.dt
    lam_e, lam_i = periodic_mode_symbols(p)
    lam = lam_e + lam_i
    den = 1.0 - dt * lam_i
    y0 = np.fft.fft(np.asarray(u0, dtype=np.float64))
    traj = [y0]
    for _ in range(nt):                               # eq. (pred)
        traj.append((traj[-1] + dt * lam_e * traj[-1]) / den)
    finals = [traj[-1]]
    for j in range(1, order):                         # eq. (corr)
        prev = traj
        traj = [y0]
        for n in range(nt):
            nodes, w = corrector_weights(n, j)
            quad = np.zeros_like(y0)
            for node, wk in zip(nodes, w):
                quad += wk * (lam * prev[node])
            rhs = (traj[n] + dt * (lam_e * traj[n])
                   - dt * (lam_i * prev[n + 1] + lam_e * prev[n])
                   + dt * quad)
            traj.append(rhs / den)
        finals.append(traj[-1])
    return [np.real(np.fft.ifft(y)) for y in finals]


def rel_l2(x: np.ndarray, ref: np.ndarray) -> float:
    """Discrete relative L2 error ``||x - ref||_2 / ||ref||_2`` over all unknowns."""
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(np.asarray(x, dtype=np.float64) - ref) / np.linalg.norm(ref))
