"""Plain FP64 CPU oracle for two extensions of semi-implicit RIDC.

Ong, Melfi and Christlieb, "Parallel Semi-Implicit Time Integrators" (arXiv:1209.4297).

TEST INFRASTRUCTURE ONLY, like ``oracle.ridc_oracle``: only the test suite, the package smoke
check and the CPU-baseline leg of the benchmark import it; the product path never calls, links
or imports anything here, and nothing here imports the product package.

1. ARK-based RIDC (section III-D, Thm 2).  The predictor and every corrector may be any of the
   IMEX Runge-Kutta pairs of section II: the third- and fourth-order pairs printed there, or
   forward-backward Euler written as a two-stage pair.  With a p_0-order predictor and
   p_1..p_j-order correctors, level j has order ``S_j = p_0 + ... + p_j``.

   * Predictor (section II): the ARK step ``y_{n+1} = y_n + dt sum_i (b^S_i K^S_i +
     b^N_i K^N_i)`` with the stages of section II.
   * Corrector: the same pair applied to the integral form of the error equation
     (section III-A, eq. error_eqn).  Writing ``eta`` for the previous level, ``y`` for the new
     one and ``I(t) = int_{t_n}^t f(eta)``, the stages are
     ``Y_i = y_n + I(t_n + c_i dt) + dt sum_l (a^S_il K^S_l + a^N_il K^N_l)`` with
     ``K^S_i = f^S(Y_i) - f^S(eta(t_n + c_i dt))`` and ``K^N_i = f^N(Y_i) - f^N(eta(...))``.
     With forward-backward Euler this is eq. (corr) (the same terms summed in another order).
   * ``eta(t)`` and ``I(t)`` come from the Lagrange interpolant of level j-1 through ``S_j``
     equispaced stored nodes, chosen as in section III-C: the trailing nodes
     ``t_{n+2-S_j} .. t_{n+1}`` once they exist, else ``t_0 .. t_{S_j-1}``.  With ``S_j = j+1``
     (every level forward-backward Euler) these are the paper's nodes.  A window of ``S_j``
     nodes makes the quadrature exact to degree ``S_j - 1``, which the order ``S_j`` of level j
     needs (Thm 2); this reading is the build's, the paper states only the orders.
   * The previous level's state between nodes is its interpolant (``f^N`` and ``f^S`` are
     evaluated at the interpolated state).
   * Every pair used here is stiffly accurate (``b`` equals the last stage's row and
     ``c_s = 1``), so ``y_{n+1}`` is the last stage value, and the stiff stage derivative of an
     implicit stage is taken from its stage equation, ``f^S(Y_i) = (Y_i - rhs_i) / (dt a^S_ii)``:
     both equal the printed formulas in exact arithmetic, and neither multiplies the rounding of
     ``Y_i`` by ``dt`` times the stiff operator's norm.

2. A nonlinear stiff term (section III-B, after eq. pred: the implicit equation is solved by
   Newton's method).  ``f^S(u) = nu Lap_h u + kappa g(u)`` with the pointwise reaction
   ``g(u) = u(1-u)`` ("logistic") or ``g(u) = u - u^3`` ("cubic"), on Dirichlet 1D grids.
   Every implicit equation ``y - tau f^S(y) = rhs`` is solved by Newton's method with the
   tridiagonal Jacobian ``I - tau (nu D2 + kappa diag g'(y))`` solved by a banded LU, iterated
   until the update reaches rounding.

Everything is plain NumPy/SciPy FP64, written step by step in the paper's order.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass
from fractions import Fraction

import numpy as np
import scipy.linalg

from .ridc_oracle import (Problem, f_explicit, f_implicit, lagrange_integral_weights,
                          solve_implicit)

__all__ = [
    "Tableau",
    "FBE",
    "ARK3",
    "ARK4",
    "SCHEMES",
    "reaction",
    "reaction_prime",
    "f_stiff",
    "solve_stage",
    "newton_solve",
    "ark_step",
    "ark_integrate",
    "window_nodes",
    "stage_interp_weights",
    "stage_quad_weights",
    "ridc_ark_sequential",
    "ridc_ark_pipelined",
    "ark_level_orders",
    "ark_delays",
    "ark_ring_slots",
]


# ---------------------------------------------------------------------------------------------
# IMEX Runge-Kutta pairs (section II)
# ---------------------------------------------------------------------------------------------
def _rows(rows):
    return tuple(tuple(Fraction(x) for x in r) for r in rows)


@dataclass(frozen=True)
class Tableau:
    """An IMEX pair: diagonally implicit ``AS`` (stiff part) and explicit ``AN`` (non-stiff
    part), weights ``bS``/``bN``, both with abscissae ``c_i = sum_l AS_il``."""
    name: str
    AS: tuple
    AN: tuple
    bS: tuple
    bN: tuple
    order: int

    @property
    def s(self) -> int:
        return len(self.bS)

    @property
    def c(self) -> tuple:
        return tuple(sum(r) for r in self.AS)

    def stiffly_accurate(self) -> bool:
        return (tuple(self.bS) == tuple(self.AS[-1]) and tuple(self.bN) == tuple(self.AN[-1])
                and self.c[-1] == 1)


# forward-backward Euler as a two-stage pair: stage 1 at t_n (explicit), stage 2 at t_{n+1}
FBE = Tableau("fbe", AS=_rows([[0, 0], [0, 1]]), AN=_rows([[0, 0], [1, 0]]),
              bS=_rows([[0, 1]])[0], bN=_rows([[1, 0]])[0], order=1)

# the third-order pair of section II (five stages, first stage explicit)
ARK3 = Tableau(
    "ark3",
    AS=_rows([[0, 0, 0, 0, 0],
              [0, "1/2", 0, 0, 0],
              ["1/4", "-5/12", "2/3", 0, 0],
              [2, "-7/2", "1/2", 2, 0],
              ["1/6", 0, "2/3", "-5/6", 1]]),
    AN=_rows([[0, 0, 0, 0, 0],
              ["1/2", 0, 0, 0, 0],
              ["1/4", "1/4", 0, 0, 0],
              [0, 1, 0, 0, 0],
              ["1/6", 0, "2/3", "1/6", 0]]),
    bS=_rows([["1/6", 0, "2/3", "-5/6", 1]])[0],
    bN=_rows([["1/6", 0, "2/3", "1/6", 0]])[0],
    order=3)

# the fourth-order pair of section II (seven stages, first stage explicit)
ARK4 = Tableau(
    "ark4",
    AS=_rows([[0, 0, 0, 0, 0, 0, 0],
              ["-1/6", "1/2", 0, 0, 0, 0, 0],
              ["1/6", "-1/3", "1/2", 0, 0, 0, 0],
              ["3/8", "-3/8", 0, "1/2", 0, 0, 0],
              ["1/8", 0, "3/8", "-1/2", "1/2", 0, 0],
              ["-1/2", 0, 3, -3, 1, "1/2", 0],
              ["1/6", 0, 0, 0, "2/3", "-1/2", "2/3"]]),
    AN=_rows([[0, 0, 0, 0, 0, 0, 0],
              ["1/3", 0, 0, 0, 0, 0, 0],
              ["1/6", "1/6", 0, 0, 0, 0, 0],
              ["1/8", 0, "3/8", 0, 0, 0, 0],
              ["1/8", 0, "3/8", 0, 0, 0, 0],
              ["1/2", 0, "-3/2", 0, 2, 0, 0],
              ["1/6", 0, 0, 0, "2/3", "1/6", 0]]),
    bS=_rows([["1/6", 0, 0, 0, "2/3", "-1/2", "2/3"]])[0],
    bN=_rows([["1/6", 0, 0, 0, "2/3", "1/6", 0]])[0],
    order=4)

SCHEMES = {"fbe": FBE, "ark3": ARK3, "ark4": ARK4}


def _tab(t) -> Tableau:
    return SCHEMES[t] if isinstance(t, str) else t


# ---------------------------------------------------------------------------------------------
# The stiff term and its implicit equations
# ---------------------------------------------------------------------------------------------
def reaction(p: Problem, u: np.ndarray) -> np.ndarray:
    """``kappa g(u)``: 0 for pure diffusion, ``kappa u(1-u)`` or ``kappa (u - u^3)``."""
    if p.fi == "diffusion":
        return np.zeros_like(u)
    if p.fi == "logistic":
        return p.kappa * (u * (1.0 - u))
    if p.fi == "cubic":
        return p.kappa * (u - u * u * u)
    raise ValueError(f"unknown stiff term {p.fi!r}")


def reaction_prime(p: Problem, u: np.ndarray) -> np.ndarray:
    """``kappa g'(u)``, the diagonal of the reaction's Jacobian."""
    if p.fi == "diffusion":
        return np.zeros_like(u)
    if p.fi == "logistic":
        return p.kappa * (1.0 - 2.0 * u)
    if p.fi == "cubic":
        return p.kappa * (1.0 - 3.0 * u * u)
    raise ValueError(f"unknown stiff term {p.fi!r}")


def f_stiff(p: Problem, u: np.ndarray) -> np.ndarray:
    """``f^S(u) = nu Lap_h u + kappa g(u)``."""
    return f_implicit(p, u) + reaction(p, u)


def newton_solve(p: Problem, rhs: np.ndarray, tau: float, guess: np.ndarray,
                 history: list | None = None, maxit: int = 50) -> np.ndarray:
    """Solve ``y - tau f^S(y) = rhs`` (1D Dirichlet) by Newton's method (section III-B).

    Each iterate solves ``J delta = rhs - (y - tau f^S(y))`` with the tridiagonal Jacobian
    ``J = I - tau (nu D2 + kappa diag g'(y))`` by a banded LU and sets ``y += delta``.  The
    iteration stops when ``max|delta| <= 1e-15 max(1, max|y|)``, or when an update already
    below ``1e-11 max(1, max|y|)`` is above half the previous one (rounding noise).
    ``history`` (optional) receives ``max|delta|`` of every iterate.
    """
    if p.dim != 1 or p.bc != "dirichlet":
        raise ValueError("the Newton solve is defined on 1D Dirichlet grids")
    n = p.n
    r = tau * p.nu / (p.h * p.h)
    y = np.array(guess, dtype=np.float64, copy=True)
    last = np.inf
    for _ in range(maxit):
        res = rhs - (y - tau * f_stiff(p, y))
        ab = np.empty((3, n))
        ab[0, :] = -r
        ab[1, :] = 1.0 + 2.0 * r - tau * reaction_prime(p, y)
        ab[2, :] = -r
        delta = scipy.linalg.solve_banded((1, 1), ab, res)
        y = y + delta
        size = float(np.max(np.abs(delta)))
        if history is not None:
            history.append(size)
        scale = max(1.0, float(np.max(np.abs(y))))
        if size <= 1e-15 * scale or (size <= 1e-11 * scale and size > 0.5 * last):
            break
        last = size
    return y


def solve_stage(p: Problem, rhs: np.ndarray, tau: float, guess: np.ndarray) -> np.ndarray:
    """Solve the implicit stage equation ``y - tau f^S(y) = rhs``: the linear solve of
    ``oracle.ridc_oracle`` (coefficient ``tau``) for pure diffusion, Newton's method
    otherwise."""
    if p.fi == "diffusion":
        return solve_implicit(dataclasses.replace(p, dt=tau), rhs)
    return newton_solve(p, rhs, tau, guess)


# ---------------------------------------------------------------------------------------------
# Predictor: one step of an IMEX pair (section II)
# ---------------------------------------------------------------------------------------------
def _stages(p: Problem, tab: Tableau, base: np.ndarray, extra_rhs, sub_s, sub_n, guess):
    """The stages of one step of ``tab``.  Stage i solves
    ``Y_i - dt a_ii f^S(Y_i) = base + extra_rhs(i) + dt sum_{l<i} (a^S_il K^S_l + a^N_il K^N_l)
    - dt a_ii sub_s(i)`` and sets ``K^S_i = f^S(Y_i) - sub_s(i)``, ``K^N_i = f^N(Y_i) -
    sub_n(i)`` (the subtracted terms are zero for the predictor).  Returns the last stage
    value (the pair is stiffly accurate)."""
    if not tab.stiffly_accurate():
        raise ValueError(f"{tab.name}: only stiffly accurate pairs are supported")
    dt = p.dt
    KS, KN = [], []
    Y = base
    for i in range(tab.s):
        rhs = base + extra_rhs(i)
        for l in range(i):
            rhs = rhs + dt * (float(tab.AS[i][l]) * KS[l] + float(tab.AN[i][l]) * KN[l])
        a = float(tab.AS[i][i])
        ss = sub_s(i)
        if a == 0.0:
            Y = rhs
            fs = f_stiff(p, Y)
        else:
            rhs = rhs - dt * a * ss
            Y = solve_stage(p, rhs, dt * a, guess(i))
            fs = (Y - rhs) / (dt * a)
        KS.append(fs - ss)
        KN.append(f_explicit(p, Y) - sub_n(i))
    return Y


def ark_step(p: Problem, tab, y: np.ndarray) -> np.ndarray:
    """One step of the IMEX pair ``tab`` from ``y`` (section II); Newton guesses: ``y``."""
    tab = _tab(tab)
    zero = np.zeros_like(y)
    return _stages(p, tab, y, lambda i: zero, lambda i: zero, lambda i: zero, lambda i: y)


def ark_integrate(p: Problem, tab, u0: np.ndarray, nt: int) -> np.ndarray:
    """``nt`` steps of ``tab`` alone (the predictor of every ARK-based RIDC)."""
    u = np.asarray(u0, dtype=np.float64).copy()
    for _ in range(nt):
        u = ark_step(p, tab, u)
    return u


# ---------------------------------------------------------------------------------------------
# Corrector windows and weights (section III-C, widened to S nodes)
# ---------------------------------------------------------------------------------------------
def window_nodes(n: int, S: int) -> list:
    """Time indices of the ``S`` interpolation nodes for the step ``t_n -> t_{n+1}``: the
    trailing nodes ``t_{n+2-S} .. t_{n+1}`` when ``n >= S-2``, else ``t_0 .. t_{S-1}``
    (ascending)."""
    start = n + 2 - S if n >= S - 2 else 0
    return list(range(start, start + S))


def _lagrange_values(nodes, t) -> list:
    """Exact ``l_k(t)`` of the Lagrange basis on ``nodes`` (rationals)."""
    out = []
    for k, tk in enumerate(nodes):
        v = Fraction(1)
        for i, ti in enumerate(nodes):
            if i != k:
                v *= Fraction(t - ti) / Fraction(tk - ti)
        out.append(v)
    return out


def stage_interp_weights(n: int, S: int, c) -> list:
    """``l_k(t_n + c dt)`` for the window of ``window_nodes(n, S)`` (exact rationals)."""
    nodes = window_nodes(n, S)
    return _lagrange_values(nodes, Fraction(n) + Fraction(c))


def stage_quad_weights(n: int, S: int, c) -> list:
    """``(1/dt) int_{t_n}^{t_n + c dt} l_k`` for the window of ``window_nodes(n, S)``."""
    nodes = window_nodes(n, S)
    return lagrange_integral_weights(nodes, Fraction(n), Fraction(n) + Fraction(c))


# ---------------------------------------------------------------------------------------------
# ARK-based RIDC
# ---------------------------------------------------------------------------------------------
def ark_level_orders(schemes) -> list:
    """``S_j = p_0 + ... + p_j``: the order of level j and its corrector's window size."""
    out, acc = [], 0
    for t in schemes:
        acc += _tab(t).order
        out.append(acc)
    return out


def _check_ark(nt: int, schemes):
    if len(schemes) < 1:
        raise ValueError("need at least the predictor")
    if nt < 0:
        raise ValueError("nt must be >= 0")
    S = ark_level_orders(schemes)
    if len(schemes) > 1 and 0 < nt < S[-1] - 1:
        raise ValueError("the start-up window of the top corrector needs nt >= S - 1")


def _corrector_step(p: Problem, tab: Tableau, S: int, n: int, y_n: np.ndarray, prev):
    """One step ``t_n -> t_{n+1}`` of a corrector of pair ``tab`` whose window holds ``S``
    nodes of the previous level (``prev(m)`` returns its value at ``t_m``)."""
    dt = p.dt
    nodes = window_nodes(n, S)
    eta = [prev(m) for m in nodes]
    F = [f_stiff(p, v) + f_explicit(p, v) for v in eta]
    interp, state_s, state_n, integ = [], [], [], []
    for i in range(tab.s):
        L = stage_interp_weights(n, S, tab.c[i])
        Q = stage_quad_weights(n, S, tab.c[i])
        e = np.zeros_like(y_n)
        q = np.zeros_like(y_n)
        for k in range(S):
            e = e + float(L[k]) * eta[k]
            q = q + float(Q[k]) * F[k]
        interp.append(e)
        state_s.append(f_stiff(p, e))
        state_n.append(f_explicit(p, e))
        integ.append(dt * q)
    return _stages(p, tab, y_n, lambda i: integ[i], lambda i: state_s[i], lambda i: state_n[i],
                   lambda i: interp[i])


def ridc_ark_sequential(p: Problem, u0: np.ndarray, nt: int, schemes) -> list:
    """ARK-based RIDC, level by level over whole trajectories.  ``schemes[0]`` is the
    predictor's pair, ``schemes[j]`` corrector j's.  Every level starts from ``u0`` (section
    III-E).  Returns every level's final value."""
    schemes = [_tab(t) for t in schemes]
    _check_ark(nt, schemes)
    S = ark_level_orders(schemes)
    u0 = np.asarray(u0, dtype=np.float64)
    traj = [u0.copy()]
    for _ in range(nt):
        traj.append(ark_step(p, schemes[0], traj[-1]))
    finals = [traj[-1]]
    for j in range(1, len(schemes)):
        prev_traj = traj
        traj = [u0.copy()]
        for n in range(nt):
            traj.append(_corrector_step(p, schemes[j], S[j], n, traj[n],
                                        lambda m: prev_traj[m]))
        finals.append(traj[-1])
    return finals


def ark_delays(schemes) -> list:
    """Pipeline start of each level: level j computes ``t_m`` at pipeline step ``m + d_j`` with
    ``d_0 = 0`` and ``d_j = d_{j-1} + S_j - 1`` (its first step needs the previous level up to
    the window's last start-up node ``t_{S_j - 1}``).  All-Euler levels give ``j(j+1)/2``
    (section III-E)."""
    S = ark_level_orders(schemes)
    d = [0]
    for j in range(1, len(S)):
        d.append(d[-1] + S[j] - 1)
    return d


def ark_ring_slots(schemes) -> list:
    """Values of each level kept alive by the pipeline: the ``2 S_{j+1} - 1`` nodes between
    the oldest one level j+1 still reads and the one level j writes in the same step; the top
    level keeps its latest two."""
    S = ark_level_orders(schemes)
    P = len(S)
    return [2 * S[j + 1] - 1 if j + 1 < P else 2 for j in range(P)]


def ridc_ark_pipelined(p: Problem, u0: np.ndarray, nt: int, schemes, trace=None) -> list:
    """ARK-based RIDC as a lagged pipeline: at step ``sigma`` level j computes
    ``t_{sigma - d_j}`` (``ark_delays``).  Each level is a ring of ``ark_ring_slots`` values:
    writing ``t_m`` deletes ``t_{m - slots}`` before the step's reads, so a read of an
    overwritten value raises ``KeyError`` (and a read of a value not yet computed does too).  ``trace(sigma, j, m)`` (optional) sees every
    level-step.  Returns every level's final value, equal to ``ridc_ark_sequential``'s."""
    schemes = [_tab(t) for t in schemes]
    _check_ark(nt, schemes)
    S = ark_level_orders(schemes)
    d = ark_delays(schemes)
    slots = ark_ring_slots(schemes)
    P = len(schemes)
    u0 = np.asarray(u0, dtype=np.float64)
    hist = [{0: u0.copy()} for _ in range(P)]
    total = nt + d[-1] if nt > 0 else 0
    for sigma in range(1, total + 1):
        # the slot a level writes this step held its value from slots[j] steps back: gone before
        # any level of this step reads (all levels of a step run concurrently)
        for j in range(P):
            m = sigma - d[j]
            if 1 <= m <= nt:
                hist[j].pop(m - slots[j], None)
        produced = []
        for j in range(P):
            m = sigma - d[j]
            if not 1 <= m <= nt:
                continue
            if trace is not None:
                trace(sigma, j, m)
            if j == 0:
                val = ark_step(p, schemes[0], hist[0][m - 1])
            else:
                ph = hist[j - 1]
                val = _corrector_step(p, schemes[j], S[j], m - 1, hist[j][m - 1],
                                      lambda k: ph[k])
            produced.append((j, m, val))
        for j, m, val in produced:
            hist[j][m] = val
    return [hist[j][nt] for j in range(P)]
