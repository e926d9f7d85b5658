"""Pins for the oracle's quadrature weights (section III-C) against closed forms.

Nothing here recomputes a weight the way the oracle does: the checks are the textbook
Adams-Moulton coefficients, exact integrals of monomials, and symmetry/consistency laws.
"""
import os
from fractions import Fraction

import pytest

from oracle import corrector_nodes, corrector_weights, lagrange_integral_weights

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "adams_moulton.txt")


def _adams_moulton():
    table = {}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            vals = [int(x) for x in line.split()]
            k, den, coef = vals[0], vals[1], vals[2:]
            table[k] = [Fraction(c, den) for c in coef]
    return table


def _exact_rows(j):
    """All j rows of corrector j's weight table, exact, in the oracle's node order."""
    rows = []
    for n in range(j):                        # n = 0..j-1 covers every distinct offset
        nodes = corrector_nodes(n, j)
        lo = min(nodes)
        rows.append((n, nodes, lagrange_integral_weights([x - lo for x in nodes],
                                                          n - lo, n - lo + 1)))
    return rows


@pytest.mark.parametrize("j", [1, 2, 3, 4])
def test_steady_state_row_is_adams_moulton(j):
    am = _adams_moulton()[j]
    n = j + 5                                 # any n >= j-1 gives the steady-state stencil
    nodes = corrector_nodes(n, j)
    assert nodes == [n + 1 - k for k in range(j + 1)]
    lo = min(nodes)
    w = lagrange_integral_weights([x - lo for x in nodes], n - lo, n - lo + 1)
    assert w == am                            # nodes are t_{n+1}, t_n, ..., t_{n+1-j}


@pytest.mark.parametrize("j", [1, 2, 3, 4, 5])
def test_rows_exact_on_polynomials(j):
    for n, nodes, w in _exact_rows(j):
        for deg in range(j + 1):
            quad = sum(wk * Fraction(t) ** deg for wk, t in zip(w, [x - min(nodes) for x in nodes]))
            a, b = Fraction(n - min(nodes)), Fraction(n - min(nodes) + 1)
            exact = (b ** (deg + 1) - a ** (deg + 1)) / (deg + 1)
            assert quad == exact, (j, n, deg)
        # and not exact one degree higher (the rule really has degree j)
        deg = j + 1
        quad = sum(wk * Fraction(t) ** deg for wk, t in zip(w, [x - min(nodes) for x in nodes]))
        a, b = Fraction(n - min(nodes)), Fraction(n - min(nodes) + 1)
        assert quad != (b ** (deg + 1) - a ** (deg + 1)) / (deg + 1)


@pytest.mark.parametrize("j", [1, 2, 3, 4, 5, 6])
def test_rows_sum_to_one_and_reflect(j):
    rows = _exact_rows(j)
    by_offset = {}
    for n, nodes, w in rows:
        assert sum(w) == 1
        lo = min(nodes)
        asc = sorted(zip([x - lo for x in nodes], w))
        by_offset[n - lo] = [v for _, v in asc]
    assert sorted(by_offset) == list(range(j))
    for r in range(j):                        # reflection t -> j - t maps interval r to j-1-r
        assert by_offset[r] == list(reversed(by_offset[j - 1 - r]))


def test_start_up_stencil_matches_text():
    # corrector 3 before it can use a trailing window integrates over [t_0,t_1] and [t_1,t_2]
    # with the nodes t_0..t_3
    assert corrector_nodes(0, 3) == [0, 1, 2, 3]
    assert corrector_nodes(1, 3) == [0, 1, 2, 3]
    assert corrector_nodes(2, 3) == [3, 2, 1, 0]
    assert corrector_nodes(3, 3) == [4, 3, 2, 1]
    # start-up row r=0 of corrector 2 is the reflected Adams-Moulton 2-step rule
    nodes, w = corrector_weights(0, 2)
    assert nodes == [0, 1, 2]
    assert w == pytest.approx([5 / 12, 8 / 12, -1 / 12], abs=1e-16)


def test_float_weights_match_exact():
    for j in range(1, 6):
        for n in range(j + 3):
            nodes, w = corrector_weights(n, j)
            lo = min(nodes)
            exact = lagrange_integral_weights([x - lo for x in nodes], n - lo, n - lo + 1)
            assert w == [float(x) for x in exact]
