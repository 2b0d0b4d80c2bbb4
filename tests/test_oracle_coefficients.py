"""Pins of the oracle's finite-difference, interpolation and axis coefficients (section 2.3, 2.4).

The oracle computes every weight from a closed Lagrange product.  Here the same weights are derived a
second, independent way: by solving the moment (exactness) conditions that define each formula, in
exact rational arithmetic.  The 10th-order axis weights are also checked against the values printed in
the paper (tests/golden/axis_weights_order10.txt), and low orders against textbook stencils.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def solve_exact(A, b):
    """Gaussian elimination over the rationals."""
    n = len(A)
    M = [list(map(Fraction, row)) + [Fraction(rhs)] for row, rhs in zip(A, b)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [x - f * y for x, y in zip(M[r], M[col])]
    return [M[i][n] / M[i][i] for i in range(n)]


def exact_staggered(nd):
    # f'(0) = sum_j a_j [f(x_j) - f(-x_j)],  x_j = (2j-1)/2, exact on x^(2p-1), p = 1..nd
    xs = [Fraction(2 * j - 1, 2) for j in range(1, nd + 1)]
    A = [[2 * x ** (2 * p - 1) for x in xs] for p in range(1, nd + 1)]
    return solve_exact(A, [1 if p == 1 else 0 for p in range(1, nd + 1)])


def exact_halfshift(nd):
    # f(0) = sum_j s_j [f(x_j) + f(-x_j)], exact on x^(2p), p = 0..nd-1
    xs = [Fraction(2 * j - 1, 2) for j in range(1, nd + 1)]
    A = [[2 * x ** (2 * p) for x in xs] for p in range(nd)]
    return solve_exact(A, [1 if p == 0 else 0 for p in range(nd)])


def exact_d1(nd):
    A = [[2 * Fraction(j) ** (2 * p - 1) for j in range(1, nd + 1)] for p in range(1, nd + 1)]
    return solve_exact(A, [1 if p == 1 else 0 for p in range(1, nd + 1)])


def exact_d2(nd):
    A = [[2 * Fraction(j) ** (2 * p) for j in range(1, nd + 1)] for p in range(1, nd + 1)]
    b = solve_exact(A, [2 if p == 1 else 0 for p in range(1, nd + 1)])
    return [-2 * sum(b)] + b


def exact_axis(nd):
    # value at rho = 0 of an even polynomial of degree <= 2nd-2 from its values at rho = k, k = 1..nd
    A = [[Fraction(k * k) ** p for k in range(1, nd + 1)] for p in range(nd)]
    return solve_exact(A, [1 if p == 0 else 0 for p in range(nd)])


EXACT = {"staggered": exact_staggered, "halfshift": exact_halfshift, "d1": exact_d1,
         "d2": exact_d2, "axis": exact_axis}


@pytest.mark.parametrize("kind", sorted(EXACT))
@pytest.mark.parametrize("nd", list(range(1, 17)))
def test_coefficients_match_moment_conditions(kind, nd):
    got = oracle.coef(kind, nd)
    want = np.array([float(x) for x in EXACT[kind](nd)])
    scale = np.max(np.abs(want))
    assert np.max(np.abs(got - want)) <= 4e-15 * nd * scale, (got, want)


def test_axis_weights_printed_in_paper():
    with open(os.path.join(GOLDEN, "axis_weights_order10.txt")) as fh:
        vals = [Fraction(line.strip()) for line in fh if line.strip() and not line.startswith("#")]
    assert vals == exact_axis(5)  # the independent derivation reproduces the printed rationals
    got = oracle.coef("axis", 5)
    assert np.allclose(got, [float(v) for v in vals], rtol=1e-15, atol=0)


def test_textbook_low_orders():
    assert np.allclose(oracle.coef("staggered", 1), [1.0])                       # Yee
    assert np.allclose(oracle.coef("staggered", 2), [9 / 8, -1 / 24])
    assert np.allclose(oracle.coef("halfshift", 1), [0.5])                      # linear midpoint
    assert np.allclose(oracle.coef("halfshift", 2), [9 / 16, -1 / 16])
    assert np.allclose(oracle.coef("d1", 1), [0.5])
    assert np.allclose(oracle.coef("d1", 2), [2 / 3, -1 / 12])
    assert np.allclose(oracle.coef("d2", 1), [-2.0, 1.0])
    assert np.allclose(oracle.coef("d2", 2), [-5 / 2, 4 / 3, -1 / 12])


@pytest.mark.parametrize("nd", [4, 8, 16])
def test_staggered_symbol_is_the_spectral_limit(nd):
    # The staggered stencil's symbol 2 sum a_j sin((2j-1)x/2) approximates x to order 2nd near 0
    a = oracle.coef("staggered", nd)
    x = 0.05
    sym = 2 * sum(a[j] * np.sin((2 * j + 1) * x / 2) for j in range(nd))
    assert abs(sym - x) < 1e-15 + x ** (2 * nd + 1)
