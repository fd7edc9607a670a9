"""Coefficients of the polynomial q in sin_phase64 (phase64.hpp).

sin r = r + r^3 q(r^2) on |r| <= pi/2, with q of degree 7 in s = r^2: the
polynomial interpolating (sin r - r) / r^3 = sum_k (-s)^k / (2k + 3)! at the
8 Chebyshev nodes of [0, (pi/2)^2], computed in exact rational arithmetic
from the Maclaurin series (summed to 55 digits) and rounded to binary64.
Interpolating at Chebyshev nodes spreads the truncation error over the
interval instead of leaving it all at its end, so 8 coefficients do what 10
Maclaurin coefficients do.  Prints the coefficients (highest degree first)
and the largest relative error of r + r^3 q(r^2) over 4000 points of
(0, pi/2], evaluated exactly with the rounded coefficients.

    python3 phase64_coefficients.py
"""
import math
from decimal import Decimal, getcontext
from fractions import Fraction

getcontext().prec = 60
PI = Decimal("3.14159265358979323846264338327950288419716939937510582097494459230781640628620899862803")
DEGREE = 7


def q_series(s: Decimal) -> Decimal:
    total, term, k = Decimal(0), Decimal(-1) / Decimal(6), 1
    while abs(term) >= Decimal(10) ** -55:
        total += term
        term = term * (-s) / (Decimal(2 * k + 2) * Decimal(2 * k + 3))
        k += 1
    return total


def coefficients(degree: int = DEGREE) -> list:
    n = degree + 1
    top = (PI / 2) ** 2
    nodes = [top / 2 * (1 + Decimal(math.cos((2 * k + 1) * math.pi / (2 * n)))) for k in range(n)]
    rows = [[Fraction(x) ** j for j in range(n)] + [Fraction(q_series(x))] for x in nodes]
    for c in range(n):  # Gauss-Jordan elimination, exact
        piv = max(range(c, n), key=lambda r: abs(rows[r][c]))
        rows[c], rows[piv] = rows[piv], rows[c]
        for r in range(n):
            if r != c and rows[r][c] != 0:
                f = rows[r][c] / rows[c][c]
                rows[r] = [a - f * b for a, b in zip(rows[r], rows[c])]
    return [float(rows[i][n] / rows[i][i]) for i in range(n)]


def max_relative_error(coef: list) -> float:
    worst = 0.0
    for t in range(1, 4001):
        r = (PI / 2) * Decimal(t) / Decimal(4000)
        s = r * r
        p = Decimal(0)
        for c in reversed(coef):
            p = p * s + Decimal(c)
        exact = r + r ** 3 * q_series(s)
        worst = max(worst, float(abs(r + r ** 3 * p - exact) / exact))
    return worst


if __name__ == "__main__":
    coef = coefficients()
    for j in reversed(range(len(coef))):
        print(f"s^{j}: {coef[j]!r}")
    print(f"max relative error: {max_relative_error(coef):.2e}")
