"""Exact rational arithmetic on cardinal B-splines, written independently of the oracle.

The cardinal B-spline of degree p on the integer knots 0..p+1 is the truncated-power
sum  B(x) = (1/p!) sum_{k=0}^{p+1} (-1)^k C(p+1, k) (x - k)_+^p,  and its derivative
is the same sum of degree p-1 divided by (p-1)!.  On each unit interval [e, e+1] it
is a polynomial, expanded here with Fractions, so products integrate exactly.
"""
from fractions import Fraction
from math import comb, factorial, floor

import mpmath as mp


def _poly_shift_power(k, n):
    """Coefficients (ascending powers of x) of (x - k)^n."""
    return [Fraction(comb(n, m)) * Fraction(-k) ** (n - m) for m in range(n + 1)]


def _add(a, b):
    out = [Fraction(0)] * max(len(a), len(b))
    for i, v in enumerate(a):
        out[i] += v
    for i, v in enumerate(b):
        out[i] += v
    return out


def _scale(a, s):
    return [v * s for v in a]


def _mul(a, b):
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, u in enumerate(a):
        for j, v in enumerate(b):
            out[i + j] += u * v
    return out


def piece(p, e, deriv=False, shift=0):
    """Polynomial of B(x - shift) (or B'(x - shift)) on [e, e+1] (ascending coefficients)."""
    n = p - 1 if deriv else p
    norm = Fraction(1, factorial(n))
    out = [Fraction(0)]
    for k in range(p + 2):
        if k + shift <= e:                     # (x - shift - k)_+ is active on [e, e+1]
            term = _poly_shift_power(k + shift, n)
            out = _add(out, _scale(term, norm * (-1) ** k * comb(p + 1, k)))
    return out


def evaluate(poly, x):
    if isinstance(x, Fraction):
        return sum(c * x ** i for i, c in enumerate(poly))
    x = mp.mpf(x)
    return sum(mp.mpf(c.numerator) / c.denominator * x ** i for i, c in enumerate(poly))


def value(p, x, deriv=False):
    """B(x) or B'(x) for rational or mpmath x (0 outside [0, p+1])."""
    e = floor(x) if isinstance(x, Fraction) else int(mp.floor(x))
    if e < 0 or e > p:
        return Fraction(0) if isinstance(x, Fraction) else mp.mpf(0)
    return evaluate(piece(p, e, deriv), x)


def gram(p, offset, deriv=False):
    """Exact integral of B(x) B(x - offset) (or of the derivatives) over [0, p+1]."""
    total = Fraction(0)
    for e in range(p + 1):
        prod = _mul(piece(p, e, deriv), piece(p, e, deriv, shift=offset))
        for i, c in enumerate(prod):
            total += c * (Fraction(e + 1) ** (i + 1) - Fraction(e) ** (i + 1)) / (i + 1)
    return total
