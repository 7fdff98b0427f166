"""B-spline basis on open uniform knot vectors (oracle; test infrastructure only).

Sec. 2.2: per direction the knot vector is open (the end knots repeated p+1
times) with simple interior knots, so the space has maximal continuity C^{p-1}
(eq:Gmap3) and dimension p + N_el (eq:DimUni).

Values come from the Cox-de Boor recursion written out directly.  The function
works with any number type that supports + - * / and comparison (Python float,
``fractions.Fraction``, ``mpmath.mpf``), so the same code serves the
high-precision rule derivation and FP64 checks.
"""


def open_uniform_knots(p, n_el, one=1):
    """Knot vector of eq:Gmap3 in *element units*: p+1 zeros, 1..N_el-1, p+1 copies of N_el.

    ``one`` fixes the number type (1, Fraction(1), mpf(1)).  Multiply by h = 1/N_el
    for the parametric domain [0, 1].
    """
    zero = one * 0
    return [zero] * p + [one * k for k in range(n_el + 1)] + [one * n_el] * p


def basis(knots, i, p, x):
    """B_{i,p}(x) by the Cox-de Boor recursion.

    Degree-0 pieces are right-continuous indicator functions of [t_k, t_{k+1});
    at the very last knot the last non-empty interval is taken closed so that the
    basis still sums to one at the right end of the domain.
    """
    last = knots[-1]
    # degree 0 values for the p+1 consecutive intervals that B_{i,p} rests on
    vals = []
    for k in range(i, i + p + 1):
        a, b = knots[k], knots[k + 1]
        inside = (a <= x < b) or (x == last and b == last and a < b)
        vals.append(x * 0 + (1 if inside else 0))
    # raise the degree one step at a time
    for deg in range(1, p + 1):
        nxt = []
        for k in range(i, i + p + 1 - deg):
            term = x * 0
            d1 = knots[k + deg] - knots[k]
            if d1 != 0:
                term = term + (x - knots[k]) / d1 * vals[k - i]
            d2 = knots[k + deg + 1] - knots[k + 1]
            if d2 != 0:
                term = term + (knots[k + deg + 1] - x) / d2 * vals[k - i + 1]
            nxt.append(term)
        vals = nxt
    return vals[0]


def basis_deriv(knots, i, p, x):
    """d/dx B_{i,p}(x) from the standard derivative formula for B-splines.

    B'_{i,p} = p/(t_{i+p}-t_i) B_{i,p-1} - p/(t_{i+p+1}-t_{i+1}) B_{i+1,p-1},
    with a term dropped when its knot span is empty.
    """
    out = x * 0
    d1 = knots[i + p] - knots[i]
    if d1 != 0:
        out = out + p / d1 * basis(knots, i, p - 1, x)
    d2 = knots[i + p + 1] - knots[i + 1]
    if d2 != 0:
        out = out - p / d2 * basis(knots, i + 1, p - 1, x)
    return out
