"""Pins for the oracle's rule derivation and B-spline evaluation (CPU only).

Each check ties the oracle to something other than itself: the digits and closed
forms the paper prints, exact rational integrals from the truncated-power form of
the cardinal B-spline, classical identities of the B-spline basis, and numpy's
Gauss-Legendre rule.
"""
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

import exact_cardinal as ec
import golden_io
from oracle import bspline, rules

mp.mp.dps = 40


def _as_mp(v):
    return mp.mpf(v.numerator) / v.denominator if isinstance(v, Fraction) else mp.mpf(v)


# --- B-spline evaluation -------------------------------------------------------------

@pytest.mark.parametrize("p", [2, 3])
def test_cardinal_basis_equals_truncated_power_form(p):
    # interior functions of an open uniform knot vector are cardinal translates
    n_el = 4 * p + 3
    knots = bspline.open_uniform_knots(p, n_el, Fraction(1))
    j = 2 * p                                 # knots j..j+p+1 are simple
    shift = j - p                             # support of B_j starts at element shift
    for num in range(0, 4 * (p + 1) + 1):
        x = Fraction(num, 4) + shift
        for deriv in (False, True):
            f = bspline.basis_deriv if deriv else bspline.basis
            got = f(knots, j, p, x)
            want = ec.value(p, x - shift, deriv)
            if deriv and (x - shift) in (0, p + 1):
                continue                      # one-sided at the support ends
            assert got == want, (p, x, deriv)


@pytest.mark.parametrize("p,n_el", [(2, 3), (2, 7), (3, 4), (3, 9)])
def test_open_basis_partition_of_unity_and_marsden(p, n_el):
    # sum_i B_i = 1 and sum_i xi_i B_i = x with Greville abscissae xi_i = (t_{i+1}+..+t_{i+p})/p,
    # and the derivatives sum to 0 -- exact in rational arithmetic at rational points
    knots = bspline.open_uniform_knots(p, n_el, Fraction(1))
    n = n_el + p
    grev = [sum(knots[i + 1:i + p + 1]) / p for i in range(n)]
    for num in range(0, 7 * n_el + 1):
        x = Fraction(num, 7)
        vals = [bspline.basis(knots, i, p, x) for i in range(n)]
        assert sum(vals) == 1
        assert sum(g * v for g, v in zip(grev, vals)) == x
        assert all(v >= 0 for v in vals)
        ders = [bspline.basis_deriv(knots, i, p, x) for i in range(n)]
        assert sum(ders) == 0


@pytest.mark.parametrize("p", [2, 3])
def test_clamped_end_function(p):
    # B_0 = (1 - x)^p on the first element of an open knot vector (element units)
    knots = bspline.open_uniform_knots(p, 6, Fraction(1))
    for num in range(0, 9):
        x = Fraction(num, 8)
        assert bspline.basis(knots, 0, p, x) == (1 - x) ** p
        assert bspline.basis_deriv(knots, 0, p, x) == -p * (1 - x) ** (p - 1)


def test_gauss_legendre_matches_numpy():
    for m in (3, 4, 6, 8):
        xs, ws = rules.gauss_legendre(m)
        ref_x, ref_w = np.polynomial.legendre.leggauss(m)
        np.testing.assert_allclose([float(x) for x in xs], (ref_x + 1) / 2, rtol=0, atol=1e-15)
        np.testing.assert_allclose([float(w) for w in ws], ref_w / 2, rtol=0, atol=1e-15)


# --- exact integrals behind the rules ------------------------------------------------

@pytest.mark.parametrize("key,value", sorted(golden_io.gram_rhs().items()))
def test_printed_rhs_equals_exact_cardinal_gram(key, value):
    kind, p, off = key
    assert ec.gram(p, off, deriv=(kind == "stiffness")) == value


@pytest.mark.parametrize("kind", ["mass", "stiffness"])
@pytest.mark.parametrize("p", [2, 3])
def test_oracle_integrals_equal_exact_gram(kind, p):
    # oracle's own basis + element-wise Gauss-Legendre reproduce the rational values
    n_el = 4 * p + 4
    knots = bspline.open_uniform_knots(p, n_el, mp.mpf(1))
    f = bspline.basis if kind == "mass" else bspline.basis_deriv
    j = 2 * p + 1
    for off in range(p + 1):
        got = rules.integrate(lambda x: f(knots, j, p, x) * f(knots, j + off, p, x),
                              j - p, j + 1, 2 * p + 2)
        assert abs(got - _as_mp(ec.gram(p, off, kind == "stiffness"))) < mp.mpf(10) ** -35


# --- interior rules --------------------------------------------------------------------

@pytest.mark.parametrize("kind,p", [("mass", 2), ("mass", 3), ("stiffness", 2), ("stiffness", 3)])
def test_interior_rule_reproduces_printed_digits(kind, p):
    printed = golden_io.interior_rules()[(kind, p)]
    tau, om = rules.interior_rule(p, kind)
    names = {"tau1": tau[0], "tau2": tau[1], "omega1": om[0], "omega2": om[1]}
    for name, want in printed.items():
        # 20 printed decimals: agreement to 1e-19 (last digit rounded)
        assert abs(names[name] - _as_mp(want)) < mp.mpf("1e-19"), (kind, p, name)
    # symmetric partners
    assert abs(tau[-1] - (p + 1 - tau[0])) < mp.mpf(10) ** -30
    assert om[-1] == om[0]


def test_cubic_stiffness_tau1_closed_form():
    # eq:CubicStiffTau1 with omega_1 = 1, and tau_1 a root of eq:CubicStiffTau1W
    tau, om = rules.interior_rule(3, "stiffness")
    closed = mp.mpf(1) / 2 - mp.sqrt(225 - 30 * mp.sqrt(30)) / 30
    assert abs(tau[0] - closed) < mp.mpf(10) ** -30
    x = tau[0]
    assert abs(30 * x ** 4 - 60 * x ** 3 + 30 * x ** 2 - 1) < mp.mpf(10) ** -30


@pytest.mark.parametrize("kind,p", [("mass", 2), ("mass", 3), ("stiffness", 2), ("stiffness", 3)])
def test_printed_rules_are_exact(kind, p):
    # the printed rule, evaluated with the truncated-power basis, integrates every
    # product of interacting cardinal functions exactly (eq:GaussQuadSys, eq:GaussQuadSysStiff)
    pr = golden_io.interior_rules()[(kind, p)]
    t = [_as_mp(pr["tau1"]), _as_mp(pr["tau2"])]
    w = [_as_mp(pr["omega1"]), _as_mp(pr["omega2"])]
    if p == 2:
        tau, om = [t[0], t[1], 3 - t[0]], [w[0], w[1], w[0]]
    else:
        tau, om = [t[0], t[1], 4 - t[1], 4 - t[0]], [w[0], w[1], w[1], w[0]]
    deriv = kind == "stiffness"
    for off in range(-p, p + 1):
        quad = sum(o * ec.value(p, x, deriv) * ec.value(p, x - off, deriv) for x, o in zip(tau, om))
        exact = _as_mp(ec.gram(p, abs(off), deriv))
        assert abs(quad - exact) < mp.mpf("1e-19"), (kind, p, off)


def test_printed_reduced_systems_and_errata():
    # the paper's reduced systems at its printed solutions; two printed lines only hold
    # after the corrections read into them (sign of the second quadratic-stiffness
    # line; tau_1 instead of tau_2 in the omega_1 term of the third cubic-stiffness line)
    r = golden_io.interior_rules()
    eps = mp.mpf("1e-18")
    t1, w1, w2 = (_as_mp(r[("mass", 2)][k]) for k in ("tau1", "omega1", "omega2"))
    assert abs(w1 * t1 ** 2 * (1 - t1) ** 2 / 4 - mp.mpf(1) / 120) < eps
    assert abs(w1 * t1 ** 2 * (-2 * t1 ** 2 + 2 * t1 + 1) / 4 + 3 * w2 / 32 - mp.mpf(13) / 60) < eps
    assert abs(w1 * t1 ** 4 / 2 + 9 * w2 / 16 - mp.mpf(11) / 20) < eps

    def cubic_mass(t1, t2, w1, w2):
        g = t2 ** 3 - 4 * t2 ** 2 + 4 * t2 - mp.mpf(4) / 3
        return [w1 * t1 ** 3 * (1 - t1) ** 3 / 36 - mp.mpf(1) / 5040,
                w1 * t1 ** 3 * (t1 ** 3 / 12 - t1 ** 2 / 6 + mp.mpf(1) / 9) - w2 * (2 - t2) ** 3 * g / 12
                - mp.mpf(1) / 42,
                -w1 * t1 ** 3 * (t1 ** 3 - t1 ** 2 - t1 - mp.mpf(1) / 3) / 12
                - w2 * (t2 ** 3 - mp.mpf(9) / 2 * t2 ** 2 + 6 * t2 - mp.mpf(3) / 2) * g / 3 - mp.mpf(397) / 1680,
                w1 * t1 ** 6 / 18 + w2 * g ** 2 / 2 - mp.mpf(151) / 315]
    c = r[("mass", 3)]
    assert max(abs(v) for v in cubic_mass(*(_as_mp(c[k]) for k in ("tau1", "tau2", "omega1", "omega2")))) < eps
    # the spurious root printed as a warning also solves the reduced system
    wr = golden_io.wrong_cubic_root()
    assert max(abs(v) for v in cubic_mass(wr["tau1"], wr["tau2"], wr["omega1"], wr["omega2"])) < eps

    t1, w1 = mp.mpf(3) / 4, mp.mpf(8) / 9
    assert abs(w1 * t1 * (1 - t1) - mp.mpf(1) / 6) < eps
    assert abs(w1 * t1 * (1 - 2 * t1) - mp.mpf(1) / 3) > mp.mpf("0.5")       # as printed: fails
    assert abs(w1 * t1 * (1 - 2 * t1) + mp.mpf(1) / 3) < eps                 # corrected sign
    assert abs(2 * w1 * t1 ** 2 - 1) < eps

    s = r[("stiffness", 3)]
    t1, t2, w1, w2 = (_as_mp(s[k]) for k in ("tau1", "tau2", "omega1", "omega2"))
    assert abs(w1 * t1 ** 2 * (1 - t1) ** 2 / 4 - mp.mpf(1) / 120) < eps
    assert abs(w1 * t1 ** 3 * (4 - 3 * t1) / 4 - 3 * w2 * (t2 - 2) ** 3 * (t2 - mp.mpf(2) / 3) / 4
               - mp.mpf(1) / 5) < eps
    third = lambda a: (w1 * t1 ** 2 * (3 * a ** 2 - 2 * a - 1) / 4
                       + 3 * w2 * (t2 - 1) * (t2 - 2) ** 2 * (t2 - mp.mpf(2) / 3) - mp.mpf(1) / 8)
    assert abs(third(t2)) > mp.mpf("0.01")                                      # as printed: fails
    assert abs(third(t1)) < eps                                                 # corrected
    assert abs(w1 * t1 ** 4 / 2 + 9 * w2 * (t2 - 2) ** 2 * (t2 - mp.mpf(2) / 3) ** 2 / 2
               - mp.mpf(2) / 3) < eps


def test_wrong_cubic_root_fails_true_exactness():
    # it solves the reduced polynomial system yet breaks exactness: node 2 left its element
    wr = golden_io.wrong_cubic_root()
    t = [wr["tau1"], wr["tau2"], 4 - wr["tau2"], 4 - wr["tau1"]]
    w = [wr["omega1"], wr["omega2"], wr["omega2"], wr["omega1"]]
    quad = sum(o * ec.value(3, x) ** 2 for x, o in zip(t, w))
    assert abs(quad - _as_mp(ec.gram(3, 0))) > mp.mpf("0.04")
    # ... and the oracle's validator refuses it on a real interior row
    n_el, j = 12, 7
    nodes = [float((j - 3 + x) / n_el) for x in t]
    oms = [float(o / n_el) for o in w]
    assert rules.exactness_residual(3, n_el, "mass", j, nodes, oms) > 1e-2


# --- boundary rules and whole-direction tables ----------------------------------------

@pytest.mark.parametrize("key", sorted(rules.BOUNDARY_PRESCRIPTION))
def test_boundary_rule_admissible_and_exact(key):
    p, kind, j = key
    tau, om = rules.boundary_rule(p, kind, j)
    n, _ = rules.BOUNDARY_PRESCRIPTION[key]
    assert len(tau) == n <= p + 1
    assert all(0 < t < j + 1 for t in tau)
    assert all(abs(t - mp.nint(t)) > 1e-6 for t in tau)
    assert all(a < b for a, b in zip(tau, tau[1:]))
    assert all(w > 0 for w in om)
    # high-precision exactness residual on every interacting column
    n_el = 4 * p + 4
    knots = bspline.open_uniform_knots(p, n_el, mp.mpf(1))
    f = bspline.basis if kind == "mass" else bspline.basis_deriv
    for i in range(0, j + p + 1):
        quad = sum(o * f(knots, i, p, x) * f(knots, j, p, x) for x, o in zip(tau, om))
        exact = rules.integrate(lambda x: f(knots, i, p, x) * f(knots, j, p, x), 0, j + 1, 2 * p + 2)
        assert abs(quad - exact) < mp.mpf(10) ** -30


@pytest.mark.parametrize("p,n_el", [(2, 3), (2, 5), (2, 9), (3, 4), (3, 7), (3, 10)])
@pytest.mark.parametrize("kind", ["mass", "stiffness"])
def test_direction_tables_exact(p, n_el, kind):
    xs, ws = rules.direction_table(p, n_el, kind)
    n = n_el + p
    for j in range(n):
        assert rules.exactness_residual(p, n_el, kind, j, xs[j], ws[j]) < 1e-14


@pytest.mark.parametrize("p,n_el", [(2, 6), (3, 8)])
def test_direction_table_layout(p, n_el):
    h = 1.0 / n_el
    n = n_el + p
    for kind in ("mass", "stiffness"):
        xs, ws = rules.direction_table(p, n_el, kind)
        assert len(xs) == n and all(len(r) == p + 1 for r in xs)
        for j in range(n):
            lo = max(0, j - p) * h
            hi = min(n_el, j + 1) * h
            for x, w in zip(xs[j], ws[j]):
                assert lo < x < hi
                assert abs(x / h - round(x / h)) > 1e-9
                assert w >= 0
            # mirror symmetry of the whole table
            mj = n - 1 - j
            real = [x for x, w in zip(xs[j], ws[j]) if w > 0]
            mirror = [1 - x for x, w in zip(xs[mj], ws[mj]) if w > 0]
            np.testing.assert_allclose(sorted(real), sorted(mirror), rtol=0, atol=1e-15)
        # interior rows are translates of the cardinal rule scaled by h
        tau, om = rules.interior_rule(p, kind)
        for j in range(p, n - p):
            np.testing.assert_allclose(xs[j], [(j - p + float(t)) * h for t in tau], rtol=0, atol=1e-15)
            np.testing.assert_allclose(ws[j], [float(o) * h for o in om], rtol=1e-15)
