"""Weighted Gaussian quadrature rules for B-splines (oracle; test infrastructure only).

What is computed here, and where the paper states it:

* A rule for row j (weight function B_j, kind "mass") is a set of nodes tau_k and
  weights omega_k with  integral(B_i B_j) = sum_k omega_k B_i(tau_k) B_j(tau_k)  for
  every i whose support meets supp(B_j)  (eq:GaussQuadSys, Sec. 3.1).  For kind
  "stiffness" the same with derivatives, B'_i B'_j  (eq:GaussQuadSysStiff, Sec. 3.2).
  The weights multiply the product of both basis functions; the printed solutions
  are exact only under that reading (eq:GaussQuadW writes omega on f alone).
* Interior rows on uniform knots use the cardinal rules of Sec. 3.1.1
  (eq:WQquadratic), Sec. 3.1.2 (eq:WQcubic), Sec. 3.2.1 (eq:WQquadraticStiff) and
  Sec. 3.2.2 (eq:WQcubicStiff).  They are re-derived here from the exactness
  conditions with the paper's own extra choices: symmetry about the centre of the
  support, middle node 3/2 for p = 2, omega_1 = 1 and the smaller admissible
  tau_1 for the cubic stiffness family (eq:CubicStiffTau1W, eq:CubicStiffTau1).
  The quadratic-stiffness middle weight multiplies B'_j(3/2) = 0, so exactness
  leaves it free; the printed value 8/9 is used.
* Boundary rows (the p rows per side whose support touches the repeated end
  knots) get no rule in the paper; its closing remark of Sec. 3.2 asks for a
  modified system or standard Gauss.  Reading used here: the same exactness
  conditions on that row's interacting functions, completed to a square system
  by exactness against the first few functions of the sequence
  x^{deg+1}, (x-1)_+^{deg+1}, ...  (x in element units from the clamped end,
  deg = p for mass and p-1 for stiffness), with the node counts listed in
  ``BOUNDARY_PRESCRIPTION``.  Every such system has exactly one admissible root
  (nodes strictly inside the support, off knots, increasing; all omega > 0).
  Parity unpinned: the paper gives no boundary-row values, so the node positions
  of these rows are pinned only through their exactness (and the library's own
  solver agreeing with this one), not against printed numbers.

All solving is done with mpmath at 40 significant digits; tables handed to the
FP64 assembly are rounded once at the end.
"""
import functools

import mpmath as mp

from .bspline import basis, basis_deriv, open_uniform_knots

DPS = 40

# (p, kind, row j) -> (number of nodes n, list of extra exactness functions by index
# into the sequence x^{deg+1}, (x-1)_+^{deg+1}, (x-2)_+^{deg+1}, ...).
# Node count n = ceil(m / 2) for m independent exactness conditions, except the
# cubic stiffness row 1 where the square 2-node system has no real root.
BOUNDARY_PRESCRIPTION = {
    (2, "mass", 0): (2, 1),
    (2, "mass", 1): (2, 0),
    (3, "mass", 0): (2, 0),
    (3, "mass", 1): (3, 1),
    (3, "mass", 2): (3, 0),
    (2, "stiffness", 0): (1, 0),
    (2, "stiffness", 1): (2, 1),
    (3, "stiffness", 0): (2, 1),
    (3, "stiffness", 1): (3, 2),
    (3, "stiffness", 2): (3, 1),
}

KINDS = ("mass", "stiffness")


def _phi(kind):
    return basis if kind == "mass" else basis_deriv


@functools.lru_cache(maxsize=None)
def gauss_legendre(m):
    """m-point Gauss-Legendre nodes and weights on [0, 1] (mpmath, DPS digits).

    Nodes are the roots of the Legendre polynomial P_m, found by Newton from the
    usual cosine guesses; weights 2 / ((1 - y^2) P_m'(y)^2) mapped to [0, 1].
    """
    with mp.workdps(DPS + 10):
        nodes, weights = [], []
        for k in range(m):
            y = mp.cos(mp.pi * (k + mp.mpf(3) / 4) / (m + mp.mpf(1) / 2))
            for _ in range(100):
                p0, p1 = mp.mpf(1), y
                for n in range(2, m + 1):
                    p0, p1 = p1, ((2 * n - 1) * y * p1 - (n - 1) * p0) / n
                dp = m * (y * p1 - p0) / (y * y - 1)
                dy = p1 / dp
                y -= dy
                if abs(dy) < mp.mpf(10) ** (-(DPS + 8)):
                    break
            p0, p1 = mp.mpf(1), y
            for n in range(2, m + 1):
                p0, p1 = p1, ((2 * n - 1) * y * p1 - (n - 1) * p0) / n
            dp = m * (y * p1 - p0) / (y * y - 1)
            w = 2 / ((1 - y * y) * dp * dp)
            nodes.append((1 - y) / 2)
            weights.append(w / 2)
        order = sorted(range(m), key=lambda k: nodes[k])
        return tuple(nodes[k] for k in order), tuple(weights[k] for k in order)


def integrate(f, lo, hi, m):
    """Integral of f over [lo, hi] (integers, element units), element by element with
    m-point Gauss-Legendre: exact for piecewise polynomials of degree <= 2m-1 whose
    breakpoints are integers."""
    xs, ws = gauss_legendre(m)
    total = mp.mpf(0)
    for e in range(lo, hi):
        for x, w in zip(xs, ws):
            total += w * f(e + x)
    return total


def _exactness_system(knots, p, kind, j, tests):
    """Residual function of the exactness conditions for row j:
    r_g(nodes, omegas) = sum_k omega_k g(tau_k) phi_j(tau_k) - int_{supp B_j} g phi_j,
    one entry per test function g.  The integrals are computed once, exactly."""
    phi = _phi(kind)
    lo = int(knots[j])
    hi = int(knots[j + p + 1])
    exact = [integrate(lambda x, g=g: g(x) * phi(knots, j, p, x), lo, hi, 2 * p + 2) for g in tests]

    def residuals(nodes, omegas):
        wphi = [(x, w * phi(knots, j, p, x)) for x, w in zip(nodes, omegas)]
        return [sum(wp * g(x) for x, wp in wphi) - e for g, e in zip(tests, exact)]
    return residuals


def _column_tests(knots, p, kind, cols):
    phi = _phi(kind)
    return [(lambda x, i=i: phi(knots, i, p, x)) for i in cols]


def newton(F, x0, tol=None, maxsteps=60):
    """Plain Newton-Raphson for a square system F(x) = 0 (the method the paper names for
    the cubic rules, Sec. 3.1.2).  The Jacobian is taken by forward differences with a
    step far below the working precision's square root, so convergence is quadratic up
    to ~1e-30 and the final residual is checked by the caller.  Returns None when an
    iteration meets a singular Jacobian or does not settle within ``maxsteps``."""
    tol = tol if tol is not None else mp.mpf(10) ** (-(DPS - 8))
    x = [mp.mpf(v) for v in x0]
    n = len(x)
    step = mp.mpf(10) ** (-(DPS // 2 + 2))
    for _ in range(maxsteps):
        f = F(*x)
        if max(abs(v) for v in f) < tol:
            return x
        J = mp.matrix(n, n)
        for c in range(n):
            xp = list(x)
            xp[c] += step
            fp = F(*xp)
            for r in range(n):
                J[r, c] = (fp[r] - f[r]) / step
        try:
            dx = mp.lu_solve(J, mp.matrix(f))
        except (ZeroDivisionError, TypeError):   # mpmath signals a zero pivot either way
            return None
        x = [x[k] - dx[k] for k in range(n)]
        if any(not mp.isfinite(v) or abs(v) > 1e6 for v in x):
            return None
    f = F(*x)
    return x if max(abs(v) for v in f) < tol else None


def _solve(F, starts, admissible):
    """Newton from each start in turn; the first admissible root wins."""
    for x0 in starts:
        vec = newton(F, x0)
        if vec is not None and admissible(vec):
            return vec
    return None


@functools.lru_cache(maxsize=None)
def interior_rule(p, kind):
    """Cardinal rule for an interior row: (tau, omega), tau on the support [0, p+1].

    Unknowns and extra conditions follow the paper (Sec. 3.1.1, 3.1.2, 3.2.1, 3.2.2);
    the equations are the exactness conditions eq:GaussQuadSys / eq:GaussQuadSysStiff
    against the interacting cardinal B-splines of column offsets 0..p (offsets -1..-p
    follow from the symmetry of the rule).
    """
    if p not in (2, 3) or kind not in KINDS:
        raise ValueError("rules exist for p in {2, 3} and kind in {mass, stiffness}")
    with mp.workdps(DPS):
        n_el = 4 * p + 4
        knots = open_uniform_knots(p, n_el, mp.mpf(1))
        j = 2 * p + 1                       # all 2p+1 interacting functions are cardinal
        base = j - p                        # left end of supp(B_j), element units
        half = mp.mpf(p + 1) / 2

        def rule_from(v):
            if p == 2 and kind == "mass":
                t1, w1, w2 = v
                return [t1, half, 2 * half - t1], [w1, w2, w1]
            if p == 3 and kind == "mass":
                t1, t2, w1, w2 = v
                return [t1, t2, 2 * half - t2, 2 * half - t1], [w1, w2, w2, w1]
            if p == 2:                      # stiffness, middle weight free (B'_j(3/2) = 0)
                t1, w1 = v
                return [t1, half, 2 * half - t1], [w1, mp.mpf(8) / 9, w1]
            t1, t2, w2 = v                  # cubic stiffness, omega_1 = 1
            return [t1, t2, 2 * half - t2, 2 * half - t1], [mp.mpf(1), w2, w2, mp.mpf(1)]

        n_unknown = {(2, "mass"): 3, (3, "mass"): 4, (2, "stiffness"): 2, (3, "stiffness"): 3}[(p, kind)]
        tests = _column_tests(knots, p, kind, [j + off for off in range(n_unknown)])

        system = _exactness_system(knots, p, kind, j, tests)

        def F(*v):
            tau, om = rule_from(list(v))
            return system([base + t for t in tau], om)

        def admissible(v):
            tau, om = rule_from(v)
            in_elem = all(q < tau[q] < q + 1 for q in range(p + 1))
            if p == 3 and kind == "stiffness":
                # the two admissible roots are 1/2 +- d (eq:CubicStiffTau1); take the smaller
                in_elem = in_elem and tau[0] < mp.mpf(1) / 2
            return in_elem and all(w > 0 for w in om)

        starts = []
        for off in (mp.mpf(1) / 2, mp.mpf(1) / 4, mp.mpf(3) / 4, mp.mpf(1) / 3):
            for w in (mp.mpf(1), mp.mpf(1) / 2):
                if p == 2 and kind == "mass":
                    starts.append([off, w, w])
                elif p == 3 and kind == "mass":
                    starts.append([off, 1 + off, w, w])
                elif p == 2:
                    starts.append([off, w])
                else:
                    starts.append([off, 1 + off, w])
        root = _solve(F, starts, admissible)
        if root is None:
            raise RuntimeError(f"no admissible interior rule found for p={p}, {kind}")
        tau, om = rule_from(root)
        return tuple(tau), tuple(om)


def _extra_function(k, deg):
    # k-th member of x^{deg+1}, (x-1)_+^{deg+1}, (x-2)_+^{deg+1}, ...
    def g(x):
        y = x - k
        return y ** (deg + 1) if y > 0 else mp.mpf(0)
    return g


@functools.lru_cache(maxsize=None)
def boundary_rule(p, kind, j):
    """Rule for left boundary row j < p: (tau, omega), tau in element units from the
    clamped end, on supp(B_j) = [0, j+1].  Rows at the right end mirror it (tau -> -tau
    about the right end; omega unchanged)."""
    if (p, kind, j) not in BOUNDARY_PRESCRIPTION:
        raise ValueError(f"no boundary rule for p={p}, {kind}, row {j}")
    n, n_extra = BOUNDARY_PRESCRIPTION[(p, kind, j)]
    with mp.workdps(DPS):
        n_el = 4 * p + 4
        knots = open_uniform_knots(p, n_el, mp.mpf(1))
        cols = list(range(0, j + p + 1))
        if kind == "stiffness":
            cols = cols[:-1]                 # sum_i B'_i = 0 makes one condition dependent
        deg = p if kind == "mass" else p - 1
        tests = _column_tests(knots, p, kind, cols) + [_extra_function(k, deg) for k in range(n_extra)]
        assert len(tests) == 2 * n, (p, kind, j, len(tests), n)

        system = _exactness_system(knots, p, kind, j, tests)

        def F(*v):
            return system(list(v[:n]), list(v[n:]))

        def admissible(v):
            tau, om = v[:n], v[n:]
            ok = all(0 < t < j + 1 for t in tau)
            ok = ok and all(tau[k] < tau[k + 1] for k in range(n - 1))
            ok = ok and all(abs(t - mp.nint(t)) > mp.mpf(10) ** -8 for t in tau)
            return ok and all(w > 0 for w in om)

        starts = []
        L = mp.mpf(j + 1)
        for shift in (mp.mpf(1) / 2, mp.mpf(1) / 4, mp.mpf(3) / 4, mp.mpf(1) / 3, mp.mpf(2) / 3):
            for spread in (mp.mpf(1), mp.mpf(3) / 4):
                tau0 = [L * (k + shift) / n * spread + L * (1 - spread) / 2 for k in range(n)]
                for w in (mp.mpf(1) / 2, mp.mpf(1)):
                    starts.append(tau0 + [w] * n)
        v = _solve(F, starts, admissible)
        if v is None:
            raise RuntimeError(f"no admissible boundary rule for p={p}, {kind}, row {j}")
        return tuple(v[:n]), tuple(v[n:])


def row_rule(p, n_el, kind, j):
    """Rule for row j of an N_el-element open uniform space, in element units on [0, N_el].

    Returns (nodes, omegas) as mpmath numbers, padded to Q = p+1 entries: padding nodes
    carry weight 0 and sit in the middle of the support's outermost element (h/2 from
    the clamped end), so that every row samples exactly Q points per direction.
    """
    n = n_el + p
    Q = p + 1
    if not 0 <= j < n:
        raise IndexError(j)
    if p <= j < n - p:
        tau, om = interior_rule(p, kind)
        return [mp.mpf(j - p) + t for t in tau], list(om)
    if j < p:
        tau, om = boundary_rule(p, kind, j)
        nodes, oms = list(tau), list(om)
        pad = mp.mpf(1) / 2
    else:
        tau, om = boundary_rule(p, kind, n - 1 - j)
        nodes = [mp.mpf(n_el) - t for t in reversed(tau)]
        oms = list(reversed(om))
        pad = mp.mpf(n_el) - mp.mpf(1) / 2
    while len(nodes) < Q:
        nodes.append(pad)
        oms.append(mp.mpf(0))
    return nodes, oms


def direction_table(p, n_el, kind):
    """FP64 rule table of one direction: nodes x[j][q] in [0, 1] and physical weights
    omega[j][q] (= h * omega in element units; the same factor serves mass and
    stiffness because B' carries 1/h).  Lists of n = N_el + p rows of Q = p+1 floats."""
    xs, ws = [], []
    with mp.workdps(DPS):
        h = mp.mpf(1) / n_el
        for j in range(n_el + p):
            nodes, oms = row_rule(p, n_el, kind, j)
            xs.append([float(x * h) for x in nodes])
            ws.append([float(w * h) for w in oms])
    return xs, ws


def exactness_residual(p, n_el, kind, j, nodes, omegas):
    """Largest |sum_q omega_q phi_i(x_q) phi_j(x_q) - int phi_i phi_j| over the columns i
    interacting with row j, for a row rule given in parametric units on [0, 1]
    (floats).  Evaluated in mpmath, relative to the largest exact entry of the row."""
    with mp.workdps(DPS):
        knots = open_uniform_knots(p, n_el, mp.mpf(1))
        phi = _phi(kind)
        n = n_el + p
        el = [mp.mpf(x) * n_el for x in nodes]
        om = [mp.mpf(w) * n_el for w in omegas]
        lo, hi = int(knots[j]), int(knots[j + p + 1])
        worst, scale = mp.mpf(0), mp.mpf(0)
        for i in range(max(0, j - p), min(n, j + p + 1)):
            quad = sum(w * phi(knots, i, p, x) * phi(knots, j, p, x) for x, w in zip(el, om))
            exact = integrate(lambda x: phi(knots, i, p, x) * phi(knots, j, p, x), lo, hi, 2 * p + 2)
            worst = max(worst, abs(quad - exact))
            scale = max(scale, abs(exact))
        return float(worst / scale)
