"""Weighted Gaussian rules on non-uniform knots by homotopy continuation (oracle; test
infrastructure only).

The paper derives its rules for uniform knots and names non-uniform knots as future work:
Newton needs a good initial guess, and the cited way to get one is to start from a known
rule and move the knot vector continuously to the target one, tracking the root
(Sec. 1 on homotopy continuation; remark on the cubic system in Sec. 3.1.2; Conclusion).
Here every row is tracked separately along the straight path
    t(lam) = (1 - lam) t_uniform + lam t_target,  lam in [0, 1],
of its open knot vector in element units (breakpoints b_k scaled by N_el, so the uniform
space has integer knots), starting from that row's uniform rule (``oracle.rules``).

The exactness conditions are those of the uniform rules (eq:GaussQuadSys,
eq:GaussQuadSysStiff) on the row's interacting functions.  The uniform interior rules
fix their remaining freedom by symmetry (and, for the cubic stiffness rule, omega_1 = 1);
on non-uniform knots symmetry is gone, so it is replaced by the condition it leaves in
each element's own coordinate r = (x - t_e) / (t_{e+1} - t_e) of the node's element e:
  * quadratic mass rows: the middle node at r = 1/2 (the paper's tau_2 = 3/2);
  * cubic mass and stiffness rows: the outer nodes mirrored, r_1 + r_4 = 1; the cubic
    stiffness rows also keep omega_1 equal to the length of the first element of the
    support in element units (1 on uniform knots, the paper's choice);
  * quadratic stiffness rows: the middle node at the zero of B'_j in the middle element
    (3/2 on uniform knots), where its weight multiplies 0 and keeps the printed 8/9.
(A first attempt with exactness for an odd power about the support centre folded back
within a small deformation; these linear conditions follow the rules smoothly.)

A path can end in a genuine singularity: the stiffness weight function B'_j changes sign,
and on strongly perturbed knots a node of a stiffness rule can meet its zero, where the
node's weight diverges.  The row then has no rule of this family and the solver raises.
Boundary rows keep their square systems (the exactness conditions completed by the
truncated powers (x - t)_+^(deg+1) at the first distinct knots from the clamped end,
``rules.BOUNDARY_PRESCRIPTION``), now with the actual knots.

Parity unpinned: the paper prints no rule on non-uniform knots.  These rules are pinned
by their exactness on the target knots, by reducing to the paper's rules on uniform
breakpoints, and by the conditions above holding; the particular member of each family
is this reading's choice.
"""
import functools

import mpmath as mp

from . import rules
from .bspline import basis, basis_deriv

DPS = rules.DPS
DPS_PATH = 30        # digits along the path; the end point is polished at DPS


def knot_vector(p, breaks):
    """Open knot vector in element units from breakpoints 0 = b_0 < ... < b_N = 1."""
    N = len(breaks) - 1
    b = [mp.mpf(x) * N for x in breaks]
    return [b[0]] * p + b + [b[-1]] * p


def _uniform_knot_vector(p, N):
    return [mp.mpf(0)] * p + [mp.mpf(k) for k in range(N + 1)] + [mp.mpf(N)] * p


def _integrate(f, kv, lo, hi, m):
    """Integral of f over the knot spans [kv[e], kv[e+1]], e = lo .. hi-1, m-point
    Gauss-Legendre per span: exact for piecewise polynomials of degree <= 2m-1 with
    breakpoints at the knots."""
    xs, ws = rules.gauss_legendre(m)
    total = mp.mpf(0)
    for e in range(lo, hi):
        a, b = kv[e], kv[e + 1]
        if b <= a:
            continue
        L = b - a
        for x, w in zip(xs, ws):
            total += w * L * f(a + L * x)
    return total


class _Row:
    """The square system of one row on a given knot vector: unknown vector v, expand(v)
    -> (nodes, omegas) in element units, residual F(v), admissibility."""

    def __init__(self, p, kind, j, n):
        self.p, self.kind, self.j, self.n = p, kind, j, n
        self.phi = basis if kind == "mass" else basis_deriv
        self.interior = p <= j < n - p

    def setup(self, kv):
        p, j, n, phi = self.p, self.j, self.n, self.phi
        self.kv = kv
        tests = []
        if self.interior:
            cols = list(range(j - p, j + p + 1))
            if self.kind == "mass":
                tests = [lambda x, i=i: phi(kv, i, p, x) for i in cols]
            else:
                tests = [lambda x, i=i: phi(kv, i, p, x) for i in cols[:-1]]
                if p == 2:
                    # zero of B'_j in the middle element, where B'_j is linear
                    a, b = kv[j + 1], kv[j + 2]
                    da, db = phi(kv, j, p, a), phi(kv, j, p, b)      # B'_j is continuous (C^1 space)
                    self.mid = a + da * (b - a) / (da - db)
        else:
            left = j < p
            jj = j if left else n - 1 - j
            nn, extra = rules.BOUNDARY_PRESCRIPTION[(p, self.kind, jj)]
            self.nn = nn
            deg = p if self.kind == "mass" else p - 1
            if left:
                cols = list(range(0, j + p + 1))
                if self.kind == "stiffness":
                    cols = cols[:-1]
                tests = [lambda x, i=i: phi(kv, i, p, x) for i in cols]
                for k in range(extra):
                    t = kv[p + k]
                    tests.append(lambda x, t=t: (x - t) ** (deg + 1) if x > t else mp.mpf(0))
            else:
                cols = list(range(j - p, n))
                if self.kind == "stiffness":
                    cols = cols[1:]
                tests = [lambda x, i=i: phi(kv, i, p, x) for i in cols]
                for k in range(extra):
                    t = kv[n - k]
                    tests.append(lambda x, t=t: (t - x) ** (deg + 1) if x < t else mp.mpf(0))
        self.tests = tests
        m = 2 * p + 2
        self.exact = [_integrate(lambda x, g=g: g(x) * phi(kv, j, p, x), kv, j, j + p + 1, m) for g in tests]

    def _rel(self, q, x):
        # coordinate of x in element q of the support, 0 .. 1
        a, b = self.kv[self.j + q], self.kv[self.j + q + 1]
        return (x - a) / (b - a)

    def expand(self, v):
        p, kv, j = self.p, self.kv, self.j
        if not self.interior:
            return list(v[:self.nn]), list(v[self.nn:])
        if self.kind == "mass" and p == 2:
            return [v[0], (kv[j + 1] + kv[j + 2]) / 2, v[1]], list(v[2:])
        if self.kind == "mass":
            return list(v[:4]), list(v[4:])
        if p == 2:
            return [v[0], self.mid, v[1]], [v[2], mp.mpf(8) / 9, v[3]]
        return list(v[:4]), [kv[j + 1] - kv[j]] + list(v[4:])

    def unknowns(self, tau, om):
        p = self.p
        if not self.interior:
            return list(tau) + list(om)
        if self.kind == "mass" and p == 2:
            return [tau[0], tau[2]] + list(om)
        if self.kind == "mass":
            return list(tau) + list(om)
        if p == 2:
            return [tau[0], tau[2], om[0], om[2]]
        return list(tau) + list(om[1:])

    def F(self, *v):
        tau, om = self.expand(v)
        wphi = [(x, w * self.phi(self.kv, self.j, self.p, x)) for x, w in zip(tau, om)]
        out = [sum(wp * g(x) for x, wp in wphi) - e for g, e in zip(self.tests, self.exact)]
        if self.interior and self.p == 3:
            out.append(self._rel(0, tau[0]) + self._rel(3, tau[3]) - 1)
        return out

    def admissible(self, v):
        tau, om = self.expand(v)
        kv, j, p = self.kv, self.j, self.p
        if self.interior:
            ok = all(kv[j + q] < tau[q] < kv[j + q + 1] for q in range(p + 1))
            if p == 3 and self.kind == "stiffness":
                ok = ok and tau[0] < (kv[j] + kv[j + 1]) / 2
        else:
            lo, hi = kv[j], kv[j + p + 1]
            ok = all(lo < t < hi for t in tau) and all(tau[k] < tau[k + 1] for k in range(len(tau) - 1))
            ok = ok and all(min(abs(t - k) for k in kv) > mp.mpf(10) ** -8 for t in tau)
        return ok and all(w > 0 for w in om)


def _uniform_start(p, kind, j, n, N):
    """The uniform rule of row j in element units, unpadded."""
    if p <= j < n - p:
        tau, om = rules.interior_rule(p, kind)
        return [mp.mpf(j - p) + t for t in tau], list(om)
    if j < p:
        tau, om = rules.boundary_rule(p, kind, j)
        return list(tau), list(om)
    tau, om = rules.boundary_rule(p, kind, n - 1 - j)
    return [mp.mpf(N) - t for t in reversed(tau)], list(reversed(om))


@functools.lru_cache(maxsize=None)
def row_rule(p, breaks, kind, j):
    """Rule of row j on the knots with breakpoints ``breaks`` (tuple of floats), traced
    from the uniform rule.  Returns (nodes, omegas) in element units, padded to Q = p+1
    entries like ``rules.row_rule`` (weight-0 nodes mid-way in the outermost element)."""
    N = len(breaks) - 1
    n = N + p
    row = _Row(p, kind, j, n)
    with mp.workdps(DPS_PATH):
        k0 = _uniform_knot_vector(p, N)
        k1 = knot_vector(p, breaks)
        tau, om = _uniform_start(p, kind, j, n, N)
        v = row.unknowns(tau, om)
        lam, step = mp.mpf(0), mp.mpf(1) / 4
        tol = mp.mpf(10) ** (-(DPS_PATH - 8))
        while lam < 1:
            nxt = min(mp.mpf(1), lam + step)
            row.setup([a + nxt * (b - a) for a, b in zip(k0, k1)])
            w = rules.newton(row.F, v, tol=tol)
            if w is not None and row.admissible(w):
                v, lam = w, nxt
                step = min(step * 2, mp.mpf(1) / 4)
            else:
                step /= 2
                if step < mp.mpf(1) / 4096:
                    raise RuntimeError(f"homotopy lost the rule of row {j} (p={p}, {kind}) at lam={lam}")
    with mp.workdps(DPS):
        row.setup(knot_vector(p, breaks))
        w = rules.newton(row.F, v)
        if w is None or not row.admissible(w):
            raise RuntimeError(f"final polish failed for row {j} (p={p}, {kind})")
        tau, om = row.expand(w)
        kv = row.kv
        pad = (kv[p] + kv[p + 1]) / 2 if j < p else (kv[n - 1] + kv[n]) / 2
        while len(tau) < p + 1:
            tau.append(pad)
            om.append(mp.mpf(0))
        return tau, om


def direction_table(p, breaks, kind):
    """FP64 rule table of one direction with breakpoints ``breaks``: nodes in [0, 1] and
    physical weights (element units over N_el), like ``rules.direction_table``."""
    breaks = tuple(float(b) for b in breaks)
    N = len(breaks) - 1
    xs, ws = [], []
    with mp.workdps(DPS):
        for j in range(N + p):
            tau, om = row_rule(p, breaks, kind, j)
            xs.append([float(t / N) for t in tau])
            ws.append([float(w / N) for w in om])
    return xs, ws


def exactness_residual(p, breaks, kind, j, nodes, omegas):
    """Largest |sum_q omega_q phi_i(x_q) phi_j(x_q) - int phi_i phi_j| over the columns
    interacting with row j (rule in parametric units), relative to the largest exact
    entry; integrals span by span with Gauss-Legendre on the actual knots."""
    N = len(breaks) - 1
    n = N + p
    phi = basis if kind == "mass" else basis_deriv
    with mp.workdps(DPS):
        kv = knot_vector(p, breaks)
        el = [mp.mpf(x) * N for x in nodes]
        om = [mp.mpf(w) * N for w in omegas]
        worst, scale = mp.mpf(0), mp.mpf(0)
        for i in range(max(0, j - p), min(n, j + p + 1)):
            quad = sum(w * phi(kv, i, p, x) * phi(kv, j, p, x) for x, w in zip(el, om))
            exact = _integrate(lambda x: phi(kv, i, p, x) * phi(kv, j, p, x), kv, j, j + p + 1, p + 2)
            worst = max(worst, abs(quad - exact))
            scale = max(scale, abs(exact))
        return float(worst / scale)
